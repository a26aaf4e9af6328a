"""Throughput of the boosted-frame FDTD/PIC step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W]

Headline workload: the 256x256x2048 mesh with 16,777,216 macro-particles in
the float split form (float fields and push, int32 cell + float offset
positions, double-precision reductions), the largest configuration.  One
step is the whole hot path: potential update + Mur boundary, gather +
undulator + Boris push, binning, charge-conserving deposition, and the
double-precision diagnostics.  Inputs are synthetic (seeded generator) and
resident in HBM before timing starts.  Also timed by default: the same shape
in double precision (speedup, and the float form's error against it), the
64-simulation parameter scan against 64 sequential runs, the mid
configuration (128x128x512, double) with its variants, and the CPU oracle on
a slab of the headline workload, on one thread and on all threads.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s + particle-pushes/s per step, FP32 vs FP64, % of HBM BW"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(kind, w, rs, nb_points=0):
    """Algorithmic HBM bytes of one launch (each state array moved once)."""
    ncell, npart = w.ncell, w.np
    ncomp = 4 if w.space_charge else 3
    if kind == "stencil":  # read psi^s, psi^{s-1}, source; write psi^{s+1}
        return 4 * rs * ncomp * ncell
    if kind == "push":  # key, offset, momentum in and out; start record out
        return npart * (4 + 6 * rs + 4 + 6 * rs + 4 + 3 * rs)
    if kind == "deposit":  # both positions in; J and rho written at every cell
        return npart * (8 + 6 * rs) + ncell * 4 * rs
    if kind == "scan":  # counts read twice, starts written
        nkeys = 1
        for a in range(3):
            nkeys *= (w.n[a] + 7) // 8
        return nkeys * 512 * 12
    if kind == "scatter":  # key, id, offset, momentum moved
        return 2 * npart * (8 + 6 * rs)
    if kind == "boundary":  # six reads and one write per boundary point
        return nb_points * 7 * rs
    return 0


def x_faces_in_stencil(w, tile_x):
    """The library's rule: the stencil pass updates the x faces when no high
    x face column falls on the first lane of a wavefront (all axes Mur here)."""
    comps = 4 if w.space_charge else 3
    return tile_x >= 2 and all((w.n[0] - (1 if c == 0 else 0) - 1) % tile_x % 64 != 0
                               for c in range(comps))


def boundary_points(w, tile_x=None):
    """Points the boundary kernel updates: every face, edge and corner point of
    each component grid, less the x faces (y, z inside) when the stencil pass
    takes them."""
    tot = 0
    comps = 4 if w.space_charge else 3
    fused = tile_x is not None and x_faces_in_stencil(w, tile_x)
    for c in range(comps):
        ext = [w.n[a] - (1 if c == a else 0) for a in range(3)]
        tot += ext[0] * ext[1] * ext[2] - (ext[0] - 2) * (ext[1] - 2) * (ext[2] - 2)
        if fused:
            tot -= 2 * (ext[1] - 2) * (ext[2] - 2)
    return tot


def mur2_boundary_bytes(w, rs):
    """Algorithmic bytes of the second-order Mur launches per step: a face
    point reads 13 values (psi^{s-1}, psi^s of itself and its inward
    neighbour, psi^{s+1} of the neighbour, psi^s of the four transverse
    neighbours of both) and writes one; an edge point 20 + 1; a corner 24 + 1."""
    comps = 4 if w.space_charge else 3
    faces = edges = corners = 0
    for c in range(comps):
        ext = [w.n[a] - (1 if c == a else 0) for a in range(3)]
        ni = [e - 2 for e in ext]
        for a in range(3):
            u, v = [t for t in range(3) if t != a]
            faces += 2 * ni[u] * ni[v]
            edges += 4 * ni[a]
        corners += 8
    return (14 * faces + 21 * edges + 25 * corners) * rs


def source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "mithra_internal.hpp"):
        with open(os.path.join(ROOT, "paper_1612_03310_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kind, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when there is none or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "%s_%s_traffic.txt" % (kind, workload))
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def gain_length(power, dz_step, smooth=60, lo=0.02, hi=0.4):
    """Power gain length from a per-step power series: the power is smoothed
    over `smooth` steps (about one rest-frame radiation period), and ln P is
    fitted by a line over the samples before the saturation peak whose power
    lies between lo and hi of the peak.  Returns (gain length [m], undulator
    distance of the peak [m], peak power, first and last fitted step)."""
    Ps = np.convolve(power, np.ones(smooth) / smooth, mode="valid")
    i_sat = int(np.argmax(Ps))
    peak = float(Ps[i_sat])
    sel = np.nonzero((Ps[:i_sat] > lo * peak) & (Ps[:i_sat] < hi * peak))[0]
    if len(sel) < 2:
        return None, (i_sat + smooth // 2) * dz_step, peak, None, None
    slope = np.polyfit(sel, np.log(Ps[sel]), 1)[0]
    return dz_step / slope, (i_sat + smooth // 2) * dz_step, peak, int(sel[0]), int(sel[-1])


def fel_theory(gamma, K, lambda_u, sigma_x, current, sigma_delta):
    """One-dimensional FEL parameter and power gain length of a round Gaussian
    beam (peak current, rms radius), and the three-dimensional gain length
    from M. Xie's published fit (zero emittance).  Not from the paper: a
    textbook yardstick for the example's growth."""
    from scipy.special import j0, j1
    ia = 17045.0  # Alfven current [A]
    xi = K * K / (4 + 2 * K * K)
    jj = j0(xi) - j1(xi)
    ku = 2 * np.pi / lambda_u
    rho = ((current / ia) * (K * jj) ** 2 / (16 * gamma ** 3 * sigma_x ** 2 * ku ** 2)) ** (1 / 3)
    l1 = lambda_u / (4 * np.pi * np.sqrt(3) * rho)
    kr = 2 * np.pi / (lambda_u * (1 + K * K / 2) / (2 * gamma ** 2))
    ed, eg = l1 / (2 * kr * sigma_x ** 2), 4 * np.pi * (l1 / lambda_u) * sigma_delta
    # the terms of the fit without emittance: diffraction, energy spread, both
    lam = 0.45 * ed ** 0.57 + 3 * eg ** 2 + 51 * ed ** 0.95 * eg ** 3
    return float(rho), float(l1), float(l1 * (1 + lam))


def example1_run(steps, torch, native, W):
    """The paper's infrared FEL example (job-file reading), run to saturation;
    returns timing, the fitted gain length and the yardsticks."""
    w = W.example1(steps=steps)
    sim = native.sim_from_workload(w, precision="f64", every=100, capacity=steps + 8,
                                   spectrum=False)
    sim.run(8)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(steps - 8)
    sim.sync()
    dt = time.perf_counter() - t0
    dg = sim.get_diag()
    info = sim.info()
    sim.close()
    dz_step = info["gamma0"] * info["beta0"] * 299792458.0 * info["dt"]
    lg, z_sat, p_sat, a, b = gain_length(dg["power"], dz_step)
    rho, l1, l3 = fel_theory(w.gamma_beam, w.K, w.lambda_u, 260e-6, 88.5, 1e-4)
    # lab-frame power through the plate, smoothed like the rest-frame one; the
    # one-dimensional saturation estimate rho * P_beam (beam power: the
    # electrons' energy times the current) and M. Xie's three-dimensional one,
    # 1.6 rho (L_1D / L_G)^2 P_beam with the fitted gain length
    lab = np.convolve(dg["power_lab"], np.ones(60) / 60, mode="valid")
    p_beam = (w.gamma_beam * 0.51099895e6) * 88.5
    p_3d = 1.6 * rho * (l1 / lg) ** 2 * p_beam if lg else None
    return {"workload": w.name, "particles": w.np, "steps": steps,
            "ms_per_step": round(dt * 1e3 / (steps - 8), 5),
            "gain_length_m": None if lg is None else round(lg, 4),
            "fit_steps": [a, b], "saturation_at_m": round(z_sat, 3),
            "peak_power_rest_frame_W": round(p_sat, 2),
            "peak_power_lab_W": float("%.4g" % lab.max()),
            "saturation_power_1d_W": float("%.4g" % (rho * p_beam)),
            "saturation_power_3d_W": None if p_3d is None else float("%.4g" % p_3d),
            "lost": int(dg["lost"][-1]),
            "bunching_max": round(float(dg["bunching"][:, 0].max()), 4),
            "rho_1d": round(rho, 5), "gain_length_1d_m": round(l1, 4),
            "gain_length_3d_xie_m": round(l3, 4), "gain_length_paper_m": 0.22}


def timed_run(sim, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(steps)
    sim.sync()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def measure(w, precision, steps, warmup, torch, native, tune=True, every=100, seed=None,
            shapes=None):
    """Graph-replayed timed region, then an event-timed region of the same
    length for the per-kernel durations.  The library captures its step graph
    on the first run, so the warm-up run builds it before timing starts.
    shapes: (stencil tile, particle brick) set instead of tuning."""
    t_setup = time.perf_counter()
    sim = native.sim_from_workload(w, precision=precision, every=every, spectrum=False,
                                   capacity=2 * steps + warmup + 8)
    if seed is not None:
        sim.set_seed(**seed)
    if shapes is not None:
        sim.set_shapes(*shapes)
    elif tune:
        sim.tune(3)
    sim.run(max(warmup, 1))
    sim.sync()
    log("  set-up + warm-up %.1f s, tile %s, brick %s" % (
        time.perf_counter() - t_setup, sim.info()["stencil_tile"], sim.info()["particle_brick"]))
    dt = timed_run(sim, steps, torch)
    sim.set_timing(True)
    sim.get_timing(reset=True)
    dt_ev = timed_run(sim, steps, torch)
    ms, calls = sim.get_timing(reset=True)
    sim.set_timing(False)
    dg = sim.get_diag()
    info = sim.info()
    sim.close()
    per_launch = {k: ms[k] / calls[k] for k in ms if calls[k] > 0}
    return dt, dt_ev, per_launch, dg, info


def occupied_tiles(w):
    """8x8x8-cell tiles holding at least one particle of the workload (the
    tiles whose potentials the push reads)."""
    c = np.floor((w.x - np.asarray(w.origin)) / np.asarray(w.d)).astype(np.int64) // 8
    nt = [(w.n[a] + 7) // 8 for a in range(3)]
    return int(np.unique((c[:, 2] * nt[1] + c[:, 1]) * nt[0] + c[:, 0]).size)


def roofline_block(kind, t_ms, nbytes, traffic=None, **extra):
    achieved = nbytes / (t_ms * 1e-3) / 1e9
    out = {"bound": "hbm", "kernel": kind, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
           "algorithmic_bytes_per_launch": int(nbytes), "avg_launch_ms": round(t_ms, 5)}
    out.update(extra)
    return out


def kernels_table(per, w, rs, nbp):
    out = {}
    for kind, t in per.items():
        b = kernel_bytes(kind, w, rs, nbp)
        out[kind] = {"ms": round(t, 5)}
        if b:
            out[kind]["algorithmic_GBs"] = round(b / (t * 1e-3) / 1e9, 1)
            out[kind]["frac_hbm"] = round(b / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return out


def push_roofline(per, w, rs, tiles, profile_name):
    """The push against HBM: particle bytes plus the potentials of the
    occupied tiles it gathers from (A^s, A^{s+1}, phi: 7 values per cell)."""
    part = kernel_bytes("push", w, rs)
    gather = tiles * 512 * 7 * rs
    t = per["push"]
    return roofline_block("push", t, part + gather, traffic_from_profile("push", profile_name),
                          particle_bytes=int(part), gather_bytes=int(gather),
                          occupied_tiles=tiles,
                          frac_particle_bytes_only=round(part / (t * 1e-3) / 1e9
                                                         / HBM_PEAK_GBS, 4))


def rel_l2(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def slab_of(w, planes):
    """A bounded sample of a workload for the CPU baseline: the full
    transverse mesh over `planes` z-planes at the bunch centre, with every
    k-th of the particles inside them so that the sample holds as many
    particles per cell as the whole job (its cell-updates/s then stand for
    the whole job's)."""
    import dataclasses
    k0 = (w.n[2] - planes) // 2
    z0 = w.origin[2] + k0 * w.d[2]
    zc = (w.x[:, 2] - z0) / w.d[2]
    sel = np.nonzero((zc >= 3.0) & (zc < planes - 4.0))[0]
    want = w.np * (w.n[0] * w.n[1] * planes) / w.ncell
    sel = sel[::max(1, int(round(len(sel) / want)))]
    n = (w.n[0], w.n[1], planes)
    kp = planes // 2
    return dataclasses.replace(w, name=w.name + "-slab", n=n,
                               origin=(w.origin[0], w.origin[1], z0), x=w.x[sel].copy(),
                               u=w.u[sel].copy(), probe=(n[0] // 2, n[1] // 2, kp), kp=kp)


def cpu_baseline(w, planes, steps_1t, steps_all):
    """The oracle as it stands on a bounded sample of the headline workload:
    one thread (the plain build), then every host thread (the OpenMP build of
    the same source, which parallelises the loops over disjoint points and
    particles and keeps every sum sequential).  Set-up excluded."""
    import oracle

    ws = slab_of(w, planes)
    res = {}
    for par, steps in ((False, steps_1t), (True, steps_all)):
        sim = oracle.from_workload(ws, parallel=par)
        t0 = time.perf_counter()
        sim.step(steps)
        dt = time.perf_counter() - t0
        res[par] = (ws.ncell * steps / dt, ws.np * steps * ws.substeps / dt, dt, steps)
        del sim
    nthreads = oracle.threads(True)
    cu, pp, dt, st = res[True]
    cu1, pp1, dt1, st1 = res[False]
    return {"value": cu, "unit": "cell-updates/s", "cores": nthreads, "kind": "oracle",
            "particle_pushes_per_s": pp, "cpu_model": cpu_model(),
            "single_thread": {"value": cu1, "unit": "cell-updates/s", "cores": 1,
                              "particle_pushes_per_s": pp1, "seconds": round(dt1, 2),
                              "steps": st1},
            "sample": "%d and %d full steps (one thread, %d threads) of a %dx%dx%d slab at the "
                      "bunch centre of the %s workload with %d of its particles (the whole "
                      "job's particles per cell; %.1f s and %.1f s, set-up excluded), plain C "
                      "double precision"
                      % (st1, st, nthreads, ws.n[0], ws.n[1], ws.n[2], w.name, ws.np, dt1, dt)}


def batch_leg(nb, torch, native, W):
    """The parameter scan: 64 simulations of uneven meshes and bunches in one
    graph-replayed batch against the same 64 run one after another."""
    ws = W.batch_configs(64, steps=nb)
    b = native.batch_from_workloads(ws, precision="f32", every=100, spectrum=False,
                                    capacity=nb + 16)
    b.tune(2)
    b.run(8)
    b.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(nb)
    b.sync()
    dtb = time.perf_counter() - t0
    b.close()
    seq = 0.0
    for wi in ws:
        s = native.sim_from_workload(wi, precision="f32", every=100, spectrum=False,
                                     capacity=nb + 16)
        s.run(8)
        s.sync()
        seq += timed_run(s, nb, torch)
        s.close()
    cells = sum(x.ncell for x in ws)
    parts = sum(x.np for x in ws)
    return {"workload": "scan-64-sims-32..96x32..96x128..384", "simulations": 64,
            "precision": "f32 split", "steps": nb, "cells": cells, "particles": parts,
            "batched_s": round(dtb, 4), "sequential_s": round(seq, 4),
            "speedup": round(seq / dtb, 3), "cell_updates_per_s": cells * nb / dtb,
            "particle_pushes_per_s": parts * nb / dtb,
            "sequential_cell_updates_per_s": cells * nb / seq}


def mid_legs(args, K, Wm, torch, native, W):
    """The mid configuration in double precision and its variants (second-order
    Mur, a TF/SF seed) and the paper's infrared FEL example."""
    import dataclasses
    out = {}
    w = W.config(1)
    km = max(50, K)
    log("mid configuration %s, %d particles, f64, %d steps" % (w.n, w.np, km))
    dt, dt_ev, per, dg, info = measure(w, "f64", km, Wm, torch, native)
    nbp = boundary_points(w, info["stencil_tile"][0])
    t_st = per["stencil"]
    out["mid_f64"] = {
        "workload": "mid-128x128x512-1M-particles", "precision": "f64", "steps": km,
        "ms_per_step": round(dt * 1e3 / km, 5),
        "event_region_ms_per_step": round(dt_ev * 1e3 / km, 5),
        "cell_updates_per_s": w.ncell * km / dt, "particle_pushes_per_s": w.np * km / dt,
        "kernels": kernels_table(per, w, 8, nbp),
        "roofline_stencil": roofline_block("stencil", t_st, kernel_bytes("stencil", w, 8),
                                           traffic_from_profile("stencil", "mid"))}
    log("  %.4f ms/step" % (dt * 1e3 / km))
    if not args.no_mur2:
        w2 = dataclasses.replace(w, bc=(2, 2, 2))
        log("second-order Mur on the mid configuration, %d steps" % km)
        dt2, _, per2, _, _ = measure(w2, "f64", km, Wm, torch, native)
        b2 = mur2_boundary_bytes(w2, 8)
        out["mur2_mid"] = {
            "bc": [2, 2, 2], "steps": km, "ms_per_step": round(dt2 * 1e3 / km, 5),
            "cell_updates_per_s": w2.ncell * km / dt2, "boundary_ms": round(per2["boundary"], 5),
            "boundary_algorithmic_GBs": round(b2 / (per2["boundary"] * 1e-3) / 1e9, 1),
            "boundary_frac_hbm": round(b2 / (per2["boundary"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "kernels_ms": {k: round(v, 5) for k, v in per2.items()}}
        log("  %.4f ms/step, boundary %.4f ms" % (dt2 * 1e3 / km, per2["boundary"]))
    if not args.no_seed:
        # a modulated-Gaussian plane wave at the rest-frame resonant
        # wavelength (32 cells), a0 = 0.1, entering through z_min
        c_light, q_e, m_e = 299792458.0, 1.602176634e-19, 9.1093837015e-31
        lam = 32 * w.d[2]
        tau = 40 * w.d[2] / c_light
        seed = dict(amplitude=0.1 * m_e * c_light / q_e, polarization=(1.0, 0.0),
                    frequency=c_light / lam, t0=3 * tau, tau=tau, cep=0.0, signal="gaussian",
                    z_ref=w.origin[2])
        log("seeded mid configuration (TF/SF plane wave), %d steps" % km)
        dt3, _, per3, dg3, _ = measure(w, "f64", km, Wm, torch, native, seed=seed)
        out["seed_mid"] = {
            "steps": km, "ms_per_step": round(dt3 * 1e3 / km, 5),
            "cell_updates_per_s": w.ncell * km / dt3, "stencil_ms": round(per3["stencil"], 5),
            "probe_Ex_max": float(np.max(np.abs(dg3["probe_E"][:, 0]))) if len(dg3) else None}
        log("  %.4f ms/step, stencil %.4f ms" % (dt3 * 1e3 / km, per3["stencil"]))
    if not args.no_example1:
        log("infrared FEL example: 64x64x2800, 131072 particles, 6000 steps")
        ex = example1_run(6000, torch, native, W)
        out["example1"] = ex
        log("  %.4f ms/step, gain length %s m (1D %.3f, 3D fit %.3f, paper 0.22), "
            "saturation at %.2f m" % (ex["ms_per_step"], ex["gain_length_m"],
                                       ex["gain_length_1d_m"], ex["gain_length_3d_xie_m"],
                                       ex["saturation_at_m"]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-planes", type=int, default=64,
                    help="z-planes of the large mesh in the CPU baseline's sample")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 1 GiB device-to-device 5 times (a kernel of known "
                         "traffic, to scale hardware byte counters)")
    ap.add_argument("--no-f64", action="store_true",
                    help="skip the same shape in double precision")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-simulation scan against 64 sequential runs")
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--no-mid", action="store_true",
                    help="skip the mid configuration (128x128x512, f64) and its variants")
    ap.add_argument("--no-mur2", action="store_true",
                    help="skip the second-order Mur leg (mid configuration, bc code 2)")
    ap.add_argument("--no-seed", action="store_true",
                    help="skip the seeded leg (mid configuration with a TF/SF plane-wave seed)")
    ap.add_argument("--no-example1", action="store_true",
                    help="skip the paper's infrared FEL example (64x64x2800, 131072 "
                         "particles, run to saturation, gain length fitted)")
    ap.add_argument("--only-headline", action="store_true",
                    help="time the headline workload only (for profiling runs)")
    ap.add_argument("--profile-leg", choices=("large", "large-f64", "mid"),
                    help="run only this workload's timed regions (for counter runs under "
                         "rocprofv3, with --copy-probe for the counter scale); prints no "
                         "JSON line")
    ap.add_argument("--shapes", metavar="TX,TY,KZ,BX,BY,BZ",
                    help="with --profile-leg: set this stencil tile and particle brick "
                         "instead of tuning (the tuner's timings mean little under a "
                         "profiler that serializes kernels)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(the z-slab sharding is a design note only); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if args.only_headline:
        args.no_f64 = args.no_batch = args.no_mid = args.no_cpu = True

    import torch

    from paper_1612_03310_amd import native
    from paper_1612_03310_amd import workloads as W

    torch.cuda.set_device(0)
    K, Wm = args.steps, args.warmup
    if args.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: 5 x 1 GiB read + 1 GiB written")
        del src, dst

    if args.profile_leg:
        wl = W.config(1) if args.profile_leg == "mid" else W.config(3)
        prec = "f32" if args.profile_leg == "large" else "f64"
        log("profile leg %s: %s, %d particles, %s, %d steps" % (args.profile_leg, wl.n, wl.np,
                                                               prec, K))
        shapes = None
        if args.shapes:
            v = [int(x) for x in args.shapes.split(",")]
            if len(v) != 6:
                ap.error("--shapes takes six integers: TX,TY,KZ,BX,BY,BZ")
            shapes = (v[:3], v[3:])
        dtp, _, perp, _, infop = measure(wl, prec, K, Wm, torch, native, shapes=shapes)
        log("  %.4f ms/step, tile %s, brick %s, kernels %s" % (
            dtp * 1e3 / K, infop["stencil_tile"], infop["particle_brick"],
            {k: round(v, 4) for k, v in perp.items()}))
        return

    # ---- headline: the large configuration, float split form -----------------
    w = W.config(3)
    wname = "large-256x256x2048-16.8M-particles"
    log("large configuration %s, %d particles, f32 split, %d steps" % (w.n, w.np, K))
    dt, dt_ev, per, dg, info = measure(w, "f32", K, Wm, torch, native)
    ms_step = dt * 1e3 / K
    value = w.ncell * K / dt
    pushes = w.np * K * w.substeps / dt
    log("  %.4f ms/step (event-timed %.4f), %.3e cell-updates/s, %.3e pushes/s"
        % (ms_step, dt_ev * 1e3 / K, value, pushes))
    tiles = occupied_tiles(w)
    nbp = boundary_points(w, info["stencil_tile"][0])
    kernels = kernels_table(per, w, 4, nbp)
    roofline = roofline_block("stencil", per["stencil"], kernel_bytes("stencil", w, 4),
                              traffic_from_profile("stencil", "large"))
    roof_push = push_roofline(per, w, 4, tiles, "large")
    step_bytes = sum(kernel_bytes(k, w, 4, nbp) for k in per)

    out_extra = {}
    if not args.no_f64:
        log("same shape in f64, %d steps" % K)
        dt64, dt64_ev, per64, dg64, info64 = measure(w, "f64", K, Wm, torch, native)
        nbp64 = boundary_points(w, info64["stencil_tile"][0])
        n = min(len(dg), len(dg64))
        acc = {"rows": n,
               "probe_Ex_rel_l2": rel_l2(dg["probe_E"][:n, 0], dg64["probe_E"][:n, 0]),
               "power_rel_l2": rel_l2(dg["power"][:n], dg64["power"][:n])}
        out_extra["fp64_same_shape"] = {
            "workload": wname, "dtype": "f64", "steps": K,
            "ms_per_step": round(dt64 * 1e3 / K, 5),
            "event_region_ms_per_step": round(dt64_ev * 1e3 / K, 5),
            "cell_updates_per_s": w.ncell * K / dt64,
            "particle_pushes_per_s": w.np * K * w.substeps / dt64,
            "kernels": kernels_table(per64, w, 8, nbp64),
            "roofline": roofline_block("stencil", per64["stencil"],
                                       kernel_bytes("stencil", w, 8),
                                       traffic_from_profile("stencil", "large-f64")),
            "roofline_push": push_roofline(per64, w, 8, tiles, "large-f64")}
        out_extra["speedup_fp32_vs_fp64"] = round(dt64 / dt, 3)
        out_extra["fp32_vs_fp64_accuracy"] = acc
        log("  %.4f ms/step; f32 against f64 over %d rows: probe Ex %.2e, power %.2e"
            % (dt64 * 1e3 / K, n, acc["probe_Ex_rel_l2"], acc["power_rel_l2"]))
    if not args.no_batch:
        log("batched scan: 64 simulations, %d steps, against 64 sequential runs"
            % args.batch_steps)
        out_extra["batch"] = batch_leg(args.batch_steps, torch, native, W)
        log("  batched %.3f s, sequential %.3f s" % (out_extra["batch"]["batched_s"],
                                                     out_extra["batch"]["sequential_s"]))
    if not args.no_mid:
        out_extra.update(mid_legs(args, K, Wm, torch, native, W))

    cpu = None
    if not args.no_cpu:
        log("cpu baseline: oracle on a %d-plane slab of the large configuration"
            % args.cpu_planes)
        cpu = cpu_baseline(w, args.cpu_planes, 3, 6)
        log("  %.3e cell-updates/s on %d threads, %.3e on one" % (
            cpu["value"], cpu["cores"], cpu["single_thread"]["value"]))

    line = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": K,
        "warmup": Wm, "ms_per_step": round(ms_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wname, "mesh": list(w.n), "particles": w.np,
                   "precision": "f32 split (int32 cell + f32 offset, f64 reductions)",
                   "courant": w.courant, "nsfd_A": info["nsfd_A"], "substeps": w.substeps,
                   "space_charge": w.space_charge, "gamma": w.gamma_beam, "K": w.K,
                   "lambda_u": w.lambda_u, "mesh_diag_every": 100,
                   "stencil_tile": info["stencil_tile"],
                   "particle_brick": info["particle_brick"]},
        "particle_pushes_per_s": pushes,
        "event_region_ms_per_step": round(dt_ev * 1e3 / K, 5),
        "whole_step_algorithmic_GBs": round(step_bytes / (ms_step * 1e-3) / 1e9, 1),
        "roofline": roofline,
        "roofline_push": roof_push,
        "kernels": kernels,
        "lost": int(dg["lost"][-1]) if len(dg) else 0,
        "nonfinite": bool(dg["nonfinite"].any()) if len(dg) else False,
        "cpu_baseline": cpu,
    }
    line.update(out_extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
