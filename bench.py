"""Throughput of the boosted-frame FDTD/PIC step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--extra]

Default workload: the 128x128x512 mesh with 1,048,576 macro-particles in
double precision (the mid configuration).  One step is the whole hot path:
potential update + Mur boundary, gather + undulator + Boris push, binning,
charge-conserving deposition, and the double-precision diagnostics.  Inputs
are synthetic (seeded generator) and resident in HBM before timing starts.

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
    return {"workload": w.name, "particles": w.np, "steps": steps,
            "ms_per_step": round(dt * 1e3 / (steps - 8), 5),
            "gain_length_m": None if lg is None else round(lg, 4),
            "fit_steps": [a, b], "saturation_at_m": round(z_sat, 3),
            "peak_power_rest_frame_W": round(p_sat, 2), "lost": int(dg["lost"][-1]),
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


def measure(w, precision, steps, warmup, torch, native, tune=True, every=100, seed=None):
    """Graph-replayed timed region, then an event-timed region of the same
    length for the per-kernel durations."""
    t_setup = time.perf_counter()
    sim = native.sim_from_workload(w, precision=precision, every=every, spectrum=False)
    if seed is not None:
        sim.set_seed(**seed)
    if tune:
        sim.tune(3)
    sim.run(warmup)
    sim.sync()
    log("  set-up + warm-up %.1f s, tile %s" % (time.perf_counter() - t_setup,
                                                sim.info()["stencil_tile"]))
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


def cpu_baseline(w, steps):
    """The oracle as it stands, single thread, on a bounded sample of the same
    workload (whole steps of the full mesh and bunch; set-up excluded)."""
    import oracle

    sim = oracle.from_workload(w)
    t0 = time.perf_counter()
    sim.step(steps)
    dt = time.perf_counter() - t0
    return {"value": w.ncell * steps / dt, "unit": "cell-updates/s", "cores": 1,
            "kind": "oracle", "particle_pushes_per_s": w.np * steps / dt,
            "sample": "%d full steps of the %dx%dx%d mesh with %d particles (%.1f s, set-up "
                      "excluded), plain C double precision, one thread"
                      % (steps, w.n[0], w.n[1], w.n[2], w.np, dt)}


def large_measurements(wl, kl, torch, native):
    """The large configuration in float split form and the same shape in double."""
    log("large configuration %s, %d particles, f32 split, %d steps" % (wl.n, wl.np, kl))
    dtl, _, perl, dgl, _ = measure(wl, "f32", kl, 5, torch, native)
    log("  %.3f ms/step" % (dtl * 1e3 / kl))
    kl64 = max(10, kl // 4)
    log("same shape in f64, %d steps" % kl64)
    dtl64, _, perl64, _, _ = measure(wl, "f64", kl64, 3, torch, native)
    log("  %.3f ms/step" % (dtl64 * 1e3 / kl64))
    return {"fp32_large": {
        "workload": "large-256x256x2048-16.8M-particles", "precision": "f32 split",
        "steps": kl, "ms_per_step": round(dtl * 1e3 / kl, 4),
        "cell_updates_per_s": wl.ncell * kl / dtl, "particle_pushes_per_s": wl.np * kl / dtl,
        "kernels_ms": {k: round(v, 4) for k, v in perl.items()},
        "stencil_frac_hbm": round(kernel_bytes("stencil", wl, 4) / (perl["stencil"] * 1e-3)
                                  / 1e9 / HBM_PEAK_GBS, 4),
        "push_frac_hbm": round(kernel_bytes("push", wl, 4) / (perl["push"] * 1e-3)
                               / 1e9 / HBM_PEAK_GBS, 4),
        "lost": int(dgl["lost"][-1]), "nonfinite": bool(dgl["nonfinite"].any()),
        "fp64_same_shape_ms_per_step": round(dtl64 * 1e3 / kl64, 4),
        "speedup_fp32_vs_fp64": round((dtl64 / kl64) / (dtl / kl), 3),
    }}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--extra", action="store_true", help="also time the batched scan")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 1 GiB device-to-device 5 times (a kernel of known "
                         "traffic, to scale hardware byte counters)")
    ap.add_argument("--skip-large", action="store_true")
    ap.add_argument("--no-mur2", action="store_true",
                    help="skip the second-order Mur leg (mid configuration, bc code 2)")
    ap.add_argument("--no-seed", action="store_true",
                    help="skip the seeded leg (mid configuration with a TF/SF plane-wave seed)")
    ap.add_argument("--no-example1", action="store_true",
                    help="skip the paper's infrared FEL example (64x64x2800, 131072 "
                         "particles, run to saturation, gain length fitted)")
    ap.add_argument("--workload", choices=("mid", "large"), default="mid",
                    help="headline workload: mid (128x128x512, 1M particles, f64, the "
                         "default) or large (256x256x2048, 16.8M particles, f32 split)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(the z-slab sharding is a design note only); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

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

    # ---- headline: the mid configuration in double precision ----------------
    if args.workload == "mid":
        w, wname, prec, rs = W.config(1), "mid-128x128x512-1M-particles", "f64", 8
    else:
        w, wname, prec, rs = W.config(3), "large-256x256x2048-16.8M-particles", "f32", 4
        args.skip_large = True
    log("%s configuration %s, %d particles, %s, %d steps" % (args.workload, w.n, w.np, prec, K))
    dt, dt_ev, per, dg, info = measure(w, prec, K, Wm, torch, native)
    ms_step = dt * 1e3 / K
    value = w.ncell * K / dt
    pushes = w.np * K * w.substeps / dt
    log("  %.4f ms/step, %.3e cell-updates/s, %.3e pushes/s" % (ms_step, value, pushes))

    nbp = boundary_points(w, info["stencil_tile"][0])
    kernels = {}
    for kind, t in per.items():
        b = kernel_bytes(kind, w, rs, nbp)
        kernels[kind] = {"ms": round(t, 5)}
        if b:
            kernels[kind]["algorithmic_GBs"] = round(b / (t * 1e-3) / 1e9, 1)
            kernels[kind]["frac_hbm"] = round(b / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    dom = max((k for k in per if kernel_bytes(k, w, rs, nbp)), key=lambda k: per[k])
    dom_bytes = kernel_bytes(dom, w, rs, nbp)
    achieved = dom_bytes / (per[dom] * 1e-3) / 1e9
    traffic = traffic_from_profile(dom, args.workload)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "algorithmic_bytes_per_launch": dom_bytes,
                "avg_launch_ms": round(per[dom], 5)}
    step_bytes = sum(kernel_bytes(k, w, rs, nbp) for k in per)

    # ---- the large float configuration and the same shape in double ---------
    out_extra = {}
    if args.workload == "mid" and not args.no_mur2:
        import dataclasses
        w2 = dataclasses.replace(w, bc=(2, 2, 2))
        k2 = max(50, K // 4)
        log("second-order Mur on the mid configuration, %d steps" % k2)
        dt2, _, per2, _, info2 = measure(w2, prec, k2, Wm, torch, native)
        b2 = mur2_boundary_bytes(w2, rs)
        out_extra["mur2_mid"] = {
            "bc": [2, 2, 2], "steps": k2, "ms_per_step": round(dt2 * 1e3 / k2, 5),
            "cell_updates_per_s": w2.ncell * k2 / dt2, "boundary_ms": round(per2["boundary"], 5),
            "boundary_algorithmic_GBs": round(b2 / (per2["boundary"] * 1e-3) / 1e9, 1),
            "boundary_frac_hbm": round(b2 / (per2["boundary"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "kernels_ms": {k: round(v, 5) for k, v in per2.items()}}
        log("  %.4f ms/step, boundary %.4f ms" % (dt2 * 1e3 / k2, per2["boundary"]))
    if args.workload == "mid" and not args.no_seed:
        # a modulated-Gaussian plane wave at the rest-frame resonant
        # wavelength (32 cells), a0 = 0.1, entering through z_min
        c_light, q_e, m_e = 299792458.0, 1.602176634e-19, 9.1093837015e-31
        lam = 32 * w.d[2]
        tau = 40 * w.d[2] / c_light
        seed = dict(amplitude=0.1 * m_e * c_light / q_e, polarization=(1.0, 0.0),
                    frequency=c_light / lam, t0=3 * tau, tau=tau, cep=0.0, signal="gaussian",
                    z_ref=w.origin[2])
        k3 = max(50, K // 4)
        log("seeded mid configuration (TF/SF plane wave), %d steps" % k3)
        dt3, _, per3, dg3, _ = measure(w, prec, k3, Wm, torch, native, seed=seed)
        out_extra["seed_mid"] = {
            "steps": k3, "ms_per_step": round(dt3 * 1e3 / k3, 5),
            "cell_updates_per_s": w.ncell * k3 / dt3, "stencil_ms": round(per3["stencil"], 5),
            "probe_Ex_max": float(np.max(np.abs(dg3["probe_E"][:, 0]))) if len(dg3) else None}
        log("  %.4f ms/step, stencil %.4f ms" % (dt3 * 1e3 / k3, per3["stencil"]))
    if args.workload == "mid" and not args.no_example1:
        log("infrared FEL example: 64x64x2800, 131072 particles, 6000 steps")
        ex = example1_run(6000, torch, native, W)
        out_extra["example1"] = ex
        log("  %.4f ms/step, gain length %s m (1D %.3f, 3D fit %.3f, paper 0.22), "
            "saturation at %.2f m" % (ex["ms_per_step"], ex["gain_length_m"],
                                       ex["gain_length_1d_m"], ex["gain_length_3d_xie_m"],
                                       ex["saturation_at_m"]))
    wl = None if args.skip_large else W.config(3)
    kl = max(20, min(200, K // 10))
    if wl is not None:
        out_extra.update(large_measurements(wl, kl, torch, native))

    if args.extra:
        log("batched scan: 64 simulations")
        ws = W.batch_configs(64, steps=100)
        b = native.batch_from_workloads(ws, precision="f32", every=100, spectrum=False)
        b.tune(2)
        b.run(8)
        b.sync()
        nb = 100
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run(nb)
        b.sync()
        dtb = time.perf_counter() - t0
        b.close()
        seq = 0.0
        for i, wi in enumerate(ws):
            s = native.sim_from_workload(wi, precision="f32", every=100, spectrum=False)
            s.run(8)
            s.sync()
            seq += timed_run(s, nb, torch)
            s.close()
        cells = sum(x.ncell for x in ws)
        out_extra["batch"] = {"simulations": 64, "steps": nb, "batched_s": round(dtb, 4),
                              "sequential_s": round(seq, 4), "speedup": round(seq / dtb, 3),
                              "cell_updates_per_s": cells * nb / dtb}

    cpu = None
    if not args.no_cpu and args.workload == "mid":  # a large step takes minutes on one core
        log("cpu baseline: oracle, %d steps of the mid configuration" % args.cpu_steps)
        cpu = cpu_baseline(w, args.cpu_steps)
        log("  %.3e cell-updates/s" % cpu["value"])

    line = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": K,
        "warmup": Wm, "ms_per_step": round(ms_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {"workload": wname, "mesh": list(w.n), "particles": w.np,
                   "precision": prec, "courant": w.courant, "nsfd_A": info["nsfd_A"],
                   "substeps": w.substeps, "space_charge": w.space_charge,
                   "gamma": w.gamma_beam, "K": w.K, "lambda_u": w.lambda_u,
                   "mesh_diag_every": 100, "stencil_tile": info["stencil_tile"]},
        "particle_pushes_per_s": pushes,
        "whole_step_algorithmic_GBs": round(step_bytes / (ms_step * 1e-3) / 1e9, 1),
        "roofline": roofline,
        "kernels": kernels,
        "event_region_ms_per_step": round(dt_ev * 1e3 / K, 5),
        "lost": int(dg["lost"][-1]) if len(dg) else 0,
        "cpu_baseline": cpu,
    }
    line.update(out_extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
