"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (any
finding aborts) and its asserts on, run over seeded workloads that exercise
every part of the step: the tiny configuration with the plane spectrum at a
sweep of normalized frequencies, further plates and particles leaving the
mesh; a finite undulator whose exit sweeps through the bunch; second-order
Mur faces; and a periodic box narrower than eight cells.  A planted overrun
shows that the build does catch one."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1612_03310_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "oracle_sanitized_driver.c")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


def _build(tmp_path, src=oracle._SRC, name="drv"):
    exe = str(tmp_path / name)
    cmd = ["gcc", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-Wall",
           "-Wno-unknown-pragmas", *SAN, "-o", exe, src, DRIVER, "-lm"]
    subprocess.check_call(cmd)
    return exe


def _write(path, w, steps, nu=(), und_length=0.0, extra=(-1, -1, -1)):
    head = (list(w.n) + list(w.d) + list(w.origin) + [w.courant, w.nsfd_A, w.substeps,
            w.space_charge] + list(w.bc) + [w.lambda_u, w.K, w.gamma_beam, w.z_e, w.q, w.m,
            len(w.x), steps] + list(w.probe) + [w.kp, und_length, len(nu)] + list(extra))
    assert len(head) == 33
    with open(path, "wb") as f:
        np.asarray(head, dtype=np.float64).tofile(f)
        np.asarray(nu, dtype=np.float64).tofile(f)
        np.ascontiguousarray(w.x, dtype=np.float64).tofile(f)
        np.ascontiguousarray(w.u, dtype=np.float64).tofile(f)


def _run(exe, inp):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(inp)], capture_output=True, text=True, timeout=600, env=env)
    return r


def _cases():
    w0 = W.config(0, n_particles=1500, steps=40)
    x = w0.x.copy()
    x[:20, 2] = w0.origin[2] + (w0.n[2] - 3.2) * w0.d[2]  # near the +z end: lost within the run
    w0.x = x
    w1 = W.config(0, n_particles=800, steps=60)
    g0 = w1.gamma_beam / np.sqrt(1 + w1.K ** 2 / 2)
    zc = g0 * (0.0 - w1.z_e)
    L = (np.floor(zc / w1.lambda_u) + 1) * w1.lambda_u  # the exit passes the bunch
    w2 = W.config(0, n_particles=600, steps=30)
    w2.bc = (2, 2, 2)  # second-order Mur on every face
    w3 = W.make_workload("narrow", (8, 8, 64), 300, 110.0, 1.2, 0.015, 1e-4, 5, 30)
    w3.bc = (1, 1, 0)
    return [("tiny+spectrum", w0, 40, np.arange(0.5, 2.01, 0.25), 0.0, (10, 20, -1)),
            ("finite undulator", w1, 60, (1.0, 2.0, 3.0), L, (-1, -1, -1)),
            ("mur2", w2, 30, (), 0.0, (-1, -1, -1)),
            ("narrow periodic", w3, 30, (1.0,), 0.0, (-1, -1, -1))]


def test_sanitized_oracle_runs_clean(tmp_path):
    exe = _build(tmp_path)
    for name, w, steps, nu, L, extra in _cases():
        inp = tmp_path / ("in_%d.bin" % abs(hash(name)))
        _write(inp, w, steps, nu, L, extra)
        r = _run(exe, inp)
        print(name, r.stdout.strip())
        assert r.returncode == 0, (name, r.stderr[-3000:])
        assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, (name, r.stderr[-3000:])
        step, rows, lost, chk = r.stdout.split()
        assert int(step) == steps and int(rows) == steps and np.isfinite(float(chk)), name


def test_sanitized_build_catches_a_planted_overrun(tmp_path):
    """The field update made to read one plane past the end of the mesh: the
    sanitized build stops with a heap overflow."""
    src = open(oracle._SRC).read()
    anchor = "void orc_field_update(orc_sim *s)\n{"
    assert src.count(anchor) == 1
    planted = src.replace(anchor, anchor + "\n    volatile double probe_past_end = "
                          "s->pot[s->lcur][0][s->ncell]; (void)probe_past_end;")
    p = tmp_path / "planted.c"
    p.write_text(planted)
    exe = _build(tmp_path, str(p), "planted")
    w = W.config(0, n_particles=64, steps=2)
    inp = tmp_path / "in.bin"
    _write(inp, w, 2)
    r = _run(exe, inp)
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr
