"""The seeded input generators (no GPU): the published configurations, the
parameter scan and the infrared FEL example's loading."""
import math

import numpy as np

from paper_1612_03310_amd import workloads as W


def test_halton_is_the_radical_inverse():
    assert np.allclose(W.halton(np.arange(1, 8), 2), [0.5, 0.25, 0.75, 0.125, 0.625, 0.375, 0.875])
    assert np.allclose(W.halton(np.arange(1, 5), 3), [1 / 3, 2 / 3, 1 / 9, 4 / 9])


def test_tapered_flat_top_puts_the_flat_share_in_the_core():
    """Flat top of length L with half-Gaussian edges of width s at the same
    density: a fraction L / (L + sqrt(2 pi) s) lies in the core, the edges are
    symmetric and their spread is that of a half-Gaussian."""
    L, s = 100.0, 3.0
    u = (np.arange(200000) + 0.5) / 200000
    z = W._tapered_flat_top(u, L, s)
    core = np.abs(z) <= L / 2
    assert abs(core.mean() - L / (L + math.sqrt(2 * math.pi) * s)) < 1e-4
    head = z[z > L / 2] - L / 2
    tail = -L / 2 - z[z < -L / 2]
    assert abs(len(head) - len(tail)) <= 1
    assert abs(np.sqrt(np.mean(head ** 2)) - s) < 0.01 * s
    assert np.all(np.diff(z) >= 0)  # an inverse distribution is monotonic


def test_example1_loading():
    w = W.example1()
    g0 = w.gamma_beam / math.sqrt(1 + w.K ** 2 / 2)
    kb = 2 * g0 * 2 * math.pi / w.lambda_u
    assert w.np == 131072 and w.n == (64, 64, 2800)
    # bunching factor close to the requested 0.01, harmonics 2 and 3 small
    b = [abs(np.exp(1j * h * kb * w.x[:, 2]).mean()) for h in (1, 2, 3)]
    assert abs(b[0] - 0.01) < 5e-4 and b[1] < 1e-3 and b[2] < 1e-3, b
    # every particle inside the safe interior, total charge 29.5 pC
    c = np.floor((w.x - np.array(w.origin)) / np.array(w.d))
    assert np.all(c >= 2) and np.all(c <= np.array(w.n) - 3)
    assert abs(w.q * w.np + 29.5e-12) < 1e-18
    # matched transverse momenta: |u_x| <= K, the lab energy as loaded
    assert np.max(np.abs(w.u[:, 0])) <= w.K * (1 + 1e-12)
    b0 = math.sqrt(1 - 1 / g0 ** 2)
    glab = g0 * (np.sqrt(1 + (w.u ** 2).sum(1)) + b0 * w.u[:, 2])
    assert abs(glab.mean() / w.gamma_beam - 1) < 1e-5 and abs(glab.std() / w.gamma_beam - 1e-4) < 2e-5


def test_configurations_have_the_published_shapes():
    """The tiny, mid and precision workloads: mesh, particle count,
    beam and undulator parameters, bunch widths n/8 cells, every particle
    inside the safe interior and seeded (same inputs on every call)."""
    want = {0: ((32, 32, 64), 4096, 100.0, 1.0, 0.015), 1: ((128, 128, 512), 1 << 20, 100.0, 1.0, 0.015),
            2: ((32, 32, 64), 4096, 100.0, 1.0, 0.015)}
    for idx, (n, npart, gamma, K, lam) in want.items():
        w = W.config(idx)
        assert tuple(w.n) == n and w.np == npart
        assert (w.gamma_beam, w.K, w.lambda_u) == (gamma, K, lam)
        c = np.floor((w.x - np.asarray(w.origin)) / np.asarray(w.d))
        assert np.all(c >= 2) and np.all(c <= np.asarray(n) - 3)
        sig = np.std(c, axis=0)
        assert np.all(np.abs(sig / (np.asarray(n) / 8) - 1) < 0.15), sig
        assert np.array_equal(W.config(idx).x, w.x)


def test_batch_scan_draws_within_the_published_ranges():
    """64 simulations: meshes from 32x32x128 to 96x96x384 (n_z = 4 n_x),
    16K-256K particles, K in [0.8, 2.0], gamma in [80, 250]."""
    ws = W.batch_configs(64, steps=10)
    assert len(ws) == 64
    for w in ws:
        nx, ny, nz = w.n
        assert nx == ny and nz == 4 * nx and 32 <= nx <= 96 and nx % 8 == 0
        assert 16 * 1024 <= w.np <= 256 * 1024
        assert 0.8 <= w.K <= 2.0 and 80.0 <= w.gamma_beam <= 250.0
    assert len({w.n for w in ws}) > 5 and len({w.np for w in ws}) > 30
