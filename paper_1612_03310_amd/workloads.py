"""Seeded synthetic workloads: meshes and electron bunches in the bunch rest frame.

This module only builds inputs.  It holds no step of the time-marching method
and imports neither the GPU library nor the CPU oracle, so both can be fed
from it.

Recipe (the paper prints no performance workload, so the shapes follow its
examples and the published configuration list):

* the frame moves with the mean longitudinal velocity of the bunch in the
  undulator, gamma0 = gamma / sqrt(1 + K^2 / 2) (section "Lorentz
  Transformation");
* the longitudinal cell is dz = lambda_u / (gamma0 * n_lambda), i.e.
  n_lambda cells per rest-frame undulator period (= per rest-frame
  radiation wavelength); the transverse cells are ``aspect`` times larger,
  which keeps (dz/dx)^2 + (dz/dy)^2 < 1 as the NSFD scheme requires;
* the mesh is centred on the undulator axis: x = y = z = 0 at its centre;
* guiding centres: independent Gaussian per axis with sigma = n_d / 8
  cells, truncated at 3 sigma by re-drawing (numpy PCG64, seeded);
* lab energy gamma' = gamma * (1 + sigma_delta * N(0, 1)); momenta matched to
  the undulator at the particle's lab phase, u'_x = -K cos(k_u z'),
  u'_y = 0, u'_z from gamma', then boosted to the rest frame, taken at the
  leapfrog's time level of u (half a particle sub-step before the positions,
  which belong to dt/2);
* each particle sits at its guiding centre plus its wiggle offset,
  x = x_c - K / (gamma0 k_u sqrt(1 + K^2/2)) sin(k_u z'), so that its
  transverse oscillation is centred on x_c (a particle started at its
  centre would swing up to twice the amplitude to one side);
* the undulator entrance z_e lies one cell behind the mesh, so every
  particle starts inside the periodic field.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

# CODATA 2018
C_LIGHT = 299792458.0
Q_E = 1.602176634e-19
M_E = 9.1093837015e-31

BASE_SEED = 1612033100
BUNCH_CHARGE = 29.5e-12  # C, the bunch charge of the paper's infrared example


@dataclasses.dataclass
class Workload:
    name: str
    n: Tuple[int, int, int]
    d: Tuple[float, float, float]
    origin: Tuple[float, float, float]
    courant: float
    nsfd_A: float
    substeps: int
    space_charge: int
    bc: Tuple[int, int, int]
    lambda_u: float
    K: float
    gamma_beam: float
    z_e: float
    x: np.ndarray  # (np, 3) rest-frame positions [m]
    u: np.ndarray  # (np, 3) gamma * beta
    q: float  # macro-particle charge [C]
    m: float  # macro-particle mass [kg]
    probe: Tuple[int, int, int]
    kp: int
    steps: int
    und_length: float = 0.0  # lab length of the undulator [m], whole periods; 0: unbounded

    @property
    def ncell(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def np(self) -> int:
        return int(self.x.shape[0])


def _truncated_normal(rng: np.random.Generator, size: int, cut: float) -> np.ndarray:
    out = rng.standard_normal(size)
    bad = np.abs(out) > cut
    while bad.any():
        out[bad] = rng.standard_normal(int(bad.sum()))
        bad = np.abs(out) > cut
    return out


def _matched(x, gp, gamma0, beta0, K, ku, z_e, dt, substeps):
    """Momenta matched to the undulator, u'_x = -K cos(k_u z'), u'_y = 0,
    u'_z from the lab energy gp, boosted to the rest frame, at the leapfrog's
    time level of u: the positions x belong to t = dt/2 and the momenta to
    half a particle sub-step before, so the lab phase is taken at that time
    and at the particle's position then.  Also returns the x positions moved
    by the wiggle offset at the positions' own phase, so that the transverse
    oscillation is centred on the input x (a particle started at its centre
    would swing up to twice the amplitude to one side)."""
    t_u = 0.5 * dt - 0.5 * dt / substeps
    zu = x[:, 2].copy()
    for _ in range(8):
        zlab = gamma0 * (zu - z_e + beta0 * C_LIGHT * t_u)
        uxp = -K * np.cos(ku * zlab)
        uzp = np.sqrt(gp * gp - 1.0 - uxp * uxp)
        uz = gamma0 * (uzp - beta0 * gp)  # boost of the 4-momentum along z
        gr = np.sqrt(1.0 + uxp * uxp + uz * uz)
        zu = x[:, 2] - (0.5 * dt - t_u) * C_LIGHT * uz / gr
    zx = gamma0 * (x[:, 2] - z_e + beta0 * C_LIGHT * 0.5 * dt)
    u = np.zeros((len(gp), 3))
    u[:, 0] = uxp
    u[:, 2] = uz
    x0 = x[:, 0] - K / (gamma0 * ku * math.sqrt(1.0 + K * K / 2.0)) * np.sin(ku * zx)
    return u, x0


def make_workload(name: str, n, n_particles: int, gamma: float, K: float, lambda_u: float,
                  sigma_delta: float, seed: int, steps: int, *, n_lambda: int = 32,
                  aspect: float = 4.0, courant: float = 0.9, sigma_cells=None,
                  substeps: int = 1, space_charge: int = 1, bc=(0, 0, 0),
                  charge: float = BUNCH_CHARGE, cut: float = 3.0) -> Workload:
    n = tuple(int(v) for v in n)
    gamma0 = gamma / math.sqrt(1.0 + K * K / 2.0)
    beta0 = math.sqrt(1.0 - 1.0 / (gamma0 * gamma0))
    dz = lambda_u / (gamma0 * n_lambda)
    d = (aspect * dz, aspect * dz, dz)
    origin = tuple(-(n[a] - 1) / 2.0 * d[a] for a in range(3))
    z_e = origin[2] - d[2]
    if sigma_cells is None:
        sigma_cells = tuple(n[a] / 8.0 for a in range(3))
    rng = np.random.Generator(np.random.PCG64(seed))
    x = np.empty((n_particles, 3))
    for a in range(3):
        x[:, a] = _truncated_normal(rng, n_particles, cut) * sigma_cells[a] * d[a]
    ku = 2.0 * math.pi / lambda_u
    gp = gamma * (1.0 + sigma_delta * rng.standard_normal(n_particles))
    u, x[:, 0] = _matched(x, gp, gamma0, beta0, K, ku, z_e, courant * d[2] / C_LIGHT, substeps)
    q = -charge / n_particles
    m = M_E * (charge / Q_E) / n_particles
    kp = int(round(0.893 * n[2]))
    kp = min(max(kp, 1), n[2] - 2)
    probe = (n[0] // 2, n[1] // 2, kp)
    return Workload(name=name, n=n, d=d, origin=origin, courant=courant, nsfd_A=-1.0,
                    substeps=substeps, space_charge=space_charge, bc=tuple(bc),
                    lambda_u=lambda_u, K=K, gamma_beam=gamma, z_e=z_e, x=x, u=u, q=q, m=m,
                    probe=probe, kp=kp, steps=steps)


def halton(index: np.ndarray, base: int) -> np.ndarray:
    """Radical inverse of the integers ``index`` in ``base`` (Halton sequence)."""
    index = np.asarray(index, dtype=np.int64).copy()
    out = np.zeros(index.shape)
    f = 1.0 / base
    while np.any(index > 0):
        out += f * (index % base)
        index //= base
        f /= base
    return out


def _tapered_flat_top(u: np.ndarray, length: float, sigma: float) -> np.ndarray:
    """Inverse cumulative distribution of a flat top of the given length with
    half-Gaussian edges of width sigma at the same peak density (the two
    halves of a small Gaussian bunch moved to tail and head), for u in (0, 1)."""
    from scipy.special import ndtri
    m_t = math.sqrt(math.pi / 2.0) * sigma  # mass of one edge at unit density
    total = length + 2.0 * m_t
    w = np.asarray(u) * total
    z = np.empty_like(w)
    lo = w < m_t
    hi = w >= m_t + length
    mid = ~lo & ~hi
    z[lo] = -length / 2.0 + sigma * ndtri(w[lo] / m_t / 2.0)
    z[mid] = -length / 2.0 + (w[mid] - m_t)
    z[hi] = length / 2.0 + sigma * ndtri(0.5 + (w[hi] - m_t - length) / m_t / 2.0)
    return z


def example1(*, n=(64, 64, 2800), n_particles: int = 131072, steps: int = 17900,
             seed: int = BASE_SEED + 10, bunching: float = 0.01,
             substeps: int = 2, transverse: str = "gaussian", flat_top: float = 100.5e-6,
             sigma_t: float = 260e-6) -> Workload:
    """The paper's infrared FEL example (section "Example 1: Infrared FEL"),
    lab parameters from its table and job file, taken into the rest frame.

    Lab frame: gamma = 100.41, sigma_delta = 1e-4, charge 29.5 pC; undulator
    lambda_u = 3 cm, K = 1.417; mesh 3200 x 3200 x 280 um at 50 x 50 x 0.1 um
    (64 x 64 x 2800 cells); transverse Gaussian of sigma 260 um cut at
    1040 um; a flat top of 100.5 um with Gaussian edges of one radiation
    wavelength (3 um); initial bunching factor 0.01; second-order Mur, no
    space charge.  Rest frame: dz = gamma0 * 0.1 um, c dt = dz, two particle
    sub-steps per field step (the job's bunch time step 1.6 ps in the lab is
    below the field step).  The matched momenta belong to the leapfrog's
    time level of u, half a sub-step before the positions at dt/2.

    Loading (quiet start, as the paper's Halton filling): z from the Halton
    sequence of base 2 through the inverse distribution of the tapered flat
    top, the transverse Gaussian by Box-Muller from bases 3 and 5; then
    z -> gamma0 z, the bunching modulation z -> z + (2 b / K_b) sin(K_b z)
    with K_b = 2 gamma0 k_u (which gives the bunching factor J_1(2 b) = b to
    first order), and momenta matched to the undulator as in make_workload.
    The bunch starts inside the undulator (entrance one cell behind the mesh).
    The power plane sits 110 um (lab) ahead of the bunch centre.
    ``transverse="uniform"`` loads the table's reading instead: a uniform
    260 x 260 um square (the printed electron density 2.72e13 cm^-3).
    ``flat_top`` and ``sigma_t`` (lab) change the flat top's length and the
    transverse width at the same peak density (the charge scales with them):
    a longer bunch slips fewer of its cooperation lengths, a wider one
    diffracts less.  The plane then sits 59.75 um ahead of the flat top's head.
    """
    n = tuple(int(v) for v in n)
    gamma, K, lambda_u, sigma_delta = 100.41, 1.417, 0.03, 1e-4
    gamma0 = gamma / math.sqrt(1.0 + K * K / 2.0)
    beta0 = math.sqrt(1.0 - 1.0 / (gamma0 * gamma0))
    ku = 2.0 * math.pi / lambda_u
    lam_r = lambda_u / (2.0 * gamma0 * gamma0)  # lab radiation wavelength
    d = (50e-6, 50e-6, 0.1e-6 * gamma0)
    origin = tuple(-(n[a] - 1) / 2.0 * d[a] for a in range(3))
    z_e = origin[2] - d[2]
    # quiet start: Halton points, indices from 1; keep the first n_particles
    # whose transverse radius is inside the 4-sigma cut
    sig_t, cut = sigma_t, 4.0 * sigma_t
    idx = np.arange(1, int(n_particles * 1.01) + 64)
    r = sig_t * np.sqrt(-2.0 * np.log(halton(idx, 3)))
    keep = r <= cut
    idx = idx[keep][:n_particles]
    r = r[keep][:n_particles]
    th = 2.0 * math.pi * halton(idx, 5)
    zl = _tapered_flat_top(halton(idx, 2), flat_top, lam_r)
    x = np.empty((n_particles, 3))
    if transverse == "uniform":
        x[:, 0] = (halton(idx, 3) - 0.5) * sig_t
        x[:, 1] = (halton(idx, 5) - 0.5) * sig_t
    else:
        x[:, 0] = r * np.cos(th)
        x[:, 1] = r * np.sin(th)
    kb = 2.0 * gamma0 * ku
    zr = gamma0 * zl
    x[:, 2] = zr + (2.0 * bunching / kb) * np.sin(kb * zr)
    rng = np.random.Generator(np.random.PCG64(seed))
    gp = gamma * (1.0 + sigma_delta * rng.standard_normal(n_particles))
    u, x[:, 0] = _matched(x, gp, gamma0, beta0, K, ku, z_e, 1.0 * d[2] / C_LIGHT, substeps)
    charge = BUNCH_CHARGE * (flat_top / 100.5e-6) * (sigma_t / 260e-6) ** 2
    q = -charge / n_particles
    m = M_E * (charge / Q_E) / n_particles
    ahead = flat_top / 2.0 + 59.75e-6  # 110 um ahead of the centre for the job's bunch
    kp = min(n[2] // 2 + int(round(gamma0 * ahead / d[2])), n[2] - 3)
    return Workload(name="example1-%dx%dx%d" % n, n=n, d=d, origin=origin, courant=1.0,
                    nsfd_A=-1.0, substeps=substeps, space_charge=0, bc=(2, 2, 2),
                    lambda_u=lambda_u, K=K, gamma_beam=gamma, z_e=z_e, x=x, u=u, q=q, m=m,
                    probe=(n[0] // 2, n[1] // 2, kp), kp=kp, steps=steps)


# The published configurations, in order (index 0..4), plus the parity subcase.
def config(index: int, *, n_particles: Optional[int] = None, steps: Optional[int] = None,
           seed: Optional[int] = None) -> Workload:
    s = BASE_SEED + index if seed is None else seed
    if index in (0, 2):  # 32x32x64, 4096 particles, gamma 100, K 1.0, lambda_u 1.5 cm
        return make_workload("tiny-32x32x64" if index == 0 else "precision-32x32x64",
                             (32, 32, 64), n_particles or 4096, 100.0, 1.0, 0.015, 1e-4, s,
                             steps or 200)
    if index == 1:  # 128x128x512, 1M particles, 2000 steps
        return make_workload("mid-128x128x512", (128, 128, 512), n_particles or 1 << 20, 100.0,
                             1.0, 0.015, 1e-4, s, steps or 2000)
    if index == 3:  # 256x256x2048, 16M particles, gamma 200, K 1.5, lambda_u 1.8 cm
        return make_workload("large-256x256x2048", (256, 256, 2048), n_particles or 1 << 24,
                             200.0, 1.5, 0.018, 2e-4, s, steps or 5000)
    raise ValueError("config index must be 0..3 (4 is the batch, see batch_configs)")


def mid_subcase(*, steps: int = 2000, n_particles: int = 65536) -> Workload:
    """64x64x128 with 65536 particles: the oracle-checkable slice of the mid case."""
    return make_workload("mid-subcase-64x64x128", (64, 64, 128), n_particles, 100.0, 1.0, 0.015,
                         1e-4, BASE_SEED + 1, steps)


def batch_configs(nsim: int = 64, *, steps: int = 1000, seed: Optional[int] = None,
                  particle_scale: float = 1.0) -> List[Workload]:
    """The undulator/beam parameter scan: uneven meshes and bunches, one per simulation."""
    base = BASE_SEED + 4 if seed is None else seed
    out = []
    for s in range(nsim):
        rng = np.random.Generator(np.random.PCG64(base + 1000 * s))
        scale = rng.uniform(1.0, 3.0)
        nx = 8 * int(round(4 * scale))
        nz = 4 * nx
        npart = 1024 * int(rng.integers(16, 257))
        npart = max(256, int(npart * particle_scale))
        gamma = float(rng.uniform(80.0, 250.0))
        K = float(rng.uniform(0.8, 2.0))
        out.append(make_workload("scan-%02d-%dx%dx%d" % (s, nx, nx, nz), (nx, nx, nz), npart,
                                 gamma, K, 0.015, 1e-4, base + 1000 * s + 1, steps))
    return out
