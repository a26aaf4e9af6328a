"""Pins of the oracle's energy and power diagnostics (section "FEL-OUTPUT"
names the radiated power; the energies follow the field and particle
definitions of chapter "Methodology"), each against a closed form that does
not reuse the oracle's own sums:

* uniform E and B (potentials linear in space and time): the field energy
  and the Poynting flux through the power plane are products of constants
  and point counts;
* a transversely uniform plane wave at c dt = dz in a periodic box (an exact
  discrete solution, one cell per step): the flux through the plane and the
  field energy follow from the discrete E and B of the wave in closed form,
  for both polarizations and both directions of travel;
* particles whose Lorentz factors are whole numbers, one at rest and one lost:
  the kinetic energy is m c^2 times a whole number; and the work done by a
  uniform field on a particle equals its kinetic-energy gain to the order of
  the scheme.

Then each pin is shown to catch a plausible mistake: the oracle is rebuilt
from its source with one mistake planted (a dropped 1/2, mu0 in the wrong
place, a flipped sign, a plane range one point short, gamma for gamma - 1),
and the pin must fail on that build.
"""
import math
import os
import subprocess

import numpy as np
import pytest

import oracle

C = 299792458.0
QE = 1.602176634e-19
ME = 9.1093837015e-31
EPS0 = 8.8541878128e-12
MU0 = 1.0 / (EPS0 * C * C)

COL_POWER, COL_FIELD, COL_KIN = 4, 5, 6


def _mesh(n, dz=1e-6, ax=4.0, ay=3.0):
    d = (ax * dz, ay * dz, dz)
    origin = tuple(-(n[a] - 1) / 2.0 * d[a] for a in range(3))
    return d, origin


def _empty(sim):
    sim.set_particles(np.zeros((0, 3)), np.zeros((0, 3)), -QE, ME)


# ---------------------------------------------------------------------------
# uniform fields
# ---------------------------------------------------------------------------

def pin_uniform_fields():
    """A_x = alpha z + beta t, A_y = g x + delta t, A_z = eps y, phi = -zeta z
    give E = (-beta, -delta, zeta) and B = (eps, alpha, g) everywhere.  On a
    mesh with absorbing faces the diagnostics cover the vertices 1..n-2 of
    each axis, so the field energy is (eps0 E^2/2 + B^2/(2 mu0)) dV times the
    number of such vertices, and the flux through plane k is
    (E_x B_y - E_y B_x)/mu0 dx dy times the plane's (nx-2)(ny-2) points."""
    n = (9, 7, 12)
    d, origin = _mesh(n)
    sim = oracle.OracleSim(n, d, origin, courant=0.9, bc=(0, 0, 0), space_charge=1, K=0.0)
    _empty(sim)
    kp = 7
    sim.config_diag((4, 3, 6), kp)
    dt = sim.const["dt"]
    alpha, beta, g, delta, eps, zeta = 0.7, 2.1e8, -0.4, -1.3e8, 0.25, 0.9e8
    kk, jj, ii = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    X = origin[0] + ii * d[0]
    Y = origin[1] + jj * d[1]
    Z = origin[2] + kk * d[2]
    # each component varies only across its own axis, so the staggered
    # sample points (reading R5) take the vertex coordinates
    for lev, t in (("cur", 0.0), ("next", dt)):
        sim.pot(0, lev)[:] = alpha * Z + beta * t
        sim.pot(1, lev)[:] = g * X + delta * t
        sim.pot(2, lev)[:] = eps * Y
    sim.pot(3, "cur")[:] = -zeta * Z
    sim.vertex_fields()
    row = sim.diag_row_now()
    E = np.array([-beta, -delta, zeta])
    B = np.array([eps, alpha, g])
    nint = (n[0] - 2) * (n[1] - 2) * (n[2] - 2)
    dV = d[0] * d[1] * d[2]
    w_ref = (0.5 * EPS0 * E.dot(E) + 0.5 * B.dot(B) / MU0) * dV * nint
    p_ref = (E[0] * B[1] - E[1] * B[0]) / MU0 * d[0] * d[1] * (n[0] - 2) * (n[1] - 2)
    assert abs(row[COL_FIELD] / w_ref - 1.0) < 1e-12, (row[COL_FIELD], w_ref)
    assert abs(row[COL_POWER] / p_ref - 1.0) < 1e-12, (row[COL_POWER], p_ref)


def test_uniform_fields_energy_and_flux():
    pin_uniform_fields()


# ---------------------------------------------------------------------------
# discrete plane wave at c dt = dz
# ---------------------------------------------------------------------------

def pin_plane_wave(comp, direction):
    """A_comp^s(k) = a cos(kappa (k - direction s) + 0.4) is an exact solution
    of the update at c dt = dz when it does not vary across the mesh
    (kappa = 2 pi m / n_z).  The vertex fields of row s (levels s and s+1,
    time (s+1/2) dt) are then, with phase f = kappa k - direction theta (s+1/2)
    + 0.4 and theta = kappa,
        E_comp = -direction (2a/dt) sin(theta/2) sin f,
        dA_comp/dz (central, mean of both levels) = -(a/dz) sin kappa cos(theta/2) sin f,
    so the flux through plane k_p is
        P_s = direction a^2 sin(theta) sin(kappa) / (dt dz mu0) sin^2 f(k_p) dx dy nx ny
    for either polarization (B_y = dA_x/dz, B_x = -dA_y/dz), and the field
    energy, with sum_k sin^2 f = n_z/2 over whole periods, is
        W = nx ny dV n_z/2 [eps0/2 (2a/dt)^2 sin^2(theta/2)
                            + (a sin(kappa)/dz)^2 cos^2(theta/2) / (2 mu0)]."""
    n = (6, 5, 48)
    d, origin = _mesh(n)
    sim = oracle.OracleSim(n, d, origin, courant=1.0, bc=(1, 1, 1), space_charge=1, K=0.0)
    _empty(sim)
    kp = 17
    sim.config_diag((2, 2, kp), kp)
    m, a = 5, 2.5e-9
    kappa = 2.0 * math.pi * m / n[2]
    theta = kappa
    kk = np.arange(n[2])
    f = lambda s: a * np.cos(kappa * (kk - direction * s) + 0.4)
    sim.pot(comp, "cur")[:] = f(0)[:, None, None]
    sim.pot(comp, "prev")[:] = f(-1)[:, None, None]
    steps = 30
    sim.step(steps)
    dg = sim.diag()
    dt, dz = sim.const["dt"], d[2]
    s = np.arange(steps)
    ph = kappa * kp - direction * theta * (s + 0.5) + 0.4
    amp = a * a * math.sin(theta) * math.sin(kappa) / (dt * dz * MU0) * d[0] * d[1] * n[0] * n[1]
    p_ref = direction * amp * np.sin(ph) ** 2
    assert np.max(np.abs(dg[:, COL_POWER] - p_ref)) < 1e-11 * amp, (dg[:5, COL_POWER], p_ref[:5])
    dV = d[0] * d[1] * d[2]
    w_ref = n[0] * n[1] * dV * n[2] / 2.0 * (
        0.5 * EPS0 * (2.0 * a / dt) ** 2 * math.sin(theta / 2) ** 2
        + (a * math.sin(kappa) / dz) ** 2 * math.cos(theta / 2) ** 2 / (2.0 * MU0))
    assert np.max(np.abs(dg[:, COL_FIELD] / w_ref - 1.0)) < 1e-11, (dg[:3, COL_FIELD], w_ref)


@pytest.mark.parametrize("comp", [0, 1])
@pytest.mark.parametrize("direction", [1, -1])
def test_plane_wave_flux_and_energy(comp, direction):
    pin_plane_wave(comp, direction)


# ---------------------------------------------------------------------------
# kinetic energy
# ---------------------------------------------------------------------------

def pin_kinetic_whole_gammas():
    """u = gamma beta with gamma = 1, 2, 3, 5 (|u|^2 = gamma^2 - 1 = 0, 3, 8, 24
    in assorted directions) and one particle outside the live cells: the
    kinetic energy of the live ones is m c^2 (0 + 1 + 2 + 4)."""
    n = (12, 12, 16)
    d, origin = _mesh(n)
    sim = oracle.OracleSim(n, d, origin, courant=0.9, bc=(0, 0, 0), space_charge=1, K=0.0)
    x = np.array([[0.1, -0.2, 0.3], [0.5, 0.4, -1.2], [-0.7, 0.2, 0.9], [0.3, 0.3, 0.3],
                  [0.0, 0.0, 0.0]]) * np.array(d)
    x[4] = (origin[0] + 0.5 * d[0], 0.0, 0.0)  # cell 0 along x: lost at load (reading R17)
    u = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, math.sqrt(3.0)], [2.0, -2.0, 0.0],
                  [3.0, 0.0, math.sqrt(15.0)], [9.0, 9.0, 9.0]])
    m = 7.0 * ME
    sim.set_particles(x, u, -7.0 * QE, m)
    assert sim.lost == 1
    row = sim.diag_row_now()
    ref = m * C * C * (0.0 + 1.0 + 2.0 + 4.0)
    assert abs(row[COL_KIN] / ref - 1.0) < 1e-13, (row[COL_KIN], ref)


def test_kinetic_energy_of_whole_lorentz_factors():
    pin_kinetic_whole_gammas()


def pin_work_energy():
    """A particle starting at rest in a uniform E_z (no B, no undulator) gains
    the kinetic energy q E_z (z_end - z_start): the work-energy theorem, to
    the first order in dt/T of the leapfrog's half-step offset (here about 1%
    over 100 steps, so the bound is 3%)."""
    n = (12, 12, 64)
    d, origin = _mesh(n)
    sim = oracle.OracleSim(n, d, origin, courant=0.9, bc=(0, 0, 0), space_charge=0, K=0.0)
    x = np.array([[0.0, 0.0, origin[2] + 8.3 * d[2]]])
    sim.set_particles(x, np.zeros((1, 3)), QE, ME)
    dt = sim.const["dt"]
    steps = 100
    # u grows by q E dt / (m c) per step: reach u = 1 (v = c/sqrt 2) at the end
    Ez = ME * C / (QE * dt * steps)
    w0 = sim.diag_row_now()[COL_KIN]
    z0 = sim.x[0, 2]
    for _ in range(steps):
        sim.E(2)[:] = Ez
        sim.push()
    w1 = sim.diag_row_now()[COL_KIN]
    work = QE * Ez * (sim.x[0, 2] - z0)
    assert w0 == 0.0
    assert abs((w1 - w0) / work - 1.0) < 0.03, (w1 - w0, work)


def test_kinetic_energy_gain_equals_the_work_of_a_uniform_field():
    pin_work_energy()


# ---------------------------------------------------------------------------
# planted mistakes: each pin must catch one
# ---------------------------------------------------------------------------

MUTANTS = [
    # (name, anchor, old text, new text, pin)
    ("field energy without 1/2 on E", "void orc_diag_row",
     "0.5 * ORC_EPS0 * e2", "ORC_EPS0 * e2", pin_uniform_fields),
    ("field energy with mu0 multiplied", "void orc_diag_row",
     "0.5 * b2 / ORC_MU0", "0.5 * b2 * ORC_MU0", pin_uniform_fields),
    ("flux with the E_y B_x sign flipped", "static double plane_power(",
     "- s->E[1][p] * s->B[0][p]", "+ s->E[1][p] * s->B[0][p]",
     lambda: pin_plane_wave(1, 1)),
    ("flux without dy", "static double plane_power(",
     "/ ORC_MU0 * s->d[0] * s->d[1]", "/ ORC_MU0 * s->d[0]", pin_uniform_fields),
    ("flux plane one row short", "static double plane_power(",
     "j <= hi[1]", "j < hi[1]", pin_uniform_fields),
    ("kinetic energy with gamma for gamma - 1", "void orc_diag_row",
     " - 1.0) * s->m * ORC_C * ORC_C", ") * s->m * ORC_C * ORC_C",
     pin_kinetic_whole_gammas),
    ("kinetic energy counting lost particles", "void orc_diag_row",
     "if (!s->alive[p]) continue;\n        const double *u",
     "const double *u", pin_kinetic_whole_gammas),
]


def _plant(src, anchor, old, new):
    at = src.index(anchor)
    where = src.index(old, at)
    return src[:where] + new + src[where + len(old):]


@pytest.mark.parametrize("mutant", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_catches_a_planted_mistake(mutant, tmp_path):
    name, anchor, old, new, pin = mutant
    pin()  # holds on the oracle as written
    with open(oracle._SRC) as f:
        src = _plant(f.read(), anchor, old, new)
    csrc = os.path.join(str(tmp_path), "mutant.c")
    with open(csrc, "w") as f:
        f.write(src)
    lib = os.path.join(str(tmp_path), "libmutant.so")
    subprocess.check_call(oracle.gcc_command(csrc, lib))
    before = oracle.use_library(lib)
    try:
        with pytest.raises(AssertionError):
            pin()
    finally:
        oracle.restore_library(before)
