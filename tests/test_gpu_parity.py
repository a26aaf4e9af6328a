"""GPU path (through the C ABI) against the FP64 CPU oracle, element by element.

Bar: relative L2 <= 1e-10 for the double-precision path; for the float path
with split positions, relative L2 <= 1e-3 of the on-axis probe field series
and of the radiated-power series.  Every input comes from the seeded
generator; no expected value comes from the GPU path.
"""
import math

import numpy as np
import pytest

import oracle
import subbox
from paper_1612_03310_amd import native
from paper_1612_03310_amd import workloads as W

pytestmark = pytest.mark.gpu

C = 299792458.0
QE = 1.602176634e-19
ME = 9.1093837015e-31

TOL64 = 1e-10
POT = ("Ax", "Ay", "Az", "phi")


def say(*a):
    print(*a, flush=True)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)


VECTORS = {"A": ("Ax", "Ay", "Az"), "A_prev": ("Ax_prev", "Ay_prev", "Az_prev"),
           "J": ("Jx", "Jy", "Jz"), "E": ("Ex", "Ey", "Ez"), "B": ("Bx", "By", "Bz")}
# Per-component guard.  A component that is tiny next to its vector (J_y,
# A_y: the bunch barely moves in y) is ill-conditioned: its edge currents are
# differences of nearly equal linear weights, so a one-ulp difference in how a
# position is held (SI metres in the oracle, cell + offset on the GPU) is
# amplified by the ratio of the weight to the y-displacement.  The bar is the
# relative L2 of each vector field; a component must still agree to 1e-8,
# which any real error in one component (a sign, an index) fails by far.
COMPONENT_GUARD = 1e-8


def _oracle_field(orc, name):
    table = {"Ax": lambda: orc.pot(0, "cur"), "Ay": lambda: orc.pot(1, "cur"),
             "Az": lambda: orc.pot(2, "cur"), "phi": lambda: orc.pot(3, "cur"),
             "Ax_prev": lambda: orc.pot(0, "prev"), "Ay_prev": lambda: orc.pot(1, "prev"),
             "Az_prev": lambda: orc.pot(2, "prev"), "phi_prev": lambda: orc.pot(3, "prev"),
             "Jx": lambda: orc.J(0), "Jy": lambda: orc.J(1), "Jz": lambda: orc.J(2),
             "rho": lambda: orc.rho, "rho_prev": lambda: orc.rho_prev,
             "Ex": lambda: orc.E(0), "Ey": lambda: orc.E(1), "Ez": lambda: orc.E(2),
             "Bx": lambda: orc.B(0), "By": lambda: orc.B(1), "Bz": lambda: orc.B(2)}
    return table[name]()


def compare_state(sim, orc, tol, what=""):
    """Every stored mesh quantity, the derived E/B and the particles."""
    errs, comp = {}, {}
    for vec, names in VECTORS.items():
        g = np.stack([sim.get_field(n) for n in names])
        o = np.stack([_oracle_field(orc, n) for n in names])
        errs[vec] = rel_l2(g, o)
        for n, gi, oi in zip(names, g, o):
            comp[n] = rel_l2(gi, oi)
    for n in ("phi", "phi_prev", "rho", "rho_prev"):
        errs[n] = rel_l2(sim.get_field(n), _oracle_field(orc, n))
    if orc.np > 0:
        pos, u, alive = sim.get_particles()
        assert np.array_equal(alive, orc.alive), what
        errs["pos"] = rel_l2(pos[alive], orc.x[alive])
        errs["u"] = rel_l2(u, orc.u)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    bad.update({k: v for k, v in comp.items() if not v <= COMPONENT_GUARD})
    say(what, "worst", max(errs, key=errs.get), max(errs.values()),
        "worst component", max(comp, key=comp.get), max(comp.values()))
    assert not bad, (what, bad)
    return errs


def compare_diag(gd, od, tol, what=""):
    assert len(gd) == len(od), (len(gd), len(od))
    assert np.array_equal(gd["step"], od[:, 0].astype(np.int64))
    assert np.array_equal(gd["lost"], od[:, 13].astype(np.int64))
    assert not gd["nonfinite"].any()
    cols = {"total_charge": 2, "power": 4, "field_energy": 5, "kinetic_energy": 6}
    errs = {k: rel_l2(gd[k], od[:, c]) for k, c in cols.items()}
    errs["probe_E"] = rel_l2(gd["probe_E"], od[:, 7:10])
    errs["probe_B"] = rel_l2(gd["probe_B"], od[:, 10:13])
    errs["bunching"] = rel_l2(gd["bunching"], od[:, 16:19])
    errs["power_harmonic"] = rel_l2(gd["power_harmonic"], od[:, 20:23])
    errs["power_extra"] = rel_l2(gd["power_extra"], od[:, 24:27])
    # continuity: the residual equals the oracle's on every row (on a step
    # that loses particles their charge leaves rho without a current), and
    # holds to round-off of the fixed-point deposit on the other rows
    errs["continuity_residual"] = rel_l2(gd["continuity_residual"], od[:, 3]) if np.any(
        od[:, 3] > 1e-9) else 0.0
    bad = {k: v for k, v in errs.items() if not v <= tol}
    say(what, "diag", errs)
    assert not bad, (what, bad)
    steady = np.concatenate([[gd["lost"][0] == 0], np.diff(gd["lost"]) == 0])
    assert np.max(gd["continuity_residual"][steady]) < 1e-11


def run_pair(w, steps, precision="f64", every=1):
    say("case", w.name, w.n, w.np, "steps", steps, precision)
    orc = oracle.from_workload(w)
    sim = native.sim_from_workload(w, precision=precision, every=every)
    sim.run(steps)
    sim.sync()
    orc.step(steps)
    return sim, orc


# ---------------------------------------------------------------------------
# potential update and boundary alone
# ---------------------------------------------------------------------------

def _random_fields(n, bc, rng):
    """Random potentials; the unused last layer of an edge grid along its own
    Mur axis is zero."""
    nx, ny, nz = n
    out = {}
    for c, name in enumerate(POT):
        a = rng.standard_normal((nz, ny, nx))
        if c < 3 and bc[c] != 1:  # an absorbing axis (Mur of either order)
            idx = [slice(None)] * 3
            idx[2 - c] = -1
            a[tuple(idx)] = 0.0
        out[name] = a
    return out


@pytest.mark.parametrize("bc,n", [((0, 0, 0), (40, 36, 50)), ((1, 1, 0), (40, 36, 50)),
                                  ((1, 1, 1), (40, 36, 50)), ((0, 1, 0), (40, 36, 50)),
                                  ((0, 0, 0), (65, 36, 50)), ((2, 2, 2), (40, 36, 50)),
                                  ((1, 1, 2), (40, 36, 50)), ((2, 1, 2), (40, 36, 50)),
                                  ((2, 2, 1), (40, 36, 50)), ((2, 2, 2), (65, 36, 50))])
def test_potential_update_and_mur_match_oracle(bc, n):
    """One step of eq. (updateEquation) plus first-order Mur on faces, edges
    and corners, with random potentials and sources, on meshes whose sizes are
    not multiples of the 8-cell tiles.  At 40 cells along x the stencil pass
    updates the x faces itself; at 65 the high x face of the potentials
    falls on the first lane of a wavefront and the boundary kernel takes
    them.  Code 2 selects second-order Mur (faces, edges and corners in the
    boundary kernels)."""
    dz = 2e-6
    d = (4 * dz, 3 * dz, dz)
    origin = tuple(-(n[a] - 1) / 2 * d[a] for a in range(3))
    say("case stencil", n, bc)
    rng = np.random.default_rng(11)
    cur = _random_fields(n, bc, rng)
    prev = _random_fields(n, bc, rng)
    J = [rng.standard_normal((n[2], n[1], n[0])) * 1e4 for _ in range(3)]
    rho = rng.standard_normal((n[2], n[1], n[0])) * 1e-2
    orc = oracle.OracleSim(n, d, origin, courant=0.9, bc=bc, space_charge=1, K=0.0,
                           gamma_beam=50.0)
    orc.set_particles(np.zeros((0, 3)), np.zeros((0, 3)), -QE, ME)
    sim = native.Sim(n, d, origin, courant=0.9, bc=bc, space_charge=1, K=0.0, gamma_beam=50.0)
    sim.set_particles(np.zeros((0, 3)), np.zeros((0, 3)), -QE, ME)
    for c, name in enumerate(POT):
        orc.pot(c, "cur")[:] = cur[name]
        orc.pot(c, "prev")[:] = prev[name]
        sim.set_field(name, cur[name])
        sim.set_field(name + "_prev", prev[name])
    for c, name in enumerate(("Jx", "Jy", "Jz")):
        orc.J(c)[:] = J[c]
        sim.set_field(name, J[c])
    orc.rho[:] = rho
    sim.set_field("rho", rho)
    orc.field_update()
    sim.run(1)
    sim.sync()
    for c, name in enumerate(POT):
        e = rel_l2(sim.get_field(name), orc.pot(c, "next"))
        assert e < TOL64, (name, e)
        # the boundary layer alone (faces, edges, corners)
        g = sim.get_field(name)
        o = orc.pot(c, "next")
        mask = np.zeros_like(g, dtype=bool)
        mask[0], mask[-1], mask[:, 0], mask[:, -1], mask[:, :, 0], mask[:, :, -1] = (True,) * 6
        if np.any(o[mask] != 0):
            assert rel_l2(g[mask], o[mask]) < TOL64, name


@pytest.mark.parametrize("courant,precision", [(1.0, "f64"), (0.9, "f64"), (0.9, "f32")])
def test_seed_plane_wave_matches_oracle(courant, precision):
    """A modulated-Gaussian seed enters at z_min through the TF/SF planes and
    crosses the mesh (periodic across, Mur along z): all four potentials
    against the oracle after 150 steps."""
    n = (8, 8, 160)
    dz = 1e-6
    d = (2 * dz, 2 * dz, dz)
    origin = (0.0, 0.0, 0.0)
    bc = (1, 1, 0)
    tau = 15 * dz / C
    seed = dict(polarization=(0.6, 0.8), frequency=C / (20 * dz), t0=4 * tau, tau=tau, cep=0.3,
                signal="gaussian", z_ref=0.0)
    say("case seed", n, courant, precision)
    orc = oracle.OracleSim(n, d, origin, courant=courant, bc=bc, K=0.0, gamma_beam=50.0)
    orc.set_particles(np.zeros((0, 3)), np.zeros((0, 3)), -QE, ME)
    orc.set_seed(1e-3, **seed)
    sim = native.Sim(n, d, origin, courant=courant, bc=bc, K=0.0, gamma_beam=50.0,
                     precision=precision)
    sim.set_particles(np.zeros((0, 3)), np.zeros((0, 3)), -QE, ME)
    sim.set_seed(1e-3, **seed)
    orc.step(150)
    sim.run(150)
    sim.sync()
    tol = TOL64 if precision == "f64" else 1e-4
    for c, name in enumerate(POT):
        g, o = sim.get_field(name), orc.pot(c, "cur")
        if c < 2:
            assert np.max(np.abs(o)) > 1e-4  # the seed is in the mesh
            assert rel_l2(g, o) < tol, (name, rel_l2(g, o))
        else:
            assert np.max(np.abs(g)) == 0.0, name


def _gaussian_seed_case(precision, courant=0.9):
    """A round, nearly collimated Gaussian beam (k z_R = 100, waist 5.6
    cells) entering through the TF/SF planes, focused 60 cells in; Mur on
    every face."""
    dz = 1e-6
    n, d = (40, 40, 100), (8 * dz, 8 * dz, dz)
    origin = (-156 * dz, -156 * dz, 0.0)
    lam, tau = 20 * dz, 15 * dz / C
    k = 2 * np.pi / lam
    zr = 100.0 / k
    seed = dict(polarization=(0.6, 0.8), frequency=C / lam, t0=4 * tau, tau=tau, cep=0.3,
                signal="gaussian", z_ref=0.0)
    beam = dict(beam="gaussian", rayleigh=(zr, 0.7 * zr), focus=(8e-6, -5e-6, 60 * dz))
    orc = oracle.OracleSim(n, d, origin, courant=courant, bc=(0, 0, 0), K=0.0, gamma_beam=50.0)
    orc.set_particles(np.zeros((0, 3)), np.zeros((0, 3)), -QE, ME)
    sim = native.Sim(n, d, origin, courant=courant, bc=(0, 0, 0), K=0.0, gamma_beam=50.0,
                     precision=precision)
    sim.set_particles(np.zeros((0, 3)), np.zeros((0, 3)), -QE, ME)
    return orc, sim, seed, beam


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_gaussian_seed_matches_oracle(precision):
    """The Gaussian-beam seed: 30 steps as a plane wave, then the beam shape
    switched on (the captured step is rebuilt with the corrections kernel)
    and 60 more steps; all four potentials against the oracle, which the
    beam shape moves far from the plane-wave run."""
    orc, sim, seed, beam = _gaussian_seed_case(precision)
    plane, _, _, _ = _gaussian_seed_case(precision)
    say("case gaussian seed", precision, beam)
    for o in (orc, plane):
        o.set_seed(1e-3, **seed)
        o.step(30)
    sim.set_seed(1e-3, **seed)
    sim.run(30)
    sim.sync()
    orc.set_seed_beam(**beam)
    sim.set_seed_beam(**beam)
    orc.step(60)
    plane.step(60)
    sim.run(60)
    sim.sync()
    tol = TOL64 if precision == "f64" else 1e-4
    for c, name in enumerate(POT):
        g, o = sim.get_field(name), orc.pot(c, "cur")
        if c < 2:
            assert np.max(np.abs(o)) > 1e-4
            assert rel_l2(g, o) < tol, (name, rel_l2(g, o))
            shaped = rel_l2(o, plane.pot(c, "cur"))
            say(name, "rel-L2", rel_l2(g, o), "beam against plane wave", shaped)
            assert shaped > 0.1
        else:
            assert np.max(np.abs(g)) == 0.0, name


def test_batch_with_gaussian_and_plane_seeds_equals_separate_runs():
    _, _, seed, beam = _gaussian_seed_case("f64")
    dz = 1e-6
    n, d = (40, 40, 100), (8 * dz, 8 * dz, dz)
    origin = (-156 * dz, -156 * dz, 0.0)
    mesh = native.make_mesh(n, d, origin, 0.9, -1.0, 1, 1, (0, 0, 0))
    und = native.make_undulator(0.015, 0.0, 50.0, 0.0)
    b = native.Batch([mesh, mesh], [und, und], precision="f64")
    for s in range(2):
        b.set_particles(s, np.zeros((0, 3)), np.zeros((0, 3)), -QE, ME)
        b.set_seed(s, 1e-3, **seed)
    b.set_seed_beam(1, **beam)
    b.run(70)
    b.sync()
    for s in range(2):
        sim = native.Sim(n, d, origin, courant=0.9, bc=(0, 0, 0), K=0.0, gamma_beam=50.0)
        sim.set_particles(np.zeros((0, 3)), np.zeros((0, 3)), -QE, ME)
        sim.set_seed(1e-3, **seed)
        if s == 1:
            sim.set_seed_beam(**beam)
        sim.run(70)
        sim.sync()
        for name in ("Ax", "Ay"):
            assert np.array_equal(b.get_field(s, name), sim.get_field(name)), (s, name)
    assert not np.array_equal(b.get_field(0, "Ax"), b.get_field(1, "Ax"))
    b.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_background_charge_matches_oracle(precision):
    """The tiny bunch with a static background equal to minus its initial
    charge density (a neutral system): 60 steps against the oracle with the
    same background; phi differs far from the run without it."""
    w = W.config(0, steps=60)
    orc = oracle.from_workload(w)
    bg = -orc.rho.copy()
    orc.set_background(bg)
    bare = oracle.from_workload(w)
    sim = native.sim_from_workload(w, precision=precision, every=1)
    sim.set_background(bg)
    sim.run(60)
    sim.sync()
    orc.step(60)
    bare.step(60)
    if precision == "f64":
        compare_state(sim, orc, TOL64, "background")
        compare_diag(sim.get_diag(), orc.diag(), TOL64, "background")
    else:
        err = rel_l2(sim.get_field("phi"), orc.pot(3, "cur"))
        say("background f32 phi rel-L2", err)
        assert err < 1e-4, err
    moved = rel_l2(orc.pot(3, "cur"), bare.pot(3, "cur"))
    say("phi, with background against without", moved)
    assert moved > 0.5
    with pytest.raises(native.MithraError) as e:
        bad = bg.copy()
        bad.flat[5] = np.nan
        sim.set_background(bad)
    assert e.value.status == native.EINVAL


def test_background_removed_is_the_plain_run_bitwise():
    w = W.config(0, steps=20)
    outs = []
    for toggle in (False, True):
        sim = native.sim_from_workload(w, precision="f64")
        if toggle:
            sim.set_background(np.ones((w.n[2], w.n[1], w.n[0])))
            sim.set_background(None)
        sim.run(20)
        sim.sync()
        outs.append((sim.get_field("phi"), sim.get_diag().tobytes()))
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1]


def test_seeded_full_loop_f64():
    """A seed and a bunch together, Mur on every face: the whole state and
    the diagnostics against the oracle."""
    n = (40, 44, 72)
    w = W.make_workload("seeded", n, 3000, 120.0, 1.3, 0.015, 1e-4, 91, 60)
    tau = 10 * w.d[2] / C
    seed = dict(polarization=(1.0, 0.0), frequency=C / (16 * w.d[2]), t0=3 * tau, tau=tau,
                cep=0.0, signal="flat-top", z_ref=w.origin[2])
    say("case seeded full loop", n)
    orc = oracle.from_workload(w)
    orc.set_seed(2e-4, **seed)
    sim = native.sim_from_workload(w, precision="f64", every=1)
    sim.set_seed(2e-4, **seed)
    sim.run(60)
    sim.sync()
    orc.step(60)
    compare_state(sim, orc, TOL64, "seeded")
    compare_diag(sim.get_diag(), orc.diag(), TOL64, "seeded")


def _optical_wave(w, a0=0.5):
    """A Gaussian-enveloped plane wave towards -z (rest frame), a0 = 0.5,
    wavelength 32 cells, crossing the bunch during the run."""
    tau = 64 * w.d[2] / C
    return a0 * ME * C / QE, dict(polarization=(0.6, 0.8), frequency=C / (32 * w.d[2]),
                                   t0=2 * tau, tau=tau, cep=0.2, signal="gaussian",
                                   z_ref=w.origin[2] + (w.n[2] - 1) * w.d[2] / 2)


def _bunch_at_rest(w):
    """The bunch at rest in the central half of the mesh along z (momenta
    matched to the static undulator would carry it out of the mesh once the
    wave replaces that field)."""
    zc = w.origin[2] + (w.n[2] - 1) * w.d[2] / 2
    x = w.x.copy()
    x[:, 2] = zc + 0.5 * (x[:, 2] - zc)
    w.x = x
    w.u = np.zeros_like(w.u)
    return w


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_optical_undulator_full_loop_matches_oracle(precision):
    """The tiny bunch driven by the optical undulator (a plane wave towards -z
    in place of the static undulator) for 60 steps: the whole state and the
    diagnostics against the oracle."""
    w = _bunch_at_rest(W.config(0, steps=60))
    amp, wave = _optical_wave(w)
    say("case optical undulator", w.n, precision)
    orc = oracle.from_workload(w)
    orc.set_optical_undulator(amp, **wave)
    sim = native.sim_from_workload(w, precision=precision, every=1)
    sim.set_optical_undulator(amp, **wave)
    sim.run(60)
    sim.sync()
    orc.step(60)
    if precision == "f64":
        compare_state(sim, orc, TOL64, "optical")
        compare_diag(sim.get_diag(), orc.diag(), TOL64, "optical")
    else:
        pos, u, alive = sim.get_particles()
        assert np.array_equal(alive, orc.alive)
        err = rel_l2(u, orc.u)
        say("optical f32 u rel-L2", err)
        assert err < 1e-4, err
    # the wave really drives the particles (they started at rest), none lost
    assert np.max(np.abs(orc.u[:, 1])) > 0.05 and orc.lost == 0


def _gaussian_beam(w):
    """An astigmatic Gaussian beam for the wave of _optical_wave: waist 6
    cells along the polarization and 6/sqrt(2) across it, focused one cell
    off the bunch axis and 10 cells ahead of its centre."""
    k = 2 * np.pi / (32 * w.d[2])
    w0 = 6 * w.d[0]
    zr = k * w0 * w0 / 2
    c = [w.origin[a] + (w.n[a] - 1) * w.d[a] / 2 for a in range(3)]
    return dict(beam="gaussian", rayleigh=(zr, 0.5 * zr),
                focus=(c[0] + w.d[0], c[1] - w.d[1], c[2] + 10 * w.d[2]))


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_gaussian_beam_optical_undulator_full_loop_matches_oracle(precision):
    """As the plane-wave case, with the wave shaped as an astigmatic Gaussian
    beam whose waist is comparable to the bunch: the whole state and the
    diagnostics against the oracle; the beam shape changes the momenta by
    far more than the bar."""
    w = _bunch_at_rest(W.config(0, steps=60))
    amp, wave = _optical_wave(w)
    beam = _gaussian_beam(w)
    say("case Gaussian-beam optical undulator", w.n, precision, beam)
    orc = oracle.from_workload(w)
    orc.set_optical_undulator(amp, **wave)
    orc.set_optical_beam(**beam)
    plane = oracle.from_workload(w)
    plane.set_optical_undulator(amp, **wave)
    sim = native.sim_from_workload(w, precision=precision, every=1)
    sim.set_optical_beam(**beam)        # kept when the wave is set afterwards
    sim.set_optical_undulator(amp, **wave)
    sim.run(60)
    sim.sync()
    orc.step(60)
    plane.step(60)
    if precision == "f64":
        compare_state(sim, orc, TOL64, "gaussian beam")
        compare_diag(sim.get_diag(), orc.diag(), TOL64, "gaussian beam")
    else:
        pos, u, alive = sim.get_particles()
        assert np.array_equal(alive, orc.alive)
        err = rel_l2(u, orc.u)
        say("gaussian beam f32 u rel-L2", err)
        assert err < 1e-4, err
    shaped = rel_l2(orc.u, plane.u)
    say("momenta, Gaussian beam against plane wave", shaped)
    assert shaped > 1e-2 and orc.lost == 0


def test_optical_beam_rejects_bad_parameters_and_plane_is_the_default():
    w = W.config(0, steps=10)
    amp, wave = _optical_wave(w)
    sim = native.sim_from_workload(w, precision="f64")
    for kw in (dict(beam=5), dict(beam="gaussian", rayleigh=(0.0, 1e-3)),
               dict(beam="gaussian", rayleigh=(1e-3, float("inf"))),
               dict(beam="gaussian", rayleigh=(1e-3, 1e-3), focus=(0.0, float("nan"), 0.0))):
        with pytest.raises(native.MithraError) as e:
            sim.set_optical_beam(**kw)
        assert e.value.status == native.EINVAL, kw
    outs = []
    for explicit in (False, True):
        s = native.sim_from_workload(_bunch_at_rest(W.config(0, steps=10)), precision="f64")
        s.set_optical_undulator(amp, **wave)
        if explicit:
            s.set_optical_beam(**_gaussian_beam(w))
            s.set_optical_beam("plane")
        s.run(10)
        s.sync()
        outs.append(s.get_particles()[1])
    assert np.array_equal(outs[0], outs[1])


def test_optical_undulator_switched_off_is_the_static_one_bitwise():
    w = W.config(0, steps=20)
    amp, wave = _optical_wave(w)
    outs = []
    for toggle in (False, True):
        sim = native.sim_from_workload(w, precision="f64")
        if toggle:
            sim.set_optical_undulator(amp, **wave)
            sim.set_optical_undulator(0.0)
        sim.run(20)
        sim.sync()
        outs.append(list(sim.get_particles()) + [sim.get_field("Ax"), sim.get_field("Ez")])
        sim.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b, equal_nan=True)


def test_optical_undulator_switched_on_mid_run_matches_oracle():
    """Steps replayed from a captured graph, then the wave switched on (the
    batch launches another push variant, so the graph is captured again),
    then more steps: the state against the oracle doing the same.  (A weak
    static undulator, K = 0.01, keeps the bunch in place before the wave.)"""
    w = _bunch_at_rest(W.make_workload("optical-switch", (32, 32, 64), 4096, 100.0, 0.01, 0.015,
                                       1e-4, 58, 40))
    amp, wave = _optical_wave(w)
    orc = oracle.from_workload(w)
    sim = native.sim_from_workload(w, precision="f64", every=1)
    sim.run(20)
    orc.step(20)
    sim.set_optical_undulator(amp, **wave)
    orc.set_optical_undulator(amp, **wave)
    sim.run(20)
    sim.sync()
    orc.step(20)
    compare_state(sim, orc, TOL64, "optical mid-run")
    compare_diag(sim.get_diag(), orc.diag(), TOL64, "optical mid-run")


def test_batch_mixing_optical_and_static_undulators_equals_separate_runs():
    """One simulation with the optical undulator, one with the static one and
    one with the optical undulator shaped as a Gaussian beam, in one batch
    (all through the optical push variant): each equals its own separate run
    bit for bit."""
    ws = [_bunch_at_rest(W.config(0, steps=30)),
          W.make_workload("static", (32, 32, 96), 3000, 120.0, 1.2, 0.015, 1e-4, 77, 30),
          _bunch_at_rest(W.config(0, steps=30, seed=991))]
    amp, wave = _optical_wave(ws[0])
    beam = _gaussian_beam(ws[2])
    b = native.batch_from_workloads(ws, precision="f64")
    b.set_optical_undulator(0, amp, **wave)
    b.set_optical_undulator(2, amp, **wave)
    b.set_optical_beam(2, **beam)
    b.run(30)
    b.sync()
    for s, w in enumerate(ws):
        sim = native.sim_from_workload(w, precision="f64")
        if s != 1:
            sim.set_optical_undulator(amp, **wave)
        if s == 2:
            sim.set_optical_beam(**beam)
        sim.run(30)
        sim.sync()
        for name in ("Ax", "Ay", "phi", "rho", "Jx"):
            assert np.array_equal(b.get_field(s, name), sim.get_field(name)), (s, name)
        for x, y in zip(b.get_particles(s), sim.get_particles()):
            assert np.array_equal(x, y, equal_nan=True), s
        assert b.get_diag(s).tobytes() == sim.get_diag().tobytes(), s
        sim.close()
    b.close()


def test_optical_undulator_rejects_bad_waves():
    w = W.config(0, steps=1)
    sim = native.sim_from_workload(w, precision="f64")
    amp, wave = _optical_wave(w)
    for bad in (dict(tau=0.0), dict(tau=-1.0), dict(frequency=-1.0), dict(signal=7),
                dict(cep=float("nan"))):
        with pytest.raises(native.MithraError) as e:
            sim.set_optical_undulator(amp, **{**wave, **bad})
        assert e.value.status == native.EINVAL
    sim.close()


def test_plane_wave_dispersion_on_gpu():
    """Property at any size: a plane wave with the frequency of eq.
    (NSFDDispersionCD) stays an exact discrete solution on the GPU too."""
    n = (32, 32, 64)
    dz = 1e-6
    d = (4 * dz, 4 * dz, dz)
    origin = (0.0, 0.0, 0.0)
    sim = native.Sim(n, d, origin, courant=0.9, bc=(1, 1, 1), space_charge=1, K=0.0,
                     gamma_beam=50.0)
    sim.set_particles(np.zeros((0, 3)), np.zeros((0, 3)), -QE, ME)
    info = sim.info()
    dt, A = info["dt"], info["nsfd_A"]
    k = (2 * math.pi / (n[0] * d[0]), 2 * math.pi * 3 / (n[1] * d[1]),
         2 * math.pi * 5 / (n[2] * d[2]))
    sx = math.sin(k[0] * d[0] / 2) ** 2 / d[0] ** 2
    sy = math.sin(k[1] * d[1] / 2) ** 2 / d[1] ** 2
    szr = math.sin(k[2] * d[2] / 2) ** 2
    w = 2.0 / dt * math.asin(C * dt * math.sqrt((1 - 4 * A * szr) * (sx + sy) + szr / d[2] ** 2))
    kk, jj, ii = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    ph = k[0] * ii * d[0] + k[1] * jj * d[1] + k[2] * kk * d[2]
    for name in POT:
        sim.set_field(name, np.cos(ph))
        sim.set_field(name + "_prev", np.cos(ph + w * dt))
    say("case plane wave")
    sim.run(150)
    sim.sync()
    for name in POT:
        assert np.max(np.abs(sim.get_field(name) - np.cos(ph - 150 * w * dt))) < 1e-10


# ---------------------------------------------------------------------------
# the whole step
# ---------------------------------------------------------------------------

def test_tiny_config_full_loop_f64():
    """32x32x64, 4096 particles, 200 steps: every array and every diagnostic."""
    w = W.config(0)
    sim, orc = run_pair(w, 200)
    compare_state(sim, orc, TOL64, "tiny")
    compare_diag(sim.get_diag(), orc.diag(), TOL64, "tiny")
    assert orc.lost == 0


@pytest.mark.parametrize("variant", ["ragged_substeps", "no_space_charge", "courant_one",
                                     "standard_scheme", "mur2"])
def test_variants_full_loop_f64(variant):
    kw = dict()
    n = (40, 44, 72)
    if variant == "ragged_substeps":
        kw = dict(substeps=2)
    elif variant == "no_space_charge":
        kw = dict(space_charge=0)
    elif variant == "courant_one":
        kw = dict(courant=1.0)
    elif variant == "mur2":
        kw = dict(bc=(2, 2, 2))
    w = W.make_workload(variant, n, 3000, 120.0, 1.3, 0.015, 1e-4, 77, 60, **kw)
    if variant == "standard_scheme":
        w.nsfd_A = 0.0
        w.courant = 0.5
    sim, orc = run_pair(w, 60)
    compare_state(sim, orc, TOL64, variant)
    compare_diag(sim.get_diag(), orc.diag(), TOL64, variant)


def test_mid_subcase_full_loop_f64():
    """64x64x128 with 65536 particles (the oracle-checkable slice of the mid
    configuration), 100 steps."""
    w = W.mid_subcase(steps=100)
    sim, orc = run_pair(w, 100)
    compare_state(sim, orc, TOL64, "mid-subcase")
    compare_diag(sim.get_diag(), orc.diag(), TOL64, "mid-subcase")


@pytest.mark.timeout(1200)
def test_mid_subcase_2000_steps_f64():
    """The oracle-checkable slice of the mid configuration (64x64x128, 65536
    particles) over the configuration's full 2000 steps: every diagnostic row
    and, at the end, every array and particle.  The oracle runs its OpenMP
    build (the same results as the plain one, bit for bit)."""
    w = W.mid_subcase(steps=2000)
    say("case", w.name, w.n, w.np, "steps", 2000, "f64 (oracle on %d threads)"
        % oracle.threads(True))
    sim = native.sim_from_workload(w, precision="f64", every=1, capacity=2048)
    sim.run(2000)
    sim.sync()
    orc = oracle.from_workload(w, parallel=True)
    for _ in range(20):
        orc.step(100)
        say("  oracle at step", orc.step_count)
    compare_state(sim, orc, TOL64, "mid-subcase-2000")
    compare_diag(sim.get_diag(), orc.diag(), TOL64, "mid-subcase-2000")


def _host_counting_sort(sim, w):
    """Bin keys of the particles from their positions (read back in SI and
    mapped to cells on the host) and the bucket starts of a counting sort.
    Positions within 1e-9 of a cell face may map to either cell on the host;
    for those the device's key must be one of the two, and it is kept."""
    pos, u, alive = sim.get_particles()
    keys, ids, starts, nkeys = sim.get_bins()
    nt = [(w.n[a] + 7) // 8 for a in range(3)]
    assert nkeys == nt[0] * nt[1] * nt[2] * 512
    dev_key = np.empty(w.np, dtype=np.int64)
    dev_key[ids] = keys  # key the device gave particle id
    v = (pos - np.asarray(w.origin)) / np.asarray(w.d)
    v[~alive] = 0.0

    def key_of(c):
        t = ((c[:, 2] // 8) * nt[1] + c[:, 1] // 8) * nt[0] + c[:, 0] // 8
        return t * 512 + ((c[:, 2] % 8) * 8 + c[:, 1] % 8) * 8 + c[:, 0] % 8

    c = np.floor(v).astype(np.int64)
    near = (v - c > 1.0 - 1e-9) & alive[:, None]
    exp_key = key_of(c)
    up = key_of(c + near.astype(np.int64))
    amb = near.any(axis=1)
    assert np.all((dev_key[amb] == exp_key[amb]) | (dev_key[amb] == up[amb]))
    exp_key[amb] = dev_key[amb]
    exp_key[~alive] = nkeys
    counts = np.bincount(exp_key, minlength=nkeys + 1)
    exp_starts = np.concatenate([[0], np.cumsum(counts)])
    return keys, ids, starts, exp_key, exp_starts, int(amb.sum())


@pytest.mark.parametrize("precision,steps", [("f64", 7), ("f32", 8), ("f32", 15)])
def test_binning_is_a_counting_sort(precision, steps):
    """After a step the particle buffer is the counting sort of the particles
    by cell key: the bucket starts equal the host's exclusive prefix sums of
    the per-key counts, exactly; every slot holds a particle of its bucket's
    key; the slots hold every particle once (lost ones in the last bucket).
    The order inside a bucket is free and not compared."""
    w = W.make_workload("bins", (64, 48, 96), 20000, 120.0, 1.3, 0.015, 1e-4, 4242, steps,
                        sigma_cells=(6.0, 5.0, 10.0))
    # a few particles start outside the live cells (lost at load)
    w.x[:5, 0] = w.origin[0] + 0.5 * w.d[0]
    say("case bins", w.n, w.np, precision, steps)
    sim = native.sim_from_workload(w, precision=precision)
    sim.run(steps)
    sim.sync()
    keys, ids, starts, exp_key, exp_starts, namb = _host_counting_sort(sim, w)
    say("  ambiguous positions", namb, "lost", int(np.sum(exp_key == len(exp_starts) - 2)))
    assert np.array_equal(starts, exp_starts)
    assert np.array_equal(np.sort(ids), np.arange(w.np))
    assert np.array_equal(keys.astype(np.int64), exp_key[ids])
    slot = np.arange(w.np)
    assert np.all((starts[keys] <= slot) & (slot < starts[keys + 1]))
    sim.close()


def test_mid_config_full_size_f64():
    """128x128x512, 1M particles, in the launch configuration the benchmark
    times: a few steps against the oracle at full size."""
    w = W.config(1)
    sim, orc = run_pair(w, 3, every=1)
    compare_state(sim, orc, TOL64, "mid-full")
    compare_diag(sim.get_diag(), orc.diag(), TOL64, "mid-full")


def _prebunched(w, ka=0.3):
    """Particles shifted along z by a sin(K z) (K = 2 gamma0 k_u), which
    gives a bunching factor near J_1(K a), far above the shot noise."""
    g0 = w.gamma_beam / math.sqrt(1.0 + w.K ** 2 / 2.0)
    kb = 2.0 * g0 * 2.0 * math.pi / w.lambda_u
    x = w.x.copy()
    x[:, 2] += (ka / kb) * np.sin(kb * x[:, 2])
    w.x = x
    return w


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_bunching_factor_matches_oracle(precision):
    """Bunching factor at harmonics 1..3 along 40 steps of a pre-bunched tiny
    bunch; FP64 with mesh terms every 4th step (the rows between hold 0)."""
    w = _prebunched(W.config(0, steps=40))
    every = 4 if precision == "f64" else 1
    tol = TOL64 if precision == "f64" else 1e-4
    sim, orc = run_pair(w, 40, precision=precision, every=every)
    gd, od = sim.get_diag(), orc.diag()
    has = gd["has_mesh_terms"] == 1
    assert has.sum() == 40 // every
    assert np.all(gd["bunching"][~has] == 0.0)
    err = rel_l2(gd["bunching"][has], od[has][:, 16:19])
    say("bunching", precision, "b1 first/last", gd["bunching"][has][0, 0],
        gd["bunching"][has][-1, 0], "rel-L2", err)
    assert gd["bunching"][has][0, 0] > 0.1
    assert err <= tol, err


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_harmonic_power_of_a_pure_tone(precision):
    """At c dt = dz a transversely uniform wave in a periodic box is an exact
    tone at the power plane (6 periods in 64 steps), and lambda_u puts the
    second harmonic of the resonant frequency on it.  Every row matches the
    oracle; after the 64 steps the second harmonic carries the mean Poynting
    flux and the first and third carry none."""
    n = (8, 8, 64)
    dz = 1e-6
    d = (4 * dz, 4 * dz, dz)
    origin = tuple(-(n[a] - 1) / 2.0 * d[a] for a in range(3))
    m, gamma, h = 6, 50.0, 2
    lambda_u = h * gamma * math.sqrt(1.0 - 1.0 / gamma ** 2) * n[2] * d[2] / m
    kw = dict(courant=1.0, bc=(1, 1, 1), K=0.0, gamma_beam=gamma, lambda_u=lambda_u)
    orc = oracle.OracleSim(n, d, origin, **kw)
    orc.set_particles(np.zeros((0, 3)), np.zeros((0, 3)), -QE, ME)
    sim = native.Sim(n, d, origin, precision=precision, **kw)
    sim.config_diag((n[0] // 2, n[1] // 2, n[2] // 2), n[2] // 2, spectrum=True)
    sim.set_particles(np.zeros((0, 3)), np.zeros((0, 3)), -QE, ME)
    kk = np.arange(n[2])
    f = lambda z: 3.0e-9 * np.cos(2.0 * math.pi * m * z / n[2] + 0.4)
    cur = np.broadcast_to(f(kk)[:, None, None], (n[2], n[1], n[0]))
    prev = np.broadcast_to(f(kk + 1)[:, None, None], (n[2], n[1], n[0]))
    orc.pot(0, "cur")[:] = cur
    orc.pot(0, "prev")[:] = prev
    sim.set_field("Ax", cur)
    sim.set_field("Ax_prev", prev)
    orc.step(n[2])
    sim.run(n[2])
    sim.sync()
    gd, od = sim.get_diag(), orc.diag()
    tol = TOL64 if precision == "f64" else 1e-5
    err = rel_l2(gd["power_harmonic"], od[:, 20:23])
    mean = gd["power"].mean()
    P = gd["power_harmonic"][-1]
    say("pure tone", precision, "P", P, "mean power", mean, "rel-L2 vs oracle", err)
    assert err <= tol, err
    assert abs(P[h - 1] / mean - 1.0) <= tol
    assert abs(P[0]) <= tol * mean and abs(P[2]) <= tol * mean


def test_further_sampling_plates_match_oracle():
    """Two further plates (one on the main plane, one nearer the bunch) on the
    tiny configuration, 60 steps: every row against the oracle; the plate on
    the main plane repeats the main power bit for bit; the unused one is 0."""
    w = W.config(0, steps=60)
    extra = (w.kp, w.kp - 12)
    orc = oracle.from_workload(w)
    orc.config_diag(w.probe, w.kp, extra_planes=extra)
    sim = native.sim_from_workload(w, precision="f64", every=1)
    sim.config_diag(w.probe, w.kp, every=1, spectrum=True, extra_planes=extra)
    sim.run(60)
    sim.sync()
    orc.step(60)
    gd = sim.get_diag()
    compare_diag(gd, orc.diag(), TOL64, "plates")
    assert np.array_equal(gd["power_extra"][:, 0], gd["power"])
    assert not gd["power_extra"][:, 2].any()
    assert np.abs(gd["power_extra"][:, 1]).max() > 0
    with pytest.raises(native.MithraError) as e:
        sim.config_diag(w.probe, w.kp, spectrum=True, extra_planes=(w.n[2],))
    assert e.value.status == native.EINVAL


def test_power_spectrum_is_off_by_default_and_fixed_after_the_first_step():
    w = W.config(0, steps=5)
    sim = native.sim_from_workload(w, spectrum=False)
    sim.run(5)
    sim.sync()
    dg = sim.get_diag()
    assert np.all(dg["power_harmonic"] == 0.0) and np.any(dg["power"] != 0.0)
    with pytest.raises(native.MithraError) as e:
        sim.config_diag(w.probe, w.kp, spectrum=True)
    assert e.value.status == native.ESTATE
    sim.close()


# ---------------------------------------------------------------------------
# float path with split positions
# ---------------------------------------------------------------------------

def test_precision_config_f32_split():
    """Float fields and push, int32 cell + float offset positions, double
    diagnostics: probe field and radiated power within 1e-3 of the FP64 oracle."""
    w = W.config(2)
    sim, orc = run_pair(w, 200, precision="f32")
    gd, od = sim.get_diag(), orc.diag()
    errs = {
        "probe_Ex": rel_l2(gd["probe_E"][:, 0], od[:, 7]),
        "power": rel_l2(gd["power"], od[:, 4]),
    }
    other = {
        "probe_E": rel_l2(gd["probe_E"], od[:, 7:10]),
        "probe_B": rel_l2(gd["probe_B"], od[:, 10:13]),
        "field_energy": rel_l2(gd["field_energy"], od[:, 5]),
        "kinetic_energy": rel_l2(gd["kinetic_energy"], od[:, 6]),
        "charge": rel_l2(gd["total_charge"], od[:, 2]),
        "Ax": rel_l2(sim.get_field("Ax"), orc.pot(0, "cur")),
        "phi": rel_l2(sim.get_field("phi"), orc.pot(3, "cur")),
    }
    # a particle lost at the mesh edge takes its charge along, which the
    # continuity residual of that step reports; check the other steps
    steady = np.concatenate([[gd["lost"][0] == 0], np.diff(gd["lost"]) == 0])
    cont = np.max(gd["continuity_residual"][steady])
    say("f32 split", errs, other, "continuity", cont, "lost", gd["lost"][-1], orc.lost)
    assert errs["probe_Ex"] <= 1e-3 and errs["power"] <= 1e-3, errs
    assert other["charge"] < 1e-6
    assert cont < 1e-5
    assert not gd["nonfinite"].any()
    assert gd["lost"][-1] == orc.lost


@pytest.mark.parametrize("index,steps", [(1, 200), (3, 100)])
def test_precision_form_on_the_mid_and_large_shapes(index, steps):
    """The float path with split positions on the 128x128x512 mesh with 1M
    particles (200 steps) and on the 256x256x2048 mesh with 16.8M particles
    (100 steps), against the double path on the GPU (which equals the oracle
    to 1e-10 on the mid mesh, see the full-size test above, and in one step
    on a box of the large one): on-axis field and radiated power within the
    float bar of 1e-3, charge within 1e-6 -- the accuracy at which the
    benchmark reports the float path's speedup."""
    w = W.config(index, steps=steps)
    say("case precision form", w.n, w.np, steps)
    rows = {}
    for precision in ("f64", "f32"):
        sim = native.sim_from_workload(w, precision=precision, every=50, spectrum=False)
        sim.run(steps)
        sim.sync()
        rows[precision] = sim.get_diag()
        sim.close()
    g, o = rows["f32"], rows["f64"]
    mesh = o["has_mesh_terms"] == 1
    errs = {"probe_Ex": rel_l2(g["probe_E"][:, 0], o["probe_E"][:, 0]),
            "power": rel_l2(g["power"], o["power"]),
            "charge": rel_l2(g["total_charge"][mesh], o["total_charge"][mesh])}
    say("precision form", errs, "lost", g["lost"][-1], o["lost"][-1])
    assert errs["probe_Ex"] <= 1e-3 and errs["power"] <= 1e-3 and errs["charge"] < 1e-6, errs
    assert not g["nonfinite"].any() and g["lost"][-1] == o["lost"][-1]


# ---------------------------------------------------------------------------
# determinism, batch, checkpoint
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_run_twice_is_bitwise_identical(precision):
    w = W.config(0, steps=50)
    outs = []
    for _ in range(2):
        sim = native.sim_from_workload(w, precision=precision)
        sim.run(50)
        sim.sync()
        outs.append(([sim.get_field(f) for f in ("Ax", "Az", "phi", "Jx", "rho", "Ex")],
                     sim.get_particles(), sim.get_diag()))
        sim.close()
    for a, b in zip(outs[0][0], outs[1][0]):
        assert np.array_equal(a, b)
    for a, b in zip(outs[0][1], outs[1][1]):
        assert np.array_equal(a, b, equal_nan=True)
    assert outs[0][2].tobytes() == outs[1][2].tobytes()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_tuned_shapes_do_not_change_the_bits(precision):
    """The tuner picks the stencil tile and the brick of tiles dealt to each
    XCD; neither changes any result: a tuned run after a few steps equals an
    untuned run bit for bit (the 64x64x128 subcase, whose tile grid admits
    several brick shapes, 24 steps)."""
    w = W.mid_subcase(steps=24)
    outs = []
    for tuned in (False, True):
        sim = native.sim_from_workload(w, precision=precision)
        sim.run(6)
        if tuned:
            sim.tune(1)
        sim.run(18)
        sim.sync()
        info = sim.info()
        say("tuned" if tuned else "default", info["stencil_tile"], info["particle_brick"])
        outs.append(([sim.get_field(f) for f in ("Ax", "Az", "phi", "Jx", "Jz", "rho")],
                     sim.get_particles(), sim.get_diag()))
        sim.close()
    for a, b in zip(outs[0][0], outs[1][0]):
        assert np.array_equal(a, b)
    for a, b in zip(outs[0][1], outs[1][1]):
        assert np.array_equal(a, b, equal_nan=True)
    assert outs[0][2].tobytes() == outs[1][2].tobytes()


def test_set_shapes_applies_them_and_keeps_the_bits():
    """Shapes set directly (what a profiler run or a tuned deployment uses)
    are the ones the launches take, give the default run's bits, and a shape
    outside the built set is refused without changing the current ones (the
    64x64x128 subcase, 16 steps, float)."""
    w = W.mid_subcase(steps=16)
    outs = []
    for shapes in (None, ([128, 2, 32], [8, 8, 1]), ([32, 8, 16], [2, 2, 16])):
        sim = native.sim_from_workload(w, precision="f32")
        if shapes is not None:
            sim.run(4)
            sim.set_shapes(*shapes)
            info = sim.info()
            assert info["stencil_tile"] == shapes[0] and info["particle_brick"] == shapes[1]
            for bad in (([100, 2, 32], [8, 8, 1]), ([128, 2, 0], [8, 8, 1]),
                        ([128, 2, 32], [0, 8, 1])):
                with pytest.raises(native.MithraError):
                    sim.set_shapes(*bad)
            assert sim.info()["stencil_tile"] == shapes[0]
            sim.run(12)
        else:
            sim.run(16)
        sim.sync()
        outs.append(([sim.get_field(f) for f in ("Ax", "Az", "phi", "Jx", "rho")],
                     sim.get_particles(), sim.get_diag()))
        sim.close()
    for o in outs[1:]:
        for a, b in zip(outs[0][0], o[0]):
            assert np.array_equal(a, b)
        for a, b in zip(outs[0][1], o[1]):
            assert np.array_equal(a, b, equal_nan=True)
        assert outs[0][2].tobytes() == o[2].tobytes()
    # the batch form: one shape for every simulation
    ws = [W.make_workload("s%d" % i, n, npart, g, K, 0.015, 1e-4, 300 + i, 12)
          for i, (n, npart, g, K) in enumerate([((32, 32, 128), 3000, 90.0, 0.9),
                                                  ((48, 48, 96), 6000, 150.0, 1.6)])]
    res = []
    for shapes in (None, ([64, 2, 16], [2, 2, 2])):
        b = native.batch_from_workloads(ws, precision="f32")
        if shapes is not None:
            b.set_shapes(*shapes)
            with pytest.raises(native.MithraError):
                b.set_shapes([64, 3, 16], [2, 2, 2])
            assert b.info(1)["stencil_tile"] == shapes[0]
        b.run(12)
        b.sync()
        res.append([b.get_field(s, f) for s in range(2) for f in ("Ax", "phi", "Jz")] +
                   [b.get_diag(s).tobytes() for s in range(2)])
        b.close()
    for x, y in zip(res[0], res[1]):
        assert np.array_equal(x, y) if isinstance(x, np.ndarray) else x == y


def test_graph_with_two_streams_equals_kernel_by_kernel_bitwise():
    """The captured step runs the scan and scatter on a second stream beside
    the deposit; kernel-by-kernel execution on one stream (timing mode) must
    give the same bits (64x64x128 subcase, 30 steps, more steps than one
    captured graph)."""
    w = W.mid_subcase(steps=30)
    outs = []
    for timed in (False, True):
        sim = native.sim_from_workload(w, precision="f32")
        sim.set_timing(timed)
        sim.run(30)
        sim.sync()
        outs.append(([sim.get_field(f) for f in ("Ax", "Ay", "phi", "Jx", "Jz", "rho")],
                     sim.get_particles(), sim.get_diag()))
        sim.close()
    for a, b in zip(outs[0][0], outs[1][0]):
        assert np.array_equal(a, b)
    for a, b in zip(outs[0][1], outs[1][1]):
        assert np.array_equal(a, b, equal_nan=True)
    assert outs[0][2].tobytes() == outs[1][2].tobytes()


def test_batch_equals_separate_runs_bitwise():
    ws = [W.make_workload("b%d" % i, n, npart, g, K, 0.015, 1e-4, 100 + i, 40)
          for i, (n, npart, g, K) in enumerate([((32, 32, 128), 3000, 90.0, 0.9),
                                                  ((48, 48, 192), 8000, 150.0, 1.6),
                                                  ((40, 40, 160), 5000, 220.0, 1.2)])]
    say("case batch", [w.n for w in ws])
    b = native.batch_from_workloads(ws, precision="f32")
    b.run(40)
    b.sync()
    for s, w in enumerate(ws):
        sim = native.sim_from_workload(w, precision="f32")
        sim.run(40)
        sim.sync()
        for f in ("Ax", "Ay", "Az", "phi", "Jz", "rho", "Ex", "By"):
            assert np.array_equal(b.get_field(s, f), sim.get_field(f)), (s, f)
        pb, ub, ab = b.get_particles(s)
        ps, us, as_ = sim.get_particles()
        assert np.array_equal(ab, as_)
        assert np.array_equal(pb[ab], ps[as_]) and np.array_equal(ub, us)
        assert b.get_diag(s).tobytes() == sim.get_diag().tobytes()
        sim.close()


def test_batch_with_mixed_boundaries_equals_separate_runs():
    """A batch whose simulations use first-order Mur, second-order Mur and a
    periodic axis with second-order Mur on the others matches the separate
    runs bit for bit (per-simulation boundary tables and stencil faces)."""
    specs = [((32, 32, 128), 3000, 90.0, 0.9, (0, 0, 0)),
             ((40, 40, 160), 4000, 150.0, 1.6, (2, 2, 2)),
             ((48, 48, 128), 5000, 220.0, 1.2, (1, 2, 2))]
    ws = [W.make_workload("m%d" % i, n, npart, g, K, 0.015, 1e-4, 500 + i, 30, bc=bc)
          for i, (n, npart, g, K, bc) in enumerate(specs)]
    say("case mixed-boundary batch", [(w.n, w.bc) for w in ws])
    b = native.batch_from_workloads(ws, precision="f32")
    b.run(30)
    b.sync()
    for s, w in enumerate(ws):
        sim = native.sim_from_workload(w, precision="f32")
        sim.run(30)
        sim.sync()
        for f in ("Ax", "Ay", "Az", "phi", "Jx", "rho", "Ez", "Bx"):
            assert np.array_equal(b.get_field(s, f), sim.get_field(f)), (s, f)
        assert b.get_diag(s).tobytes() == sim.get_diag().tobytes()
        sim.close()
    b.close()


@pytest.mark.timeout(900)
def test_batch_config_full_size_sims_equal_separate_runs_bitwise():
    """The 64-simulation scan at its full sizes, 200 steps in one batch; the
    simulations with the fewest and the most cells and the median one, each
    run alone for 200 steps, give the same fields, particles and diagnostic
    rows bit for bit."""
    steps = 200
    ws = W.batch_configs(64, steps=steps)
    say("case full batch, bitwise", len(ws), "simulations", steps, "steps")
    b = native.batch_from_workloads(ws, precision="f32", every=10, spectrum=False,
                                    capacity=steps + 8)
    b.run(steps)
    b.sync()
    order = sorted(range(len(ws)), key=lambda i: ws[i].ncell)
    for s in (order[0], order[len(order) // 2], order[-1]):
        w = ws[s]
        say("  simulation", s, w.n, w.np)
        sim = native.sim_from_workload(w, precision="f32", every=10, spectrum=False,
                                       capacity=steps + 8)
        sim.run(steps)
        sim.sync()
        for f in ("Ax", "Ay", "Az", "phi", "Jx", "Jy", "Jz", "rho", "Ex", "By"):
            assert np.array_equal(b.get_field(s, f), sim.get_field(f)), (s, f)
        pb, ub, ab = b.get_particles(s)
        ps, us, as_ = sim.get_particles()
        assert np.array_equal(ab, as_), s
        assert np.array_equal(pb[ab], ps[as_]) and np.array_equal(ub, us), s
        assert b.get_diag(s).tobytes() == sim.get_diag().tobytes(), s
        sim.close()
    b.close()


def test_batch_tuned_matches_oracle_f64():
    ws = [W.make_workload("t%d" % i, n, npart, g, K, 0.015, 1e-4, 300 + i, 30)
          for i, (n, npart, g, K) in enumerate([((32, 32, 64), 2000, 100.0, 1.0),
                                                  ((40, 32, 96), 3000, 140.0, 1.5)])]
    b = native.batch_from_workloads(ws, precision="f64")
    b.tune(2)
    b.run(30)
    b.sync()
    for s, w in enumerate(ws):
        orc = oracle.from_workload(w)
        orc.step(30)
        for c, name in enumerate(POT):
            assert rel_l2(b.get_field(s, name), orc.pot(c, "cur")) < TOL64
        pos, u, alive = b.get_particles(s)
        assert rel_l2(u, orc.u) < TOL64
        compare_diag(b.get_diag(s), orc.diag(), TOL64, "batch-f64-%d" % s)


def test_batch_config_full_size_f32():
    """The 64-simulation parameter scan at its full sizes (32x32x128 to
    96x96x384, 16K-256K particles each), tuned and run as the benchmark runs
    it, in float with split positions.  Every simulation: charge equal to the
    live particles' charge, continuity to float round-off, finite values.
    Three sampled simulations (fewest cells, most cells, the median) against
    the oracle on the float bar."""
    steps = 12
    ws = W.batch_configs(64, steps=steps)
    say("case full batch", len(ws), "cells", sum(w.ncell for w in ws),
        "particles", sum(w.np for w in ws))
    b = native.batch_from_workloads(ws, precision="f32", every=1, spectrum=False)
    b.tune(2)
    say("tuned", b.info(0)["stencil_tile"])
    b.run(steps)
    b.sync()
    diag = [b.get_diag(s) for s in range(len(ws))]  # reading marks the rows read
    for s, w in enumerate(ws):
        gd = diag[s]
        assert len(gd) == steps and not gd["nonfinite"].any(), s
        live = w.np - gd["lost"]
        assert np.all(np.abs(gd["total_charge"] - live * w.q) <= 1e-6 * abs(w.np * w.q)), s
        steady = np.concatenate([[gd["lost"][0] == 0], np.diff(gd["lost"]) == 0])
        assert np.max(gd["continuity_residual"][steady]) < 1e-5, s
    order = sorted(range(len(ws)), key=lambda i: ws[i].ncell)
    for s in (order[0], order[len(order) // 2], order[-1]):
        w = ws[s]
        say("oracle for simulation", s, w.n, w.np)
        orc = oracle.from_workload(w)
        orc.step(steps)
        gd, od = diag[s], orc.diag()
        assert np.array_equal(gd["lost"], od[:, 13].astype(np.int64)), s
        errs = {"probe_Ex": rel_l2(gd["probe_E"][:, 0], od[:, 7]),
                "power": rel_l2(gd["power"], od[:, 4]),
                "charge": rel_l2(gd["total_charge"], od[:, 2])}
        say("simulation", s, errs)
        assert errs["probe_Ex"] <= 1e-3 and errs["power"] <= 1e-3 and errs["charge"] < 1e-6, errs
        pos, u, alive = b.get_particles(s)
        assert np.array_equal(alive, orc.alive), s
    b.close()


def test_checkpoint_resume_is_bitwise():
    w = W.config(0, steps=30)
    sim = native.sim_from_workload(w)
    sim.run(10)
    blob = sim.get_state()
    sim.run(20)
    sim.sync()
    ref = [sim.get_field(f) for f in ("Ax", "phi", "Jy", "rho", "Bz")] + list(sim.get_particles())
    sim2 = native.sim_from_workload(w)
    sim2.set_state(blob)
    sim2.run(20)
    sim2.sync()
    got = [sim2.get_field(f) for f in ("Ax", "phi", "Jy", "rho", "Bz")] + list(sim2.get_particles())
    for a, b in zip(ref, got):
        assert np.array_equal(a, b, equal_nan=True)
    # the rows after the restart too, the plane spectrum included
    assert sim.get_diag()[10:].tobytes() == sim2.get_diag().tobytes()


def test_corrupt_checkpoints_are_rejected_and_change_nothing():
    """A blob with a negative step or particle count, a live particle outside
    the safe interior, an offset outside [0, 1] or non-finite momenta, or one
    cut short, is refused before anything changes: the simulation then runs
    exactly as one that was never given it."""
    w = W.config(0, steps=10)
    src = native.sim_from_workload(w)
    src.run(3)
    blob = bytearray(src.get_state())
    head = 56                               # magic, 6 int32, step, np, ncell
    ncell, npart = w.ncell, w.np
    parts = head + 13 * ncell * 8           # after 13 FP64 mesh arrays
    alive = np.frombuffer(bytes(blob[parts:parts + npart]), dtype=np.uint8)
    p = int(np.argmax(alive == 1))
    cell_at = parts + npart + 12 * p        # int32 cell of particle p, x
    off_at = parts + npart + 12 * npart + 24 * p
    mom_at = parts + npart + 12 * npart + 24 * npart + 24 * p

    def patched(at, fmt, value):
        b = bytearray(blob)
        b[at:at + np.dtype(fmt).itemsize] = np.array([value], dtype=fmt).tobytes()
        return bytes(b)

    bad = {"negative step": patched(32, np.int64, -1),
           "negative count": patched(40, np.int64, -5),
           "cell far outside": patched(cell_at, np.int32, 1 << 20),
           "cell in the lost margin": patched(cell_at, np.int32, 1),
           "offset above one": patched(off_at, np.float64, 2.0),
           "momentum not finite": patched(mom_at, np.float64, np.inf),
           "cut short": bytes(blob[:-8])}
    sim = native.sim_from_workload(w)
    ref = native.sim_from_workload(w)
    for what, b in bad.items():
        say("case corrupt blob:", what)
        with pytest.raises(native.MithraError) as e:
            sim.set_state(b)
        assert e.value.status == native.EINVAL, what
    for s in (sim, ref):
        s.run(5)
        s.sync()
    for f in ("Ax", "phi", "Jz", "rho"):
        assert np.array_equal(sim.get_field(f), ref.get_field(f)), f
    assert sim.get_diag().tobytes() == ref.get_diag().tobytes()
    sim.set_state(bytes(blob))  # the intact blob is still accepted


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------

def test_empty_bunch_and_minimal_mesh():
    n = (8, 8, 8)
    d = (4e-6, 4e-6, 1e-6)
    origin = (-14e-6, -14e-6, -3.5e-6)
    sim = native.Sim(n, d, origin)
    sim.set_particles(np.zeros((0, 3)), np.zeros((0, 3)), -QE, ME)
    sim.run(10)
    sim.sync()
    assert np.all(sim.get_field("Ax") == 0.0)
    dg = sim.get_diag()
    assert len(dg) == 10 and not dg["nonfinite"].any()


def test_particles_outside_the_safe_interior_are_counted_lost():
    w = W.config(0, n_particles=64, steps=1)
    x = w.x.copy()
    x[3] = [w.origin[0] + 0.5 * w.d[0], 0.0, 0.0]           # cell 0 in x
    x[7] = [0.0, 0.0, w.origin[2] + (w.n[2] - 2.5) * w.d[2]]  # cell n-3 is the last allowed
    x[9] = [0.0, 0.0, w.origin[2] + (w.n[2] - 1.5) * w.d[2]]  # cell n-2: lost
    w.x = x
    sim, orc = run_pair(w, 1)
    pos, u, alive = sim.get_particles()
    assert not alive[3] and alive[7] and not alive[9]
    assert np.array_equal(alive, orc.alive)
    assert sim.get_diag()["lost"][-1] == orc.lost == 2
    compare_state(sim, orc, TOL64, "lost")


def test_many_lost_particles_are_carried_along():
    """Lost particles stay in their bucket from step to step, in more than one
    block's worth (600), next to live ones; every particle keeps its data."""
    w = W.config(0, n_particles=1000, steps=6)
    rng = np.random.default_rng(11)
    x = w.x.copy()
    far = rng.choice(len(x), 600, replace=False)
    x[far, 2] = w.origin[2] + (w.n[2] - 1.5) * w.d[2]  # cell n-2 in z: lost in step 1
    w.x = x
    sim, orc = run_pair(w, 6)
    pos, u, alive = sim.get_particles()
    assert orc.lost >= 600 and sim.get_diag()["lost"][-1] == orc.lost
    assert not alive[far].any()
    compare_state(sim, orc, TOL64, "many lost")


def test_invalid_meshes_are_rejected():
    n = (16, 16, 16)
    d = (1e-6, 1e-6, 1e-6)  # cubic cells: unstable for the NSFD scheme at courant 0.9
    with pytest.raises(native.MithraError) as e:
        native.Sim(n, d, (0, 0, 0), courant=0.9)
    assert e.value.status == native.EINVAL and "unstable" in str(e.value)
    with pytest.raises(native.MithraError) as e:
        native.Sim(n, (4e-6, 4e-6, 1e-6), (0, 0, 0), courant=1.2)
    assert e.value.status == native.EINVAL
    with pytest.raises(native.MithraError) as e:
        native.Sim((4, 16, 16), (4e-6, 4e-6, 1e-6), (0, 0, 0))
    assert e.value.status == native.EINVAL
    with pytest.raises(native.MithraError) as e:  # Mur orders cannot be mixed
        native.Sim(n, (4e-6, 4e-6, 1e-6), (0, 0, 0), bc=(0, 2, 2))
    assert e.value.status == native.EINVAL and "mixed" in str(e.value)
    with pytest.raises(native.MithraError) as e:
        native.Sim(n, (4e-6, 4e-6, 1e-6), (0, 0, 0), bc=(3, 0, 0))
    assert e.value.status == native.EINVAL
    sim = native.Sim(n, (4e-6, 4e-6, 1e-6), (0, 0, 0), bc=(0, 0, 1))
    with pytest.raises(native.MithraError) as e:  # the seed enters through z_min
        sim.set_seed(1e-3, tau=1e-15)
    assert e.value.status == native.EINVAL and "z axis" in str(e.value)
    sim.close()
    sim = native.Sim(n, (4e-6, 4e-6, 1e-6), (0, 0, 0))
    for bad in (dict(tau=0.0), dict(tau=1e-15, signal=7), dict(tau=1e-15, frequency=-1.0),
                dict(tau=1e-15, t0=float("nan"))):
        with pytest.raises(native.MithraError) as e:
            sim.set_seed(1e-3, **bad)
        assert e.value.status == native.EINVAL, bad
    sim.set_seed(0.0)  # clearing is always valid
    sim.close()


def test_run_before_particles_is_a_state_error():
    sim = native.Sim((16, 16, 16), (4e-6, 4e-6, 1e-6), (0, 0, 0))
    with pytest.raises(native.MithraError) as e:
        sim.run(1)
    assert e.value.status == native.ESTATE


def test_device_bytes_follow_reallocations():
    """device_bytes is what the simulation holds: a re-laid diagnostic ring
    (and its per-row spectra) replaces the old one, and re-loading particles
    leaves no blocks behind."""
    w = W.config(0, steps=4)
    sim = native.sim_from_workload(w)  # ring of 4096 rows of 29 doubles
    row = 29 * 8  # bytes of one row of the device ring
    srow = 2 * 3 * 8  # and of its spectrum row (3 frequencies, bunch frame and lab)

    def block(n):  # device blocks are sized in multiples of 256 bytes
        return (n + 255) // 256 * 256

    b0 = sim.info()["device_bytes"]
    sim.config_diag(w.probe, w.kp, capacity=100)
    b1 = sim.info()["device_bytes"]
    assert b0 - b1 == (block(4096 * row) - block(100 * row) + block(4096 * srow) -
                       block(100 * srow))
    sim.config_diag(w.probe, w.kp, capacity=4096)
    assert sim.info()["device_bytes"] == b0
    sim.set_particles(w.x, w.u, w.q, w.m)
    assert sim.info()["device_bytes"] == b0
    sim.run(1)
    sim.sync()
    b2 = sim.info()["device_bytes"]
    with pytest.raises(native.MithraError) as e:  # fixed once stepping began
        sim.config_diag(w.probe, w.kp, capacity=100)
    assert e.value.status == native.ESTATE
    assert sim.info()["device_bytes"] == b2
    sim.run(3)
    sim.sync()
    assert len(sim.get_diag()) == 4


def test_particle_count_beyond_32_bit_offsets_is_rejected():
    """More particles than 32-bit bucket offsets hold are refused before any
    array is read (the count alone decides; the arrays passed are short)."""
    sim = native.Sim((16, 16, 16), (4e-6, 4e-6, 1e-6), (0, 0, 0))
    pos = np.zeros((1, 3))
    too_many = (1 << 31) - (1 << 20) + 1
    st = sim._lib.mithra_set_particles(sim._h, too_many, native._dptr(pos), native._dptr(pos),
                                       -QE, ME)
    assert st == native.EINVAL
    assert b"at most" in sim._lib.mithra_last_error()
    sim.set_particles(np.zeros((0, 3)), np.zeros((0, 3)), -QE, ME)  # still usable
    sim.run(1)
    sim.sync()


def test_overflowing_field_is_reported_as_numeric_error():
    """A potential that overflows the float range makes the momenta non-finite;
    the particle is counted lost and sync reports ENUMERIC."""
    w = W.config(0, n_particles=256, steps=2)
    sim = native.sim_from_workload(w, precision="f32")
    big = np.full((w.n[2], w.n[1], w.n[0]), 3e38)
    big[::2] = -3e38
    sim.set_field("Ax", big)
    sim.run(1)
    with pytest.raises(native.MithraError) as e:
        sim.sync()
    assert e.value.status == native.ENUMERIC
    sim.sync()  # the flag is cleared once reported


# ---------------------------------------------------------------------------
# the large float configuration at full size (properties that hold at any size)
# ---------------------------------------------------------------------------

def test_large_config_f32_properties():
    """256x256x2048 with 16.8M particles: charge conserved, continuity at
    round-off of the float deposit, nothing lost, everything finite."""
    w = W.config(3)
    say("case large", w.n, w.np)
    sim = native.sim_from_workload(w, precision="f32", every=5)
    sim.run(10)
    sim.sync()
    dg = sim.get_diag()
    mesh = dg[dg["has_mesh_terms"] == 1]
    total = w.q * w.np
    assert len(mesh) == 2
    assert np.max(np.abs(mesh["total_charge"] / total - 1.0)) < 1e-5
    assert np.max(mesh["continuity_residual"]) < 1e-5
    assert dg["lost"][-1] == 0 and not dg["nonfinite"].any()
    assert np.all(np.isfinite(dg["power"]))


@pytest.mark.parametrize("precision,bar", [("f32", 1e-6), ("f64", 1e-12)])
def test_large_config_one_step_against_the_oracle_on_a_box(precision, bar):
    """256x256x2048 with 16.8M particles, in float with split positions and
    in double, tuned as the benchmark runs them: after a few steps, one more
    step of the whole mesh against one oracle step of a 48x48x64-cell box at
    the bunch centre (about 360K particles) loaded with the state before it.
    Away from the box faces the two compute the same quantities (the box cut
    is checked on the CPU).  Both sides start from the same state, so what
    differs is the rounding of one step's arithmetic: in float a few units of
    2^-24, bar 1e-6 relative L2 (16 units); in double a few units of 2^-53,
    bar 1e-12; for every field, the momenta and, in cells, the positions."""
    w = W.config(3)
    say("case large box", w.n, w.np, precision)
    sim = native.sim_from_workload(w, precision=precision, every=100, spectrum=False)
    sim.tune(3)
    sim.run(4)
    sim.sync()
    step = sim.info()["step"]
    lo, hi = (104, 104, 992), (152, 152, 1056)
    sl = subbox.box_slices(lo, hi)
    names = list(subbox.POT) + [n + "_prev" for n in subbox.POT] + list(subbox.SRC)
    fields = {n: sim.get_field(n)[sl].copy() for n in names}
    x0, u0, alive0 = sim.get_particles()
    assert alive0.all()
    box, sel = subbox.load_box(w, lo, hi, fields, x0, u0, alive0, step)
    keep = subbox.compared_particles(w, lo, hi, x0, sel)
    say("step", step, "loaded", int(sel.sum()), "compared", int(keep.sum()))
    sim.run(1)
    sim.sync()
    box.step(1)
    assert box.lost == 0
    errs = {}
    for c, name in enumerate(subbox.POT):
        errs[name] = rel_l2(subbox.inner(sim.get_field(name)[sl], subbox.MARGIN_POT),
                            subbox.inner(box.pot(c, "cur"), subbox.MARGIN_POT))
    for v, get in (("E", box.E), ("B", box.B)):
        g = np.stack([subbox.inner(sim.get_field(v + a)[sl], subbox.MARGIN_EB) for a in "xyz"])
        o = np.stack([subbox.inner(get(c), subbox.MARGIN_EB) for c in range(3)])
        errs[v] = rel_l2(g, o)
    g = np.stack([subbox.inner(sim.get_field(n)[sl], subbox.MARGIN_SRC) for n in subbox.SRC[:3]])
    o = np.stack([subbox.inner(box.J(c), subbox.MARGIN_SRC) for c in range(3)])
    errs["J"] = rel_l2(g, o)
    errs["rho"] = rel_l2(subbox.inner(sim.get_field("rho")[sl], subbox.MARGIN_SRC),
                         subbox.inner(box.rho, subbox.MARGIN_SRC))
    x1, u1, alive1 = sim.get_particles()
    assert alive1.all()
    errs["u"] = rel_l2(u1[sel][keep], box.u[keep])
    errs["x_cells"] = float(np.max(np.abs(x1[sel][keep] - box.x[keep]) / np.asarray(w.d)))
    say("large box", errs)
    bad = {k: v for k, v in errs.items() if not v <= bar}
    assert not bad, (bad, errs)
    sim.close()


# ---------------------------------------------------------------------------
# the paper's infrared FEL example, run to saturation
# ---------------------------------------------------------------------------

def test_example1_grows_exponentially_and_saturates():
    """Example 1 (64x64x2800, 131072 particles, job-file reading: Gaussian
    transverse profile, tapered flat top, bunching 0.01, second-order Mur, no
    space charge), 6000 steps = 3 m of undulator.  The power through the plane
    ahead of the bunch grows exponentially and saturates; the fitted power gain
    length lies between M. Xie's three-dimensional estimate for this beam and
    1.5 times it.  (The paper reports 0.22 m, about its one-dimensional value;
    this run gives about 0.5 m: the bunch is only a few cooperation lengths
    long, see the longer-bunch test below.)"""
    import bench
    w = W.example1(steps=6000)
    say("case example1", w.n, w.np)
    sim = native.sim_from_workload(w, precision="f64", every=100, capacity=6100)
    sim.run(6000)
    sim.sync()
    dg = sim.get_diag()
    info = sim.info()
    dz_step = info["gamma0"] * info["beta0"] * C * info["dt"]
    lg, z_sat, p_sat, a, b = bench.gain_length(dg["power"], dz_step)
    rho, l1, l3 = bench.fel_theory(w.gamma_beam, w.K, w.lambda_u, 260e-6, 88.5, 1e-4)
    say("example1 gain length", lg, "1D", l1, "3D fit", l3, "saturation at", z_sat, "m, peak",
        p_sat, "W, fit steps", a, b, "lost", dg["lost"][-1])
    assert not dg["nonfinite"].any()
    assert dg["lost"][-1] < 0.01 * w.np
    assert 1.5 < z_sat < 2.95  # the peak lies inside the run, not at its end
    assert b - a > 1000  # more than half a metre of exponential growth
    assert l3 < lg < 1.5 * l3, (lg, l1, l3)


def _example1_gain_length(**kw):
    import bench
    w = W.example1(steps=6000, **kw)
    sim = native.sim_from_workload(w, precision="f64", every=100, capacity=6100, spectrum=False)
    sim.run(6000)
    sim.sync()
    dg = sim.get_diag()
    info = sim.info()
    sim.close()
    assert not dg["nonfinite"].any() and dg["lost"][-1] < 0.01 * w.np
    dz_step = info["gamma0"] * info["beta0"] * C * info["dt"]
    return bench.gain_length(dg["power"], dz_step)[0]


def test_example1_longer_bunch_grows_faster():
    """Slippage: the job's flat top (100.5 um) is only a few cooperation
    lengths lambda_r / (4 pi rho) long, so the radiation leaves the bunch
    before it has grown much.  Four times the flat top at the same density
    (402 um, 524288 particles, 64x64x6400) grows clearly faster, and still no
    faster than the one-dimensional limit of this density."""
    import bench
    lg1 = _example1_gain_length()
    lg4 = _example1_gain_length(n=(64, 64, 6400), n_particles=524288, flat_top=402e-6)
    rho, l1, l3 = bench.fel_theory(100.41, 1.417, 0.03, 260e-6, 88.5, 1e-4)
    say("example1 gain length, job bunch", lg1, "four times longer", lg4, "1D", l1)
    assert lg4 < 0.85 * lg1, (lg1, lg4)
    assert lg4 > l1, (lg4, l1)


def test_plain_c_caller_equals_the_binding_bitwise(tmp_path):
    """The library used from C alone (tests/abi_driver.c: no Python, no
    PyTorch, device memory from hipMalloc, its own stream) gives the same
    diagnostic rows and A_x, bit for bit, as the Python binding on PyTorch's
    allocator and stream: the tiny configuration, 40 steps."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pkg = os.path.join(root, "paper_1612_03310_amd")
    exe = tmp_path / "abi_driver"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(root, "include"),
                           os.path.join(root, "tests", "abi_driver.c"), "-L", pkg, "-lmithra",
                           "-Wl,-rpath," + pkg, "-Wl,-rpath-link,/opt/rocm/lib", "-o", str(exe)])
    w = W.config(0, steps=40)
    head = (list(w.n) + list(w.d) + list(w.origin) + [w.courant, w.nsfd_A, w.substeps,
            w.space_charge] + list(w.bc) + [w.lambda_u, w.K, w.gamma_beam, w.z_e, w.q, w.m,
            w.np, 40] + list(w.probe) + [w.kp, w.und_length, 0.0])
    inp = tmp_path / "in.bin"
    with open(inp, "wb") as f:
        np.asarray(head, dtype=np.float64).tofile(f)
        np.ascontiguousarray(w.x, dtype=np.float64).tofile(f)
        np.ascontiguousarray(w.u, dtype=np.float64).tofile(f)
    out = tmp_path / "out.bin"
    say("case plain C caller", w.n, w.np)
    subprocess.run([str(exe), str(inp), str(out)], check=True, timeout=120)
    raw = out.read_bytes()
    nrows = int(np.frombuffer(raw[:8], dtype=np.int64)[0])
    rowbytes = native.DIAG_DTYPE.itemsize * nrows
    c_rows = raw[8:8 + rowbytes]
    c_ax = np.frombuffer(raw[8 + rowbytes:], dtype=np.float64).reshape(w.n[2], w.n[1], w.n[0])
    sim = native.sim_from_workload(w, precision="f64", every=1, spectrum=False)
    sim.run(40)
    sim.sync()
    assert nrows == 40
    assert sim.get_diag().tobytes() == c_rows
    assert np.array_equal(sim.get_field("Ax"), c_ax)
