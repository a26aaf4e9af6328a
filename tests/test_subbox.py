"""The box-cut oracle step used by the full-size checks, checked on the CPU:
a step of a box loaded from a whole-mesh state equals, away from the box
faces, the step of the whole mesh."""
import numpy as np

import oracle
import subbox
from paper_1612_03310_amd import workloads as W

TOL = 1e-10


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def snapshot(orc, sl):
    f = {}
    for c, name in enumerate(subbox.POT):
        f[name] = orc.pot(c, "cur")[sl].copy()
        f[name + "_prev"] = orc.pot(c, "prev")[sl].copy()
    for c in range(3):
        f[subbox.SRC[c]] = orc.J(c)[sl].copy()
    f["rho"] = orc.rho[sl].copy()
    return f


def test_box_step_equals_whole_mesh_step():
    w = W.config(0, steps=4)
    whole = oracle.from_workload(w)
    whole.step(3)
    lo, hi = (2, 3, 6), (30, 29, 58)
    sl = subbox.box_slices(lo, hi)
    fields = snapshot(whole, sl)
    x0, u0, alive0 = whole.x.copy(), whole.u.copy(), whole.alive.copy()
    box, sel = subbox.load_box(w, lo, hi, fields, x0, u0, alive0, whole.step_count)
    assert sel.sum() > 0.9 * w.np
    whole.step(1)
    box.step(1)
    assert box.lost == 0 and whole.lost == 0
    errs = {}
    for c, name in enumerate(subbox.POT):
        errs[name] = rel(subbox.inner(box.pot(c, "cur"), subbox.MARGIN_POT),
                         subbox.inner(whole.pot(c, "cur")[sl], subbox.MARGIN_POT))
    for c in range(3):
        errs["E%d" % c] = rel(subbox.inner(box.E(c), subbox.MARGIN_EB),
                              subbox.inner(whole.E(c)[sl], subbox.MARGIN_EB))
        errs["B%d" % c] = rel(subbox.inner(box.B(c), subbox.MARGIN_EB),
                              subbox.inner(whole.B(c)[sl], subbox.MARGIN_EB))
    J_box = np.stack([subbox.inner(box.J(c), subbox.MARGIN_SRC) for c in range(3)])
    J_whole = np.stack([subbox.inner(whole.J(c)[sl], subbox.MARGIN_SRC) for c in range(3)])
    errs["J"] = rel(J_box, J_whole)
    errs["rho"] = rel(subbox.inner(box.rho, subbox.MARGIN_SRC),
                      subbox.inner(whole.rho[sl], subbox.MARGIN_SRC))
    keep = subbox.compared_particles(w, lo, hi, x0, sel)
    assert keep.sum() > 0.5 * w.np
    errs["x"] = rel(box.x[keep], whole.x[sel][keep])
    errs["u"] = rel(box.u[keep], whole.u[sel][keep])
    print(errs)
    assert all(v <= TOL for v in errs.values()), errs


def test_box_margins_are_needed():
    """The comparison fails when it reaches into the face layers: the box
    faces are absorbing, the whole mesh has interior values there."""
    w = W.config(0, steps=4)
    whole = oracle.from_workload(w)
    whole.step(3)
    lo, hi = (2, 3, 6), (30, 29, 58)
    sl = subbox.box_slices(lo, hi)
    fields = snapshot(whole, sl)
    box, _ = subbox.load_box(w, lo, hi, fields, whole.x.copy(), whole.u.copy(),
                             whole.alive.copy(), whole.step_count)
    whole.step(1)
    box.step(1)
    assert rel(box.pot(3, "cur"), whole.pot(3, "cur")[sl]) > 1e-6
