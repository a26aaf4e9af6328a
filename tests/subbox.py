"""One oracle step on a box of cells cut out of a larger mesh.

The box is loaded with a state taken elsewhere: the potentials at levels n and
n-1, the sources J^n and rho^{n+1/2}, the particles whose cell lies inside it
and the step counter.  Away from the box faces one oracle step of the box
equals one step of the whole mesh, because every part of the step is local:
the potential update (eq. updateEquation) reaches one cell, E and B at a
vertex (section "Field Evaluation") one more, the linear gather the cell's
eight vertices, and the charge-conserving deposit the vertices and edges of
the start and end cells.  The margins below follow from those reaches; the
box faces themselves get the oracle's absorbing boundary, which the whole
mesh does not have there.
"""
import numpy as np

import oracle

POT = ("Ax", "Ay", "Az", "phi")
SRC = ("Jx", "Jy", "Jz", "rho")

# cells kept away from the box faces, per quantity compared
MARGIN_POT = 2      # potentials at n+1: the update's reach plus the face layer
MARGIN_EB = 3       # E, B at n+1/2: central differences of the potentials
PART_LO = 5         # particles compared: start cell in [PART_LO, n - 1 - PART_LO]
MARGIN_SRC = 7      # J^{n+1}, rho^{n+3/2}: every particle that reaches the cell is in the box
LOAD_LO = 3         # particles loaded: cell in [LOAD_LO, n - 1 - LOAD_LO]


def box_slices(lo, hi):
    """Index of the box in a (nz, ny, nx) array; lo, hi in (x, y, z) order."""
    return (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))


def inner(a, m):
    """The part of a (nz, ny, nx) box array at least m cells from its faces."""
    return a[m:a.shape[0] - m, m:a.shape[1] - m, m:a.shape[2] - m]


def cells(w, x):
    """Cell index (x, y, z) of positions in the whole mesh of workload w."""
    return np.floor((x - np.asarray(w.origin)) / np.asarray(w.d)).astype(np.int64)


def load_box(w, lo, hi, fields, x, u, alive, step):
    """Oracle on the box [lo, hi) of w's mesh holding `fields` (box arrays,
    (nz, ny, nx), by name: Ax..phi, Ax_prev..phi_prev, Jx..Jz, rho), the live
    particles x, u whose cell lies at least LOAD_LO cells inside the box, and
    the step counter.  Returns the oracle and the mask of loaded particles."""
    lo = np.asarray(lo)
    hi = np.asarray(hi)
    n = tuple(int(v) for v in hi - lo)
    d = np.asarray(w.d)
    origin = tuple(float(v) for v in np.asarray(w.origin) + lo * d)
    orc = oracle.OracleSim(n, w.d, origin, w.courant, w.nsfd_A, w.substeps, w.space_charge,
                           w.bc, w.lambda_u, w.K, w.gamma_beam, w.z_e)
    c = cells(w, np.where(alive[:, None], x, 0.0)) - lo
    sel = alive & np.all((c >= LOAD_LO) & (c <= np.asarray(n) - 1 - LOAD_LO), axis=1)
    orc.set_particles(np.ascontiguousarray(x[sel]), np.ascontiguousarray(u[sel]), w.q, w.m)
    assert orc.lost == 0
    # the sources after the particles: loading particles deposits rho afresh
    for comp, name in enumerate(POT):
        orc.pot(comp, "cur")[:] = fields[name]
        orc.pot(comp, "prev")[:] = fields[name + "_prev"]
    for comp in range(3):
        orc.J(comp)[:] = fields[SRC[comp]]
    orc.rho[:] = fields["rho"]
    orc.set_step(step)
    return orc, sel


def compared_particles(w, lo, hi, x0, sel):
    """Of the loaded particles (mask sel over all), those whose start cell
    lies at least PART_LO cells inside the box, as a mask over the loaded."""
    n = np.asarray(hi) - np.asarray(lo)
    c = cells(w, x0[sel]) - np.asarray(lo)
    return np.all((c >= PART_LO) & (c <= n - 1 - PART_LO), axis=1)
