"""The allocation-free read-back (mithra_get_field_noalloc) against
mithra_get_field, through the C ABI: every field, both precisions, bit for
bit, on two calls in a row, the second on a smaller mesh; a mesh whose
z-plane exceeds the scratch is refused."""
import numpy as np
import pytest

from paper_1612_03310_amd import native
from paper_1612_03310_amd import workloads as W

FIELDS = ("Ax", "Ay", "Az", "phi", "Jx", "Jy", "Jz", "rho", "Ex", "Ey", "Ez", "Bx", "By",
          "Bz", "Ax_prev", "phi_prev", "rho_prev")

pytestmark = pytest.mark.gpu


def _sim(n, npart, precision, steps, seed):
    w = W.make_workload("noalloc", n, npart, 110.0, 1.2, 0.015, 1e-4, seed, steps)
    sim = native.sim_from_workload(w, precision=precision)
    sim.run(steps)
    sim.sync()
    return sim


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_noalloc_read_back_equals_get_field(precision):
    # 64x64x150: 4096 points per plane, 64 planes per chunk, so three chunks
    # (64, 64, 22 planes); then 32x32x64 in one chunk
    for n, npart, steps, seed in (((64, 64, 150), 6000, 9, 71), ((32, 32, 64), 2000, 5, 72)):
        print("case noalloc", precision, n, npart, steps, flush=True)
        sim = _sim(n, npart, precision, steps, seed)
        out = np.empty(sim.ncell)
        for f in FIELDS:
            ref = sim.get_field(f)
            out[:] = np.nan
            got = sim.get_field_noalloc(f, out)
            assert got.tobytes() == ref.tobytes(), (precision, n, f)
            if f in ("Ex", "Bz", "Jz"):
                assert np.any(ref != 0.0), (n, f)
        sim.close()


def test_noalloc_refuses_a_plane_beyond_the_scratch():
    n = (520, 520, 8)  # 270400 points per z-plane, above the 262144 of the scratch
    d = (4e-6, 4e-6, 1e-6)
    origin = tuple(-(n[a] - 1) / 2.0 * d[a] for a in range(3))
    print("case noalloc refusal", n, flush=True)
    sim = native.Sim(n, d, origin, precision="f32")
    sim.set_particles(np.zeros((0, 3)), np.zeros((0, 3)), -1.602176634e-19, 9.1093837015e-31)
    sim.run(1)
    sim.sync()
    with pytest.raises(native.MithraError, match="z-plane") as e:
        sim.get_field_noalloc("Ex")
    assert e.value.status == native.EINVAL
    sim.close()
