"""ctypes binding of ``libmithra.so`` (the C ABI in ``include/mithra.h``).

Argument marshalling only: every step of the method runs in the HIP kernels of
the library.  PyTorch supplies the stream (``torch.cuda.current_stream()``)
and, through the allocator hook, the device memory.  There is no fallback: if
the library is missing or cannot load, constructing a simulation raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmithra.so")

OK, EINVAL, ENOMEM, EDEVICE, ENUMERIC, ESTATE = range(6)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ENUMERIC", 5: "ESTATE"}
F64, F32_SPLIT = 0, 1
MUR1, PERIODIC = 0, 1
FIELDS = {"Ax": 0, "Ay": 1, "Az": 2, "phi": 3, "Jx": 4, "Jy": 5, "Jz": 6, "rho": 7,
          "Ex": 8, "Ey": 9, "Ez": 10, "Bx": 11, "By": 12, "Bz": 13,
          "Ax_prev": 14, "Ay_prev": 15, "Az_prev": 16, "phi_prev": 17, "rho_prev": 18}
KINDS = ("stencil", "boundary", "push", "deposit", "scan", "scatter", "diag")

# every exported function of the C ABI (checked by the symbol test)
ABI_FUNCTIONS = (
    "mithra_create", "mithra_set_allocator", "mithra_set_particles", "mithra_config_diag",
    "mithra_run", "mithra_sync", "mithra_get_field", "mithra_set_field", "mithra_get_particles",
    "mithra_get_diag", "mithra_get_info", "mithra_get_state", "mithra_set_state",
    "mithra_set_timing", "mithra_get_timing", "mithra_tune", "mithra_last_error",
    "mithra_destroy", "mithra_batch_create", "mithra_batch_set_particles",
    "mithra_batch_config_diag", "mithra_batch_tune", "mithra_batch_run", "mithra_batch_sync",
    "mithra_batch_get_diag", "mithra_batch_get_field", "mithra_batch_get_particles",
    "mithra_batch_get_info", "mithra_batch_set_timing", "mithra_batch_get_timing",
    "mithra_batch_destroy", "mithra_set_seed", "mithra_batch_set_seed",
    "mithra_set_optical_undulator", "mithra_batch_set_optical_undulator",
    "mithra_set_optical_beam", "mithra_batch_set_optical_beam",
    "mithra_set_seed_beam", "mithra_batch_set_seed_beam", "mithra_set_background",
    "mithra_get_bins", "mithra_get_field_noalloc", "mithra_set_spectrum", "mithra_get_spectrum",
    "mithra_batch_set_spectrum", "mithra_batch_get_spectrum", "mithra_set_shapes",
    "mithra_batch_set_shapes",
)

MAX_FREQ = 32

SIGNALS = {"neumann": 0, "gaussian": 1, "secant": 2, "flat-top": 3}


class Mesh(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("d", ctypes.c_double * 3),
                ("origin", ctypes.c_double * 3), ("courant", ctypes.c_double),
                ("nsfd_A", ctypes.c_double), ("substeps", ctypes.c_int32),
                ("space_charge", ctypes.c_int32), ("bc", ctypes.c_int32 * 3)]


class Undulator(ctypes.Structure):
    _fields_ = [("lambda_u", ctypes.c_double), ("K", ctypes.c_double),
                ("gamma_beam", ctypes.c_double), ("z_entrance", ctypes.c_double),
                ("length", ctypes.c_double)]


class Seed(ctypes.Structure):
    _fields_ = [("amplitude", ctypes.c_double), ("polarization", ctypes.c_double * 2),
                ("frequency", ctypes.c_double), ("t0", ctypes.c_double), ("tau", ctypes.c_double),
                ("cep", ctypes.c_double), ("z_ref", ctypes.c_double), ("signal", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


def make_seed(amplitude, polarization=(1.0, 0.0), frequency=0.0, t0=0.0, tau=1.0, cep=0.0,
              signal="gaussian", z_ref=0.0) -> Seed:
    s = Seed()
    s.amplitude = float(amplitude)
    s.polarization[0] = float(polarization[0])
    s.polarization[1] = float(polarization[1])
    s.frequency = float(frequency)
    s.t0 = float(t0)
    s.tau = float(tau)
    s.cep = float(cep)
    s.z_ref = float(z_ref)
    s.signal = SIGNALS[signal] if isinstance(signal, str) else int(signal)
    return s


class Beam(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("rayleigh", ctypes.c_double * 2), ("focus", ctypes.c_double * 3)]


BEAMS = {"plane": 0, "gaussian": 1}


def make_beam(beam="plane", rayleigh=(0.0, 0.0), focus=(0.0, 0.0, 0.0)) -> Beam:
    b = Beam()
    b.type = BEAMS[beam] if isinstance(beam, str) else int(beam)
    for a in range(2):
        b.rayleigh[a] = float(rayleigh[a])
    for a in range(3):
        b.focus[a] = float(focus[a])
    return b


class DiagCfg(ctypes.Structure):
    _fields_ = [("probe", ctypes.c_int32 * 3), ("power_plane_k", ctypes.c_int32),
                ("mesh_diag_every", ctypes.c_int32), ("capacity", ctypes.c_int32),
                ("power_spectrum", ctypes.c_int32), ("extra_planes", ctypes.c_int32 * 3)]


class DiagRow(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("t", ctypes.c_double),
                ("total_charge", ctypes.c_double), ("continuity_residual", ctypes.c_double),
                ("power", ctypes.c_double), ("field_energy", ctypes.c_double),
                ("kinetic_energy", ctypes.c_double), ("probe_E", ctypes.c_double * 3),
                ("probe_B", ctypes.c_double * 3), ("lost", ctypes.c_int64),
                ("nonfinite", ctypes.c_int32), ("has_mesh_terms", ctypes.c_int32),
                ("bunching", ctypes.c_double * 3), ("power_harmonic", ctypes.c_double * 3),
                ("power_extra", ctypes.c_double * 3), ("power_lab", ctypes.c_double),
                ("z_undulator", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("dtb", ctypes.c_double), ("nsfd_A", ctypes.c_double),
                ("gamma0", ctypes.c_double), ("beta0", ctypes.c_double), ("B0", ctypes.c_double),
                ("ku", ctypes.c_double), ("step", ctypes.c_int64), ("np", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("stencil_tile", ctypes.c_int32 * 3),
                ("precision", ctypes.c_int32), ("particle_brick", ctypes.c_int32 * 3),
                ("pad", ctypes.c_int32)]


DIAG_DTYPE = np.dtype([("step", np.int64), ("t", np.float64), ("total_charge", np.float64),
                       ("continuity_residual", np.float64), ("power", np.float64),
                       ("field_energy", np.float64), ("kinetic_energy", np.float64),
                       ("probe_E", np.float64, 3), ("probe_B", np.float64, 3),
                       ("lost", np.int64), ("nonfinite", np.int32),
                       ("has_mesh_terms", np.int32), ("bunching", np.float64, 3),
                       ("power_harmonic", np.float64, 3), ("power_extra", np.float64, 3),
                       ("power_lab", np.float64), ("z_undulator", np.float64)])
assert DIAG_DTYPE.itemsize == ctypes.sizeof(DiagRow)


class MithraError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), msg))
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library; raises if it is missing (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libmithra.so is not built (run __graft_entry__.build() or "
                           "python -m paper_1612_03310_amd.build): %s" % path)
    # torch ships its own HIP runtime (same SONAME, different file name).  Load
    # it first so that the library binds to that copy: two runtimes in one
    # process cannot share the device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "mithra_create": [ctypes.POINTER(Mesh), ctypes.POINTER(Undulator), I32, P, pp],
        "mithra_set_allocator": [P, P, P],
        "mithra_set_particles": [P, I64, dp, dp, D, D],
        "mithra_config_diag": [P, ctypes.POINTER(DiagCfg)],
        "mithra_set_seed": [P, ctypes.POINTER(Seed)],
        "mithra_batch_set_seed": [P, I32, ctypes.POINTER(Seed)],
        "mithra_set_optical_undulator": [P, ctypes.POINTER(Seed)],
        "mithra_batch_set_optical_undulator": [P, I32, ctypes.POINTER(Seed)],
        "mithra_set_optical_beam": [P, ctypes.POINTER(Beam)],
        "mithra_batch_set_optical_beam": [P, I32, ctypes.POINTER(Beam)],
        "mithra_set_seed_beam": [P, ctypes.POINTER(Beam)],
        "mithra_set_background": [P, dp],
        "mithra_batch_set_seed_beam": [P, I32, ctypes.POINTER(Beam)],
        "mithra_run": [P, I64],
        "mithra_sync": [P],
        "mithra_get_field": [P, I32, dp],
        "mithra_get_field_noalloc": [P, I32, dp],
        "mithra_set_field": [P, I32, dp],
        "mithra_get_particles": [P, dp, dp, ctypes.POINTER(ctypes.c_uint8),
                                 ctypes.POINTER(ctypes.c_int64)],
        "mithra_get_diag": [P, ctypes.POINTER(DiagRow), I64, ctypes.POINTER(ctypes.c_int64)],
        "mithra_get_bins": [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)],
        "mithra_get_info": [P, ctypes.POINTER(Info)],
        "mithra_get_state": [P, P, ctypes.POINTER(ctypes.c_size_t)],
        "mithra_set_state": [P, P, ctypes.c_size_t],
        "mithra_set_timing": [P, I32],
        "mithra_get_timing": [P, dp, ctypes.POINTER(ctypes.c_int64), I32, I32],
        "mithra_tune": [P, I32],
        "mithra_set_shapes": [P, ctypes.POINTER(I32), ctypes.POINTER(I32)],
        "mithra_batch_create": [I32, ctypes.POINTER(Mesh), ctypes.POINTER(Undulator), I32, P, pp],
        "mithra_batch_set_particles": [P, I32, I64, dp, dp, D, D],
        "mithra_batch_config_diag": [P, I32, ctypes.POINTER(DiagCfg)],
        "mithra_set_spectrum": [P, dp, I32],
        "mithra_get_spectrum": [P, I64, I64, dp, dp],
        "mithra_batch_set_spectrum": [P, I32, dp, I32],
        "mithra_batch_get_spectrum": [P, I32, I64, I64, dp, dp],
        "mithra_batch_tune": [P, I32],
        "mithra_batch_set_shapes": [P, ctypes.POINTER(I32), ctypes.POINTER(I32)],
        "mithra_batch_run": [P, I64],
        "mithra_batch_sync": [P],
        "mithra_batch_get_diag": [P, I32, ctypes.POINTER(DiagRow), I64,
                                  ctypes.POINTER(ctypes.c_int64)],
        "mithra_batch_get_field": [P, I32, I32, dp],
        "mithra_batch_get_particles": [P, I32, dp, dp, ctypes.POINTER(ctypes.c_uint8),
                                       ctypes.POINTER(ctypes.c_int64)],
        "mithra_batch_get_info": [P, I32, ctypes.POINTER(Info)],
        "mithra_batch_set_timing": [P, I32],
        "mithra_batch_get_timing": [P, dp, ctypes.POINTER(ctypes.c_int64), I32, I32],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.mithra_last_error.restype = ctypes.c_char_p
    lib.mithra_last_error.argtypes = []
    lib.mithra_destroy.restype = None
    lib.mithra_destroy.argtypes = [P]
    lib.mithra_batch_destroy.restype = None
    lib.mithra_batch_destroy.argtypes = [P]
    _lib = lib
    return lib


def _check(status: int):
    if status != OK:
        msg = _lib.mithra_last_error().decode(errors="replace")
        raise MithraError(status, msg)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---- PyTorch plumbing: stream and caching allocator ------------------------

_ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_live_blocks: Dict[int, object] = {}
_hooks = []


def use_torch_allocator(enable: bool = True):
    """Route the library's device allocations through torch's caching allocator.

    The two callbacks are created once and kept for the life of the module:
    every simulation keeps the function pointers it was created with, so the
    callback objects must outlive all of them."""
    lib = load_library()
    if not enable:
        _check(lib.mithra_set_allocator(None, None, None))
        return
    if _hooks:
        a, f = _hooks
        _check(lib.mithra_set_allocator(ctypes.cast(a, ctypes.c_void_p),
                                        ctypes.cast(f, ctypes.c_void_p), None))
        return
    import torch

    def _alloc(nbytes, _ctx):
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        except Exception:  # out of memory: the library reports ENOMEM
            return None
        live[t.data_ptr()] = t
        return t.data_ptr()

    live = _live_blocks  # module globals may already be gone at interpreter exit

    def _free(ptr, _ctx):
        live.pop(int(ptr) if ptr else 0, None)

    a, f = _ALLOC_T(_alloc), _FREE_T(_free)
    _hooks.extend((a, f))
    _check(lib.mithra_set_allocator(ctypes.cast(a, ctypes.c_void_p),
                                    ctypes.cast(f, ctypes.c_void_p), None))


def _torch_stream():
    import torch
    if not torch.cuda.is_available():
        raise MithraError(EDEVICE, "no GPU visible to torch")
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_mesh(n, d, origin, courant=0.9, nsfd_A=-1.0, substeps=1, space_charge=1,
              bc=(0, 0, 0)) -> Mesh:
    m = Mesh()
    for a in range(3):
        m.n[a] = int(n[a])
        m.d[a] = float(d[a])
        m.origin[a] = float(origin[a])
        m.bc[a] = int(bc[a])
    m.courant = float(courant)
    m.nsfd_A = float(nsfd_A)
    m.substeps = int(substeps)
    m.space_charge = int(space_charge)
    return m


def make_undulator(lambda_u, K, gamma_beam, z_entrance, length=0.0) -> Undulator:
    """length: lab length of the undulator [m], whole periods; <= 0 unbounded."""
    return Undulator(float(lambda_u), float(K), float(gamma_beam), float(z_entrance),
                     float(length))


assert DIAG_DTYPE.itemsize == ctypes.sizeof(DiagRow)


def make_diag_cfg(probe, kp, every=1, capacity=4096, spectrum=False, extra_planes=()) -> DiagCfg:
    """Diagnostic settings; extra_planes: up to three further plate z indices."""
    c = DiagCfg()
    for a in range(3):
        c.probe[a] = int(probe[a])
    c.power_plane_k = int(kp)
    c.mesh_diag_every = int(every)
    c.capacity = int(capacity)
    c.power_spectrum = 1 if spectrum else 0
    k = list(extra_planes) + [-1] * (3 - len(extra_planes))
    for e in range(3):
        c.extra_planes[e] = int(k[e])
    return c


def _rows_to_array(rows, n):
    out = np.zeros(n, dtype=DIAG_DTYPE)
    ctypes.memmove(out.ctypes.data, rows, n * DIAG_DTYPE.itemsize)
    return out


class Sim:
    """One simulation on the current GPU, on torch's current stream."""

    def __init__(self, n, d, origin, courant=0.9, nsfd_A=-1.0, substeps=1, space_charge=1,
                 bc=(0, 0, 0), lambda_u=0.015, K=1.0, gamma_beam=100.0, z_entrance=0.0,
                 precision: str = "f64", stream=None, torch_allocator: bool = True,
                 length=0.0):
        self._lib = load_library()
        if torch_allocator:
            use_torch_allocator(True)
        self.n = tuple(int(v) for v in n)
        self.precision = {"f64": F64, "f32": F32_SPLIT, "f32_split": F32_SPLIT}[precision]
        mesh = make_mesh(n, d, origin, courant, nsfd_A, substeps, space_charge, bc)
        und = make_undulator(lambda_u, K, gamma_beam, z_entrance, length)
        st = stream if stream is not None else _torch_stream()
        h = ctypes.c_void_p()
        _check(self._lib.mithra_create(ctypes.byref(mesh), ctypes.byref(und), self.precision, st,
                                       ctypes.byref(h)))
        self._h = h
        self._np = 0

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mithra_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def ncell(self):
        return self.n[0] * self.n[1] * self.n[2]

    def set_particles(self, pos, u, q, m):
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 3)
        if pos.shape != u.shape:
            raise ValueError("pos and u must both be (np, 3)")
        _check(self._lib.mithra_set_particles(self._h, pos.shape[0], _dptr(pos), _dptr(u),
                                              float(q), float(m)))
        self._np = pos.shape[0]

    def set_seed(self, amplitude, **kw):
        """Seed plane wave (see mithra_set_seed); amplitude 0 clears it."""
        seed = make_seed(amplitude, **kw)
        _check(self._lib.mithra_set_seed(self._h, ctypes.byref(seed)))

    def set_optical_undulator(self, amplitude, **kw):
        """Plane wave towards -z in place of the static undulator (see
        mithra_set_optical_undulator); amplitude 0 restores the static one."""
        wave = make_seed(amplitude, **kw)
        _check(self._lib.mithra_set_optical_undulator(self._h, ctypes.byref(wave)))

    def set_optical_beam(self, beam="plane", rayleigh=(0.0, 0.0), focus=(0.0, 0.0, 0.0)):
        """Beam of the optical undulator (see mithra_set_optical_beam)."""
        b = make_beam(beam, rayleigh, focus)
        _check(self._lib.mithra_set_optical_beam(self._h, ctypes.byref(b)))

    def set_background(self, rho):
        """Static background charge density at the vertices, (nz, ny, nx) or
        None to remove it (see mithra_set_background)."""
        if rho is None:
            _check(self._lib.mithra_set_background(self._h, None))
            return
        nx, ny, nz = self.n
        a = np.ascontiguousarray(rho, dtype=np.float64).reshape(nz, ny, nx)
        _check(self._lib.mithra_set_background(self._h, _dptr(a)))

    def set_seed_beam(self, beam="plane", rayleigh=(0.0, 0.0), focus=(0.0, 0.0, 0.0)):
        """Beam of the seed (see mithra_set_seed_beam)."""
        b = make_beam(beam, rayleigh, focus)
        _check(self._lib.mithra_set_seed_beam(self._h, ctypes.byref(b)))

    def config_diag(self, probe, kp, every=1, capacity=4096, spectrum=False, extra_planes=()):
        c = make_diag_cfg(probe, kp, every, capacity, spectrum, extra_planes)
        _check(self._lib.mithra_config_diag(self._h, ctypes.byref(c)))

    def set_spectrum(self, nu):
        """Normalized frequencies of the power spectrum (at most MAX_FREQ)."""
        nu = np.ascontiguousarray(nu, dtype=np.float64).reshape(-1)
        _check(self._lib.mithra_set_spectrum(self._h, _dptr(nu), int(nu.size)))
        self._nfreq = int(nu.size)

    def get_spectrum(self, first_step, count):
        """(rest, lab), each (count, nfreq): the mean power at each frequency
        for rows first_step .. first_step + count - 1."""
        nf = getattr(self, "_nfreq", 3)
        rest = np.empty((max(count, 1), nf))
        lab = np.empty((max(count, 1), nf))
        _check(self._lib.mithra_get_spectrum(self._h, int(first_step), int(count), _dptr(rest),
                                             _dptr(lab)))
        return rest[:count], lab[:count]

    def run(self, nsteps: int):
        _check(self._lib.mithra_run(self._h, int(nsteps)))

    def sync(self):
        _check(self._lib.mithra_sync(self._h))

    def get_field(self, name: str) -> np.ndarray:
        out = np.empty(self.ncell, dtype=np.float64)
        _check(self._lib.mithra_get_field(self._h, FIELDS[name], _dptr(out)))
        return out.reshape(self.n[2], self.n[1], self.n[0])

    def get_field_noalloc(self, name: str, out=None) -> np.ndarray:
        """mithra_get_field_noalloc: the library allocates nothing; out, if
        given, is a float64 array of the mesh's size the field is written to."""
        if out is None:
            out = np.empty(self.ncell, dtype=np.float64)
        if out.dtype != np.float64 or out.size != self.ncell or not out.flags.c_contiguous:
            raise ValueError("out must be a contiguous float64 array of %d values" % self.ncell)
        _check(self._lib.mithra_get_field_noalloc(self._h, FIELDS[name], _dptr(out)))
        return out.reshape(self.n[2], self.n[1], self.n[0])

    def set_field(self, name: str, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(-1)
        if a.size != self.ncell:
            raise ValueError("field must have %d values" % self.ncell)
        _check(self._lib.mithra_set_field(self._h, FIELDS[name], _dptr(a)))

    def get_particles(self):
        npart = self._np
        pos = np.empty((max(npart, 1), 3))
        u = np.empty((max(npart, 1), 3))
        alive = np.empty(max(npart, 1), dtype=np.uint8)
        nal = ctypes.c_int64()
        _check(self._lib.mithra_get_particles(
            self._h, _dptr(pos), _dptr(u), alive.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
            ctypes.byref(nal)))
        return pos[:npart], u[:npart], alive[:npart].astype(bool)

    def get_diag(self, cap: int = 1 << 20) -> np.ndarray:
        rows = (DiagRow * cap)()
        n = ctypes.c_int64()
        _check(self._lib.mithra_get_diag(self._h, rows, cap, ctypes.byref(n)))
        return _rows_to_array(rows, n.value)

    def get_bins(self):
        """(keys [np], ids [np], starts [nkeys + 2], nkeys) of the particle
        buffer the next step reads."""
        i32 = ctypes.POINTER(ctypes.c_int32)
        nk = ctypes.c_int64()
        _check(self._lib.mithra_get_bins(self._h, None, None, None, ctypes.byref(nk)))
        npart = self._np
        keys = np.empty(max(npart, 1), dtype=np.int32)
        ids = np.empty(max(npart, 1), dtype=np.int32)
        starts = np.empty(nk.value + 2, dtype=np.int32)
        _check(self._lib.mithra_get_bins(self._h, keys.ctypes.data_as(i32),
                                         ids.ctypes.data_as(i32), starts.ctypes.data_as(i32),
                                         ctypes.byref(nk)))
        return keys[:npart], ids[:npart], starts, int(nk.value)

    def info(self) -> dict:
        i = Info()
        _check(self._lib.mithra_get_info(self._h, ctypes.byref(i)))
        return {k: (list(getattr(i, k)) if k in ("stencil_tile", "particle_brick") else getattr(i, k))
                for k, _ in Info._fields_ if k != "pad"}

    def get_state(self) -> bytes:
        n = ctypes.c_size_t()
        _check(self._lib.mithra_get_state(self._h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(self._lib.mithra_get_state(self._h, buf, ctypes.byref(n)))
        return buf.raw[:n.value]

    def set_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(self._lib.mithra_set_state(self._h, buf, len(blob)))

    def set_timing(self, on: bool):
        _check(self._lib.mithra_set_timing(self._h, 1 if on else 0))

    def get_timing(self, reset: bool = False):
        ms = np.zeros(len(KINDS))
        calls = np.zeros(len(KINDS), dtype=np.int64)
        _check(self._lib.mithra_get_timing(self._h, _dptr(ms),
                                           calls.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                           len(KINDS), 1 if reset else 0))
        return dict(zip(KINDS, ms.tolist())), dict(zip(KINDS, calls.tolist()))

    def tune(self, trials: int = 5):
        _check(self._lib.mithra_tune(self._h, int(trials)))

    def set_shapes(self, stencil_tile: Sequence[int], particle_brick: Sequence[int]):
        t = (ctypes.c_int32 * 3)(*map(int, stencil_tile))
        b = (ctypes.c_int32 * 3)(*map(int, particle_brick))
        _check(self._lib.mithra_set_shapes(self._h, t, b))


class Batch:
    """Independent simulations advanced in lockstep with shared launches."""

    def __init__(self, meshes: Sequence[Mesh], undulators: Sequence[Undulator],
                 precision: str = "f32", stream=None, torch_allocator: bool = True):
        self._lib = load_library()
        if torch_allocator:
            use_torch_allocator(True)
        self.nsim = len(meshes)
        self.n = [tuple(m.n) for m in meshes]
        self.precision = {"f64": F64, "f32": F32_SPLIT, "f32_split": F32_SPLIT}[precision]
        marr = (Mesh * self.nsim)(*meshes)
        uarr = (Undulator * self.nsim)(*undulators)
        st = stream if stream is not None else _torch_stream()
        h = ctypes.c_void_p()
        _check(self._lib.mithra_batch_create(self.nsim, marr, uarr, self.precision, st,
                                             ctypes.byref(h)))
        self._h = h
        self._np = [0] * self.nsim

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mithra_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_particles(self, s, pos, u, q, m):
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 3)
        _check(self._lib.mithra_batch_set_particles(self._h, int(s), pos.shape[0], _dptr(pos),
                                                    _dptr(u), float(q), float(m)))
        self._np[s] = pos.shape[0]

    def set_seed(self, s, amplitude, **kw):
        seed = make_seed(amplitude, **kw)
        _check(self._lib.mithra_batch_set_seed(self._h, int(s), ctypes.byref(seed)))

    def set_optical_undulator(self, s, amplitude, **kw):
        wave = make_seed(amplitude, **kw)
        _check(self._lib.mithra_batch_set_optical_undulator(self._h, int(s), ctypes.byref(wave)))

    def set_optical_beam(self, s, beam="plane", rayleigh=(0.0, 0.0), focus=(0.0, 0.0, 0.0)):
        b = make_beam(beam, rayleigh, focus)
        _check(self._lib.mithra_batch_set_optical_beam(self._h, int(s), ctypes.byref(b)))

    def set_seed_beam(self, s, beam="plane", rayleigh=(0.0, 0.0), focus=(0.0, 0.0, 0.0)):
        b = make_beam(beam, rayleigh, focus)
        _check(self._lib.mithra_batch_set_seed_beam(self._h, int(s), ctypes.byref(b)))

    def config_diag(self, s, probe, kp, every=1, capacity=4096, spectrum=False,
                    extra_planes=()):
        c = make_diag_cfg(probe, kp, every, capacity, spectrum, extra_planes)
        _check(self._lib.mithra_batch_config_diag(self._h, int(s), ctypes.byref(c)))

    def set_spectrum(self, s, nu):
        nu = np.ascontiguousarray(nu, dtype=np.float64).reshape(-1)
        _check(self._lib.mithra_batch_set_spectrum(self._h, int(s), _dptr(nu), int(nu.size)))
        if not hasattr(self, "_nfreq"):
            self._nfreq = [3] * self.nsim
        self._nfreq[s] = int(nu.size)

    def get_spectrum(self, s, first_step, count):
        nf = getattr(self, "_nfreq", [3] * self.nsim)[s]
        rest = np.empty((max(count, 1), nf))
        lab = np.empty((max(count, 1), nf))
        _check(self._lib.mithra_batch_get_spectrum(self._h, int(s), int(first_step), int(count),
                                                   _dptr(rest), _dptr(lab)))
        return rest[:count], lab[:count]

    def tune(self, trials: int = 5):
        _check(self._lib.mithra_batch_tune(self._h, int(trials)))

    def set_shapes(self, stencil_tile: Sequence[int], particle_brick: Sequence[int]):
        t = (ctypes.c_int32 * 3)(*map(int, stencil_tile))
        b = (ctypes.c_int32 * 3)(*map(int, particle_brick))
        _check(self._lib.mithra_batch_set_shapes(self._h, t, b))

    def run(self, nsteps: int):
        _check(self._lib.mithra_batch_run(self._h, int(nsteps)))

    def sync(self):
        _check(self._lib.mithra_batch_sync(self._h))

    def get_diag(self, s, cap: int = 1 << 20) -> np.ndarray:
        rows = (DiagRow * cap)()
        n = ctypes.c_int64()
        _check(self._lib.mithra_batch_get_diag(self._h, int(s), rows, cap, ctypes.byref(n)))
        return _rows_to_array(rows, n.value)

    def get_field(self, s, name: str) -> np.ndarray:
        nx, ny, nz = self.n[s]
        out = np.empty(nx * ny * nz, dtype=np.float64)
        _check(self._lib.mithra_batch_get_field(self._h, int(s), FIELDS[name], _dptr(out)))
        return out.reshape(nz, ny, nx)

    def get_particles(self, s):
        npart = self._np[s]
        pos = np.empty((max(npart, 1), 3))
        u = np.empty((max(npart, 1), 3))
        alive = np.empty(max(npart, 1), dtype=np.uint8)
        nal = ctypes.c_int64()
        _check(self._lib.mithra_batch_get_particles(
            self._h, int(s), _dptr(pos), _dptr(u),
            alive.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), ctypes.byref(nal)))
        return pos[:npart], u[:npart], alive[:npart].astype(bool)

    def info(self, s) -> dict:
        i = Info()
        _check(self._lib.mithra_batch_get_info(self._h, int(s), ctypes.byref(i)))
        return {k: (list(getattr(i, k)) if k in ("stencil_tile", "particle_brick") else getattr(i, k))
                for k, _ in Info._fields_ if k != "pad"}

    def set_timing(self, on: bool):
        _check(self._lib.mithra_batch_set_timing(self._h, 1 if on else 0))

    def get_timing(self, reset: bool = False):
        ms = np.zeros(len(KINDS))
        calls = np.zeros(len(KINDS), dtype=np.int64)
        _check(self._lib.mithra_batch_get_timing(
            self._h, _dptr(ms), calls.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            len(KINDS), 1 if reset else 0))
        return dict(zip(KINDS, ms.tolist())), dict(zip(KINDS, calls.tolist()))


def sim_from_workload(w, precision: str = "f64", every: int = 1, capacity: int = 4096,
                      spectrum: bool = True, **kw) -> Sim:
    """A simulation loaded with a workload from the seeded generator (every
    diagnostic on, the plane spectrum included, unless told otherwise)."""
    s = Sim(w.n, w.d, w.origin, w.courant, w.nsfd_A, w.substeps, w.space_charge, w.bc,
            w.lambda_u, w.K, w.gamma_beam, w.z_e, precision=precision,
            length=w.und_length, **kw)
    s.config_diag(w.probe, w.kp, every=every, capacity=capacity, spectrum=spectrum)
    s.set_particles(w.x, w.u, w.q, w.m)
    return s


def batch_from_workloads(ws, precision: str = "f32", every: int = 1, capacity: int = 4096,
                         spectrum: bool = True, **kw) -> Batch:
    meshes = [make_mesh(w.n, w.d, w.origin, w.courant, w.nsfd_A, w.substeps, w.space_charge,
                        w.bc) for w in ws]
    unds = [make_undulator(w.lambda_u, w.K, w.gamma_beam, w.z_e, w.und_length) for w in ws]
    b = Batch(meshes, unds, precision=precision, **kw)
    for s, w in enumerate(ws):
        b.config_diag(s, w.probe, w.kp, every=every, capacity=capacity, spectrum=spectrum)
        b.set_particles(s, w.x, w.u, w.q, w.m)
    return b
