"""Plain FP64 CPU oracle of MITHRA's boosted-frame FDTD/PIC step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The
product library never loads it and shares no code with it.

The arithmetic lives in ``mithra_oracle.c`` (plain C, scalar loops, SI units,
double precision).  This module builds it with gcc and marshals arrays with
ctypes; it does no arithmetic of the method itself.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mithra_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# The same source built with OpenMP: the loops that write disjoint points or
# particles (potential update, vertex fields, push, plane spectrum) run on
# all threads; sums stay sequential, so every result equals the plain
# build's bit for bit.  For long oracle runs and the all-core CPU baseline.
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

NDIAG = 29
MAXF = 32
DIAG_COLUMNS = ("step", "t", "total_charge", "continuity_residual", "power",
                "field_energy", "kinetic_energy", "Ex", "Ey", "Ez", "Bx", "By",
                "Bz", "lost", "nonfinite", "spare", "bunching1", "bunching2",
                "bunching3", "spare2", "power_h1", "power_h2", "power_h3", "spare3",
                "power_extra1", "power_extra2", "power_extra3", "power_lab", "z_undulator")

_lib = None


def gcc_command(src: str, out: str, extra=()):
    """The oracle's compile line (no fast-math, no FMA contraction); `extra`
    adds flags, e.g. sanitizers or OpenMP."""
    return ["gcc", "-O3", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
            "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas", *extra, "-o", out, src, "-lm"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc, plain and with OpenMP."""
    for lib, extra in ((_LIB, ()), (_LIB_OMP, ("-fopenmp",))):
        if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
            tmp = lib + ".tmp%d" % os.getpid()
            subprocess.check_call(gcc_command(_SRC, tmp, extra))
            os.replace(tmp, lib)
    return _LIB


_lib_omp = None


def _load_parallel():
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(_LIB_OMP) or os.path.getmtime(_LIB_OMP) < os.path.getmtime(_SRC):
            build(force=True)
        _lib_omp = _open(_LIB_OMP)
    return _lib_omp


def threads(parallel: bool = True) -> int:
    """Threads the oracle's parallel loops use (1 for the plain build)."""
    return int((_load_parallel() if parallel else _load()).orc_threads())


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    _lib = _open(_LIB)
    return _lib


def use_library(path):
    """Make simulations created from now on use the oracle built at `path`
    (the tests build copies with one planted mistake to show that a pin
    catches it).  Returns the library in use before, for restore_library."""
    global _lib
    before = _load()
    _lib = _open(path)
    return before


def restore_library(lib):
    global _lib
    _lib = lib


def _open(path):
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    D = ctypes.c_double
    I = ctypes.c_int
    L = ctypes.c_long
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.orc_create.restype = P
    lib.orc_create.argtypes = [ip, dp, dp, D, D, I, I, ip, D, D, D, D]
    lib.orc_destroy.argtypes = [P]
    lib.orc_set_particles.argtypes = [P, L, dp, dp, D, D]
    lib.orc_set_particles.restype = I
    lib.orc_set_background.argtypes = [P, dp]
    lib.orc_set_seed.argtypes = [P, I, D, D, D, D, D, D, D, I, D]
    lib.orc_set_optical.argtypes = [P, I, D, D, D, D, D, D, D, I, D]
    lib.orc_set_optical_beam.argtypes = [P, I, D, D, D, D, D]
    lib.orc_set_seed_beam.argtypes = [P, I, D, D, D, D, D]
    lib.orc_seed_incident.argtypes = [P, I, I, I, I, D]
    lib.orc_seed_incident.restype = D
    lib.orc_seed_signal.argtypes = [P, D]
    lib.orc_seed_signal.restype = D
    lib.orc_config_diag.argtypes = [P, I, I, I, I]
    lib.orc_config_extra_planes.argtypes = [P, I, I, I]
    lib.orc_set_spectrum.argtypes = [P, dp, I]
    lib.orc_set_undulator_length.argtypes = [P, D]
    for name in ("orc_field_update", "orc_vertex_fields", "orc_push", "orc_deposit",
                 "orc_rotate"):
        getattr(lib, name).argtypes = [P]
    lib.orc_step.argtypes = [P, L]
    lib.orc_set_step.argtypes = [P, L]
    lib.orc_diag_row.argtypes = [P, dp]
    lib.orc_array.restype = dp
    lib.orc_array.argtypes = [P, I]
    lib.orc_alive.restype = ctypes.POINTER(ctypes.c_ubyte)
    lib.orc_alive.argtypes = [P]
    lib.orc_info.restype = L
    lib.orc_info.argtypes = [P, I]
    lib.orc_constants.argtypes = [P, dp]
    lib.orc_undulator.argtypes = [P, D, D, D, D, dp, dp]
    lib.orc_boris.argtypes = [D, D, D, dp, dp, dp]
    lib.orc_gather.argtypes = [P, dp, dp, dp]
    lib.orc_deposit_current.argtypes = [P, dp, dp]
    lib.orc_threads.restype = I
    lib.orc_threads.argtypes = []
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


CONSTANT_NAMES = ("dt", "dtb", "A", "a1", "a2", "a4", "a6", "a8", "gamma0", "beta0",
                  "B0", "ku", "mur_b0", "mur_b1", "mu0", "eps0", "c", "e", "me")


class OracleSim:
    """One simulation held by the C oracle.

    Arrays are returned as numpy views shaped (nz, ny, nx) (x fastest), so
    ``a[k, j, i]`` is grid point (i, j, k).  Potential components are
    0: A_x at (i+1/2, j, k), 1: A_y at (i, j+1/2, k), 2: A_z at (i, j, k+1/2),
    3: phi at (i, j, k).
    """

    def __init__(self, n, d, origin, courant=0.9, nsfd_A=-1.0, substeps=1,
                 space_charge=1, bc=(0, 0, 0), lambda_u=0.015, K=1.0,
                 gamma_beam=100.0, z_e=0.0, parallel=False):
        lib = _load_parallel() if parallel else _load()
        self._lib = lib
        self.n = tuple(int(v) for v in n)
        n_c = (ctypes.c_int * 3)(*self.n)
        d_c = (ctypes.c_double * 3)(*[float(v) for v in d])
        o_c = (ctypes.c_double * 3)(*[float(v) for v in origin])
        bc_c = (ctypes.c_int * 3)(*[int(v) for v in bc])
        self._h = lib.orc_create(n_c, d_c, o_c, float(courant), float(nsfd_A), int(substeps),
                                 int(space_charge), bc_c, float(lambda_u), float(K),
                                 float(gamma_beam), float(z_e))
        if not self._h:
            raise MemoryError("oracle allocation failed")
        out = np.zeros(len(CONSTANT_NAMES))
        lib.orc_constants(self._h, _dptr(out))
        self.const = dict(zip(CONSTANT_NAMES, out.tolist()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    # ---- inputs ------------------------------------------------------------
    def set_particles(self, x, u, q, m):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 3)
        if x.shape != u.shape:
            raise ValueError("x and u must both be (np, 3)")
        self._lib.orc_set_particles(self._h, x.shape[0], _dptr(x), _dptr(u), float(q), float(m))

    def set_background(self, bg):
        bg = np.ascontiguousarray(bg, dtype=np.float64).reshape(-1)
        self._lib.orc_set_background(self._h, _dptr(bg))

    SIGNALS = {"neumann": 0, "gaussian": 1, "secant": 2, "flat-top": 3}

    def set_seed(self, a0, polarization=(1.0, 0.0), frequency=0.0, t0=0.0, tau=1.0, cep=0.0,
                 signal="gaussian", z_ref=0.0, on=True):
        self._lib.orc_set_seed(self._h, int(on), float(a0), float(polarization[0]),
                               float(polarization[1]), float(frequency), float(t0), float(tau),
                               float(cep), int(self.SIGNALS[signal]), float(z_ref))

    def seed_signal(self, t):
        return float(self._lib.orc_seed_signal(self._h, float(t)))

    def set_optical_undulator(self, amplitude, polarization=(1.0, 0.0), frequency=0.0, t0=0.0,
                              tau=1.0, cep=0.0, signal="gaussian", z_ref=0.0, on=True):
        """Plane wave towards -z in place of the static undulator (rest frame)."""
        self._lib.orc_set_optical(self._h, int(on), float(amplitude), float(polarization[0]),
                                  float(polarization[1]), float(frequency), float(t0),
                                  float(tau), float(cep), int(self.SIGNALS[signal]),
                                  float(z_ref))

    def set_seed_beam(self, beam="plane", rayleigh=(0.0, 0.0), focus=(0.0, 0.0, 0.0)):
        """Beam of the seed: "plane" or "gaussian" (travelling towards +z) with
        the Rayleigh lengths along the polarization and across it [m] and the
        focus (rest frame)."""
        self._lib.orc_set_seed_beam(self._h, {"plane": 0, "gaussian": 1}[beam],
                                    float(rayleigh[0]), float(rayleigh[1]), float(focus[0]),
                                    float(focus[1]), float(focus[2]))

    def seed_incident(self, comp, i, j, k, t):
        """Incident potential of the seed at grid point (i, j, k) of
        component comp (0: A_x, 1: A_y) at time t."""
        return self._lib.orc_seed_incident(self._h, int(comp), int(i), int(j), int(k), float(t))

    def set_optical_beam(self, beam="plane", rayleigh=(0.0, 0.0), focus=(0.0, 0.0, 0.0)):
        """Beam of the optical undulator: "plane" or "gaussian" with the
        Rayleigh lengths along the polarization and across it [m] and the
        focus (rest frame)."""
        self._lib.orc_set_optical_beam(self._h, {"plane": 0, "gaussian": 1}[beam],
                                       float(rayleigh[0]), float(rayleigh[1]), float(focus[0]),
                                       float(focus[1]), float(focus[2]))

    def config_diag(self, probe, kp, extra_planes=()):
        self._lib.orc_config_diag(self._h, int(probe[0]), int(probe[1]), int(probe[2]), int(kp))
        k = list(extra_planes) + [-1] * (3 - len(extra_planes))
        self._lib.orc_config_extra_planes(self._h, int(k[0]), int(k[1]), int(k[2]))

    def set_spectrum(self, nu):
        """Normalized frequencies nu_f (omega_f = nu_f omega_1) of the plane
        spectrum, at most 32; restarts it."""
        nu = np.ascontiguousarray(nu, dtype=np.float64).reshape(-1)
        self._nfreq = int(nu.size)
        self._lib.orc_set_spectrum(self._h, _dptr(nu), int(nu.size))

    def set_undulator_length(self, length):
        """Lab length of the static undulator [m] (whole periods); <= 0: unbounded."""
        self._lib.orc_set_undulator_length(self._h, float(length))

    def spectrum_rows(self):
        """(rest, lab): the mean power [W] at each frequency since the
        restart, one row per step, in the bunch frame and in the lab."""
        nd = int(self._lib.orc_info(self._h, 3))
        nf = getattr(self, "_nfreq", 3)
        if nd == 0:
            return np.zeros((0, nf)), np.zeros((0, nf))
        ptr = self._lib.orc_array(self._h, 27)
        a = np.ctypeslib.as_array(ptr, shape=(nd, 2, MAXF)).copy()
        return a[:, 0, :nf], a[:, 1, :nf]

    # ---- stepping ----------------------------------------------------------
    def step(self, nsteps=1):
        self._lib.orc_step(self._h, int(nsteps))

    def field_update(self):
        self._lib.orc_field_update(self._h)

    def vertex_fields(self):
        self._lib.orc_vertex_fields(self._h)

    def push(self):
        self._lib.orc_push(self._h)

    def deposit(self):
        self._lib.orc_deposit(self._h)

    def rotate(self):
        self._lib.orc_rotate(self._h)

    # ---- state ---------------------------------------------------------------
    def _mesh(self, which):
        nx, ny, nz = self.n
        ptr = self._lib.orc_array(self._h, which)
        return np.ctypeslib.as_array(ptr, shape=(nz, ny, nx))

    def pot(self, comp, level="cur"):
        base = {"cur": 0, "prev": 4, "next": 8}[level]
        return self._mesh(base + comp)

    def J(self, comp):
        return self._mesh(12 + comp)

    @property
    def rho(self):
        return self._mesh(15)

    @property
    def rho_prev(self):
        return self._mesh(16)

    def E(self, comp):
        return self._mesh(17 + comp)

    def B(self, comp):
        return self._mesh(20 + comp)

    @property
    def np(self):
        return int(self._lib.orc_info(self._h, 0))

    @property
    def step_count(self):
        return int(self._lib.orc_info(self._h, 1))

    def set_step(self, step):
        """Step counter of the state loaded by hand (no arithmetic)."""
        self._lib.orc_set_step(self._h, int(step))

    @property
    def lost(self):
        return int(self._lib.orc_info(self._h, 2))

    def _parts(self, which):
        npart = self.np
        ptr = self._lib.orc_array(self._h, which)
        return np.ctypeslib.as_array(ptr, shape=(max(npart, 1), 3))[:npart]

    @property
    def x(self):
        return self._parts(23)

    @property
    def u(self):
        return self._parts(24)

    @property
    def x_old(self):
        return self._parts(25)

    @property
    def alive(self):
        npart = self.np
        ptr = self._lib.orc_alive(self._h)
        return np.ctypeslib.as_array(ptr, shape=(max(npart, 1),))[:npart].astype(bool)

    def diag(self):
        nd = int(self._lib.orc_info(self._h, 3))
        if nd == 0:
            return np.zeros((0, NDIAG))
        ptr = self._lib.orc_array(self._h, 26)
        return np.ctypeslib.as_array(ptr, shape=(nd, NDIAG)).copy()

    def diag_row_now(self):
        row = np.zeros(NDIAG)
        self._lib.orc_diag_row(self._h, _dptr(row))
        return row

    # ---- single pieces (for the pins) -----------------------------------------
    def undulator(self, x, y, z, t):
        E = np.zeros(3)
        B = np.zeros(3)
        self._lib.orc_undulator(self._h, float(x), float(y), float(z), float(t), _dptr(E), _dptr(B))
        return E, B

    def gather(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        E = np.zeros(3)
        B = np.zeros(3)
        self._lib.orc_gather(self._h, _dptr(x), _dptr(E), _dptr(B))
        return E, B

    def deposit_current(self, x0, x1):
        x0 = np.ascontiguousarray(x0, dtype=np.float64)
        x1 = np.ascontiguousarray(x1, dtype=np.float64)
        self._lib.orc_deposit_current(self._h, _dptr(x0), _dptr(x1))


def boris(q, m, dtb, u, E, B):
    """One Boris step of eq. (BorisScheme) done by the C oracle."""
    lib = _load()
    u = np.array(u, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    lib.orc_boris(float(q), float(m), float(dtb), _dptr(u), _dptr(E), _dptr(B))
    return u


def from_workload(w, parallel=False):
    """Oracle simulation loaded with a workload from the seeded generator
    (parallel: the OpenMP build, same results)."""
    s = OracleSim(w.n, w.d, w.origin, w.courant, w.nsfd_A, w.substeps, w.space_charge,
                  w.bc, w.lambda_u, w.K, w.gamma_beam, w.z_e, parallel=parallel)
    s.config_diag(w.probe, w.kp)
    s.set_undulator_length(getattr(w, "und_length", 0.0))
    s.set_particles(w.x, w.u, w.q, w.m)
    return s
