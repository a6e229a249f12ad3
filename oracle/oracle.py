"""ctypes binding of the FP64 population-form oracle (``tslb_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Arrays are numpy float64, C order, shape
``(nz, ny, nx)`` for scalars and ``(k, nz, ny, nx)`` for k-component fields, so
the flat index is ``x + nx*(y + ny*z)`` as in the C code.  Tensor components
are ordered xx, yy, zz, xy, xz, yz.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tslb_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lock = threading.Lock()
_lib = None

BC_PERIODIC, BC_FREESLIP, BC_INLET, BC_OUTFLOW, BC_NOSLIP = 0, 1, 2, 3, 4


def library_path() -> str:
    return _LIB


def build_oracle(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 6),
        ("nu", ctypes.c_double), ("sigma", ctypes.c_double), ("width", ctypes.c_double),
        ("gamma", ctypes.c_double), ("eps", ctypes.c_double),
        ("inlet_u", ctypes.c_double), ("inlet_d", ctypes.c_double), ("inlet_noise", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("vd", ctypes.c_int32),
        ("rho_a", ctypes.c_double), ("rho_b", ctypes.c_double),
        ("nu_a", ctypes.c_double), ("nu_b", ctypes.c_double),
        ("grav", ctypes.c_double * 3),
    ]


_D = ctypes.POINTER(ctypes.c_double)


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_oracle(force=True)
        lib = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        lib.orc_create.argtypes = [ctypes.POINTER(OrcParams), ctypes.POINTER(vp)]
        lib.orc_create.restype = ctypes.c_int
        lib.orc_free.argtypes = [vp]
        lib.orc_free.restype = None
        lib.orc_set_physical.argtypes = [vp, _D, _D, _D, _D, ctypes.c_int64]
        lib.orc_set_physical.restype = None
        lib.orc_step.argtypes = [vp, ctypes.c_int64]
        lib.orc_step.restype = None
        for name in ("orc_get_physical", "orc_get_raw", "orc_get_geometry"):
            getattr(lib, name).argtypes = [vp, _D, _D, _D, _D]
            getattr(lib, name).restype = None
        lib.orc_sums.argtypes = [vp, _D, _D]
        lib.orc_sums.restype = None
        lib.orc_get_populations.argtypes = [vp, _D, _D]
        lib.orc_get_populations.restype = None
        lib.orc_omega.argtypes = [vp]
        lib.orc_omega.restype = ctypes.c_double
        lib.orc_gamma.argtypes = [vp]
        lib.orc_gamma.restype = ctypes.c_double
        lib.orc_step_count.argtypes = [vp]
        lib.orc_step_count.restype = ctypes.c_long
        lib.orc_collide.argtypes = [ctypes.c_double, _D, _D, _D, ctypes.c_double, _D]
        lib.orc_collide.restype = None
        lib.orc_collide_vd.argtypes = [ctypes.c_double, _D, _D, _D, ctypes.c_double, _D]
        lib.orc_collide_vd.restype = None
        lib.orc_get_accel.argtypes = [vp, _D, _D]
        lib.orc_get_accel.restype = None
        lib.orc_phase_collide.argtypes = [ctypes.c_double, _D, _D, ctypes.c_double, _D]
        lib.orc_phase_collide.restype = None
        lib.orc_noise.argtypes = [ctypes.c_uint64] * 5
        lib.orc_noise.restype = ctypes.c_double
        lib.orc_splitmix64_next.argtypes = [ctypes.c_uint64]
        lib.orc_splitmix64_next.restype = ctypes.c_uint64
        lib.orc_lattice.argtypes = [ctypes.POINTER(ctypes.c_int32), _D, ctypes.POINTER(ctypes.c_int32), _D]
        lib.orc_lattice.restype = None
        _lib = lib
        return lib


def lattice():
    """(c27 (27,3) int, w27 (27,), c7 (7,3) int, w7 (7,)) as the oracle defines them."""
    lib = _load()
    c27 = np.zeros((27, 3), np.int32)
    w27 = np.zeros(27)
    c7 = np.zeros((7, 3), np.int32)
    w7 = np.zeros(7)
    lib.orc_lattice(c27.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(w27),
                    c7.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(w7))
    return c27.astype(np.int64), w27, c7.astype(np.int64), w7


def collide(rho, u, P, F, omega):
    """Post-collision D3Q27 populations of one node (27,)."""
    lib = _load()
    u = np.ascontiguousarray(u, np.float64)
    P = np.ascontiguousarray(P, np.float64)
    F = np.ascontiguousarray(F, np.float64)
    f = np.zeros(27)
    lib.orc_collide(float(rho), _ptr(u), _ptr(P), _ptr(F), float(omega), _ptr(f))
    return f


def collide_vd(rho, u, P, a, omega):
    """Post-collision populations of the variable-density scheme (unit density in
    the velocity terms, rho = 1 + p*, acceleration a) at one node (27,)."""
    lib = _load()
    u = np.ascontiguousarray(u, np.float64)
    P = np.ascontiguousarray(P, np.float64)
    a = np.ascontiguousarray(a, np.float64)
    f = np.zeros(27)
    lib.orc_collide_vd(float(rho), _ptr(u), _ptr(P), _ptr(a), float(omega), _ptr(f))
    return f


def phase_collide(phi, u, n, gamma):
    """Post-collision D3Q7 phase populations of one node (7,)."""
    lib = _load()
    u = np.ascontiguousarray(u, np.float64)
    n = np.ascontiguousarray(n, np.float64)
    g = np.zeros(7)
    lib.orc_phase_collide(float(phi), _ptr(u), _ptr(n), float(gamma), _ptr(g))
    return g


def noise(seed, stream, step, node, comp):
    return _load().orc_noise(seed, stream, step, node, comp)


def splitmix64_next(state):
    return _load().orc_splitmix64_next(state)


class Oracle:
    """One FP64 population-form lattice (periodic or with boundary layers)."""

    def __init__(self, nx, ny, nz, nu, sigma=0.0, width=3.0, gamma=0.0, eps=1e-12,
                 bc=(0, 0, 0, 0, 0, 0), inlet_u=0.0, inlet_d=0.0, inlet_noise=0.0, seed=0,
                 rho_a=None, rho_b=None, nu_a=None, nu_b=None, gravity=(0.0, 0.0, 0.0)):
        """rho_a/rho_b/nu_a/nu_b given: the variable-density scheme (then the
        state's first field is rho = 1 + p*, p* the normalised pressure, and nu
        is unused); otherwise the paper's equal-density scheme."""
        self.lib = _load()
        p = OrcParams()
        p.nx, p.ny, p.nz = nx, ny, nz
        for s in range(6):
            p.bc[s] = int(bc[s])
        p.nu, p.sigma, p.width, p.gamma, p.eps = nu, sigma, width, gamma, eps
        p.inlet_u, p.inlet_d, p.inlet_noise = inlet_u, inlet_d, inlet_noise
        p.seed = seed
        if rho_a is not None:
            p.vd = 1
            p.rho_a, p.rho_b, p.nu_a, p.nu_b = float(rho_a), float(rho_b), float(nu_a), float(nu_b)
            for c in range(3):
                p.grav[c] = float(gravity[c])
        self.vd = bool(p.vd)
        h = ctypes.c_void_p()
        rc = self.lib.orc_create(ctypes.byref(p), ctypes.byref(h))
        if rc != 0:
            raise ValueError("oracle rejected the parameters (rc=%d)" % rc)
        self.h = h
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz

    def close(self):
        if getattr(self, "h", None):
            self.lib.orc_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    @property
    def omega(self):
        return self.lib.orc_omega(self.h)

    @property
    def gamma(self):
        return self.lib.orc_gamma(self.h)

    @property
    def step_count(self):
        return self.lib.orc_step_count(self.h)

    def _f(self, k=None):
        shape = self.shape if k is None else (k,) + self.shape
        return np.zeros(shape)

    def set_physical(self, rho, u, P, phi, step=0):
        c = lambda a: np.ascontiguousarray(a, np.float64)  # noqa: E731
        rho, u, P, phi = c(rho), c(u), c(P), c(phi)
        assert rho.shape == self.shape and u.shape == (3,) + self.shape
        assert P.shape == (6,) + self.shape and phi.shape == self.shape
        self.lib.orc_set_physical(self.h, _ptr(rho), _ptr(u), _ptr(P), _ptr(phi), int(step))

    def step(self, n=1):
        self.lib.orc_step(self.h, int(n))

    def physical(self):
        rho, u, P, phi = self._f(), self._f(3), self._f(6), self._f()
        self.lib.orc_get_physical(self.h, _ptr(rho), _ptr(u), _ptr(P), _ptr(phi))
        return {"rho": rho, "u": u, "P": P, "phi": phi}

    def raw(self):
        drho, ub, Q, phi = self._f(), self._f(3), self._f(6), self._f()
        self.lib.orc_get_raw(self.h, _ptr(drho), _ptr(ub), _ptr(Q), _ptr(phi))
        return {"drho": drho, "ubar": ub, "Q": Q, "phi": phi}

    def geometry(self):
        G, n, kappa, F = self._f(3), self._f(3), self._f(), self._f(3)
        self.lib.orc_get_geometry(self.h, _ptr(G), _ptr(n), _ptr(kappa), _ptr(F))
        return {"G": G, "n": n, "kappa": kappa, "F": F}

    def accel(self):
        """(acceleration a (3, ...), omega (...)) of the current state."""
        a, om = self._f(3), self._f()
        self.lib.orc_get_accel(self.h, _ptr(a), _ptr(om))
        return a, om

    def sums(self):
        m, p = ctypes.c_double(), ctypes.c_double()
        self.lib.orc_sums(self.h, ctypes.byref(m), ctypes.byref(p))
        return m.value, p.value

    def populations(self):
        f, g = self._f(27), self._f(7)
        self.lib.orc_get_populations(self.h, _ptr(f), _ptr(g))
        return f, g
