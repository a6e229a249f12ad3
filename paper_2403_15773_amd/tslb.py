"""Thin ctypes binding of ``libtslb.so`` (the C-ABI in ``include/tslb.h``).

Argument marshalling only: every step of the method runs in the HIP kernels.
The library must have been built (``__graft_entry__.build()``); there is no
fallback, and a missing library raises.  PyTorch is optional: a torch CUDA
tensor may be handed in as the device allocation and a torch stream as the
stream, but nothing here computes with torch.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtslb.so")
ABI_VERSION = 4

OK, E_INVAL, E_NOMEM, E_DEVICE, E_UNSTABLE, E_STATE = 0, -1, -2, -3, -4, -5
BC_PERIODIC, BC_FREESLIP, BC_INLET, BC_OUTFLOW, BC_NOSLIP = 0, 1, 2, 3, 4
STORE_FP32, STORE_FP16, STORE_BF16, STORE_FP16Q = 0, 1, 2, 3
STORAGE = {"fp32": STORE_FP32, "fp16": STORE_FP16, "bf16": STORE_BF16, "fp16q": STORE_FP16Q}

EXPORTS = [
    "tslb_params_init", "tslb_params_size", "tslb_required_bytes", "tslb_create", "tslb_set_state", "tslb_step", "tslb_sync",
    "tslb_moments", "tslb_phase", "tslb_state_bytes", "tslb_get_state_raw", "tslb_set_state_raw",
    "tslb_diagnostics", "tslb_step_index", "tslb_set_timing", "tslb_last_step_kernel_ms", "tslb_set_kernel",
    "tslb_copy_bandwidth", "tslb_destroy", "tslb_last_error",
    "tslb_group_create", "tslb_group_admit", "tslb_group_poll", "tslb_group_status", "tslb_group_destroy",
    "tslb_group_last_error", "tslb_stats_start", "tslb_stats_stop", "tslb_stats_get", "tslb_probe_projection",
    "tslb_set_state_rest", "tslb_step_kernel_times", "tslb_device_memory", "tslb_group_busy", "tslb_device_bytes",
    "tslb_diagnostics_noalloc", "tslb_set_tile", "tslb_tile_rows",
]
KERNEL_FUSED, KERNEL_GATHER = 0, 1


class TslbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("tslb error %d: %s" % (code, msg))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 6),
        ("nu", ctypes.c_double), ("sigma", ctypes.c_double), ("width", ctypes.c_double),
        ("gamma", ctypes.c_double), ("eps", ctypes.c_double),
        ("inlet_u", ctypes.c_double), ("inlet_d", ctypes.c_double), ("inlet_noise", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("storage", ctypes.c_int32),
        ("u_scale", ctypes.c_double),
        ("check_interval", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("device_buffer", ctypes.c_void_p),
        ("device_buffer_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
        ("components", ctypes.c_int32),
        ("max_mass_drift", ctypes.c_double),
        ("variable_density", ctypes.c_int32),
        ("density_a", ctypes.c_double), ("density_b", ctypes.c_double),
        ("nu_a", ctypes.c_double), ("nu_b", ctypes.c_double),
        ("gravity", ctypes.c_double * 3),
    ]


_lock = threading.Lock()
_lib = None
_F = ctypes.POINTER(ctypes.c_float)


def load_library(path: str = LIB_PATH):
    """Load the built library; raise if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError("libtslb.so is not built (expected at %s); run __graft_entry__.build()" % path)
        lib = ctypes.CDLL(path)
        vp, P = ctypes.c_void_p, ctypes.POINTER(Params)
        sig = {
            "tslb_params_init": (None, [P]),
            "tslb_params_size": (ctypes.c_size_t, []),
            "tslb_required_bytes": (ctypes.c_size_t, [P]),
            "tslb_create": (ctypes.c_int, [P, ctypes.POINTER(vp)]),
            "tslb_set_state": (ctypes.c_int, [vp, _F, _F, _F, _F, ctypes.c_int64]),
            "tslb_set_state_rest": (ctypes.c_int, [vp, ctypes.c_int64]),
            "tslb_step": (ctypes.c_int, [vp, ctypes.c_int64]),
            "tslb_sync": (ctypes.c_int, [vp]),
            "tslb_moments": (ctypes.c_int, [vp, _F, _F, _F]),
            "tslb_phase": (ctypes.c_int, [vp, _F]),
            "tslb_state_bytes": (ctypes.c_size_t, [vp]),
            "tslb_device_bytes": (ctypes.c_size_t, [vp]),
            "tslb_get_state_raw": (ctypes.c_int, [vp, vp, ctypes.c_size_t]),
            "tslb_set_state_raw": (ctypes.c_int, [vp, vp, ctypes.c_size_t, ctypes.c_int64]),
            "tslb_diagnostics": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                                ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]),
            "tslb_diagnostics_noalloc": (ctypes.c_int, [P, vp, vp, vp]),
            "tslb_step_index": (ctypes.c_int64, [vp]),
            "tslb_set_timing": (ctypes.c_int, [vp, ctypes.c_int]),
            "tslb_last_step_kernel_ms": (ctypes.c_double, [vp]),
            "tslb_step_kernel_times": (ctypes.c_int, [vp, _F, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
            "tslb_set_kernel": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int]),
            "tslb_set_tile": (ctypes.c_int, [vp, ctypes.c_int]),
            "tslb_tile_rows": (ctypes.c_int, [vp]),
            "tslb_copy_bandwidth": (ctypes.c_int, [ctypes.c_int, ctypes.c_size_t, ctypes.c_int,
                                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
            "tslb_probe_projection": (ctypes.c_int, [ctypes.c_int32, vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                                     ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_double)]),
            "tslb_destroy": (None, [vp]),
            "tslb_last_error": (ctypes.c_char_p, [vp]),
            "tslb_group_create": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_int32, vp, ctypes.POINTER(vp)]),
            "tslb_group_admit": (ctypes.c_int, [vp, vp, ctypes.c_int64]),
            "tslb_group_poll": (ctypes.c_int, [vp, ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
            "tslb_group_status": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_int32),
                                                 ctypes.POINTER(ctypes.c_int64)]),
            "tslb_group_busy": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
            "tslb_device_memory": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t),
                                                  ctypes.POINTER(ctypes.c_size_t)]),
            "tslb_group_destroy": (None, [vp]),
            "tslb_group_last_error": (ctypes.c_char_p, [vp]),
            "tslb_stats_start": (ctypes.c_int, [vp, ctypes.c_int32]),
            "tslb_stats_stop": (ctypes.c_int, [vp]),
            "tslb_stats_get": (ctypes.c_int, [vp, _F, _F, _F, ctypes.POINTER(ctypes.c_int64)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def make_params(nx, ny, nz, nu, sigma=0.0, width=3.0, gamma=0.0, eps=-1.0, bc=(0,) * 6, inlet_u=0.0,
                inlet_d=0.0, inlet_noise=0.0, seed=0, storage="fp32", u_scale=0.0, check_interval=0, device=0,
                device_buffer=None, device_buffer_bytes=0, stream=None, components=2, max_mass_drift=0.0,
                density_a=None, density_b=None, nu_a=None, nu_b=None, gravity=(0.0, 0.0, 0.0)) -> Params:
    """Lattice parameters.  density_a/density_b/nu_a/nu_b given select the
    variable-density step (then rho_dev of the state is the normalised pressure
    p* and nu is unused)."""
    lib = load_library()
    p = Params()
    lib.tslb_params_init(ctypes.byref(p))
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    for s in range(6):
        p.bc[s] = int(bc[s])
    p.nu, p.sigma, p.width, p.gamma, p.eps = float(nu), float(sigma), float(width), float(gamma), float(eps)
    p.inlet_u, p.inlet_d, p.inlet_noise = float(inlet_u), float(inlet_d), float(inlet_noise)
    p.seed = int(seed)
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.u_scale = float(u_scale)
    p.check_interval = int(check_interval)
    p.device = int(device)
    p.device_buffer = device_buffer
    p.device_buffer_bytes = int(device_buffer_bytes)
    p.stream = stream
    p.components = int(components)
    p.max_mass_drift = float(max_mass_drift)
    if density_a is not None:
        p.variable_density = 1
        p.density_a, p.density_b = float(density_a), float(density_b)
        p.nu_a, p.nu_b = float(nu_a), float(nu_b)
    for c in range(3):
        p.gravity[c] = float(gravity[c])
    return p


def copy_bandwidth(nbytes: int, iters: int = 20, device: int = 0):
    """(GB/s of read + written bytes, median ms) of the library's plain copy kernel."""
    lib = load_library()
    g, m = ctypes.c_double(), ctypes.c_double()
    rc = lib.tslb_copy_bandwidth(int(device), int(nbytes), int(iters), ctypes.byref(g), ctypes.byref(m))
    if rc != OK:
        raise TslbError(rc, lib.tslb_last_error(None).decode())
    return g.value, m.value


def device_memory(device: int = 0):
    """(free, total) device memory in bytes."""
    lib = load_library()
    f, t = ctypes.c_size_t(), ctypes.c_size_t()
    rc = lib.tslb_device_memory(int(device), ctypes.byref(f), ctypes.byref(t))
    if rc != OK:
        raise TslbError(rc, lib.tslb_last_error(None).decode())
    return f.value, t.value


PROJECTION_VALU, PROJECTION_MFMA = 0, 1


def projection_probe(kind, coef, reps: int, iters: int = 10, device: int = 0, want_out: bool = True):
    """(mean ms per launch, accumulated brackets (27, nodes) or None) of the
    library's moment-to-population projection probe; coef is (16, nodes)."""
    lib = load_library()
    coef = np.ascontiguousarray(coef, np.float32)
    nodes = coef.shape[1]
    out = np.empty((27, nodes), np.float32) if want_out else None
    m = ctypes.c_double()
    rc = lib.tslb_probe_projection(int(kind), coef.ctypes.data, int(nodes), int(reps), int(iters), int(device),
                                   None if out is None else out.ctypes.data, ctypes.byref(m))
    if rc != OK:
        raise TslbError(rc, lib.tslb_last_error(None).decode())
    return m.value, out


def diagnostics_noalloc(params: Params, state_ptr: int, stream_ptr, out_ptr: int) -> None:
    """Queue tslb_diagnostics_noalloc: state_ptr and out_ptr are device
    addresses (one state buffer; three doubles), stream_ptr a hipStream_t or
    None.  Nothing is allocated."""
    lib = load_library()
    rc = lib.tslb_diagnostics_noalloc(ctypes.byref(params), state_ptr, stream_ptr, out_ptr)
    if rc != OK:
        raise TslbError(rc, lib.tslb_last_error(None).decode())


def required_bytes(params: Params) -> int:
    return load_library().tslb_required_bytes(ctypes.byref(params))


def _f32(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.shape != shape:
        raise ValueError("expected shape %s, got %s" % (shape, a.shape))
    return a


class Simulation:
    """One lattice on the GPU (a ``tslb_ctx``)."""

    def __init__(self, params: Params | None = None, **kw):
        self.lib = load_library()
        self.params = params if params is not None else make_params(**kw)
        h = ctypes.c_void_p()
        rc = self.lib.tslb_create(ctypes.byref(self.params), ctypes.byref(h))
        if rc != OK:
            raise TslbError(rc, self.lib.tslb_last_error(None).decode())
        self.h = h
        self.shape = (self.params.nz, self.params.ny, self.params.nx)
        self.N = self.params.nx * self.params.ny * self.params.nz

    def _check(self, rc):
        if rc != OK:
            raise TslbError(rc, self.lib.tslb_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.tslb_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_state(self, rho_dev, u, P, phi=None, step=0):
        """Physical fields: rho_dev = rho - 1, u (3,...), P (6,...), phi (None for one component)."""
        sh = self.shape
        rho_dev, u, P = _f32(rho_dev, sh), _f32(u, (3,) + sh), _f32(P, (6,) + sh)
        phi_p = None if phi is None else _f32(phi, sh).ctypes.data_as(_F)
        self._check(self.lib.tslb_set_state(self.h, rho_dev.ctypes.data_as(_F), u.ctypes.data_as(_F),
                                            P.ctypes.data_as(_F), phi_p, int(step)))

    def set_state_rest(self, step=0):
        """Fluid at rest: rho = 1, u = 0, P = 0, phi = 0 (no host transfer)."""
        self._check(self.lib.tslb_set_state_rest(self.h, int(step)))

    def step(self, n=1):
        self._check(self.lib.tslb_step(self.h, int(n)))

    def sync(self):
        self._check(self.lib.tslb_sync(self.h))

    def moments(self):
        """(rho - 1, u, P) at the current step, float32."""
        sh = self.shape
        drho, u, P = np.empty(sh, np.float32), np.empty((3,) + sh, np.float32), np.empty((6,) + sh, np.float32)
        self._check(self.lib.tslb_moments(self.h, drho.ctypes.data_as(_F), u.ctypes.data_as(_F),
                                          P.ctypes.data_as(_F)))
        return drho, u, P

    def phase(self):
        phi = np.empty(self.shape, np.float32)
        self._check(self.lib.tslb_phase(self.h, phi.ctypes.data_as(_F)))
        return phi

    def physical(self):
        """dict with rho_dev (float32), rho = 1 + rho_dev (float64), u, P, phi."""
        drho, u, P = self.moments()
        return {"rho_dev": drho, "rho": 1.0 + drho.astype(np.float64), "u": u, "P": P, "phi": self.phase()}

    @property
    def state_bytes(self):
        return self.lib.tslb_state_bytes(self.h)

    @property
    def device_bytes(self):
        """Device memory the lattice holds now (what a serving group charges)."""
        return self.lib.tslb_device_bytes(self.h)

    def get_state_raw(self) -> np.ndarray:
        buf = np.empty(self.state_bytes, np.uint8)
        self._check(self.lib.tslb_get_state_raw(self.h, buf.ctypes.data, buf.nbytes))
        return buf

    def set_state_raw(self, buf: np.ndarray, step: int):
        buf = np.ascontiguousarray(buf, np.uint8)
        self._check(self.lib.tslb_set_state_raw(self.h, buf.ctypes.data, buf.nbytes, int(step)))

    def diagnostics(self):
        m, p = ctypes.c_double(), ctypes.c_double()
        s, f = ctypes.c_int64(), ctypes.c_int32()
        self._check(self.lib.tslb_diagnostics(self.h, ctypes.byref(m), ctypes.byref(p), ctypes.byref(s),
                                              ctypes.byref(f)))
        return {"mass": m.value, "phase": p.value, "step": s.value, "finite": bool(f.value)}

    @property
    def step_index(self):
        return self.lib.tslb_step_index(self.h)

    def set_timing(self, enable=True):
        self._check(self.lib.tslb_set_timing(self.h, 1 if enable else 0))

    def last_step_kernel_ms(self):
        return self.lib.tslb_last_step_kernel_ms(self.h)

    def step_kernel_times(self) -> np.ndarray:
        """Per-launch fused-kernel durations (ms) of the last timed step() call."""
        n = ctypes.c_int64()
        self._check(self.lib.tslb_step_kernel_times(self.h, None, 0, ctypes.byref(n)))
        out = np.empty(n.value, np.float32)
        self._check(self.lib.tslb_step_kernel_times(self.h, out.ctypes.data_as(_F), out.size, ctypes.byref(n)))
        return out

    def stats_start(self, every=1):
        """Accumulate time averages of phi, u and u_z^2 every `every` steps."""
        self._check(self.lib.tslb_stats_start(self.h, int(every)))

    def stats_stop(self):
        self._check(self.lib.tslb_stats_stop(self.h))

    def stats_samples(self) -> int:
        """Samples accumulated since the last stats_start (0 before any)."""
        n = ctypes.c_int64()
        self._check(self.lib.tslb_stats_get(self.h, None, None, None, ctypes.byref(n)))
        return n.value

    def stats(self):
        """dict: mean_phi, mean_u (3, ...), rms_uz, samples; raises with no samples."""
        sh = self.shape
        mp, mu, rz = np.empty(sh, np.float32), np.empty((3,) + sh, np.float32), np.empty(sh, np.float32)
        n = ctypes.c_int64()
        self._check(self.lib.tslb_stats_get(self.h, mp.ctypes.data_as(_F), mu.ctypes.data_as(_F),
                                            rz.ctypes.data_as(_F), ctypes.byref(n)))
        return {"mean_phi": mp, "mean_u": mu, "rms_uz": rz, "samples": n.value}

    def set_kernel(self, kernel="fused", chunk_z=0):
        k = {"fused": KERNEL_FUSED, "gather": KERNEL_GATHER}[kernel] if isinstance(kernel, str) else int(kernel)
        self._check(self.lib.tslb_set_kernel(self.h, k, int(chunk_z)))

    def set_tile(self, rows=0):
        """Fused-step tile height: 16 or 20 rows, 0 = the library's choice."""
        self._check(self.lib.tslb_set_tile(self.h, int(rows)))

    @property
    def tile_rows(self):
        return int(self.lib.tslb_tile_rows(self.h))


class Group:
    """A serving group (``tslb_group``): admitted Simulations advance together,
    one multi-domain step launch per :meth:`poll`."""

    def __init__(self, hbm_budget_bytes: int, max_domains: int = 256, stream=None):
        self.lib = load_library()
        h = ctypes.c_void_p()
        rc = self.lib.tslb_group_create(int(hbm_budget_bytes), int(max_domains), stream, ctypes.byref(h))
        if rc != OK:
            raise TslbError(rc, self.lib.tslb_group_last_error(None).decode())
        self.h = h
        self.max_domains = int(max_domains)
        self._members = {}  # ctx handle value -> Simulation

    def _check(self, rc):
        if rc != OK:
            raise TslbError(rc, self.lib.tslb_group_last_error(self.h).decode())

    def admit(self, sim: Simulation, nsteps: int) -> bool:
        """True if admitted; False if the HBM budget or the slots are full (defer)."""
        rc = self.lib.tslb_group_admit(self.h, sim.h, int(nsteps))
        if rc == E_NOMEM:
            return False
        self._check(rc)
        self._members[sim.h.value] = sim
        return True

    def poll(self):
        """Retire finished members (returned as Simulations) and launch the next step."""
        cap = max(1, len(self._members))
        arr = (ctypes.c_void_p * cap)()
        n = ctypes.c_int32()
        self._check(self.lib.tslb_group_poll(self.h, arr, cap, ctypes.byref(n)))
        return [self._members.pop(arr[i]) for i in range(n.value)]

    def status(self):
        b, m, l = ctypes.c_size_t(), ctypes.c_int32(), ctypes.c_int64()
        self._check(self.lib.tslb_group_status(self.h, ctypes.byref(b), ctypes.byref(m), ctypes.byref(l)))
        return {"bytes_in_use": b.value, "members": m.value, "launches": l.value}

    def busy(self):
        """(summed device time of the completed launches in ms, their count)."""
        b, n = ctypes.c_double(), ctypes.c_int64()
        self._check(self.lib.tslb_group_busy(self.h, ctypes.byref(b), ctypes.byref(n)))
        return b.value, n.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.tslb_group_destroy(self.h)
            self.h = None
            self._members = {}

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
