"""Python binding of liblbac.so (the C ABI in include/lbac.h).

Argument marshalling only: every step of the scheme runs in the HIP kernels
of the library.  The functions keep the C names (lbac_init, lbac_step,
lbac_phi, lbac_mass, ...); `Simulation` wraps a context for convenience.
PyTorch supplies the stream (its current stream) and, optionally, device
memory through its caching allocator.

There is no fallback: if the library cannot be loaded, `load()` raises.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

LBAC_OK, LBAC_EINVAL, LBAC_ENOMEM, LBAC_EDEVICE, LBAC_ENONFINITE, LBAC_ESTATE = 0, -1, -2, -3, -4, -5
VEL = {"zero": 0, "vortex": 1, "rotation": 2, "uniform": 3, "vortex_paper": 4}
PRECISION = {"f64": 0, "f32": 1, "f32_f16store": 2, "f32_bf16store": 3}
MODEL = {"improved": 0, "conventional": 1}

_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class lbac_allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", C.c_void_p)]


class lbac_params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("eps", C.c_double), ("tau", C.c_double), ("delta", C.c_double),
        ("vel_kind", C.c_int32),
        ("U", C.c_double), ("period_T", C.c_double),
        ("omega", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
        ("ux", C.c_double), ("uy", C.c_double),
        ("precision", C.c_int32), ("model", C.c_int32),
        ("stream", C.c_void_p),
        ("alloc", C.POINTER(lbac_allocator)),
    ]


class lbac3_params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("eps", C.c_double), ("tau", C.c_double), ("delta", C.c_double),
        ("vel_kind", C.c_int32),
        ("U", C.c_double), ("period_T", C.c_double),
        ("ux", C.c_double), ("uy", C.c_double), ("uz", C.c_double),
        ("precision", C.c_int32),
        ("stream", C.c_void_p),
    ]


EXPORTS = [
    "lbac_default_params", "lbac_init", "lbac_init_device", "lbac_free", "lbac_step", "lbac_phi",
    "lbac_phi_device", "lbac_mass", "lbac_shape_error", "lbac_time", "lbac_get_state", "lbac_set_state",
    "lbac_set_launch", "lbac_get_launch", "lbac_autotune", "lbac_set_graph_chunk", "lbac_bytes_per_node",
    "lbac_steps_per_launch",
    "lbac_copy_ceiling", "lbac_set_closure",
    "lbac_stream", "lbac_strerror", "lbac_last_error",
    "lbac_batch_init", "lbac_batch_free", "lbac_batch_run", "lbac_batch_instance", "lbac_batch_count",
    "lbac_batch_phi", "lbac_batch_mass",
    "lbac_batch_set_shape", "lbac_batch_get_shape", "lbac_batch_autotune", "lbac_batch_set_timeout",
    "lbac_batch_last_error", "lbac_batch_schedule_check",
    "lbac_mlp_create", "lbac_mlp_free", "lbac_mlp_get_weights", "lbac_mlp_set_weights", "lbac_mlp_forward",
    "lbac_mlp_loss_grad", "lbac_mlp_train_step", "lbac_mlp_last_error",
    "lbac_closure_workspace_bytes", "lbac_closure_extract", "lbac_closure_extract_noalloc",
]
# include/lbac3.h (the D3Q19 form)
EXPORTS3 = [
    "lbac3_default_params", "lbac3_init", "lbac3_step", "lbac3_phi", "lbac3_mass", "lbac3_shape_error",
    "lbac3_time", "lbac3_set_launch", "lbac3_get_launch", "lbac3_autotune", "lbac3_bytes_per_node",
    "lbac3_last_error", "lbac3_free",
]
VEL3 = {"zero": 0, "deformation": 1, "vortex_xy": 2, "uniform": 3}
MLP_NPARAM = 5954

_lib = None


def lib_path():
    return _build.LIB


def load():
    """Loads liblbac.so (building it first only if no built library exists)."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        _build.build()
    L = C.CDLL(path)
    P = C.POINTER
    ctx_pp = P(C.c_void_p)
    dp = P(C.c_double)
    L.lbac_default_params.argtypes = [P(lbac_params), C.c_int32, C.c_int32]
    L.lbac_default_params.restype = None
    L.lbac_init.argtypes = [P(lbac_params), dp, ctx_pp]
    L.lbac_init_device.argtypes = [P(lbac_params), C.c_void_p, ctx_pp]
    L.lbac_free.argtypes = [C.c_void_p]
    L.lbac_step.argtypes = [C.c_void_p, C.c_int64]
    L.lbac_phi.argtypes = [C.c_void_p, dp]
    L.lbac_phi_device.argtypes = [C.c_void_p, C.c_void_p]
    L.lbac_mass.argtypes = [C.c_void_p, dp]
    L.lbac_shape_error.argtypes = [C.c_void_p, dp, dp, dp]
    L.lbac_time.argtypes = [C.c_void_p, P(C.c_int64)]
    L.lbac_get_state.argtypes = [C.c_void_p, C.c_void_p, P(C.c_size_t)]
    L.lbac_set_state.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
    L.lbac_set_launch.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]
    L.lbac_copy_ceiling.argtypes = [C.c_void_p, C.c_int32, P(C.c_double)]
    L.lbac_get_launch.argtypes = [C.c_void_p, P(C.c_int32), P(C.c_int32), P(C.c_int32)]
    L.lbac_autotune.argtypes = [C.c_void_p, C.c_int32, dp]
    L.lbac_set_graph_chunk.argtypes = [C.c_void_p, C.c_int32]
    L.lbac_bytes_per_node.argtypes = [C.c_void_p, dp]
    L.lbac_steps_per_launch.argtypes = [C.c_void_p, P(C.c_int32)]
    L.lbac_set_closure.argtypes = [C.c_void_p, P(C.c_float), C.c_float]
    L.lbac_stream.argtypes = [C.c_void_p]
    L.lbac_stream.restype = C.c_void_p
    L.lbac_strerror.argtypes = [C.c_int]
    L.lbac_strerror.restype = C.c_char_p
    L.lbac_last_error.argtypes = [C.c_void_p]
    L.lbac_last_error.restype = C.c_char_p
    L.lbac_batch_init.argtypes = [P(lbac_params), P(P(C.c_double)), C.c_int32, ctx_pp]
    L.lbac_batch_free.argtypes = [C.c_void_p]
    L.lbac_batch_run.argtypes = [C.c_void_p, P(C.c_int64)]
    L.lbac_batch_instance.argtypes = [C.c_void_p, C.c_int32, ctx_pp]
    L.lbac_batch_count.argtypes = [C.c_void_p, P(C.c_int32)]
    L.lbac_batch_phi.argtypes = [C.c_void_p, C.c_int32, P(C.c_double)]
    L.lbac_batch_mass.argtypes = [C.c_void_p, P(C.c_double)]
    L.lbac_batch_set_shape.argtypes = [C.c_void_p, C.c_int32]
    L.lbac_batch_get_shape.argtypes = [C.c_void_p, P(C.c_int32), P(C.c_int32)]
    L.lbac_batch_autotune.argtypes = [C.c_void_p, P(C.c_int64), dp]
    L.lbac_batch_set_timeout.argtypes = [C.c_void_p, C.c_double, C.c_int32]
    L.lbac_batch_last_error.argtypes = [C.c_void_p]
    L.lbac_batch_schedule_check.argtypes = [P(C.c_int32), P(C.c_int32), P(C.c_int64), C.c_int32, C.c_int32,
                                            C.c_int32, C.c_int32, C.c_uint64, P(C.c_int32), P(C.c_int64)]
    L.lbac_batch_last_error.restype = C.c_char_p
    fp = P(C.c_float)
    L.lbac_mlp_create.argtypes = [fp, C.c_void_p, ctx_pp]
    L.lbac_mlp_free.argtypes = [C.c_void_p]
    L.lbac_mlp_get_weights.argtypes = [C.c_void_p, fp]
    L.lbac_mlp_set_weights.argtypes = [C.c_void_p, fp]
    L.lbac_mlp_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
    L.lbac_mlp_loss_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, dp, fp]
    L.lbac_mlp_train_step.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_float, dp]
    L.lbac_mlp_last_error.argtypes = [C.c_void_p]
    L.lbac_mlp_last_error.restype = C.c_char_p
    L.lbac_closure_workspace_bytes.argtypes = [C.c_int32, C.c_int32, C.c_int32]
    L.lbac_closure_workspace_bytes.restype = C.c_int64
    L.lbac_closure_extract.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                       C.c_double, C.c_float, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_int64, C.c_int64, P(C.c_int64), C.c_void_p]
    L.lbac_closure_extract_noalloc.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                               C.c_double, C.c_float, C.c_int32, C.c_void_p, C.c_void_p, C.c_int64,
                                               C.c_int64, P(C.c_int64), C.c_void_p]
    p3 = P(lbac3_params)
    L.lbac3_default_params.argtypes = [p3, C.c_int32, C.c_int32, C.c_int32]
    L.lbac3_default_params.restype = None
    L.lbac3_init.argtypes = [p3, dp, ctx_pp]
    L.lbac3_step.argtypes = [C.c_void_p, C.c_int64]
    L.lbac3_phi.argtypes = [C.c_void_p, dp]
    L.lbac3_mass.argtypes = [C.c_void_p, dp]
    L.lbac3_shape_error.argtypes = [C.c_void_p, dp, dp, dp]
    L.lbac3_time.argtypes = [C.c_void_p, P(C.c_int64)]
    L.lbac3_set_launch.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
    L.lbac3_get_launch.argtypes = [C.c_void_p, P(C.c_int32), P(C.c_int32), P(C.c_int32), P(C.c_int32), P(C.c_int32)]
    L.lbac3_autotune.argtypes = [C.c_void_p, C.c_int32, dp]
    L.lbac3_bytes_per_node.argtypes = [C.c_void_p, dp]
    L.lbac3_last_error.argtypes = [C.c_void_p]
    L.lbac3_last_error.restype = C.c_char_p
    L.lbac3_free.argtypes = [C.c_void_p]
    for name in EXPORTS + EXPORTS3:
        if name not in ("lbac_default_params", "lbac_stream", "lbac_strerror", "lbac_last_error",
                        "lbac_batch_last_error", "lbac_mlp_last_error", "lbac_closure_workspace_bytes",
                        "lbac3_default_params", "lbac3_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


class LbacError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("lbac error %d (%s): %s" % (code, load().lbac_strerror(code).decode(), msg))
        self.code = code


def _check(rc, ctx=None, what=""):
    if rc != LBAC_OK:
        msg = load().lbac_last_error(ctx).decode() if ctx else what
        raise LbacError(rc, msg or what)


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(nx, ny, eps=1.0, tau=0.8, delta=1e-10, vel="vortex", U=0.02, period_T=2000.0, omega=0.0,
                cx=None, cy=None, ux=0.0, uy=0.0, precision="f64", model="improved", stream=None, **_ignored):
    p = lbac_params()
    load().lbac_default_params(C.byref(p), int(nx), int(ny))
    p.eps, p.tau, p.delta = float(eps), float(tau), float(delta)
    p.vel_kind = VEL[vel] if isinstance(vel, str) else int(vel)
    p.U, p.period_T, p.omega = float(U), float(period_T), float(omega)
    p.cx = 0.5 * nx if cx is None else float(cx)
    p.cy = 0.5 * ny if cy is None else float(cy)
    p.ux, p.uy = float(ux), float(uy)
    p.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    p.model = MODEL[model] if isinstance(model, str) else int(model)
    p.stream = stream
    return p


class TorchAllocator:
    """Routes the library's device allocations through torch's caching allocator."""

    def __init__(self, device=None):
        import torch

        self.torch = torch
        self.device = torch.cuda.current_device() if device is None else device
        self._alloc = _ALLOC_FN(self._do_alloc)
        self._free = _FREE_FN(self._do_free)
        self.struct = lbac_allocator(self._alloc, self._free, None)

    def _do_alloc(self, nbytes, user):
        try:
            s = self.torch.cuda.current_stream(self.device)
            return self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, s)
        except Exception:
            return None

    def _do_free(self, ptr, user):
        if ptr:
            self.torch.cuda.caching_allocator_delete(ptr)


class Simulation:
    """One lattice run on the current GPU.  `case` keys mirror lbac_params."""

    def __init__(self, case, phi0, stream=None, torch_alloc=False):
        L = load()
        self._keep = []
        p = make_params(**{**case, "stream": stream})
        if torch_alloc:
            ta = TorchAllocator()
            self._keep.append(ta)
            p.alloc = C.pointer(ta.struct)
        self.nx, self.ny = p.nx, p.ny
        self.params = p
        phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(p.ny, p.nx)
        h = C.c_void_p()
        _check(L.lbac_init(C.byref(p), _dp(phi0), C.byref(h)), what="lbac_init")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().lbac_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n):
        _check(load().lbac_step(self.h, int(n)), self.h)

    def phi(self):
        out = np.empty((self.ny, self.nx))
        _check(load().lbac_phi(self.h, _dp(out)), self.h)
        return out

    def phi_device(self, out_ptr):
        _check(load().lbac_phi_device(self.h, C.c_void_p(out_ptr)), self.h)

    def mass(self):
        m = C.c_double()
        _check(load().lbac_mass(self.h, C.byref(m)), self.h)
        return m.value

    def shape_error(self, ref):
        ref = np.ascontiguousarray(ref, dtype=np.float64)
        e1, e2 = C.c_double(), C.c_double()
        _check(load().lbac_shape_error(self.h, _dp(ref), C.byref(e1), C.byref(e2)), self.h)
        return e1.value, e2.value

    def time(self):
        t = C.c_int64()
        _check(load().lbac_time(self.h, C.byref(t)), self.h)
        return t.value

    def get_state(self):
        n = C.c_size_t()
        _check(load().lbac_get_state(self.h, None, C.byref(n)), self.h)
        buf = np.empty(n.value, dtype=np.uint8)
        _check(load().lbac_get_state(self.h, buf.ctypes.data_as(C.c_void_p), C.byref(n)), self.h)
        return buf

    def set_state(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(load().lbac_set_state(self.h, buf.ctypes.data_as(C.c_void_p), buf.size), self.h)

    def set_launch(self, bx, strip_h, variant=0):
        """variant 0: block-wide tiles through LDS; 1: one tile per wavefront in
        registers; 2: block-wide with two rows of loads in flight; 3, 4: two or
        three steps per launch (FP32 storage).  bx: tile columns, 64, 128 or
        256; the multi-step variants take any multiple of 32 from 64 to 320."""
        _check(load().lbac_set_launch(self.h, int(variant), int(bx), int(strip_h)), self.h)

    def get_launch(self):
        """(bx, strip_h, variant)"""
        v, bx, sh = C.c_int32(), C.c_int32(), C.c_int32()
        _check(load().lbac_get_launch(self.h, C.byref(v), C.byref(bx), C.byref(sh)), self.h)
        return bx.value, sh.value, v.value

    def autotune(self, steps=10):
        us = C.c_double()
        _check(load().lbac_autotune(self.h, int(steps), C.byref(us)), self.h)
        return us.value

    def set_graph_chunk(self, chunk):
        _check(load().lbac_set_graph_chunk(self.h, int(chunk)), self.h)

    def set_closure(self, params, theta=0.02):
        """Learned closure on (FP32 parameter vector) or off (None)."""
        if params is None:
            _check(load().lbac_set_closure(self.h, None, 0.0), self.h)
            return
        w = np.ascontiguousarray(params, dtype=np.float32)
        assert w.size == MLP_NPARAM
        _check(load().lbac_set_closure(self.h, w.ctypes.data_as(C.POINTER(C.c_float)), float(theta)), self.h)

    def bytes_per_node(self):
        b = C.c_double()
        _check(load().lbac_bytes_per_node(self.h, C.byref(b)), self.h)
        return b.value

    def steps_per_launch(self):
        n = C.c_int32()
        _check(load().lbac_steps_per_launch(self.h, C.byref(n)), self.h)
        return n.value

    def copy_ceiling(self, launches=20):
        """Mean microseconds of a plain copy of the state in the step's access pattern."""
        us = C.c_double()
        _check(load().lbac_copy_ceiling(self.h, int(launches), C.byref(us)), self.h)
        return us.value

    def stream(self):
        return load().lbac_stream(self.h)


class _Borrowed(Simulation):
    """A context owned by a batch (not freed by this object)."""

    def __init__(self, h, nx, ny):
        self.h, self.nx, self.ny, self._keep = h, nx, ny, []

    def close(self):
        self.h = None


class Batch:
    """Independent instances advanced together by one persistent launch.
    precision: the storage of every instance ("f32", "f32_f16store" or
    "f32_bf16store"; FP32 collide in all three)."""

    def __init__(self, cases, phi0s, stream=None, precision="f32"):
        L = load()
        n = len(cases)
        params = (lbac_params * n)()
        for k, c in enumerate(cases):
            params[k] = make_params(**{**c, "precision": precision, "stream": stream if k == 0 else None})
        self._phi = [np.ascontiguousarray(p, dtype=np.float64).reshape(c["ny"], c["nx"]) for c, p in zip(cases, phi0s)]
        ptrs = (C.POINTER(C.c_double) * n)(*[_dp(a) for a in self._phi])
        h = C.c_void_p()
        _check(L.lbac_batch_init(params, ptrs, n, C.byref(h)), what="lbac_batch_init")
        self.h = h
        self.count = n
        self.shapes = [(c["nx"], c["ny"]) for c in cases]

    def _err(self, rc):
        if rc != LBAC_OK:
            raise LbacError(rc, load().lbac_batch_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            load().lbac_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, nsteps):
        ns = (C.c_int64 * self.count)(*[int(v) for v in nsteps])
        self._err(load().lbac_batch_run(self.h, ns))

    def instance(self, k):
        c = C.c_void_p()
        self._err(load().lbac_batch_instance(self.h, int(k), C.byref(c)))
        nx, ny = self.shapes[k]
        return _Borrowed(c, nx, ny)

    def phi(self, k):
        """phi of instance k (ny x nx, FP64) through lbac_batch_phi."""
        nx, ny = self.shapes[k]
        out = np.empty((ny, nx), dtype=np.float64)
        self._err(load().lbac_batch_phi(self.h, int(k), _dp(out)))
        return out

    def masses(self):
        """The mass of every instance through lbac_batch_mass."""
        out = np.empty(self.count, dtype=np.float64)
        self._err(load().lbac_batch_mass(self.h, _dp(out)))
        return out

    def set_shape(self, strip_h):
        self._err(load().lbac_batch_set_shape(self.h, int(strip_h)))

    def get_shape(self):
        """(strip height, workgroups the device keeps resident at once)."""
        a, b = C.c_int32(), C.c_int32()
        self._err(load().lbac_batch_get_shape(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def autotune(self, steps=8):
        """Tunes the strip height on dry runs of `steps` steps per instance (an
        int, or one count per instance); returns the best time in ms."""
        if np.ndim(steps) == 0:
            steps = [int(steps)] * self.count
        ns = (C.c_int64 * self.count)(*[int(v) for v in steps])
        ms = C.c_double()
        self._err(load().lbac_batch_autotune(self.h, ns, C.byref(ms)))
        return ms.value

    def set_timeout(self, seconds, test_stall=False):
        self._err(load().lbac_batch_set_timeout(self.h, float(seconds), 1 if test_stall else 0))


def batch_schedule_check(shapes, nsteps, strip_h, workers, seed=0, protocol=0):
    """Runs a slot protocol of the batched schedule on the CPU (no GPU) for
    instances of the given (nx, ny) shapes and step counts with `workers`
    workgroups running at once (protocol 0: the library's; 1: without the
    dependency waits; 2: fixed per-workgroup item lists).  Returns (verdict,
    slots run): verdict 0 = no deadlock and no hazard, 1 = deadlock, 2 =
    read or write hazard."""
    n = len(shapes)
    nx = (C.c_int32 * n)(*[int(a) for a, _ in shapes])
    ny = (C.c_int32 * n)(*[int(b) for _, b in shapes])
    ns = (C.c_int64 * n)(*[int(v) for v in nsteps])
    verdict, ran = C.c_int32(), C.c_int64()
    _check(load().lbac_batch_schedule_check(nx, ny, ns, n, int(strip_h), int(workers), int(protocol), int(seed),
                                            C.byref(verdict), C.byref(ran)), what="lbac_batch_schedule_check")
    return verdict.value, ran.value


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class Mlp:
    """The closure network on the GPU (FP32 training kernels).  Sample arrays
    are device pointers (for example torch tensors' data_ptr())."""

    def __init__(self, init, stream=None):
        w = np.ascontiguousarray(init, dtype=np.float32)
        assert w.size == MLP_NPARAM
        h = C.c_void_p()
        _check(load().lbac_mlp_create(_fp(w), stream, C.byref(h)), what="lbac_mlp_create")
        self.h = h

    def _err(self, rc):
        if rc != LBAC_OK:
            raise LbacError(rc, load().lbac_mlp_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            load().lbac_mlp_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def weights(self):
        w = np.empty(MLP_NPARAM, dtype=np.float32)
        self._err(load().lbac_mlp_get_weights(self.h, _fp(w)))
        return w

    def set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        self._err(load().lbac_mlp_set_weights(self.h, _fp(w)))

    def forward(self, x_ptr, batch, out_ptr):
        self._err(load().lbac_mlp_forward(self.h, C.c_void_p(x_ptr), int(batch), C.c_void_p(out_ptr)))

    def loss_grad(self, x_ptr, y_ptr, batch):
        L = C.c_double()
        g = np.empty(MLP_NPARAM, dtype=np.float32)
        self._err(load().lbac_mlp_loss_grad(self.h, C.c_void_p(x_ptr), C.c_void_p(y_ptr), int(batch), C.byref(L),
                                            _fp(g)))
        return L.value, g

    def train_step(self, x_ptr, y_ptr, batch, lr, want_loss=False):
        L = C.c_double()
        self._err(load().lbac_mlp_train_step(self.h, C.c_void_p(x_ptr), C.c_void_p(y_ptr), int(batch),
                                             float(lr), C.byref(L) if want_loss else None))
        return L.value if want_loss else None


def closure_extract(phi_f_ptr, nxf, nyf, r, eps_f, eps_c, delta, theta, augment, workspace_ptr, x_ptr, y_ptr,
                    base, capacity, stream=None):
    """Appends closure training samples from a fine field (device pointers);
    returns how many the field yields."""
    n = C.c_int64()
    _check(load().lbac_closure_extract(C.c_void_p(phi_f_ptr), int(nxf), int(nyf), int(r), float(eps_f),
                                       float(eps_c), float(delta), float(theta), 1 if augment else 0,
                                       C.c_void_p(workspace_ptr), C.c_void_p(x_ptr), C.c_void_p(y_ptr), int(base),
                                       int(capacity), C.byref(n), stream), what="lbac_closure_extract")
    return n.value


def closure_extract_noalloc(phi_f_ptr, nxf, nyf, r, eps_f, eps_c, delta, theta, augment, x_ptr, y_ptr, base,
                            capacity, stream=None):
    """closure_extract with the library's fixed device workspace (allocates
    nothing; coarse grids up to 512 x 512)."""
    n = C.c_int64()
    _check(load().lbac_closure_extract_noalloc(C.c_void_p(phi_f_ptr), int(nxf), int(nyf), int(r), float(eps_f),
                                               float(eps_c), float(delta), float(theta), 1 if augment else 0,
                                               C.c_void_p(x_ptr), C.c_void_p(y_ptr), int(base), int(capacity),
                                               C.byref(n), stream), what="lbac_closure_extract_noalloc")
    return n.value


def closure_workspace_bytes(nxf, nyf, r):
    return int(load().lbac_closure_workspace_bytes(int(nxf), int(nyf), int(r)))


def make_params3(nx, ny, nz, eps=1.0, tau=0.8, delta=1e-10, vel="deformation", U=0.02, period_T=None, ux=0.0,
                 uy=0.0, uz=0.0, precision="f32", stream=None, **_ignored):
    p = lbac3_params()
    load().lbac3_default_params(C.byref(p), int(nx), int(ny), int(nz))
    p.eps, p.tau, p.delta = float(eps), float(tau), float(delta)
    p.vel_kind = VEL3[vel] if isinstance(vel, str) else int(vel)
    p.U = float(U)
    if period_T is not None:
        p.period_T = float(period_T)
    p.ux, p.uy, p.uz = float(ux), float(uy), float(uz)
    p.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    p.stream = stream
    return p


def _check3(rc, h=None, what=""):
    if rc != LBAC_OK:
        msg = load().lbac3_last_error(h).decode() if h else load().lbac3_last_error(None).decode()
        raise LbacError(rc, msg or what)


class Simulation3:
    """One run of the D3Q19 form (include/lbac3.h).  `case` keys mirror
    lbac3_params; phi arrays are (nz, ny, nx)."""

    def __init__(self, case, phi0, stream=None):
        L = load()
        p = make_params3(**{**case, "stream": stream})
        self.nx, self.ny, self.nz = p.nx, p.ny, p.nz
        self.params = p
        phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(p.nz, p.ny, p.nx)
        h = C.c_void_p()
        _check3(L.lbac3_init(C.byref(p), _dp(phi0), C.byref(h)), what="lbac3_init")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().lbac3_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n):
        _check3(load().lbac3_step(self.h, int(n)), self.h)

    def phi(self):
        out = np.empty((self.nz, self.ny, self.nx))
        _check3(load().lbac3_phi(self.h, _dp(out)), self.h)
        return out

    def mass(self):
        m = C.c_double()
        _check3(load().lbac3_mass(self.h, C.byref(m)), self.h)
        return m.value

    def shape_error(self, ref):
        ref = np.ascontiguousarray(ref, dtype=np.float64).reshape(self.nz, self.ny, self.nx)
        e1, e2 = C.c_double(), C.c_double()
        _check3(load().lbac3_shape_error(self.h, _dp(ref), C.byref(e1), C.byref(e2)), self.h)
        return e1.value, e2.value

    def time(self):
        t = C.c_int64()
        _check3(load().lbac3_time(self.h, C.byref(t)), self.h)
        return t.value

    def set_launch(self, tile_x, tile_y, variant, strip_z, z_major=0):
        _check3(load().lbac3_set_launch(self.h, int(tile_x), int(tile_y), int(variant), int(strip_z), int(z_major)),
                self.h)

    def get_launch(self):
        v = [C.c_int32() for _ in range(5)]
        _check3(load().lbac3_get_launch(self.h, *[C.byref(x) for x in v]), self.h)
        return tuple(x.value for x in v)

    def autotune(self, steps=8):
        us = C.c_double()
        _check3(load().lbac3_autotune(self.h, int(steps), C.byref(us)), self.h)
        return us.value

    def bytes_per_node(self):
        b = C.c_double()
        _check3(load().lbac3_bytes_per_node(self.h, C.byref(b)), self.h)
        return b.value
