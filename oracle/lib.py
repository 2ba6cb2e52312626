"""ctypes wrapper over the FP64 C oracle (test infrastructure only).

Every function here forwards to ``lbm_oracle.c``; see that file for the
equations each one follows.  Arrays are numpy float64, shape (ny, nx), x
fastest.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

VEL_ZERO, VEL_VORTEX, VEL_ROTATION, VEL_UNIFORM, VEL_VORTEX_PAPER = range(5)
# planted mistakes for pin-sensitivity tests (see the MUT_* list in lbm_oracle.c)
MUTATIONS = {"drop_dt_phiu": 1, "no_force_factor": 2, "flux_sign": 3, "grad_swap": 4, "stream_back": 5,
             "no_clip": 6, "vel_swap": 7, "feq_no_u": 8, "diag_weight": 9}
# planted mistakes in the conventional model (Eq. (1)) and in the closure hook
MUTATIONS_CONVENTIONAL = {"conv_width4": 10, "conv_normal_psi": 11}
MUTATIONS_CLOSURE = {"closure_no_cs2": 12, "closure_stencil_t": 13}
READ_JAIN, READ_LITERAL, READ_LIANG = range(3)
# test-only perturbations (Params.noise): every post-collision population, or
# the shifted populations g_i = f*_i - w_i phi* with the node's sum kept
NOISE_POPULATIONS, NOISE_SHIFTED = range(2)
MODEL_IMPROVED, MODEL_CONVENTIONAL = range(2)


class OrcParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("eps", C.c_double), ("tau", C.c_double), ("delta", C.c_double),
        ("vel_kind", C.c_int32),
        ("U", C.c_double), ("period_T", C.c_double),
        ("omega", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
        ("ux", C.c_double), ("uy", C.c_double),
        ("reading", C.c_int32), ("model", C.c_int32),
        ("mlp", C.POINTER(C.c_double)), ("theta", C.c_double),
        ("mutation", C.c_int32),
        ("noise", C.c_double), ("noise_seed", C.c_uint64),
        ("noise_kind", C.c_int32), ("noise_every", C.c_int32),
    ]


_lib = None
_path = None  # a build other than the in-tree one (use_library)


def use_library(path):
    """Loads the oracle from `path` (another build of lbm_oracle.c, for
    example one compiled for the host's own CPU) instead of the in-tree one."""
    global _lib, _path
    _lib, _path = None, path


def lib():
    global _lib
    if _lib is None:
        path = _path or _build.LIB
        if _path is None and (not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC)):
            _build.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        L.orc_run.argtypes = [C.POINTER(OrcParams), dp, C.c_long, dp, dp]
        L.orc_run_window.argtypes = [C.POINTER(OrcParams), dp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_long, dp]
        L.orc_psi.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int]
        L.orc_psi.restype = C.c_double
        L.orc_sharpen.argtypes = [C.c_double, C.c_double, C.c_int]
        L.orc_sharpen.restype = C.c_double
        L.orc_sharpen_conventional.argtypes = [C.c_double, C.c_double, C.c_int]
        L.orc_sharpen_conventional.restype = C.c_double
        L.orc_feq.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        L.orc_forcing.argtypes = [C.c_double, C.c_double, dp]
        L.orc_gradient.argtypes = [dp, C.c_int, C.c_int, dp, dp]
        L.orc_velocity.argtypes = [C.POINTER(OrcParams), C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_flux.argtypes = [C.POINTER(OrcParams), dp, C.c_int, C.c_int, dp, dp]
        L.orc_closure_field.argtypes = [C.POINTER(OrcParams), dp, C.c_int, C.c_int, dp, dp]
        L.orc_mlp.argtypes = [dp, dp, dp]
        L.orc_lattice.argtypes = [C.POINTER(C.c_int), C.POINTER(C.c_int), dp]
        L.orc_nparam.restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Params:
    """Problem description mirrored into the C struct.  Defaults follow the
    64x64 single-vortex case: eps = 1, tau = 0.8, delta = 1e-10, U = 0.02."""

    def __init__(self, nx, ny, eps=1.0, tau=0.8, delta=1e-10, vel_kind=VEL_VORTEX, U=0.02,
                 period_T=2000.0, omega=0.0, cx=None, cy=None, ux=0.0, uy=0.0,
                 reading=READ_JAIN, model=MODEL_IMPROVED, mlp=None, theta=0.0, mutation=0, noise=0.0,
                 noise_seed=0, noise_kind=0, noise_every=1):
        self.nx, self.ny = int(nx), int(ny)
        self.eps, self.tau, self.delta = float(eps), float(tau), float(delta)
        self.vel_kind, self.U, self.period_T = int(vel_kind), float(U), float(period_T)
        self.omega = float(omega)
        self.cx = 0.5 * nx if cx is None else float(cx)
        self.cy = 0.5 * ny if cy is None else float(cy)
        self.ux, self.uy = float(ux), float(uy)
        self.reading, self.model = int(reading), int(model)
        self.mlp = None if mlp is None else np.ascontiguousarray(mlp, dtype=np.float64)
        self.theta = float(theta)
        self.mutation = int(mutation)
        self.noise, self.noise_seed = float(noise), int(noise_seed)
        self.noise_kind, self.noise_every = int(noise_kind), int(noise_every)

    def c(self):
        s = OrcParams(self.nx, self.ny, self.eps, self.tau, self.delta, self.vel_kind, self.U, self.period_T,
                      self.omega, self.cx, self.cy, self.ux, self.uy, self.reading, self.model,
                      None if self.mlp is None else _dp(self.mlp), self.theta, self.mutation, self.noise,
                      self.noise_seed, self.noise_kind, self.noise_every)
        return s


def run(p: Params, phi0, nsteps, with_mass=False):
    """phi after nsteps steps (and sum phi at t = 0..nsteps if with_mass)."""
    phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(p.ny, p.nx)
    out = np.empty_like(phi0)
    mass = np.empty(nsteps + 1) if with_mass else None
    cp = p.c()
    rc = lib().orc_run(C.byref(cp), _dp(phi0), int(nsteps), _dp(out), None if mass is None else _dp(mass))
    if rc != 0:
        raise RuntimeError("orc_run failed: %d" % rc)
    return (out, mass) if with_mass else out


def run_window(p: Params, phi0, x0, y0, wx, wy, nsteps):
    """phi on rows y0..y0+wy-1, columns x0..x0+wx-1 of the full periodic run."""
    phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(p.ny, p.nx)
    out = np.empty((wy, wx))
    cp = p.c()
    rc = lib().orc_run_window(C.byref(cp), _dp(phi0), int(x0), int(y0), int(wx), int(wy), int(nsteps), _dp(out))
    if rc != 0:
        raise RuntimeError("orc_run_window failed: %d" % rc)
    return out


def psi(phi, eps, delta, reading=READ_JAIN):
    return lib().orc_psi(float(phi), float(eps), float(delta), int(reading))


def sharpen(psi_v, eps, reading=READ_JAIN):
    return lib().orc_sharpen(float(psi_v), float(eps), int(reading))


def sharpen_conventional(phi, eps, reading=READ_JAIN):
    return lib().orc_sharpen_conventional(float(phi), float(eps), int(reading))


def feq(phi, u, v):
    out = np.empty(9)
    lib().orc_feq(float(phi), float(u), float(v), _dp(out))
    return out


def forcing(gx, gy):
    out = np.empty(9)
    lib().orc_forcing(float(gx), float(gy), _dp(out))
    return out


def gradient(chi):
    chi = np.ascontiguousarray(chi, dtype=np.float64)
    ny, nx = chi.shape
    gx, gy = np.empty_like(chi), np.empty_like(chi)
    lib().orc_gradient(_dp(chi), nx, ny, _dp(gx), _dp(gy))
    return gx, gy


def velocity(p: Params, X, Y, t):
    u, v = C.c_double(), C.c_double()
    cp = p.c()
    lib().orc_velocity(C.byref(cp), float(X), float(Y), float(t), C.byref(u), C.byref(v))
    return u.value, v.value


def flux(p: Params, phi):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    ny, nx = phi.shape
    fx, fy = np.empty_like(phi), np.empty_like(phi)
    cp = p.c()
    lib().orc_flux(C.byref(cp), _dp(phi), nx, ny, _dp(fx), _dp(fy))
    return fx, fy


def closure_field(p: Params, phi):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    ny, nx = phi.shape
    cx, cy = np.empty_like(phi), np.empty_like(phi)
    cp = p.c()
    lib().orc_closure_field(C.byref(cp), _dp(phi), nx, ny, _dp(cx), _dp(cy))
    return cx, cy


def mlp(weights, x):
    w = np.ascontiguousarray(weights, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty(2)
    lib().orc_mlp(_dp(w), _dp(x), _dp(out))
    return out


def lattice():
    cx = (C.c_int * 9)()
    cy = (C.c_int * 9)()
    w = np.empty(9)
    lib().orc_lattice(cx, cy, _dp(w))
    return np.array(cx[:]), np.array(cy[:]), w


def nparam():
    return lib().orc_nparam()
