"""ctypes wrapper over the FP64 D3Q19 oracle (test infrastructure only).

Every function forwards to ``lbm_oracle3.c``; see that file for the
equations each one follows.  Arrays are numpy float64, shape (nz, ny, nx),
x fastest.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

VEL3_ZERO, VEL3_DEFORMATION, VEL3_VORTEX_XY, VEL3_UNIFORM = range(4)
# planted mistakes for pin-sensitivity tests (see the MUT3_* list in lbm_oracle3.c)
MUTATIONS = {"edge_weight": 1, "grad_zx": 2, "stream_back": 3, "drop_gz": 4}


class Orc3Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("eps", C.c_double), ("tau", C.c_double), ("delta", C.c_double),
        ("vel_kind", C.c_int32),
        ("U", C.c_double), ("period_T", C.c_double),
        ("ux", C.c_double), ("uy", C.c_double), ("uz", C.c_double),
        ("mutation", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB3
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC3):
            _build.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.orc3_run.argtypes = [C.POINTER(Orc3Params), dp, C.c_long, dp, dp]
        L.orc3_lattice.argtypes = [ip, ip, ip, dp]
        L.orc3_velocity.argtypes = [C.POINTER(Orc3Params), C.c_double, C.c_double, C.c_double, C.c_double, dp, dp,
                                    dp]
        L.orc3_feq.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, dp]
        L.orc3_forcing.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        L.orc3_gradient.argtypes = [dp, C.c_int, C.c_int, C.c_int, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Params3:
    def __init__(self, nx, ny, nz, eps=1.0, tau=0.8, delta=1e-10, vel_kind=VEL3_DEFORMATION, U=0.02,
                 period_T=400.0, ux=0.0, uy=0.0, uz=0.0, mutation=0):
        self.nx, self.ny, self.nz = nx, ny, nz
        self.eps, self.tau, self.delta = eps, tau, delta
        self.vel_kind, self.U, self.period_T = vel_kind, U, period_T
        self.ux, self.uy, self.uz = ux, uy, uz
        self.mutation = mutation

    def c(self):
        return Orc3Params(self.nx, self.ny, self.nz, self.eps, self.tau, self.delta, self.vel_kind, self.U,
                          self.period_T, self.ux, self.uy, self.uz, self.mutation)


def lattice():
    cx, cy, cz = (C.c_int * 19)(), (C.c_int * 19)(), (C.c_int * 19)()
    w = np.zeros(19)
    lib().orc3_lattice(cx, cy, cz, _dp(w))
    return np.array(cx[:]), np.array(cy[:]), np.array(cz[:]), w


def run(p, phi0, nsteps, with_mass=False):
    phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(p.nz, p.ny, p.nx)
    out = np.empty_like(phi0)
    mass = np.empty(nsteps + 1) if with_mass else None
    rc = lib().orc3_run(C.byref(p.c()), _dp(phi0), int(nsteps), _dp(out), _dp(mass) if with_mass else None)
    if rc != 0:
        raise RuntimeError("orc3_run failed: %d" % rc)
    return (out, mass) if with_mass else out


def velocity(p, X, Y, Z, t):
    u, v, w = C.c_double(), C.c_double(), C.c_double()
    lib().orc3_velocity(C.byref(p.c()), float(X), float(Y), float(Z), float(t), C.byref(u), C.byref(v), C.byref(w))
    return u.value, v.value, w.value


def feq(phi, u, v, w):
    out = np.zeros(19)
    lib().orc3_feq(float(phi), float(u), float(v), float(w), _dp(out))
    return out


def forcing(gx, gy, gz):
    out = np.zeros(19)
    lib().orc3_forcing(float(gx), float(gy), float(gz), _dp(out))
    return out


def gradient(chi):
    chi = np.ascontiguousarray(chi, dtype=np.float64)
    nz, ny, nx = chi.shape
    gx, gy, gz = np.empty_like(chi), np.empty_like(chi), np.empty_like(chi)
    lib().orc3_gradient(_dp(chi), nx, ny, nz, _dp(gx), _dp(gy), _dp(gz))
    return gx, gy, gz
