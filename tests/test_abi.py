"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point the header declares, and rejects bad input before it
touches a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2203_05230_amd import lbac

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(lbac3?_\w+)\s*\(", src, flags=re.M))
    return sorted(names)


def test_header_declares_the_boundary():
    names = header_functions()
    for required in ("lbac_init", "lbac_step", "lbac_phi", "lbac_mass", "lbac_free"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = lbac.load()
    for name in header_functions():
        assert hasattr(L, name), name
    assert set(header_functions()) == set(lbac.EXPORTS) | set(lbac.EXPORTS3)


@pytest.mark.parametrize("struct,header", [("lbac_params", "lbac.h"), ("lbac3_params", "lbac3.h")])
def test_params_struct_layout_matches_header(tmp_path, struct, header):
    """The ctypes mirrors of lbac_params / lbac3_params have the offsets the C compiler gives the header."""
    cls = getattr(lbac, struct)
    fields = [name for name, _ in cls._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "%s"\nint main(void){\n' % header
                   + "".join('printf("%%zu\\n", offsetof(%s, %s));\n' % (struct, f) for f in fields)
                   + 'printf("%%zu\\n", sizeof(%s));return 0;}\n' % struct)
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [getattr(cls, f).offset for f in fields] + [C.sizeof(cls)]
    assert got == want


def _init(**kw):
    L = lbac.load()
    n = kw.pop("n", 16)
    phi0 = kw.pop("phi0", np.full((n, n), 0.5))
    p = lbac.make_params(n, n, **kw)
    h = C.c_void_p()
    rc = L.lbac_init(C.byref(p), phi0.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h))
    if rc == 0:
        L.lbac_free(h)
    return rc


@pytest.mark.parametrize("kw", [dict(tau=0.5), dict(tau=0.3), dict(eps=0.0), dict(eps=-1.0), dict(delta=-1e-3),
                                dict(vel="vortex", period_T=0.0), dict(vel="uniform", ux=0.3, uy=0.1),
                                dict(precision=7), dict(model=5), dict(tau=float("nan"))])
def test_invalid_parameters_rejected(kw):
    assert _init(**kw) == lbac.LBAC_EINVAL


def test_nonfinite_phi0_rejected():
    phi0 = np.full((16, 16), 0.5)
    phi0[3, 4] = np.nan
    assert _init(phi0=phi0) == lbac.LBAC_EINVAL
    phi0[3, 4] = np.inf
    assert _init(phi0=phi0) == lbac.LBAC_EINVAL


def test_bad_sizes_rejected():
    L = lbac.load()
    for nx, ny in ((0, 16), (16, 0), (-3, 4), (70000, 4), (65536, 4096)):
        p = lbac.make_params(16, 16)
        p.nx, p.ny = nx, ny
        h = C.c_void_p()
        phi0 = np.zeros(16)
        assert L.lbac_init(C.byref(p), phi0.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h)) == lbac.LBAC_EINVAL


def test_batch_rejects_instances_beyond_its_addressing():
    """The batch kernel reaches the nine planes of an instance through one
    buffer resource with offsets below 2^31 bytes: a larger instance is
    refused before anything is allocated."""
    L = lbac.load()
    ps = (lbac.lbac_params * 2)(lbac.make_params(128, 128, precision="f32"),
                                lbac.make_params(7800, 7800, precision="f32"))
    phi0 = np.zeros(16)
    ptr = phi0.ctypes.data_as(C.POINTER(C.c_double))
    ptrs = (C.POINTER(C.c_double) * 2)(ptr, ptr)
    h = C.c_void_p()
    assert L.lbac_batch_init(ps, ptrs, 2, C.byref(h)) == lbac.LBAC_EINVAL
    assert not h.value


@pytest.mark.parametrize("precs", [("f64", "f64"), ("f32", "f32_f16store"), ("f32_bf16store", "f32_f16store")])
def test_batch_rejects_fp64_and_mixed_precisions(precs):
    """Every instance of a batch has one precision, FP32 or shifted 16-bit
    storage (one kernel serves the launch); refused before anything is
    allocated."""
    L = lbac.load()
    ps = (lbac.lbac_params * 2)(*[lbac.make_params(64, 64, precision=p) for p in precs])
    phi0 = np.zeros(16)
    ptr = phi0.ctypes.data_as(C.POINTER(C.c_double))
    h = C.c_void_p()
    assert L.lbac_batch_init(ps, (C.POINTER(C.c_double) * 2)(ptr, ptr), 2, C.byref(h)) == lbac.LBAC_EINVAL
    assert not h.value


def test_batch_queries_reject_null_handles():
    L = lbac.load()
    out = np.zeros(4)
    assert L.lbac_batch_phi(None, 0, out.ctypes.data_as(C.POINTER(C.c_double))) == lbac.LBAC_EINVAL
    assert L.lbac_batch_mass(None, out.ctypes.data_as(C.POINTER(C.c_double))) == lbac.LBAC_EINVAL


def test_null_arguments_rejected():
    L = lbac.load()
    p = lbac.make_params(16, 16)
    h = C.c_void_p()
    assert L.lbac_init(C.byref(p), None, C.byref(h)) == lbac.LBAC_EINVAL
    assert L.lbac_step(None, 1) == lbac.LBAC_EINVAL
    assert L.lbac_mass(None, None) == lbac.LBAC_EINVAL
    assert L.lbac_free(None) == lbac.LBAC_OK


def test_status_strings():
    L = lbac.load()
    for code in (0, -1, -2, -3, -4, -5):
        assert L.lbac_strerror(code)
    assert L.lbac_strerror(0) == b"ok"


@pytest.mark.parametrize("kw", [dict(tau=0.5), dict(eps=0.0), dict(delta=-1.0), dict(vel=9), dict(precision=2),
                                dict(vel="deformation", period_T=0.0), dict(vel="uniform", ux=0.2, uy=0.1, uz=0.1),
                                dict(vel="deformation", U=0.2)])
def test_3d_invalid_parameters_rejected(kw):
    L = lbac.load()
    p = lbac.make_params3(8, 8, 8, **kw)
    h = C.c_void_p()
    phi0 = np.full(512, 0.5)
    assert L.lbac3_init(C.byref(p), phi0.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h)) == lbac.LBAC_EINVAL
    assert L.lbac3_last_error(None)


def test_3d_bad_sizes_and_nulls_rejected():
    L = lbac.load()
    h = C.c_void_p()
    phi0 = np.zeros(8)
    for dims in ((0, 4, 4), (4, 4, 0), (5000, 2, 2), (1024, 1024, 256)):
        p = lbac.make_params3(2, 2, 2)
        p.nx, p.ny, p.nz = dims
        assert L.lbac3_init(C.byref(p), phi0.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h)) == lbac.LBAC_EINVAL
    assert L.lbac3_init(None, None, C.byref(h)) == lbac.LBAC_EINVAL
    assert L.lbac3_step(None, 1) == lbac.LBAC_EINVAL
    assert L.lbac3_free(None) == lbac.LBAC_EINVAL
