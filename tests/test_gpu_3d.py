"""The D3Q19 form on the GPU (include/lbac3.h) against the FP64 D3Q19 oracle,
and against the 2-D form for data that do not vary along z."""
import sys

import numpy as np
import pytest

from oracle import lib3 as O3
from paper_2203_05230_amd import workloads as W

pytestmark = pytest.mark.gpu

VEL3_O = {"zero": O3.VEL3_ZERO, "deformation": O3.VEL3_DEFORMATION, "vortex_xy": O3.VEL3_VORTEX_XY,
          "uniform": O3.VEL3_UNIFORM}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oparams(c):
    return O3.Params3(c["nx"], c["ny"], c["nz"], eps=c["eps"], tau=c["tau"], delta=c["delta"],
                      vel_kind=VEL3_O[c["vel"]], U=c.get("U", 0.0), period_T=c.get("period_T", 1.0),
                      ux=c.get("ux", 0.0), uy=c.get("uy", 0.0), uz=c.get("uz", 0.0))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def assert_fp64(phi, ref, steps, eps, delta):
    """As for the 2-D form: 1e-12 on the resolved nodes (|phi| > 1e-8); where
    phi is at the level of delta the normal of Eq. (13) is set by rounding and
    the change is bounded by steps * delta / eps."""
    m = np.abs(ref) > 1e-8
    assert rel_l2(phi[m], ref[m]) <= 1e-12
    assert np.max(np.abs(phi - ref)) <= steps * delta / eps


def gpu(lb, case, phi0, steps, precision, launch=None):
    sim = lb.Simulation3({**case, "precision": precision}, phi0)
    if launch:
        sim.set_launch(*launch)
    sim.step(steps)
    return sim


def deformation(n, eps=1.0, U=0.02, T=800.0):
    return dict(nx=n, ny=n, nz=n, eps=eps, tau=0.8, delta=1e-10, vel="deformation", U=U, period_T=T)


def test_fp64_deformation_parity(gpu_lib):
    say("case: 3-D FP64 deformation 32^3, 150 steps")
    c = deformation(32)
    phi0 = W.sphere(32, 1.0, R_frac=0.2)
    ref, mass = O3.run(oparams(c), phi0, 150, with_mass=True)
    sim = gpu(gpu_lib, c, phi0, 150, "f64")
    assert_fp64(sim.phi(), ref, 150, 1.0, 1e-10)
    assert abs(sim.mass() - mass[0]) / mass[0] <= 1e-12
    e1, e2 = sim.shape_error(phi0)
    assert e2 == pytest.approx(rel_l2(ref, phi0), rel=1e-9)
    assert sim.time() == 150


@pytest.mark.parametrize("dims", [(20, 28, 36), (5, 3, 7), (1, 1, 16), (33, 1, 17)])
def test_fp64_ragged_grids_and_strips(gpu_lib, dims):
    say("case: 3-D FP64 ragged grid", dims)
    nx, ny, nz = dims
    c = dict(nx=nx, ny=ny, nz=nz, eps=1.2, tau=0.7, delta=1e-10, vel="uniform", ux=0.03, uy=-0.02, uz=0.04)
    rng = np.random.default_rng(nx * 10000 + ny * 100 + nz)
    phi0 = 0.9 * W.sphere(max(dims), 1.5, R_frac=0.3, centre_frac=(0.5, 0.5, 0.5))[:nz, :ny, :nx] \
        + 0.05 * rng.random((nz, ny, nx))
    ref = O3.run(oparams(c), phi0, 40)
    base = None
    for launch in ((32, 16, 0, 1), (32, 8, 1, 5, 1), (64, 4, 1, 32), (32, 8, 0, 3, 1), (128, 4, 2, 2), (64, 8, 2, 36),
                   (32, 16, 2, 3, 1)):
        phi = gpu(gpu_lib, c, phi0, 40, "f64", launch=launch).phi()
        assert_fp64(phi, ref, 40, 1.2, 1e-10)
        if base is None:
            base = phi
        assert np.array_equal(phi, base), launch


def test_fp32_parity_after_300_steps(gpu_lib):
    say("case: 3-D FP32 deformation 48^3, 300 steps")
    c = deformation(48, U=0.02, T=1200.0)
    phi0 = W.sphere(48, 1.0, R_frac=0.2)
    ref = O3.run(oparams(c), phi0, 300)
    sim = gpu(gpu_lib, c, phi0, 300, "f32")
    err = rel_l2(sim.phi(), ref)
    say("  FP32 rel L2 %.3e" % err)
    assert err <= 1e-5
    m0 = phi0.sum()
    assert abs(sim.mass() - m0) / m0 <= 1e-6


def test_z_invariant_data_match_the_2d_form(gpu_lib):
    """D3Q19 summed over z is D2Q9: every z plane of the 3-D form equals the
    2-D form's FP64 result (to rounding)."""
    say("case: z-invariant 3-D vs 2-D")
    nx, ny, nz = 48, 40, 4
    phi2 = W.circle(nx, 1.0, ny=ny)
    c2 = dict(nx=nx, ny=ny, eps=1.0, tau=0.8, delta=1e-10, vel="vortex", U=0.04, period_T=400.0)
    s2 = gpu_lib.Simulation({**c2, "precision": "f64"}, phi2)
    s2.step(200)
    ref = s2.phi()
    c3 = dict(nx=nx, ny=ny, nz=nz, eps=1.0, tau=0.8, delta=1e-10, vel="vortex_xy", U=0.04, period_T=400.0)
    phi3 = gpu(gpu_lib, c3, np.repeat(phi2[None], nz, axis=0), 200, "f64").phi()
    for k in range(nz):
        m = np.abs(ref) > 1e-8
        assert rel_l2(phi3[k][m], ref[m]) <= 1e-12
        assert np.max(np.abs(phi3[k] - ref)) <= 200 * 1e-10


SHAPES = {
    # (tile_x, tile_y, variant, strip_z, z_major); odd strips march down
    "f64": ((32, 16, 0, 32, 0), (32, 8, 0, 7, 1), (64, 4, 1, 4, 0), (64, 8, 1, 40, 0), (128, 4, 2, 16, 1),
            (32, 8, 2, 5, 0), (32, 16, 1, 3, 1)),
    "f32": ((32, 16, 0, 32, 0), (32, 8, 0, 7, 1), (64, 4, 1, 4, 0), (64, 8, 1, 40, 0), (128, 4, 2, 16, 1),
            (32, 8, 2, 5, 0), (32, 32, 0, 14, 1), (32, 32, 1, 9, 0), (64, 16, 2, 20, 1), (128, 8, 1, 40, 1),
            (128, 8, 0, 6, 0)),
}


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_launch_shapes_bitwise(gpu_lib, prec):
    say("case: 3-D launch shapes", prec)
    c = deformation(40)
    phi0 = W.sphere(40, 1.0, R_frac=0.2)
    base = None
    for launch in SHAPES[prec]:
        phi = gpu(gpu_lib, c, phi0, 12, prec, launch=launch).phi()
        if base is None:
            base = phi
        assert np.array_equal(phi, base), launch


def test_fp32_tall_tiles_match_oracle(gpu_lib):
    """1024-thread tiles (FP32 only) on a grid that leaves ragged tiles in x
    and y and strips marching both ways."""
    say("case: 3-D FP32 1024-column tiles, 45x70x33")
    c = dict(nx=45, ny=70, nz=33, eps=1.0, tau=0.8, delta=1e-10, vel="deformation", U=0.02, period_T=800.0)
    phi0 = W.sphere(70, 1.0, R_frac=0.25)[:33, :70, :45]
    ref = O3.run(oparams(c), phi0, 60)
    for launch in ((32, 32, 1, 5, 1), (64, 16, 2, 11, 0), (128, 8, 0, 7, 1)):
        err = rel_l2(gpu(gpu_lib, c, phi0, 60, "f32", launch=launch).phi(), ref)
        say("  launch", launch, "FP32 rel L2 %.3e" % err)
        assert err <= 1e-5


def test_launch_shape_errors(gpu_lib):
    c = deformation(16)
    phi0 = W.sphere(16, 1.0, R_frac=0.2)
    s64 = gpu_lib.Simulation3({**c, "precision": "f64"}, phi0)
    for bad in ((32, 32, 0, 8), (128, 8, 0, 8), (64, 16, 0, 8),  # 1024-thread tiles need FP32
                (32, 16, 3, 8), (32, 16, 0, 8, 2), (32, 12, 0, 8), (48, 8, 0, 8), (32, 16, 0, 0)):
        with pytest.raises(gpu_lib.LbacError):
            s64.set_launch(*bad)
    s64.set_launch(64, 8, 2, 5, 1)
    assert s64.get_launch() == (64, 8, 2, 5, 1)
    s64.close()


def test_autotune_keeps_state(gpu_lib):
    say("case: 3-D autotune")
    c = deformation(40)
    phi0 = W.sphere(40, 1.0, R_frac=0.2)
    a = gpu_lib.Simulation3({**c, "precision": "f32"}, phi0)
    b = gpu_lib.Simulation3({**c, "precision": "f32"}, phi0)
    a.step(3)
    b.step(3)
    assert a.autotune(3) > 0
    a.step(4)
    b.step(4)
    assert np.array_equal(a.phi(), b.phi())
    assert a.bytes_per_node() == 152.0
