"""Pins of the FP64 D3Q19 oracle (the 3-D form of the scheme).

The strongest pin ties it to the already pinned 2-D oracle: for data that do
not vary along one axis and a velocity without a component along it, the
D3Q19 lattice summed over that axis is exactly the D2Q9 lattice (weights
1/3 + 2/18 = 4/9, 1/18 + 2/36 = 1/9, 1/36), and its isotropic gradient is the
D2Q9 one, so every plane must reproduce the 2-D scheme.  The others compare
with textbook lattice moments, closed forms of Eq. (10)-(11), polynomial
exactness of the gradient, conservation and limit cases.  The last tests
plant each known mistake in the oracle and check that a pin fails.
"""
import numpy as np
import pytest

from oracle import lib as O
from oracle import lib3 as O3
from paper_2203_05230_amd import workloads as W


def _extrude(phi2, n, axis):
    """A 2-D field (rows = second axis, cols = first axis of the plane) made
    invariant along `axis` of an (nz, ny, nx) array."""
    if axis == 2:  # invariant along z: phi2 is (ny, nx)
        return np.repeat(phi2[None, :, :], n, axis=0)
    if axis == 0:  # invariant along x: phi2 is (nz, ny) = plane (y -> x2d, z -> y2d)
        return np.repeat(phi2[:, :, None], n, axis=2)
    return np.repeat(phi2[:, None, :], n, axis=1)  # invariant along y: phi2 is (nz, nx)


def pin_reduce_z(mutation=0, steps=150):
    """z-invariant data in the vortex field of the x-y plane: every z plane
    equals the 2-D scheme (to rounding)."""
    nx, ny = 40, 32
    phi2 = W.circle(nx, 1.0, ny=ny)
    ref = O.run(O.Params(nx, ny, eps=1.0, tau=0.8, vel_kind=O.VEL_VORTEX, U=0.04, period_T=300.0), phi2, steps)
    p = O3.Params3(nx, ny, 3, eps=1.0, tau=0.8, vel_kind=O3.VEL3_VORTEX_XY, U=0.04, period_T=300.0, mutation=mutation)
    a = O3.run(p, _extrude(phi2, 3, 2), steps)
    err = max(np.max(np.abs(a[k] - ref)) for k in range(3))
    return bool(err < 1e-12), err


def pin_reduce_x(mutation=0, steps=150):
    """x-invariant data under uniform flow (0, a, b): every x line carries the
    2-D scheme of the (y, z) plane with flow (a, b)."""
    ny, nz = 36, 28
    phi2 = W.circle(ny, 1.2, ny=nz, R_frac=0.25, yc_frac=0.45)  # (nz, ny)
    ref = O.run(O.Params(ny, nz, eps=1.2, tau=0.7, vel_kind=O.VEL_UNIFORM, ux=0.03, uy=-0.05), phi2, steps)
    p = O3.Params3(3, ny, nz, eps=1.2, tau=0.7, vel_kind=O3.VEL3_UNIFORM, ux=0.0, uy=0.03, uz=-0.05,
                   mutation=mutation)
    a = O3.run(p, _extrude(phi2, 3, 0), steps)
    err = max(np.max(np.abs(a[:, :, k] - ref)) for k in range(3))
    return bool(err < 1e-12), err


def pin_reduce_y(mutation=0, steps=150):
    """y-invariant data under uniform flow (a, 0, b): the (x, z) plane."""
    nx, nz = 30, 34
    phi2 = W.circle(nx, 0.8, ny=nz, R_frac=0.3, xc_frac=0.55, yc_frac=0.5)  # (nz, nx)
    ref = O.run(O.Params(nx, nz, eps=0.8, tau=0.9, vel_kind=O.VEL_UNIFORM, ux=-0.04, uy=0.02), phi2, steps)
    p = O3.Params3(nx, 3, nz, eps=0.8, tau=0.9, vel_kind=O3.VEL3_UNIFORM, ux=-0.04, uy=0.0, uz=0.02,
                   mutation=mutation)
    a = O3.run(p, _extrude(phi2, 3, 1), steps)
    err = max(np.max(np.abs(a[:, k, :] - ref)) for k in range(3))
    return bool(err < 1e-12), err


def pin_mass(mutation=0, steps=200):
    """Eq. (9)-(12) conserve sum phi exactly; with the deformation field too."""
    c = W.deformation_case(24, eps=1.0, U=0.03)
    p = O3.Params3(24, 24, 24, eps=1.0, tau=0.8, vel_kind=O3.VEL3_DEFORMATION, U=0.03, period_T=c["period_T"],
                   mutation=mutation)
    _, m = O3.run(p, W.sphere(24, 1.0, R_frac=0.25, centre_frac=(0.5, 0.5, 0.5)), steps, with_mass=True)
    drift = np.max(np.abs(m - m[0])) / m[0]
    return bool(np.isfinite(drift) and drift < 4 * steps * 2.0**-52), drift


def pin_translation(mutation=0):
    """Uniform diagonal flow: after one transit along every axis the ball is
    back; a quarter transit moves its centroid by a quarter period."""
    n, U = 24, 0.04
    phi0 = W.sphere(n, 1.0, R_frac=0.25, centre_frac=(0.5, 0.5, 0.5))
    p = O3.Params3(n, n, n, eps=1.0, tau=0.8, vel_kind=O3.VEL3_UNIFORM, ux=U, uy=U, uz=U, mutation=mutation)
    q = O3.run(p, phi0, int(0.25 * n / U))
    full = O3.run(p, phi0, int(n / U))

    def centroid(phi, axis):
        ang = 2 * np.pi * (np.arange(n) + 0.5) / n
        prof = phi.sum(axis=tuple(a for a in range(3) if a != axis))
        return (np.angle(np.sum(prof * np.exp(1j * ang))) % (2 * np.pi)) * n / (2 * np.pi)

    shifts = [(centroid(q, ax) - centroid(phi0, ax)) % n for ax in range(3)]
    e_full = np.linalg.norm(full - phi0) / np.linalg.norm(phi0)
    ok = all(abs(s - 0.25 * n) < 0.05 for s in shifts) and e_full < 0.05
    return bool(ok), (shifts, e_full)


def pin_stationary(mutation=0):
    """Without flow a ball of the equilibrium profile (Eq. (2)) settles within
    a few hundred steps to a nearby discrete equilibrium and then stays: the
    change from 200 to 600 steps is small, and so is the total."""
    n, eps = 24, 1.0
    phi0 = W.sphere(n, eps, R_frac=0.3, centre_frac=(0.5, 0.5, 0.5))
    p = O3.Params3(n, n, n, eps=eps, tau=0.8, vel_kind=O3.VEL3_ZERO, mutation=mutation)
    a = O3.run(p, phi0, 200)
    b = O3.run(p, phi0, 600)
    d200 = np.linalg.norm(a - phi0) / np.linalg.norm(phi0)
    d600 = np.linalg.norm(b - phi0) / np.linalg.norm(phi0)
    return bool(d600 < 0.02 and d600 - d200 < 0.005), (d200, d600)


ALL_PINS = [pin_reduce_z, pin_reduce_x, pin_reduce_y, pin_mass, pin_translation, pin_stationary]


def test_lattice_moments_are_textbook_d3q19():
    cx, cy, cz, w = O3.lattice()
    c = np.stack([cx, cy, cz], 1).astype(float)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(w @ c, 0.0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), np.eye(3) / 3.0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", w, c, c, c), 0.0, atol=1e-16)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), iso, atol=1e-16)
    # every velocity has its opposite, and the set is the 19 of length^2 <= 2
    vel = {tuple(v) for v in c.astype(int)}
    assert len(vel) == 19 and all(tuple(-np.array(v)) in vel for v in vel)
    assert all(sum(x * x for x in v) <= 2 for v in vel)


def test_equilibrium_and_forcing_moments():
    cx, cy, cz, _ = O3.lattice()
    c = np.stack([cx, cy, cz], 1).astype(float)
    rng = np.random.default_rng(3)
    for _ in range(5):
        phi, u, v, w, gx, gy, gz = rng.uniform(-1, 1, 7)
        fe = O3.feq(phi, u, v, w)
        assert fe.sum() == pytest.approx(phi, abs=1e-15)
        assert np.allclose(c.T @ fe, phi * np.array([u, v, w]), atol=1e-15)
        assert np.allclose(np.einsum("i,ia,ib->ab", fe, c, c), phi / 3.0 * np.eye(3), atol=1e-15)
        F = O3.forcing(gx, gy, gz)
        assert abs(F.sum()) < 1e-15
        assert np.allclose(c.T @ F, [gx, gy, gz], atol=1e-15)


def test_gradient_exact_on_quadratics_second_order_on_sines():
    n = 12
    Z, Y, X = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5, np.arange(n) + 0.5, indexing="ij")
    chi = 0.7 * X - 1.3 * Y + 0.4 * Z + 0.05 * X * X + 0.02 * X * Y - 0.03 * Y * Z + 0.04 * Z * Z
    gx, gy, gz = O3.gradient(chi)
    inner = (slice(1, -1),) * 3
    assert np.allclose(gx[inner], (0.7 + 0.1 * X + 0.02 * Y)[inner], atol=1e-12)
    assert np.allclose(gy[inner], (-1.3 + 0.02 * X - 0.03 * Z)[inner], atol=1e-12)
    assert np.allclose(gz[inner], (0.4 - 0.03 * Y + 0.08 * Z)[inner], atol=1e-12)
    errs = []
    for n in (24, 48):
        Z, Y, X = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5, np.arange(n) + 0.5, indexing="ij")
        k = 2 * np.pi / n
        gx, gy, gz = O3.gradient(np.sin(k * X) * np.cos(k * Y) * np.sin(k * Z))
        errs.append(np.max(np.abs(gz - k * np.sin(k * X) * np.cos(k * Y) * np.cos(k * Z))) / k)
    assert 3.8 < errs[0] / errs[1] < 4.2


def test_deformation_field_is_divergence_free_and_reverses():
    n = 32
    p = O3.Params3(n, n, n, vel_kind=O3.VEL3_DEFORMATION, U=0.02, period_T=1000.0)
    h = 1e-4
    for X, Y, Z in ((5.5, 20.5, 11.5), (17.5, 3.5, 29.5), (30.5, 30.5, 7.5)):
        d = (O3.velocity(p, X + h, Y, Z, 0)[0] - O3.velocity(p, X - h, Y, Z, 0)[0] +
             O3.velocity(p, X, Y + h, Z, 0)[1] - O3.velocity(p, X, Y - h, Z, 0)[1] +
             O3.velocity(p, X, Y, Z + h, 0)[2] - O3.velocity(p, X, Y, Z - h, 0)[2]) / (2 * h)
        assert abs(d) < 1e-9
        u0 = np.array(O3.velocity(p, X, Y, Z, 0.0))
        u1 = np.array(O3.velocity(p, X, Y, Z, 1000.0))
        assert np.allclose(u1, -u0, atol=1e-15)
        assert np.max(np.abs(u0)) <= 2 * 0.02 + 1e-15


def test_deformation_run_returns():
    """The ball is stretched by the deformation field (its relative L2
    distance from phi0 reaches ~0.7 at t = T/2) and comes back at t = T to
    within the discretisation error of a 32^3 grid."""
    T = 800.0
    phi0 = W.sphere(32, 1.0, R_frac=0.2, centre_frac=(0.35, 0.35, 0.35))
    p = O3.Params3(32, 32, 32, eps=1.0, tau=0.8, vel_kind=O3.VEL3_DEFORMATION, U=0.02, period_T=T)
    half = O3.run(p, phi0, int(T / 2))
    full = O3.run(p, phi0, int(T))
    e_half = np.linalg.norm(half - phi0) / np.linalg.norm(phi0)
    e_full = np.linalg.norm(full - phi0) / np.linalg.norm(phi0)
    assert e_half > 0.5 and e_full < 0.2 * e_half


@pytest.mark.parametrize("pin", ALL_PINS, ids=[f.__name__ for f in ALL_PINS])
def test_unmutated_oracle_passes(pin):
    ok, detail = pin()
    assert ok, detail


@pytest.mark.parametrize("name", sorted(O3.MUTATIONS))
def test_planted_mistake_is_caught(name):
    mut = O3.MUTATIONS[name]
    for pin in ALL_PINS:
        ok, _ = pin(mutation=mut)
        if not ok:
            return
    pytest.fail("mistake %s passed every pin" % name)
