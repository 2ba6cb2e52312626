"""Seeded synthetic inputs: initial order-parameter fields and run parameters.

This module holds no arithmetic of the scheme itself: it only draws problem
set-ups (shapes, sizes, widths, relaxation times) and writes the initial
phi field as a smoothed indicator of a shape, so that the library and the
CPU oracle can be fed identical inputs.  Every generator is deterministic in
its arguments (numpy PCG64 for the random ones).

Node (i, j) sits at the cell centre X = i + 1/2, Y = j + 1/2.
"""
import numpy as np


def _centres(nx, ny):
    X = np.arange(nx, dtype=np.float64) + 0.5
    Y = np.arange(ny, dtype=np.float64) + 0.5
    return np.meshgrid(X, Y)  # arrays of shape (ny, nx)


def smoothed_indicator(d, eps):
    """phi = (1 + tanh(d / (2 eps))) / 2 for a signed distance d (positive inside)."""
    return 0.5 * (1.0 + np.tanh(d / (2.0 * eps)))


def circle_distance(nx, ny, xc, yc, R):
    X, Y = _centres(nx, ny)
    return R - np.hypot(X - xc, Y - yc)


def circle(n, eps, R_frac=0.15, xc_frac=0.5, yc_frac=0.75, ny=None):
    """Disk of radius R_frac*n centred at (xc_frac*n, yc_frac*n) on an n-by-ny grid."""
    ny = n if ny is None else ny
    d = circle_distance(n, ny, xc_frac * n, yc_frac * ny, R_frac * n)
    return smoothed_indicator(d, eps)


def slotted_disk_distance(n, R_frac=0.15, xc_frac=0.5, yc_frac=0.75, slot_w_frac=0.05, slot_l_frac=0.25,
                          angle=0.0):
    """Signed distance (positive inside) of Zalesak's slotted disk.  The slot is
    slot_w_frac*n wide and slot_l_frac*n long, cut from the disk edge that faces
    the grid centre; angle rotates the slot about the disk centre."""
    X, Y = _centres(n, n)
    xc, yc, R = xc_frac * n, yc_frac * n, R_frac * n
    d_disk = R - np.hypot(X - xc, Y - yc)
    # slot frame: local axis s points from the disk centre towards the cut edge
    # (straight down for angle = 0), t across the slot
    ca, sa = np.cos(angle), np.sin(angle)
    lx, ly = X - xc, Y - yc
    s = -(lx * sa - ly * ca)  # component along (sin a, -cos a)
    t = lx * ca + ly * sa
    # box covering the slot, open past the disk edge
    s_lo, s_hi = R - slot_l_frac * n, 2.0 * R
    half_w = 0.5 * slot_w_frac * n
    qs = np.abs(s - 0.5 * (s_lo + s_hi)) - 0.5 * (s_hi - s_lo)
    qt = np.abs(t) - half_w
    outside = np.hypot(np.maximum(qs, 0.0), np.maximum(qt, 0.0)) + np.minimum(np.maximum(qs, qt), 0.0)
    return np.minimum(d_disk, outside)


def slotted_disk(n, eps, **kw):
    return smoothed_indicator(slotted_disk_distance(n, **kw), eps)


def slab(nx, ny, eps, width_frac=0.5, axis=0, centre_frac=0.5):
    """Planar band of the given width; axis=0 varies along x, axis=1 along y."""
    X, Y = _centres(nx, ny)
    if axis == 0:
        d = 0.5 * width_frac * nx - np.abs(X - centre_frac * nx)
    else:
        d = 0.5 * width_frac * ny - np.abs(Y - centre_frac * ny)
    return smoothed_indicator(d, eps)


def uniform_random(nx, ny, seed, lo=0.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, size=(ny, nx))


# ---------------------------------------------------------------------------
# run descriptions (plain dicts; keys mirror the library parameter struct)

def single_vortex_case(n, eps=1.0, tau=0.8, U=0.02, period_T=2000.0, delta=1e-10):
    """Single vortex: disk R = 0.15 n at (0.5 n, 0.75 n)."""
    return dict(nx=n, ny=n, eps=eps, tau=tau, delta=delta, vel="vortex", U=U, period_T=float(period_T))


def paper_vortex_case(eps_paper, L=200):
    """The paper's own single-vortex test (Sec. 3, Eq. (14)): an L x L grid
    (L = 200), disk R = 0.2 L at (0.5 L, 0.75 L), U0 = 0.04, mobility
    M = 0.001 (tau = 3 M + 1/2 = 0.503), period T = 6 L / U0 = 30 000 steps,
    the printed velocity signs and regulariser e^-20.  eps_paper is the
    paper's interface width (3 and 1.5 in its figures); the library's width
    convention has eps = eps_paper / 4."""
    U0, M = 0.04, 0.001
    T = 6.0 * L / U0
    return dict(nx=L, ny=L, eps=eps_paper / 4.0, tau=3.0 * M + 0.5, delta=float(np.exp(-20.0)), vel="vortex_paper",
                U=U0, period_T=T, steps=int(round(T)), phi0=("circle", dict(R_frac=0.2)))


def zalesak_case(n, eps=1.0, tau=0.8, delta=1e-10, rev_steps=None):
    """Slotted disk under solid-body rotation about the grid centre, one
    revolution in rev_steps (default 64 n) steps."""
    rev = float(64 * n if rev_steps is None else rev_steps)
    return dict(nx=n, ny=n, eps=eps, tau=tau, delta=delta, vel="rotation", omega=2.0 * np.pi / rev,
                cx=0.5 * n, cy=0.5 * n, steps=int(round(rev)))


BATCH_SIDES = (128, 192, 256, 384, 512)
BATCH_EPS = (0.5, 1.0, 2.0)


def batch_cases(count=256, seed=0, sides=BATCH_SIDES, eps_set=BATCH_EPS, tau_lo=0.6, tau_hi=1.0,
                vortex_steps_per_side=8, rev_steps_per_side=64):
    """Seeded list of independent instances: sides uniform from `sides`, eps
    from `eps_set`, tau uniform in [tau_lo, tau_hi]; the first half are
    single-vortex runs (period and length 8 n steps), the second half
    slotted disks under one revolution (64 n steps)."""
    rng = np.random.default_rng(seed)
    n = rng.choice(np.asarray(sides), size=count)
    eps = rng.choice(np.asarray(eps_set, dtype=np.float64), size=count)
    tau = rng.uniform(tau_lo, tau_hi, size=count)
    out = []
    for k in range(count):
        nk = int(n[k])
        if k < count // 2:
            T = vortex_steps_per_side * nk
            c = single_vortex_case(nk, eps=float(eps[k]), tau=float(tau[k]), period_T=float(T))
            c["steps"] = T
            c["phi0"] = ("circle", {})
        else:
            c = zalesak_case(nk, eps=float(eps[k]), tau=float(tau[k]), rev_steps=rev_steps_per_side * nk)
            c["phi0"] = ("slotted_disk", {})
        out.append(c)
    return out


def initial_field(case):
    """phi0 for a run description produced above."""
    kind, kw = case.get("phi0", ("circle", {}))
    if kind == "circle":
        return circle(case["nx"], case["eps"], **kw)
    if kind == "slotted_disk":
        return slotted_disk(case["nx"], case["eps"], **kw)
    raise ValueError(kind)


def closure_training_cases(count=64, seed=1, n=512, eps=2.0, tau=1.7):
    """Seeded vortex / slotted-disk set-ups for generating closure training
    data: centre jitter of +-0.05 n, radius in [0.12 n, 0.18 n], random slot
    orientation; first half vortex, second half slotted disk."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        jx, jy = rng.uniform(-0.05, 0.05, size=2)
        r = rng.uniform(0.12, 0.18)
        ang = rng.uniform(0.0, 2.0 * np.pi)
        geom = dict(R_frac=r, xc_frac=0.5 + jx, yc_frac=0.75 + jy)
        if k < count // 2:
            c = single_vortex_case(n, eps=eps, tau=tau, period_T=8.0 * n)
            c["steps"] = 8 * n
            c["phi0"] = ("circle", geom)
        else:
            c = zalesak_case(n, eps=eps, tau=tau)
            geom["angle"] = ang
            c["phi0"] = ("slotted_disk", geom)
        out.append(c)
    return out


# ---- three dimensions (D3Q19 form) -------------------------------------------

def sphere(nx, eps, R_frac=0.15, centre_frac=(0.35, 0.35, 0.35), ny=None, nz=None):
    """Ball of radius R_frac*nx at centre_frac*(nx, ny, nz) on an nz-by-ny-by-nx
    grid (cell centres), with the tanh profile of width eps; array (nz, ny, nx)."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    X = np.arange(nx, dtype=np.float64) + 0.5
    Y = np.arange(ny, dtype=np.float64) + 0.5
    Z = np.arange(nz, dtype=np.float64) + 0.5
    r = np.sqrt((Z[:, None, None] - centre_frac[2] * nz) ** 2 + (Y[None, :, None] - centre_frac[1] * ny) ** 2 +
                (X[None, None, :] - centre_frac[0] * nx) ** 2)
    return smoothed_indicator(R_frac * nx - r, eps)


def deformation_case(n, eps=1.0, tau=0.8, U=0.02, period_T=None, delta=1e-10):
    """Sphere (R = 0.15 n at 0.35 n in each direction) in the three-dimensional
    deformation field, amplitude U (|u| <= 2 U), reversed at t = T / 2 and back
    at t = T; by default T = 3 n / U steps (three domain lengths at speed U,
    the field's classic period)."""
    T = float(3.0 * n / U) if period_T is None else float(period_T)
    return dict(nx=n, ny=n, nz=n, eps=eps, tau=tau, delta=delta, vel="deformation", U=U, period_T=T,
                steps=int(round(T)))
