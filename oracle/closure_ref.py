"""FP64 reference of the closure's training data (test infrastructure only).

From a fine field phi_f on a grid r times finer than the coarse one:
  * restriction: phi_c = mean of each r x r block (mass per coarse cell is kept);
  * target: the sharpening flux the fine field carries, expressed per coarse
    lattice unit and averaged over the block, minus the flux the coarse scheme
    computes from phi_c:  c* = mean_block(r S_f n_f) - S_c(phi_c) n_c(phi_c),
    with S n from the oracle (Eq. (6), (7), (13));
  * samples: the 5x5 neighbourhoods of phi_c (dy = -2..2 outer, dx = -2..2
    inner, periodic) at coarse nodes inside the band theta < clip(phi_c) < 1 - theta.
"""
import numpy as np

from . import lib as O


def restrict(phi_f, r=4):
    ny, nx = phi_f.shape
    return phi_f.reshape(ny // r, r, nx // r, r).mean(axis=(1, 3))


def target(phi_f, eps_f, eps_c, delta=1e-10, r=4):
    nyf, nxf = phi_f.shape
    pf = O.Params(nxf, nyf, eps=eps_f, delta=delta)
    fx, fy = O.flux(pf, phi_f)
    phi_c = restrict(phi_f, r)
    pc = O.Params(nxf // r, nyf // r, eps=eps_c, delta=delta)
    cx, cy = O.flux(pc, phi_c)
    tx = restrict(r * fx, r) - cx
    ty = restrict(r * fy, r) - cy
    return phi_c, tx, ty


def band(phi_c, theta):
    pc = np.clip(phi_c, 0.0, 1.0)
    return (pc > theta) & (pc < 1.0 - theta)


def stencils(phi_c, mask):
    ny, nx = phi_c.shape
    jj, ii = np.nonzero(mask)
    X = np.empty((jj.size, 25))
    m = 0
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            X[:, m] = phi_c[(jj + dy) % ny, (ii + dx) % nx]
            m += 1
    return X, jj, ii
