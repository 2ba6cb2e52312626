"""Finite-volume solution of the 1-D improved conservative Allen-Cahn
equation, and of the conventional one (test infrastructure).

Solves Eq. (8) of the paper on a periodic line,
    d_t phi + d_x(phi u) = d_x( M [ d_x phi - S(psi) n ] ),
with psi = eps ln((phi_c + delta)/(1 - phi_c + delta)) (Eq. (13)),
S = (1 - tanh^2(psi / (2 eps))) / (4 eps) (Jain width convention) and
n = d_x psi / (|d_x psi| + delta), by a conservative cell-centred finite-volume
discretisation on a grid `refine` times finer than the lattice, classical
RK4 in time.  Lengths and times are in lattice units, so its solution is
what the lattice scheme must approach (Chapman-Enskog claim after Eq. (12):
the LB recovers Eq. (8) with M = c_s^2 (tau - 1/2)).

With conventional=True the flux is that of the conventional conservative
Allen-Cahn equation, Eq. (1): S = phi (1 - phi) / eps (the Jain width, the
paper's 4 phi (1 - phi) / eps with eps four times larger) evaluated at the
face, and n = d_x phi / (|d_x phi| + delta).
"""
import numpy as np


def _rhs_conventional(phi, h, u, M, eps, delta):
    phi_r = np.roll(phi, -1)
    dphi = (phi_r - phi) / h
    n = dphi / (np.abs(dphi) + delta)
    phi_f = 0.5 * (phi + phi_r)
    S = phi_f * (1.0 - phi_f) / eps
    flux = u * phi_f - M * (dphi - S * n)
    return -(flux - np.roll(flux, 1)) / h


def _rhs(phi, h, u, M, eps, delta):
    pc = np.clip(phi, 0.0, 1.0)
    psi = eps * np.log((pc + delta) / (1.0 - pc + delta))
    # face i+1/2 between cells i and i+1
    phi_r = np.roll(phi, -1)
    psi_r = np.roll(psi, -1)
    dphi = (phi_r - phi) / h
    dpsi = (psi_r - psi) / h
    n = dpsi / (np.abs(dpsi) + delta)
    psi_f = 0.5 * (psi + psi_r)
    S = (1.0 - np.tanh(psi_f / (2.0 * eps)) ** 2) / (4.0 * eps)
    flux = u * 0.5 * (phi + phi_r) - M * (dphi - S * n)
    return -(flux - np.roll(flux, 1)) / h


def solve(phi0_fine, h, u, M, eps, delta, t_end, cfl=0.2, conventional=False):
    """Integrate from phi0_fine (cell averages on spacing h) to time t_end."""
    rhs = _rhs_conventional if conventional else _rhs
    phi = np.asarray(phi0_fine, dtype=np.float64).copy()
    dt_lim = cfl * min(h * h / max(M, 1e-30), h / max(abs(u), 1e-30))
    nst = int(np.ceil(t_end / dt_lim))
    dt = t_end / nst
    for _ in range(nst):
        k1 = rhs(phi, h, u, M, eps, delta)
        k2 = rhs(phi + 0.5 * dt * k1, h, u, M, eps, delta)
        k3 = rhs(phi + 0.5 * dt * k2, h, u, M, eps, delta)
        k4 = rhs(phi + dt * k3, h, u, M, eps, delta)
        phi = phi + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return phi
