"""Independent 1-D reduction of the scheme on the D1Q3 lattice (test infrastructure).

For data that do not vary along one axis, summing the D2Q9 populations over
the velocities that share the same component along the other axis gives a
D1Q3 lattice with weights 2/3 (rest) and 1/6 (each moving direction), the
same sound speed c_s^2 = 1/3, and the isotropic gradient reduces to the
central difference (chi(x+1) - chi(x-1)) / 2.  This module writes that 1-D
scheme out directly from the paper's equations (Eq. (9)-(13), Jain width
convention), so that a 2-D implementation fed axis-invariant data must agree
with it to rounding: it pins the D2Q9 weights, velocity set, streaming
direction, gradient stencil and forcing without reusing any 2-D code.
"""
import numpy as np

C = (0, 1, -1)
W = (2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0)


def run(phi0, eps, tau, delta, nsteps, u_of_step):
    """phi after nsteps on a periodic 1-D grid.  u_of_step(n) returns the
    velocity at every node (array) or a scalar at step n."""
    phi0 = np.asarray(phi0, dtype=np.float64)
    u0 = np.broadcast_to(np.asarray(u_of_step(0), dtype=np.float64), phi0.shape)
    f = np.array([W[k] * phi0 * (1.0 + 3.0 * C[k] * u0) for k in range(3)])
    phiu_prev = phi0 * u0
    for n in range(nsteps):
        phi = f.sum(axis=0)
        pc = np.clip(phi, 0.0, 1.0)
        psi = eps * np.log((pc + delta) / (1.0 - pc + delta))
        g = 0.5 * (np.roll(psi, -1) - np.roll(psi, 1))
        nrm = g / (np.abs(g) + delta)
        S = (1.0 - np.tanh(psi / (2.0 * eps)) ** 2) / (4.0 * eps)
        u = np.broadcast_to(np.asarray(u_of_step(n), dtype=np.float64), phi.shape)
        G = phi * u - phiu_prev + S * nrm / 3.0
        new = np.empty_like(f)
        for k in range(3):
            fe = W[k] * phi * (1.0 + 3.0 * C[k] * u)
            F = 3.0 * W[k] * C[k] * G
            post = f[k] - (f[k] - fe) / tau + (1.0 - 0.5 / tau) * F
            new[k] = np.roll(post, C[k])
        f = new
        phiu_prev = phi * u
    return f.sum(axis=0)
