"""Writes the FP64 oracle's phi at t = T for the 1024^2 single vortex over one
full period (T = 16384 steps, eps = 0.5 and 1; R = 0.15 N at (0.5 N, 0.75 N),
tau = 0.8, U = 0.02, delta = 1e-10; the single-vortex test of Sec. 3 at the
sizes the precision forms are measured on), stored as FP32 (the differences
of interest are 1e-6 and larger), compressed, together with the oracle's own
response at t = T (relative L2 change of phi) to rounding-sized perturbations
of each storage form:

  resp_f32   every post-collision population times (1 + u xi) after every
             step, u = 2^-24 (FP32 arithmetic and storage);
  resp_f16   the shifted populations g_i = f*_i - w_i phi* times (1 + u xi),
             u = 2^-11, after every third step (FP16 storage of g_i, rounded
             once per three-step launch; the node's sum is kept);
  resp_bf16  the same with u = 2^-8 (BF16 storage).

xi is uniform in [-1, 1) from the oracle's counter-based generator.  Calls
only oracle/ and the seeded input generator.  About forty minutes per width
on eight cores.

    python tests/golden/make_c2_oracle.py [eps ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import lib as O  # noqa: E402
from paper_2203_05230_amd import workloads as W  # noqa: E402

N, T = 1024, 16384
PERTURBATIONS = {
    "resp_f32": dict(noise=2.0**-24, noise_kind=O.NOISE_POPULATIONS, noise_every=1),
    "resp_f16": dict(noise=2.0**-11, noise_kind=O.NOISE_SHIFTED, noise_every=3),
    "resp_bf16": dict(noise=2.0**-8, noise_kind=O.NOISE_SHIFTED, noise_every=3),
}


def path(eps):
    return os.path.join(HERE, "c2_oracle_%d_eps%g.npz" % (N, eps))


def params(eps, **kw):
    return O.Params(N, N, eps=eps, tau=0.8, delta=1e-10, vel_kind=O.VEL_VORTEX, U=0.02, period_T=float(T), **kw)


def main(eps_list):
    for eps in eps_list:
        t0 = time.time()
        phi0 = W.circle(N, eps)
        phi, mass = O.run(params(eps), phi0, T, with_mass=True)
        resp = {}
        for name, kw in PERTURBATIONS.items():
            r = O.run(params(eps, noise_seed=17, **kw), phi0, T)
            resp[name] = float(np.linalg.norm(r - phi) / np.linalg.norm(phi))
            print("eps %g: %s %.3e (%.0f s)" % (eps, name, resp[name], time.time() - t0), flush=True)
        np.savez_compressed(path(eps), phi=phi.astype(np.float32), mass0=mass[0], massT=mass[-1], steps=T,
                            eps=eps, **resp)
        print("eps %g: %.0f s, E2 vs phi0 %.4e" % (eps, time.time() - t0,
                                                   np.linalg.norm(phi - phi0) / np.linalg.norm(phi0)), flush=True)


if __name__ == "__main__":
    main([float(a) for a in sys.argv[1:]] or [0.5, 1.0])
