"""Writes the FP64 oracle's phi at t = T for the 1024^2 single vortex over one
full period (T = 16384 steps, eps = 0.5 and 1; R = 0.15 N at (0.5 N, 0.75 N),
tau = 0.8, U = 0.02, delta = 1e-10; the single-vortex test of Sec. 3 at the
sizes the precision forms are measured on), stored as FP32 (the differences
of interest are 1e-5 and larger), compressed.  Calls only oracle/ and the
seeded input generator.  About ten minutes per width on eight cores.

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


def path(eps):
    return os.path.join(HERE, "c2_oracle_%d_eps%g.npz" % (N, eps))


def main(eps_list):
    for eps in eps_list:
        t0 = time.time()
        phi0 = W.circle(N, eps)
        p = O.Params(N, N, eps=eps, tau=0.8, delta=1e-10, vel_kind=O.VEL_VORTEX, U=0.02, period_T=float(T))
        phi, mass = O.run(p, phi0, T, with_mass=True)
        np.savez_compressed(path(eps), phi=phi.astype(np.float32), mass0=mass[0], massT=mass[-1], steps=T,
                            eps=eps)
        print("eps %g: %.0f s, E2 vs phi0 %.4e" % (eps, time.time() - t0,
                                                   np.linalg.norm(phi - phi0) / np.linalg.norm(phi0)), flush=True)


if __name__ == "__main__":
    main([float(a) for a in sys.argv[1:]] or [0.5, 1.0])
