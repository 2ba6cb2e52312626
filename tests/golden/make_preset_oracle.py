"""Writes the FP64 oracle's phi at t = T for the paper's own single-vortex
set-up over one full period (Sec. 3: L = 200, R = 0.2 L at (0.5 L, 0.75 L),
U0 = 0.04, M = 0.001 so tau = 0.503, the printed velocity signs, regulariser
e^-20, T = 6 L / U0 = 30 000 steps; eps_paper 3 and 1.5), together with the
oracle's own response at t = T to moving phi0 by one ulp (down, and up) at the
nodes where it saturates at 1: where phi is saturated the regulariser makes
psi's slope ~1e8, so the normal of Eq. (13) there is set by rounding, and no
two FP64 evaluations of the scheme that round differently can agree more
closely than that response.  Calls only oracle/ and the seeded input
generator; stored in FP64, compressed.  About a minute per width on eight
cores.

    python tests/golden/make_preset_oracle.py [eps_paper ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import lib as O  # noqa: E402
from paper_2203_05230_amd import workloads as W  # noqa: E402


def path(eps_paper):
    return os.path.join(HERE, "preset_oracle_eps_paper%g.npz" % eps_paper)


def main(eps_list):
    for eps_paper in eps_list:
        t0 = time.time()
        c = W.paper_vortex_case(eps_paper)
        phi0 = W.initial_field(c)
        p = O.Params(c["nx"], c["ny"], eps=c["eps"], tau=c["tau"], delta=c["delta"], vel_kind=O.VEL_VORTEX_PAPER,
                     U=c["U"], period_T=c["period_T"])
        steps = int(c["steps"])
        ref, mass = O.run(p, phi0, steps, with_mass=True)
        resolved = np.abs(ref) > 1e-8
        bulk = phi0 == 1.0
        response = 0.0
        for toward in (0.0, 2.0):
            q = phi0.copy()
            q[bulk] = np.nextafter(1.0, toward)
            r = O.run(p, q, steps)
            response = max(response, float(np.linalg.norm(r[resolved] - ref[resolved]) /
                                           np.linalg.norm(ref[resolved])))
        np.savez_compressed(path(eps_paper), phi=ref, mass0=mass[0], massT=mass[-1], steps=steps,
                            eps_paper=eps_paper, ulp_response=response, bulk_nodes=int(bulk.sum()))
        print("eps_paper %g: %d steps, %.0f s, one-ulp response %.3e, mass drift %.1e" %
              (eps_paper, steps, time.time() - t0, response, abs(mass[-1] - mass[0]) / mass[0]), flush=True)


if __name__ == "__main__":
    main([float(a) for a in sys.argv[1:]] or [3.0, 1.5])
