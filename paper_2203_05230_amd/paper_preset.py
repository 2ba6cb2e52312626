"""The paper's own single-vortex experiment run with this scheme (Sec. 3,
Eq. (14)): L = 200, R = 0.2 L at (0.5 L, 0.75 L), U0 = 0.04, M = 0.001
(tau = 0.503), one full period T = 30 000 steps, the printed velocity signs,
regulariser e^-20.  Reports the relative L1 error of the paper (and the
relative L2 error) of phi at t = T against phi0, the mass drift, and the
shape at T/2, for a list of interface widths eps_paper (the paper's
convention; 3 and 1.5 in its figures, eps = eps_paper / 4 here).

    python -m paper_2203_05230_amd.paper_preset --eps 1,1.5,2,2.5,3,4 --precision f64
"""
import argparse
import json
import os
import sys
import time

import numpy as np

from . import lbac
from . import workloads as W


def run(eps_paper, precision="f64", graph_chunk=1000):
    case = W.paper_vortex_case(eps_paper)
    phi0 = W.initial_field(case)
    sim = lbac.Simulation({**case, "precision": precision}, phi0)
    sim.set_graph_chunk(graph_chunk)
    m0 = sim.mass()
    T = case["steps"]
    t0 = time.perf_counter()
    sim.step(T // 2)
    half = sim.phi()
    sim.step(T - T // 2)
    e1, e2 = sim.shape_error(phi0)
    seconds = time.perf_counter() - t0
    m1 = sim.mass()
    sim.close()
    return dict(eps_paper=eps_paper, eps=case["eps"], precision=precision, steps=T, e1=e1, e2=e2,
                mass_drift=abs(m1 - m0) / m0, seconds=seconds, half_min=float(half.min()), half_max=float(half.max())), half


def main(argv=None):
    ap = argparse.ArgumentParser(description="the paper's single-vortex experiment with this scheme")
    ap.add_argument("--eps", default="1,1.5,2,2.5,3,4", help="interface widths in the paper's convention")
    ap.add_argument("--precision", default="f64")
    ap.add_argument("--out", default="paper_preset_out")
    a = ap.parse_args(argv)
    lbac.load()
    os.makedirs(a.out, exist_ok=True)
    rows = []
    for e in [float(v) for v in a.eps.split(",") if v]:
        r, half = run(e, a.precision)
        np.save(os.path.join(a.out, "phi_half_eps%g_%s.npy" % (e, a.precision)), half.astype(np.float32))
        rows.append(r)
        print("eps_paper %-4g (eps %.4g) %s: E1 %.4e  E2 %.4e  mass drift %.2e  phi(T/2) in [%.3g, %.3g]  %.2f s"
              % (e, r["eps"], a.precision, r["e1"], r["e2"], r["mass_drift"], r["half_min"], r["half_max"],
                 r["seconds"]), flush=True)
    with open(os.path.join(a.out, "paper_preset_%s.json" % a.precision), "w") as fh:
        json.dump(rows, fh, indent=1)
    return rows


if __name__ == "__main__":
    main(sys.argv[1:])
