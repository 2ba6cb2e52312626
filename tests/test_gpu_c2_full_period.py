"""The 1024^2 single vortex over one full period (16 384 steps; eps 0.5 and 1;
R = 0.15 N at (0.5 N, 0.75 N), tau 0.8, U 0.02) through the C ABI: FP32
storage and the shifted FP16 and BF16 storage forms, in the three-step launch
the 8192^2 benchmark uses, against the FP64 oracle's phi(T) stored by
tests/golden/make_c2_oracle.py (the single-vortex test of Sec. 3, with the
error norm there: relative distance of phi at t = T).

Bound on the relative L2 distance to the oracle, per form:
  1e-5 + 4 (r_f32 + r_storage)
where r_f32 and r_storage are the oracle's own responses at t = T, stored
with the golden field, to perturbations of the size and pattern of the form's
rounding (every population by 2^-24 after every step; the shifted
populations by the 16-bit format's unit roundoff after every third step).
The 1e-5 term is the FP32 tolerance this scheme is held to elsewhere: the
noise model does not cover rounding that repeats identically every step
(the FP32 velocity table, the FP32 lattice weights), which accumulates
systematically.  At eps = 0.5 the scheme amplifies grid-scale perturbations
in the bulk (the sharpening flux of a one-node dip exceeds the diffusive one
when eps < 1), so the responses and the bound are large there; at eps = 1
they are small.  Also: the 16-bit forms' shape error E2 against phi0 within
5% of FP32's, and each form's mass within 1e-5 of the oracle's.
"""
import os
import sys

import numpy as np
import pytest

from paper_2203_05230_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
LAUNCH = (224, 40, 4)  # bx, strip rows, LBAC_KERNEL_FUSED3
RESP = {"f32": (), "f32_f16store": ("resp_f16",), "f32_bf16store": ("resp_bf16",)}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("eps", [1.0, 0.5])
def test_c2_full_period_against_oracle(gpu_lib, eps):
    n, T = 1024, 16384
    z = np.load(os.path.join(GOLDEN, "c2_oracle_%d_eps%g.npz" % (n, eps)))
    assert int(z["steps"]) == T
    ref = z["phi"].astype(np.float64)
    case = W.single_vortex_case(n, eps=eps, tau=0.8, U=0.02, period_T=float(T))
    phi0 = W.circle(n, eps)
    e2 = {}
    for prec, keys in RESP.items():
        say("case: 1024^2 full period, eps", eps, prec, "launch", LAUNCH)
        sim = gpu_lib.Simulation({**case, "precision": prec}, phi0)
        sim.set_launch(*LAUNCH)
        sim.set_graph_chunk(96)
        sim.step(T)
        phi = sim.phi()
        e2[prec] = sim.shape_error(phi0)[1]
        mass = sim.mass()
        sim.close()
        err = float(np.linalg.norm(phi - ref) / np.linalg.norm(ref))
        bound = 1e-5 + 4.0 * (float(z["resp_f32"]) + sum(float(z[k]) for k in keys))
        dm = abs(mass - float(z["massT"])) / float(z["massT"])
        say("  rel L2 vs oracle %.3e (bound %.3e), mass vs oracle %.2e, E2 %.5e" % (err, bound, dm, e2[prec]))
        assert err <= bound
        assert dm <= 1e-5
    for prec in ("f32_f16store", "f32_bf16store"):
        assert abs(e2[prec] / e2["f32"] - 1.0) <= 0.05, (prec, e2)
