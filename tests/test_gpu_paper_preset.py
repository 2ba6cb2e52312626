"""The paper's own single-vortex set-up (L = 200, R = 0.2 L, U0 = 0.04,
tau = 0.503, printed velocity signs, regulariser e^-20, eps_paper 3 and 1.5)
through the C ABI: FP64 parity with the oracle over the start of the period,
and a full period in FP32 against the same period in FP64."""
import sys

import numpy as np
import pytest

from oracle import lib as O
from paper_2203_05230_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oparams(c):
    return O.Params(c["nx"], c["ny"], eps=c["eps"], tau=c["tau"], delta=c["delta"], vel_kind=O.VEL_VORTEX_PAPER,
                    U=c["U"], period_T=c["period_T"])


# With the paper's regulariser e^-20 and a disk whose inside saturates at
# phi0 = 1 exactly, psi = eps ln((phi_c + delta)/(1 - phi_c + delta)) has the
# slope eps/delta ~ 1e8 there: a one-ulp difference of phi moves psi by more
# than delta, so the normal n = grad psi / (|grad psi| + delta) of Eq. (13) in
# the bulk is set by rounding while S n has the size delta/eps.  No two FP64
# evaluations that round differently can agree beyond what that allows.  The
# bound is measured with the oracle itself: its response to moving phi0 by
# one ulp (down, and up) at the saturated nodes, over the same steps.
@pytest.mark.parametrize("eps_paper,steps", [(3.0, 3000), (1.5, 1000)])
def test_paper_preset_fp64_parity(gpu_lib, eps_paper, steps):
    say("case: paper preset eps_paper", eps_paper, "FP64,", steps, "steps")
    c = W.paper_vortex_case(eps_paper)
    phi0 = W.initial_field(c)
    p = oparams(c)
    ref, mass = O.run(p, phi0, steps, with_mass=True)
    m = np.abs(ref) > 1e-8
    bulk = phi0 == 1.0
    assert bulk.sum() > 100
    response = 0.0
    for toward in (0.0, 2.0):
        q = phi0.copy()
        q[bulk] = np.nextafter(1.0, toward)
        r = O.run(p, q, steps)
        response = max(response, np.linalg.norm(r[m] - ref[m]) / np.linalg.norm(ref[m]))
    sim = gpu_lib.Simulation({**c, "precision": "f64"}, phi0)
    sim.set_graph_chunk(500)
    sim.step(steps)
    phi = sim.phi()
    err = np.linalg.norm(phi[m] - ref[m]) / np.linalg.norm(ref[m])
    say("  rel L2 on resolved nodes %.3e; oracle response to one ulp of the bulk %.3e" % (err, response))
    assert err <= response
    assert np.max(np.abs(phi - ref)) <= steps * c["delta"] / c["eps"]
    assert abs(sim.mass() - mass[0]) / mass[0] <= 1e-12


@pytest.mark.parametrize("eps_paper", [3.0, 1.5])
def test_paper_preset_full_period_fp32_vs_fp64(gpu_lib, eps_paper):
    """One full period T = 30 000 steps: the FP32 form's L1 error against phi0
    stays within 1% of the FP64 form's, and both conserve mass."""
    say("case: paper preset eps_paper", eps_paper, "full period, FP32 vs FP64")
    c = W.paper_vortex_case(eps_paper)
    phi0 = W.initial_field(c)
    out = {}
    for prec in ("f64", "f32"):
        sim = gpu_lib.Simulation({**c, "precision": prec}, phi0)
        sim.set_graph_chunk(1000)
        m0 = sim.mass()
        sim.step(c["steps"])
        e1, e2 = sim.shape_error(phi0)
        out[prec] = (e1, e2, abs(sim.mass() - m0) / m0)
        sim.close()
    say("  E1 f64 %.4e f32 %.4e; mass drift f64 %.1e f32 %.1e" % (out["f64"][0], out["f32"][0], out["f64"][2],
                                                                 out["f32"][2]))
    assert out["f64"][2] <= 1e-12 and out["f32"][2] <= 1e-5
    assert abs(out["f32"][0] - out["f64"][0]) <= 0.01 * out["f64"][0]
