"""CPU checks of the oracle's test-only perturbation option, which the GPU
tests use to measure how the iteration amplifies rounding-sized errors (the
bound a floating-point form is held to is a multiple of that response).

* Perturbing the shifted populations g_i = f*_i - w_i phi* with the rest
  population as the remainder keeps every node's sum, so the total mass moves
  only by rounding (Eq. (9) streaming is a permutation); perturbing every
  population does not.
* For small perturbations the response is linear in their size.
* noise_every = k perturbs after every k-th step and after the last one: with
  k larger than the run, only the last step is perturbed, which moves phi(T)
  by no more than the perturbation itself.
"""
import numpy as np

from oracle import lib as O
from paper_2203_05230_amd import workloads as W


def _params(**kw):
    return O.Params(48, 40, eps=1.0, tau=0.8, delta=1e-10, vel_kind=O.VEL_VORTEX, U=0.03, period_T=200.0, **kw)


def _phi0():
    return W.circle(48, 1.0, ny=40)


def test_shifted_noise_keeps_mass():
    phi0 = _phi0()
    _, m = O.run(_params(noise=1e-3, noise_seed=3, noise_kind=O.NOISE_SHIFTED), phi0, 60, with_mass=True)
    assert abs(m[-1] - m[0]) / m[0] <= 1e-13
    _, m2 = O.run(_params(noise=1e-3, noise_seed=3, noise_kind=O.NOISE_POPULATIONS), phi0, 60, with_mass=True)
    assert abs(m2[-1] - m2[0]) / m2[0] >= 1e-6


def test_response_is_linear_for_small_perturbations():
    phi0 = _phi0()
    ref = O.run(_params(), phi0, 60)
    for kind in (O.NOISE_POPULATIONS, O.NOISE_SHIFTED):
        r = [np.linalg.norm(O.run(_params(noise=a, noise_seed=5, noise_kind=kind), phi0, 60) - ref)
             for a in (1e-9, 2e-9)]
        assert r[0] > 0 and abs(r[1] / r[0] - 2.0) <= 0.02, (kind, r)


def test_shifted_noise_touches_only_the_shifted_part():
    """At rest and with phi uniform the post-collision populations are w_i phi
    exactly, so g_i = 0 and the shifted perturbation changes nothing."""
    phi0 = np.full((40, 48), 0.37)
    p = O.Params(48, 40, eps=1.0, tau=0.8, delta=1e-10, vel_kind=O.VEL_ZERO)
    ref = O.run(p, phi0, 10)
    q = O.Params(48, 40, eps=1.0, tau=0.8, delta=1e-10, vel_kind=O.VEL_ZERO, noise=1e-2, noise_seed=1,
                 noise_kind=O.NOISE_SHIFTED)
    assert np.max(np.abs(O.run(q, phi0, 10) - ref)) <= 1e-15


def test_noise_every():
    phi0 = _phi0()
    ref = O.run(_params(), phi0, 30)
    a = 1e-6
    last_only = O.run(_params(noise=a, noise_seed=9, noise_every=1000), phi0, 30)
    every = O.run(_params(noise=a, noise_seed=9, noise_every=1), phi0, 30)
    third = O.run(_params(noise=a, noise_seed=9, noise_every=3), phi0, 30)
    d_last, d_every, d_third = (np.max(np.abs(x - ref)) for x in (last_only, every, third))
    # the last step's perturbation reaches phi(T) through one streaming step:
    # at most the nine perturbed populations, each below a w_i-weighted phi
    assert 0 < d_last <= 9 * a * np.max(phi0)
    assert d_last < d_third < d_every
