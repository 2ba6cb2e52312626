"""Pins of the FP64 closure references: the MLP against an independent
implementation (the C oracle's loops), its gradient against central finite
differences, GELU limits, Adam's closed-form first step, and the training
targets' restriction and consistency properties."""
import numpy as np
import pytest

from oracle import closure_ref as CR
from oracle import lib as O
from oracle import mlp as M
from paper_2203_05230_amd import workloads as W


def test_parameter_count_matches_c_oracle():
    assert M.N_PARAM == O.nparam() == 5954


def test_forward_matches_c_loops():
    w = M.init_weights(1, scale=1.5)
    w[M.N_PARAM - 2:] = [0.3, -0.2]
    X = np.random.default_rng(2).uniform(-1, 2, size=(50, 25))
    out, _ = M.forward(w, X)
    for s in range(50):
        assert np.allclose(out[s], O.mlp(w, X[s]), rtol=1e-13, atol=1e-13)


def test_gelu_limits():
    assert M.gelu(0.0) == 0.0
    assert M.gelu(10.0) == pytest.approx(10.0, rel=1e-12)
    assert abs(M.gelu(-10.0)) < 1e-12
    assert M.gelu_grad(0.0) == pytest.approx(0.5)
    x = np.linspace(-4, 4, 101)
    h = 1e-6
    assert np.allclose(M.gelu_grad(x), (M.gelu(x + h) - M.gelu(x - h)) / (2 * h), atol=1e-8)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    w = M.init_weights(3, scale=1.2) + 0.01 * rng.standard_normal(M.N_PARAM)
    X = rng.uniform(0, 1, size=(16, 25))
    Y = rng.normal(0, 0.1, size=(16, 2))
    L, g = M.loss_and_grad(w, X, Y)
    assert L == pytest.approx(M.loss(w, X, Y))
    idx = rng.choice(M.N_PARAM, size=200, replace=False)
    idx = np.concatenate([idx, [0, 1599, 1600, 1663, 1664, 5759, 5760, 5823, 5824, 5951, 5952, 5953]])
    h = 1e-6
    for i in idx:
        e = np.zeros(M.N_PARAM)
        e[i] = h
        fd = (M.loss(w + e, X, Y) - M.loss(w - e, X, Y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, i


def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    w = np.array([1.0, 2.0, 3.0, 4.0])
    w1, m, v = M.adam(w, g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8))


def test_loss_zero_at_own_output():
    w = M.init_weights(5)
    X = np.random.default_rng(6).uniform(0, 1, size=(8, 25))
    out, _ = M.forward(w, X)
    L, g = M.loss_and_grad(w, X, out)
    assert L == 0.0 and np.all(g == 0.0)


def test_restriction_keeps_mass_and_stencil_layout():
    phi_f = W.circle(64, 2.0)
    phi_c = CR.restrict(phi_f, 4)
    assert phi_c.shape == (16, 16)
    assert phi_c.sum() * 16 == pytest.approx(phi_f.sum(), rel=1e-14)
    mask = np.zeros((16, 16), bool)
    mask[3, 5] = True
    X, jj, ii = CR.stencils(phi_c, mask)
    assert X[0, 12] == phi_c[3, 5] and X[0, 13] == phi_c[3, 6] and X[0, 7] == phi_c[2, 5]
    assert X[0, 0] == phi_c[1, 3] and X[0, 24] == phi_c[5, 7]


def test_target_vanishes_under_refinement_for_equilibrium_band():
    """For a planar equilibrium band the fine and coarse fluxes describe the
    same profile, so the target is a discretisation residual that falls
    as the coarse width in nodes grows (eps_c = 1 -> 2)."""
    res = []
    for eps_c in (1.0, 2.0):
        n = int(32 * eps_c)
        phi_f = W.slab(4 * n, 4 * n, 4 * eps_c)
        phi_c, tx, ty = CR.target(phi_f, 4 * eps_c, eps_c)
        S = (1.0 / (4 * eps_c))
        res.append(np.max(np.abs(tx)) / S)
        assert np.max(np.abs(ty)) < 1e-10
    assert res[1] < res[0] / 3
