"""The closure network's GPU training kernels against the FP64 oracle
(oracle/mlp.py): forward outputs, loss, gradient, Adam updates.  FP32
arithmetic: tolerances are a few hundred FP32 unit roundoffs relative to the
size of the quantity compared."""
import sys

import numpy as np
import pytest

from oracle import mlp as M

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def data(seed, B):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.0, 1.0, size=(B, 25)).astype(np.float32)
    Y = rng.normal(0.0, 0.05, size=(B, 2)).astype(np.float32)
    return X, Y


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_forward_matches_oracle(gpu_lib):
    import torch

    say("case: mlp forward")
    w = M.init_weights(11, scale=1.3).astype(np.float32)
    X, _ = data(1, 1000)
    net = gpu_lib.Mlp(w)
    xd, od = dev(torch, X), torch.empty((1000, 2), dtype=torch.float32, device="cuda")
    net.forward(xd.data_ptr(), 1000, od.data_ptr())
    torch.cuda.synchronize()
    ref, _ = M.forward(w.astype(np.float64), X.astype(np.float64))
    got = od.cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-5 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("B", [1, 37, 512, 3000])
def test_loss_and_gradient_match_oracle(gpu_lib, B):
    import torch

    say("case: mlp loss/grad, batch", B)
    w = M.init_weights(12, scale=1.3).astype(np.float32)
    X, Y = data(2 + B, B)
    net = gpu_lib.Mlp(w)
    xd, yd = dev(torch, X), dev(torch, Y)
    L, g = net.loss_grad(xd.data_ptr(), yd.data_ptr(), B)
    Lr, gr = M.loss_and_grad(w.astype(np.float64), X.astype(np.float64), Y.astype(np.float64))
    assert L == pytest.approx(Lr, rel=1e-5)
    assert np.linalg.norm(g - gr) <= 2e-5 * np.linalg.norm(gr)
    assert np.max(np.abs(g - gr)) <= 2e-5 * np.max(np.abs(gr))


def test_adam_steps_match_oracle(gpu_lib):
    """Each GPU Adam step equals the oracle's Adam step applied to the GPU's own
    gradient (the gradient itself is compared in the test above): this
    isolates the update arithmetic, which for near-zero gradients is only
    defined up to the gradient's sign."""
    import torch

    say("case: mlp adam")
    w = M.init_weights(13, scale=1.0).astype(np.float32)
    X, Y = data(5, 256)
    net = gpu_lib.Mlp(w)
    xd, yd = dev(torch, X), dev(torch, Y)
    wr, m, v = w.astype(np.float64), np.zeros(M.N_PARAM), np.zeros(M.N_PARAM)
    lr = 1e-3
    for t in range(1, 4):
        _, g = net.loss_grad(xd.data_ptr(), yd.data_ptr(), 256)
        net.train_step(xd.data_ptr(), yd.data_ptr(), 256, lr)
        wr, m, v = M.adam(wr, g.astype(np.float64), m, v, t, lr)
        got = net.weights().astype(np.float64)
        assert np.max(np.abs(got - wr) - 4 * 2.0**-24 * np.abs(wr)) <= 1e-5 * lr * t
        wr = got  # continue from the GPU's FP32 weights


def test_training_reduces_loss(gpu_lib):
    import torch

    say("case: mlp training reduces loss")
    teacher = M.init_weights(21, scale=0.8)
    rng = np.random.default_rng(9)
    X = rng.uniform(0, 1, size=(4096, 25))
    Y, _ = M.forward(teacher, X)
    net = gpu_lib.Mlp(M.init_weights(22, scale=0.8).astype(np.float32))
    xd, yd = dev(torch, X.astype(np.float32)), dev(torch, Y.astype(np.float32))
    first = net.train_step(xd.data_ptr(), yd.data_ptr(), 4096, 3e-3, want_loss=True)
    for _ in range(300):
        net.train_step(xd.data_ptr(), yd.data_ptr(), 4096, 3e-3)
    last = net.train_step(xd.data_ptr(), yd.data_ptr(), 4096, 3e-3, want_loss=True)
    assert last < 0.1 * first
