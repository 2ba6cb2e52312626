"""Learned closure: data generation, training and evaluation driver.

Every arithmetic step runs in the library's kernels: the fine runs (batched
persistent form), the restriction / flux-target / band-sample extraction
(lbac_closure_extract), the network's training (lbac_mlp_*), and the coarse
runs with the network fused into the step (lbac_set_closure).  torch only
holds device memory and draws minibatch indices.

Set-up (acoustic scaling between the grids, r = 4): a coarse run of side n
with width eps_c and relaxation time tau_c corresponds to a fine run of side
r n with eps_f = r eps_c, tau_f = r (tau_c - 1/2) + 1/2 (same mobility in
physical units), the same lattice velocity amplitude and r times the steps.
"""
import json
import math
import os
import sys
import time

import numpy as np

from . import lbac
from . import workloads as W

R = 4


def fine_case(case_c, r=R):
    c = dict(case_c)
    c["nx"] = c["ny"] = r * case_c["nx"]
    c["eps"] = r * case_c["eps"]
    c["tau"] = r * (case_c["tau"] - 0.5) + 0.5
    if c.get("vel") == "vortex":
        c["period_T"] = r * case_c["period_T"]
    elif c.get("vel") == "rotation":
        c["omega"] = case_c["omega"] / r
        c["cx"], c["cy"] = r * case_c["cx"], r * case_c["cy"]
    c["steps"] = r * case_c["steps"]
    kind, geom = case_c.get("phi0", ("circle", {}))
    c["phi0"] = (kind, geom)
    return c


def coarse_cases(count, seed, n=128, eps=0.5, tau=0.8):
    """Vortex / slotted-disk set-ups with jittered geometry (first half vortex)."""
    cs = W.closure_training_cases(count=count, seed=seed, n=n, eps=eps, tau=tau)
    for c in cs:
        if c["vel"] == "vortex":
            c["period_T"] = float(8 * n)
            c["steps"] = 8 * n
    return cs


def generate(cases_c, snapshots=16, theta=0.02, augment=True, capacity=None, log=print):
    """Runs the fine twins of cases_c together and extracts coarse samples at
    `snapshots` evenly spaced times of each run.  Returns device tensors X, Y."""
    import torch

    fines = [fine_case(c) for c in cases_c]
    phis = [W.initial_field(f) for f in fines]
    b = lbac.Batch(fines, phis)
    b.autotune(4)
    nf = fines[0]["nx"]
    assert all(f["nx"] == nf for f in fines)
    ws = torch.empty(lbac.closure_workspace_bytes(nf, nf, R), dtype=torch.uint8, device="cuda")
    pf = torch.empty((nf, nf), dtype=torch.float64, device="cuda")
    if capacity is None:
        capacity = len(fines) * snapshots * (8 if augment else 1) * 4096
    X = torch.empty((capacity, 25), dtype=torch.float32, device="cuda")
    Y = torch.empty((capacity, 2), dtype=torch.float32, device="cuda")
    n = 0
    chunks = [max(1, f["steps"] // snapshots) for f in fines]
    t0 = time.time()
    for s in range(snapshots):
        b.run(chunks)
        for k, f in enumerate(fines):
            inst = b.instance(k)
            inst.phi_device(pf.data_ptr())
            torch.cuda.synchronize()
            got = lbac.closure_extract(pf.data_ptr(), nf, nf, R, f["eps"], cases_c[k]["eps"], f["delta"], theta,
                                       augment, ws.data_ptr(), X.data_ptr(), Y.data_ptr(), n, capacity)
            n = min(n + got, capacity)
        log("closure data: snapshot %d/%d, %d samples, %.1f s" % (s + 1, snapshots, n, time.time() - t0))
    b.close()
    return X[:n], Y[:n]


def init_weights(seed, scale=1.0, out_scale=1.0):
    """Uniform fan-in initialisation, zero biases (layout of LBAC_MLP_NPARAM);
    the output layer is scaled by out_scale."""
    rng = np.random.default_rng(seed)
    parts = []
    for rows, cols in ((64, 25), (64, 0), (64, 64), (64, 0), (2, 64), (2, 0)):
        if cols:
            lim = scale * math.sqrt(3.0 / cols)
            parts.append(rng.uniform(-lim, lim, size=rows * cols))
        else:
            parts.append(np.zeros(rows))
    w = np.concatenate(parts)
    w[64 * 25 + 64 + 64 * 64 + 64:] *= out_scale
    return w.astype(np.float32)


def train(X, Y, steps=4000, batch=4096, lr=2e-3, seed=0, log=print):
    """Adam on the MSE of the standardised targets (cosine learning-rate
    decay); the target scale is folded back into the output layer.  Returns
    the FP32 parameter vector and the loss history."""
    import torch

    n = X.shape[0]
    scale = float(Y.std().item()) or 1.0
    Yn = (Y / scale).contiguous()
    # the minibatch gather and the training kernels share one stream, so a
    # gather never overwrites a minibatch that the previous step still reads
    st = torch.cuda.Stream()
    net = lbac.Mlp(init_weights(seed), stream=st.cuda_stream)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    hist = []
    with torch.cuda.stream(st):
        st.wait_stream(torch.cuda.default_stream())
        xb = torch.empty((batch, 25), dtype=torch.float32, device="cuda")
        yb = torch.empty((batch, 2), dtype=torch.float32, device="cuda")
        for s in range(steps):
            idx = torch.randint(0, n, (batch,), device="cuda", generator=gen)
            torch.index_select(X, 0, idx, out=xb)
            torch.index_select(Yn, 0, idx, out=yb)
            a = lr * 0.5 * (1.0 + math.cos(math.pi * s / steps))
            want = (s % 200 == 0) or s == steps - 1
            L = net.train_step(xb.data_ptr(), yb.data_ptr(), batch, a, want_loss=want)
            if want:
                hist.append((s, L))
                log("closure training: step %d loss %.4e (standardised)" % (s, L))
    st.synchronize()
    w = net.weights().astype(np.float64)
    net.close()
    # fold the target scale into W3, b3
    o3 = 64 * 25 + 64 + 64 * 64 + 64
    w[o3:] *= scale
    return w.astype(np.float32), hist, scale


def evaluate(weights, cases_c, theta=0.02, log=print):
    """E1/E2 at t = T against phi0 for: plain coarse, coarse with the closure,
    and the fine run (on its own grid, and restricted to the coarse grid)."""
    rows = []
    for c in cases_c:
        phi0 = W.initial_field(c)
        plain = lbac.Simulation({**c, "precision": "f32"}, phi0)
        plain.step(c["steps"])
        e_plain = plain.shape_error(phi0)
        cl = lbac.Simulation({**c, "precision": "f32"}, phi0)
        cl.set_closure(weights, theta=theta)
        cl.step(c["steps"])
        e_cl = cl.shape_error(phi0)
        f = fine_case(c)
        phi0f = W.initial_field(f)
        fine = lbac.Simulation({**f, "precision": "f32"}, phi0f)
        fine.step(f["steps"])
        e_fine = fine.shape_error(phi0f)
        pf = fine.phi()
        nr = c["nx"]
        restricted = pf.reshape(nr, R, nr, R).mean(axis=(1, 3))
        diff = restricted - phi0
        e_fine_c = (np.abs(diff).sum() / np.abs(phi0).sum(), np.linalg.norm(diff) / np.linalg.norm(phi0))
        row = dict(kind=c["vel"], plain=e_plain, closure=e_cl, fine=e_fine, fine_restricted=e_fine_c,
                   closure_vs_plain_truth=float(np.linalg.norm(cl.phi() - restricted) /
                                                np.linalg.norm(plain.phi() - restricted)))
        rows.append(row)
        log("closure eval %-8s E2 plain %.4e closure %.4e fine %.4e fine(restricted) %.4e; "
            "|closure - fine| / |plain - fine| = %.3f" % (c["vel"], e_plain[1], e_cl[1], e_fine[1], e_fine_c[1],
                                                            row["closure_vs_plain_truth"]))
        for s in (plain, cl, fine):
            s.close()
    return rows


def main(argv=None):
    import argparse

    import torch

    ap = argparse.ArgumentParser(description="train and evaluate the learned closure")
    ap.add_argument("--n", type=int, default=128, help="coarse side")
    ap.add_argument("--train-runs", type=int, default=64)
    ap.add_argument("--eval-runs", type=int, default=8)
    ap.add_argument("--snapshots", type=int, default=16)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--theta", type=float, default=0.02)
    ap.add_argument("--eps", type=float, default=0.5)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", default="closure_out")
    a = ap.parse_args(argv)
    torch.cuda.set_device(0)
    lbac.load()
    os.makedirs(a.out, exist_ok=True)
    log = lambda m: print(m, flush=True)  # noqa: E731
    t0 = time.time()
    train_cases = coarse_cases(a.train_runs, a.seed, n=a.n, eps=a.eps)
    X, Y = generate(train_cases, snapshots=a.snapshots, theta=a.theta, log=log)
    log("closure data: %d samples in %.1f s" % (X.shape[0], time.time() - t0))
    w, hist, scale = train(X, Y, steps=a.steps, batch=a.batch, lr=a.lr, seed=a.seed, log=log)
    np.save(os.path.join(a.out, "closure_weights.npy"), w)
    eval_cases = coarse_cases(a.eval_runs, a.seed + 1000, n=a.n, eps=a.eps)
    rows = evaluate(w, eval_cases, theta=a.theta, log=log)
    res = dict(samples=int(X.shape[0]), target_scale=scale, loss=hist, eval=rows, seconds=time.time() - t0)
    with open(os.path.join(a.out, "closure_result.json"), "w") as fh:
        json.dump(res, fh, indent=1)
    return res


if __name__ == "__main__":
    main(sys.argv[1:])
