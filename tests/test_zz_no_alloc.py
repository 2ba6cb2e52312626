"""The allocation-free closure-sample extraction (lbac_closure_extract_noalloc)
against the workspace form (lbac_closure_extract) it varies, through the C
ABI: the same sample count and bitwise the same samples, on two calls in a
row (the second on a smaller field, so that what the first left in the
library's fixed workspace must not leak into it), plus the size limit."""
import sys

import numpy as np
import pytest

from paper_2203_05230_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _field(nf, r, eps_c, seed):
    rng = np.random.default_rng(seed)
    return np.clip(W.circle(nf, r * eps_c, R_frac=0.23, xc_frac=0.47, yc_frac=0.55)
                   + 1e-3 * rng.standard_normal((nf, nf)), -0.01, 1.01)


def _extract(gpu_lib, torch, phi_f, r, eps_c, theta, augment, noalloc):
    nf = phi_f.shape[0]
    pf = torch.from_numpy(phi_f).cuda()
    cap = 8 * (nf // r) ** 2
    X = torch.full((cap, 25), -7.0, dtype=torch.float32, device="cuda")
    Y = torch.full((cap, 2), -7.0, dtype=torch.float32, device="cuda")
    if noalloc:
        n = gpu_lib.closure_extract_noalloc(pf.data_ptr(), nf, nf, r, r * eps_c, eps_c, 1e-10, theta, augment,
                                            X.data_ptr(), Y.data_ptr(), 0, cap)
    else:
        ws = torch.empty(gpu_lib.closure_workspace_bytes(nf, nf, r), dtype=torch.uint8, device="cuda")
        n = gpu_lib.closure_extract(pf.data_ptr(), nf, nf, r, r * eps_c, eps_c, 1e-10, theta, augment, ws.data_ptr(),
                                    X.data_ptr(), Y.data_ptr(), 0, cap)
    torch.cuda.synchronize()
    return n, X.cpu().numpy(), Y.cpu().numpy()


def test_noalloc_extraction_equals_workspace_form_on_two_calls(gpu_lib):
    import torch

    for nf, seed, augment in ((256, 4, True), (160, 5, False)):
        say("case: closure extraction without allocation, fine grid %d, augment %s" % (nf, augment))
        phi_f = _field(nf, 4, 1.0, seed)
        n0, X0, Y0 = _extract(gpu_lib, torch, phi_f, 4, 1.0, 0.02, augment, noalloc=False)
        n1, X1, Y1 = _extract(gpu_lib, torch, phi_f, 4, 1.0, 0.02, augment, noalloc=True)
        assert n1 == n0 > 50
        assert np.array_equal(X1, X0) and np.array_equal(Y1, Y0)


def test_noalloc_extraction_rejects_grids_beyond_its_workspace(gpu_lib):
    import torch

    say("case: closure extraction without allocation, size limit")
    nf, r = 2048, 2  # coarse 1024 x 1024: about 25 MB of workspace, beyond the 8 MiB array
    pf = torch.zeros((nf, nf), dtype=torch.float64, device="cuda")
    with pytest.raises(gpu_lib.LbacError) as ei:
        gpu_lib.closure_extract_noalloc(pf.data_ptr(), nf, nf, r, 2.0, 1.0, 1e-10, 0.02, False, 0, 0, 0, 0)
    assert ei.value.code == gpu_lib.LBAC_EINVAL
