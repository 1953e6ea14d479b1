"""The allocation-free residual norm (mg_residual_norms_static): its per-block partials
live in the library's fixed device array instead of the tree's store, and it writes the
per-domain sums into caller device memory without synchronising.  Called through the C
ABI and compared with mg_domain_residual_norms (the same kernels with the store's
partials) on two calls in a row, the second on a smaller tree, so stale partials of the
first call would show; trees beyond the array's 65536 leaf blocks are rejected."""
import ctypes

import numpy as np
import pytest

from helpers import gpu_tree, inputs
from paper_1901_11370_amd import workloads as W

pytestmark = pytest.mark.gpu


def _static_norms(t):
    import torch
    from paper_1901_11370_amd import mg
    out = torch.full((4 * t.ndom,), float("nan"), dtype=torch.float64, device="cuda")
    rc = mg._lib.mg_residual_norms_static(t.h, ctypes.c_void_p(out.data_ptr()))
    assert rc == mg.MG_OK, mg.mg_last_error(t.h)
    torch.cuda.synchronize()
    n = out.cpu().numpy().reshape(t.ndom, 4)
    mx = np.where(n[:, 2] > 0, n[:, 0] / np.where(n[:, 2] > 0, n[:, 2], 1.0), n[:, 0])
    l2 = np.sqrt(np.where(n[:, 3] > 0, n[:, 1] / np.where(n[:, 3] > 0, n[:, 3], 1.0), n[:, 1]))
    return mx, l2


def _case(w, cycles):
    t = gpu_tree(w)
    f, e = inputs(w, t)
    if w.variable_eps:
        t.set_eps(np.concatenate(e))
    t.set_rhs(np.concatenate(f))
    t.fmg()
    t.vcycle(cycles)
    return t


def test_static_norms_match_the_store_norms_on_two_calls():
    # first a refined forest of three domains with variable eps, then a smaller tree
    big = W.config5(sizes=(32, 48, 64))
    small = W.config3(nested=False, base=32)
    for w, cyc in ((big, 1), (small, 2)):
        t = _case(w, cyc)
        mx, l2 = _static_norms(t)
        ref_mx, ref_l2 = t.domain_residual_norms()
        print(w.name, mx, ref_mx, l2, ref_l2, flush=True)
        assert np.all(np.abs(mx - ref_mx) <= 1e-15 * np.abs(ref_mx))
        assert np.all(np.abs(l2 - ref_l2) <= 1e-15 * np.abs(ref_l2))
        # and once more on the same tree: the array keeps the last call's contents, the
        # next call overwrites every partial it reads
        mx2, l22 = _static_norms(t)
        assert np.array_equal(mx2, mx) and np.array_equal(l22, l2)
        del t


def test_static_norms_reject_trees_beyond_the_array():
    from paper_1901_11370_amd import mg
    # 256 x 256 x 68 cells in 4^3 blocks: 69632 leaf blocks > 65536
    d = mg.Domain(3, (256, 256, 68), (0, 0, 0), (1, 1, 68 / 256), [mg.MG_BC_DIRICHLET] * 6)
    t = mg.Tree([d], bs=4)
    import torch
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    rc = mg._lib.mg_residual_norms_static(t.h, ctypes.c_void_p(out.data_ptr()))
    assert rc == mg.MG_ERR_ARG
    assert b"65536" in mg.mg_last_error(t.h)
