"""Parity at the benchmark sizes, in the configuration bench.py times (FMG then
V(2,2) cycles, captured graphs): every leaf value of the 256^3 periodic grid and of
the literal-rule AMR tree against the reference solver after the same cycles."""
import numpy as np
import pytest

from helpers import gpu_tree, inputs, oracle_trees, rel_err
from paper_1901_11370_amd import workloads as W

pytestmark = pytest.mark.gpu


def _fmg_v(w, n_v, remove_mean=False, **params):
    import torch
    t = gpu_tree(w, **params)
    f, _ = inputs(w, t)
    t.set_rhs(torch.from_numpy(f[0]).cuda())
    t.fmg()
    t.vcycle(n_v)
    phi = t.get_phi()
    g_norm = t.residual_norm()[0]
    del t
    o = oracle_trees(w)[0]
    o.set_rhs(f[0])
    o.fmg()
    o.vcycle(n_v)
    err = rel_err(phi, o.get_phi(), remove_mean)
    o_norm = o.residual_norm()[0]
    print(w.name, "leaf cells", len(phi), "rel err", err, "norms", g_norm, o_norm, flush=True)
    return err, g_norm, o_norm


def test_periodic_256_full_size():
    err, g, o = _fmg_v(W.config2(n=256), 2, remove_mean=True)
    assert err <= 1e-11 and abs(g - o) <= 1e-6 * o


def test_periodic_256_full_size_mixed_against_fp64_reference():
    # mixed form: FP32 FMG + one refinement step; compared with the FP64 reference
    # after FMG + 2 V-cycles, both near the FP32 cycle accuracy (bound 1e-6)
    err, g, o = _fmg_v(W.config2(n=256), 2, remove_mean=True, precision=1)
    assert err <= 1e-6


def test_amr_literal_full_size():
    err, g, o = _fmg_v(W.config3(nested=False), 1)
    assert err <= 1e-11 and abs(g - o) <= 1e-6 * o
