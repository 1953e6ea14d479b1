"""Captured cycle sequences (HIP graphs) against the same kernels launched one by one.

Two trees on identical inputs, one replaying captured V-cycles, FMG cycles,
refinement steps and residual norms, one launching every kernel directly.  After
every replay (with the program's own eager work -- norms, reads, a change of the
right-hand side -- between replays) the two must agree bit for bit: the graphs hold
exactly the kernels of the direct path.
"""
import numpy as np
import pytest

from helpers import gpu_tree, inputs
from paper_1901_11370_amd import workloads as W

pytestmark = pytest.mark.gpu


def _pair(w, **params):
    import torch
    a = gpu_tree(w, graphs=1, **params)
    b = gpu_tree(w, graphs=0, **params)
    f, e = inputs(w, a)
    for t in (a, b):
        if w.variable_eps:
            t.set_eps(torch.from_numpy(np.concatenate(e)).cuda())
        t.set_rhs(torch.from_numpy(np.concatenate(f)).cuda())
    return a, b, np.concatenate(f)


def _same(a, b, what):
    pa, pb = a.get_phi(), b.get_phi()
    assert np.array_equal(pa, pb), f"{what}: max diff {np.abs(pa - pb).max():.3e}"


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replays_match_direct_launches(precision):
    import torch
    w = W.config3(nested=False, base=32)
    a, b, f = _pair(w, precision=precision)
    a.fmg(); b.fmg()
    _same(a, b, "fmg")
    for k in range(4):
        a.vcycle(); b.vcycle()
        _same(a, b, f"vcycle {k}")
        na, nb = a.residual_norm(), b.residual_norm()
        assert na == nb
    # eager work between replays: a new right-hand side, then replays again
    f2 = torch.from_numpy(0.5 * f).cuda()
    a.set_rhs(f2); b.set_rhs(f2)
    for k in range(3):
        a.vcycle(); b.vcycle()
        _same(a, b, f"vcycle after new rhs {k}")
    ca, _ = a.solve(rel_tol=1e-10, max_cycles=30)
    cb, _ = b.solve(rel_tol=1e-10, max_cycles=30)
    assert ca == cb
    _same(a, b, "solve")
    ra, _ = a.solve_stats()
    rb, _ = b.solve_stats()
    assert np.array_equal(ra, rb)


def test_graph_replays_forest_variable_eps_homogeneous_switch():
    w = W.config5(sizes=(32, 48))
    a, b, f = _pair(w, precision=1)
    for homog in (False, True, False):
        a.set_homogeneous_bc(homog); b.set_homogeneous_bc(homog)
        ca, _ = a.solve(rel_tol=1e-10, max_cycles=30)
        cb, _ = b.solve(rel_tol=1e-10, max_cycles=30)
        assert ca == cb
        _same(a, b, f"solve homogeneous={homog}")
        assert np.array_equal(a.domain_residual_norms()[0], b.domain_residual_norms()[0])
