"""Helmholtz term (the paper's equation list: div(eps grad phi) - lambda phi = f) in
the reference solver, pinned to closed forms and a dense direct solve."""
import numpy as np
import pytest

from oracle import DIRICHLET, PERIODIC, OracleTree
from paper_1901_11370_amd import workloads as W


@pytest.mark.parametrize("dim,n,hi,k,lam", [(3, (16, 16, 16), (1, 1, 1), (1, 2, 1), 5.0),
                                            (2, (32, 16), (2, 1), (3, 1), 50.0)])
def test_periodic_mode_and_constant(dim, n, hi, k, lam):
    # f = c + cos(2 pi k.x/L): the constant is not removed (the operator is regular),
    # phi = -c / lam + cos(...) / (mu_k - lam), mu_k the discrete Laplacian eigenvalue
    dom = W.Domain(dim, list(n), [0.0] * dim, list(hi), [PERIODIC] * (2 * dim))
    t = OracleTree(dim, dom.base_cells, dom.lo, dom.hi, dom.bc_kind, bs=8)
    t.set_lambda(lam)
    x = W.cell_centres(t.leaf_layout(), dom)
    mode = np.cos(2 * np.pi * sum(k[d] * x[:, d] / hi[d] for d in range(dim)))
    c = 0.7
    t.set_rhs(c + mode)
    t.solve(rel_tol=1e-13, max_cycles=40)
    h = [hi[d] / n[d] for d in range(dim)]
    mu = -sum(4.0 / h[d] ** 2 * np.sin(np.pi * k[d] * h[d] / hi[d]) ** 2 for d in range(dim))
    ref = -c / lam + mode / (mu - lam)
    assert np.abs(t.get_phi() - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("var_eps", [False, True])
def test_dense_direct_solve_refined(var_eps):
    rng = np.random.default_rng(11)
    dom = W.Domain(2, [8, 8], [0, 0], [1, 1], [DIRICHLET] * 4)
    t = OracleTree(2, dom.base_cells, dom.lo, dom.hi, dom.bc_kind, bs=4, max_refine=1,
                   refine=lambda d, lev, o, bs: lev == 0 and tuple(o[:2]) == (4, 4), variable_eps=var_eps)
    t.set_lambda(30.0)
    if var_eps:
        t.set_eps(np.exp(rng.normal(size=t.n_leaf) * 0.5))
    n = t.n_leaf
    A = np.column_stack([t.apply(np.eye(n)[j]) for j in range(n)])
    # the operator's diagonal carries -lambda on top of the Laplacian's
    t0 = OracleTree(2, dom.base_cells, dom.lo, dom.hi, dom.bc_kind, bs=4, max_refine=1,
                    refine=lambda d, lev, o, bs: lev == 0 and tuple(o[:2]) == (4, 4), variable_eps=var_eps)
    if var_eps:
        t0.set_eps(np.exp(np.random.default_rng(11).normal(size=n) * 0.5))
    A0 = np.column_stack([t0.apply(np.eye(n)[j]) for j in range(n)])
    assert np.abs(A - (A0 - 30.0 * np.eye(n))).max() <= 1e-9 * np.abs(A0).max()
    f = rng.normal(size=n)
    ref = np.linalg.solve(A, f)
    t.set_rhs(f)
    t.set_phi(np.zeros(n))
    for _ in range(40):
        t.vcycle()
    assert np.abs(t.get_phi() - ref).max() <= 1e-12 * np.abs(ref).max()
