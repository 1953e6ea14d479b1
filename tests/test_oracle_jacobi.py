"""The reference solver's weighted-Jacobi smoother (the smoother of the paper's timing
runs), pinned to closed forms and to a direct solve.

On a periodic grid with constant coefficients every Fourier mode is an eigenvector of
one weighted-Jacobi step with f = 0:  factor 1 - omega * sum_d h_d^-2 (1 - cos theta_d)
/ sum_d h_d^-2 (theta_d = 2 pi k_d h_d / L_d); the checkerboard (theta = pi on every
axis) gives 1 - 2 omega.  Multigrid with any convergent smoother has the discrete
solution as its fixed point, so Jacobi cycles must reach the dense direct solve.
"""
import numpy as np
import pytest

from oracle import DIRICHLET, PERIODIC, OracleTree
from paper_1901_11370_amd import workloads as W


def _tree(dim, n, bc, hi, bs, **kw):
    dom = W.Domain(dim, list(n), [0.0] * dim, list(hi), [bc] * (2 * dim))
    return dom, OracleTree(dim, dom.base_cells, dom.lo, dom.hi, dom.bc_kind, bs=bs, **kw)


def _one_step(t, phi, omega):
    t.set_smoother(OracleTree.JACOBI, omega)
    t.set_rhs(np.zeros(t.n_leaf))
    t.set_phi(phi)
    top = t.num_levels - 1
    t.fill_ghosts_level(top)
    t.smooth_level(top, 1)
    return t.get_phi()


@pytest.mark.parametrize("omega", [2.0 / 3.0, 0.8, 1.0])
def test_checkerboard_factor(omega):
    dom, t = _tree(3, (16, 16, 16), PERIODIC, (1.0, 1.0, 1.0), 8)
    lay = t.leaf_layout()
    s = lay[:, 1] + lay[:, 2] + lay[:, 3]
    phi = np.where(s % 2 == 0, 1.0, -1.0)
    out = _one_step(t, phi, omega)
    assert np.abs(out - (1 - 2 * omega) * phi).max() <= 1e-14


@pytest.mark.parametrize("dim,n,hi,k", [(3, (16, 16, 16), (1, 1, 1), (1, 2, 3)),
                                        (3, (16, 8, 16), (1, 0.5, 2), (3, 1, 2)),
                                        (2, (32, 16), (2, 1), (5, 3))])
def test_fourier_mode_factor(dim, n, hi, k):
    omega = 2.0 / 3.0
    dom, t = _tree(dim, n, PERIODIC, hi, 8)
    x = W.cell_centres(t.leaf_layout(), dom)
    phi = np.cos(2 * np.pi * sum(k[d] * x[:, d] / hi[d] for d in range(dim)))
    h = [hi[d] / n[d] for d in range(dim)]
    w = [1.0 / hd ** 2 for hd in h]
    theta = [2 * np.pi * k[d] * h[d] / hi[d] for d in range(dim)]
    factor = 1 - omega * sum(w[d] * (1 - np.cos(theta[d])) for d in range(dim)) / sum(w)
    out = _one_step(t, phi, omega)
    assert np.abs(out - factor * phi).max() <= 1e-13


def test_jacobi_cycles_reach_the_dense_solution():
    rng = np.random.default_rng(3)
    dom, t = _tree(2, (8, 8), DIRICHLET, (1, 1), 4, max_refine=1,
                   refine=lambda d, lev, o, bs: lev == 0 and tuple(o[:2]) == (4, 0))
    n = t.n_leaf
    A = np.column_stack([t.apply(np.eye(n)[j]) for j in range(n)])
    f = rng.normal(size=n)
    ref = np.linalg.solve(A, f)
    t.set_smoother(OracleTree.JACOBI, 2.0 / 3.0)
    t.set_phi(np.zeros(n))
    t.set_rhs(f)
    for _ in range(120):
        t.vcycle()
    assert np.abs(t.get_phi() - ref).max() <= 1e-11 * np.abs(ref).max()
