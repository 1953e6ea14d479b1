"""2D axisymmetric form of the reference solver ((1/r) d/dr (r dphi/dr) + d2phi/dz2 in
finite volumes, x = r, y = z), pinned to exactness on r^2 + z^2 (also in the cells on
the axis, whose inner face has zero radius), second-order convergence to a manufactured
solution, and the dense direct solve of a refined tree."""
import numpy as np
import pytest

from oracle import DIRICHLET, NEUMANN, OracleTree
from paper_1901_11370_amd import workloads as W


def _tree(n, bc, **kw):
    dom = W.Domain(2, [n, n], [0.0, 0.0], [1.0, 1.0], bc)
    t = OracleTree(2, dom.base_cells, dom.lo, dom.hi, dom.bc_kind, bs=8, **kw)
    t.set_axisymmetric(True)
    return dom, t


def test_exact_on_r2_plus_z2():
    dom, t = _tree(32, [NEUMANN, DIRICHLET, DIRICHLET, DIRICHLET])
    lay = t.leaf_layout()
    x = W.cell_centres(lay, dom)
    out = t.apply(x[:, 0] ** 2 + x[:, 1] ** 2)
    inner = (lay[:, 1] < 31) & (lay[:, 2] > 0) & (lay[:, 2] < 31)   # axis cells included
    assert np.abs(out[inner] - 6.0).max() <= 1e-10
    assert np.any(inner & (lay[:, 1] == 0))


def test_second_order_convergence():
    errs = []
    for n in (16, 32, 64):
        dom, t = _tree(n, [NEUMANN, DIRICHLET, NEUMANN, NEUMANN])
        x = W.cell_centres(t.leaf_layout(), dom)
        r, z = x[:, 0], x[:, 1]
        sol = (1 - r ** 2) * np.cos(np.pi * z)
        t.set_rhs(-4 * np.cos(np.pi * z) - np.pi ** 2 * sol)
        t.solve(rel_tol=1e-12, max_cycles=60)
        errs.append(np.abs(t.get_phi() - sol).max())
    print("max errors", errs)
    assert 3.5 <= errs[0] / errs[1] <= 4.5 and 3.5 <= errs[1] / errs[2] <= 4.5


@pytest.mark.parametrize("lam", [0.0, 20.0])
def test_dense_direct_solve_refined(lam):
    rng = np.random.default_rng(5)
    dom, t = _tree(8, [NEUMANN, DIRICHLET, DIRICHLET, NEUMANN], max_refine=1,
                   refine=lambda d, lev, o, bs: lev == 0 and tuple(o[:2]) == (0, 0))
    t.set_lambda(lam)
    n = t.n_leaf
    A = np.column_stack([t.apply(np.eye(n)[j]) for j in range(n)])
    f = rng.normal(size=n)
    ref = np.linalg.solve(A, f)
    t.set_rhs(f)
    t.set_phi(np.zeros(n))
    for _ in range(60):
        t.vcycle()
    assert np.abs(t.get_phi() - ref).max() <= 1e-11 * np.abs(ref).max()


def test_rejected_in_3d_or_negative_radius():
    d3 = OracleTree(3, [8, 8, 8], [0, 0, 0], [1, 1, 1], [DIRICHLET] * 6, bs=8)
    with pytest.raises(ValueError):
        d3.set_axisymmetric(True)
    neg = OracleTree(2, [8, 8], [-1, 0], [1, 1], [DIRICHLET] * 4, bs=8)
    with pytest.raises(ValueError):
        neg.set_axisymmetric(True)
