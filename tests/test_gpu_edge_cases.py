"""Degenerate and boundary cases of the GPU path against the reference solver (the
FP64 bar of 1e-11 relative after the same cycles): one-block domains (the whole
hierarchy below the block runs in the single-workgroup coarse solver), the smallest
block size on a one-block grid, coarsest grids of 3, 5 and 7 cells per axis with
periodic wrap (odd periodic coarse grids), refinement that wraps across a periodic
boundary, a forest that mixes a one-block domain with larger ones, and f = 0 (Laplace
with boundary values, where the residual norm is absolute).
"""
import numpy as np
import pytest

from helpers import gpu_tree, inputs, oracle_trees, rel_err, split
from paper_1901_11370_amd import workloads as W
from test_gpu_parity import _run

pytestmark = pytest.mark.gpu


def _gauss_workload(name, dom, bs, remove_mean=False, **kw):
    rng = np.random.default_rng(17)
    lo, hi = np.array(dom.lo, float), np.array(dom.hi, float)
    c = lo + rng.uniform(0.2, 0.8, size=(3, dom.dim)) * (hi - lo)
    g = W.Gaussians(c, np.array([1.0, -0.7, 0.4]), np.array([0.15, 0.1, 0.2]) * (hi - lo).min())

    def rhs(i, lay):
        f = g(W.cell_centres(lay, dom))
        return f - f.mean() if remove_mean else f
    return W.Workload(name, [dom], bs=bs, rhs=rhs, **kw)


@pytest.mark.parametrize("case", ["single_block_2d", "single_block_3d_periodic", "one_block_bs4"])
def test_one_block_domains(case):
    if case == "single_block_2d":
        dom = W.Domain(2, [16, 16], [0, 0], [1, 1], [W.DIRICHLET] * 4, [1.0, -1.0, 0.5, 0.0])
        _run(_gauss_workload(case, dom, 16), "fvvnv")
    elif case == "single_block_3d_periodic":
        dom = W.Domain(3, [16, 16, 16], [0, 0, 0], [1, 1, 1], [W.PERIODIC] * 6)
        _run(_gauss_workload(case, dom, 16, remove_mean=True), "fvv", remove_mean=True)
    else:
        dom = W.Domain(2, [4, 4], [0, 0], [1, 1], [W.NEUMANN, W.DIRICHLET, W.DIRICHLET, W.NEUMANN],
                       [0.5, 1.0, -0.5, 0.0])
        _run(_gauss_workload(case, dom, 4), "vvfv")


@pytest.mark.parametrize("dim", [2, 3])
def test_odd_periodic_coarsest_grids(dim):
    # 7*16 x 5*16 (x 3*16): the coarsest grid has 7 x 5 (x 3) cells, odd along every
    # periodic axis, so a colour's ghosts are refilled after each half-sweep there
    n = [112, 80] if dim == 2 else [48, 80, 112]
    dom = W.Domain(dim, n, [0.0] * dim, [float(x) / 80 for x in n], [W.PERIODIC] * (2 * dim))
    _run(_gauss_workload(f"odd{dim}", dom, 16, remove_mean=True), "fvv", remove_mean=True)


def test_refinement_wrapping_a_periodic_boundary():
    # refined blocks around the corner (0,0) of a periodic square: the refined region
    # continues across every periodic face, so coarse-fine faces meet the wrap
    dom = W.Domain(2, [64, 64], [0, 0], [1, 1], [W.PERIODIC] * 4)

    def refine(d, level, origin, bs):
        h = 1.0 / (64 << level)
        c = (np.array(origin[:2], float) + bs / 2) * h
        c = np.minimum(c, 1 - c)        # distance to the corner through the wrap
        return level < 2 and float(np.hypot(*c)) < 0.25 / (level + 1)

    w = _gauss_workload("wrap", dom, 8, remove_mean=True, max_refine=2, refine=refine)
    _run(w, "fvvn", remove_mean=True)


def test_forest_with_a_one_block_domain():
    w = W.config5(sizes=(16, 48, 64))
    _run(w, "fvvn")


def test_laplace_with_boundary_values():
    # f = 0: the solution is set by the boundary values alone; the relative residual
    # norm has no right-hand side to scale by and is reported as the absolute one
    dom = W.Domain(3, [32, 32, 32], [0, 0, 0], [1, 1, 1], [W.DIRICHLET] * 6, [1.0, 0.0, 0.5, -0.5, 0.25, 0.0])
    w = W.Workload("laplace", [dom], bs=16, rhs=lambda i, lay: np.zeros(len(lay)))
    t, refs = _run(w, "fvv")
    r0, _ = t.residual_norm()
    t.vcycle(3)
    r1, _ = t.residual_norm()
    assert np.isfinite(r0) and r1 < 5e-3 * r0   # three cycles at about 0.1 each


@pytest.mark.parametrize("precision", [0, 1])
def test_zero_cycles_and_already_converged_solves(precision):
    from paper_1901_11370_amd import mg
    dom = W.Domain(3, [32, 32, 32], [0, 0, 0], [1, 1, 1], [W.DIRICHLET] * 6)
    w = _gauss_workload("z", dom, 16)
    t = gpu_tree(w, precision=precision)
    f, _ = inputs(w, t)
    t.set_rhs(f[0])
    t.vcycle(0)
    t.fmg(0)
    assert np.all(t.get_phi() == 0.0)
    # phi = 0: the relative residual is 1, so a tolerance above it needs no cycle
    c, rc = t.solve(rel_tol=2.0, max_cycles=10, fmg_first=False)
    assert (c, rc) == (0, mg.MG_OK) and np.all(t.get_phi() == 0.0)
    for fmg in (False, True):
        c, rc = t.solve(rel_tol=1e-10, max_cycles=0, fmg_first=fmg, raise_on_fail=False)
        assert (c, rc) == (0, mg.MG_ERR_NOT_CONVERGED) and np.all(t.get_phi() == 0.0)
    c, rc = t.solve(rel_tol=1e-10, max_cycles=40)
    assert rc == mg.MG_OK and c > 0
    phi = t.get_phi()
    c, rc = t.solve(rel_tol=1e-10, max_cycles=40, fmg_first=False)
    assert (c, rc) == (0, mg.MG_OK) and np.array_equal(t.get_phi(), phi)


def test_zero_problem_stays_zero():
    # f = 0 with homogeneous boundary values: phi = 0 is exact, the (absolute) residual
    # is zero and every cycle leaves it there
    from paper_1901_11370_amd import mg
    dom = W.Domain(2, [64, 64], [0, 0], [1, 1], [W.DIRICHLET, W.NEUMANN, W.PERIODIC, W.PERIODIC])
    w = W.Workload("zero", [dom], bs=16, rhs=lambda i, lay: np.zeros(len(lay)))
    t = gpu_tree(w)
    t.set_rhs(np.zeros(t.n_leaf))
    t.fmg()
    t.vcycle(2)
    assert np.all(t.get_phi() == 0.0)
    assert t.residual_norm() == (0.0, 0.0)
    c, rc = t.solve(rel_tol=1e-10, max_cycles=5, fmg_first=False)
    assert (c, rc) == (0, mg.MG_OK)
    c, rc = t.solve(rel_tol=1e-10, max_cycles=5)   # the FP64 FMG runs before the first check
    assert (c, rc) == (1, mg.MG_OK) and np.all(t.get_phi() == 0.0)


@pytest.mark.parametrize("homogeneous", [False, True])
def test_apply_operator_matches_reference(homogeneous):
    # L phi for a random phi on a refined 3D tree with variable eps and every boundary
    # kind with non-zero values (periodic in y), against the reference operator
    dom = W.Domain(3, [32, 32, 48], [0.0, 0.0, 0.0], [1.0, 1.0, 1.5],
                   [W.DIRICHLET, W.NEUMANN, W.PERIODIC, W.PERIODIC, W.NEUMANN, W.DIRICHLET],
                   [0.7, -0.3, 0.0, 0.0, 0.4, -1.1])

    def refine(d, level, origin, bs):
        return level == 0 and origin[0] >= 16 and origin[2] < 32

    w = W.Workload("apply_op", [dom], bs=16, max_refine=1, refine=refine, variable_eps=True,
                   eps=lambda i, lay: np.exp(0.6 * np.sin(5 * W.cell_centres(lay, dom)).sum(axis=1)))
    t = gpu_tree(w)
    o = oracle_trees(w)[0]
    lay = t.leaf_layout()[:, 1:]
    assert np.array_equal(lay, o.leaf_layout())
    eps = w.eps(0, lay)
    phi = np.random.default_rng(5).standard_normal(t.n_leaf)
    t.set_eps(eps)
    o.set_eps(eps)
    if homogeneous:
        t.set_homogeneous_bc(True)
        o2 = W.Domain(dom.dim, dom.base_cells, dom.lo, dom.hi, dom.bc_kind, [0.0] * 6)
        o = oracle_trees(W.Workload("apply_op0", [o2], bs=16, max_refine=1, refine=refine,
                                    variable_eps=True))[0]
        o.set_eps(eps)
    got = t.apply_operator(phi)
    ref = o.apply(phi)
    err = rel_err(got, ref)
    print(f"homogeneous={homogeneous}: L phi rel err {err:.2e}", flush=True)
    assert err <= 1e-13
    # the tree's own phi and f are untouched: phi = 0, f = 0 still give a zero residual
    assert np.all(t.get_phi() == 0.0)


def test_nan_in_the_rhs_is_reported():
    # a NaN in f makes the residual norm non-finite: mg_residual_norm and mg_solve
    # return MG_ERR_NAN (ordinary NaN arithmetic in the kernels, no fault)
    import ctypes
    from paper_1901_11370_amd import mg
    w = W.config2(n=32)
    t = gpu_tree(w)
    f, _ = inputs(w, t)
    bad = f[0].copy()
    bad[12345] = np.nan
    t.set_rhs(bad)
    a, b = ctypes.c_double(), ctypes.c_double()
    assert mg.mg_residual_norm(t.h, ctypes.byref(a), ctypes.byref(b)) == mg.MG_ERR_NAN
    assert np.isnan(a.value)
    c = ctypes.c_int()
    assert mg.mg_solve(t.h, 1e-10, 5, 1, ctypes.byref(c)) == mg.MG_ERR_NAN
    # a plain right-hand side again: the tree solves normally
    t.set_rhs(f[0])
    t.set_phi(np.zeros(t.n_leaf))
    cycles, rc = t.solve(rel_tol=1e-10, max_cycles=30)
    assert rc == mg.MG_OK


@pytest.mark.parametrize("periodic", [False, True])
def test_conservation_on_the_amr_tree(periodic):
    # discrete conservation (Sec. 2.6, flux matching at refinement boundaries) of the
    # GPU operator on the literal-rule AMR tree of the 128^3 workload (7.5e6 leaf cells,
    # three refinement levels): for a random phi the volume-weighted sum of L phi over
    # the leaves is the boundary flux, sum over Dirichlet faces of -2 h phi_b (zero
    # boundary values), and zero on the same tree made periodic
    w = W.config3(nested=False)
    if periodic:
        d = w.domains[0]
        w.domains = [W.Domain(3, d.base_cells, d.lo, d.hi, [W.PERIODIC] * 6)]
    t = gpu_tree(w)
    lay = t.leaf_layout()
    phi = np.random.default_rng(8).standard_normal(t.n_leaf)
    lphi = t.apply_operator(phi)
    h = W.cell_widths(lay[:, 1:], w.domains[0])[:, 0]
    vol = h ** 3
    total = np.sum(vol * lphi)
    scale = np.sum(np.abs(vol * lphi))
    if periodic:
        flux = 0.0
    else:
        cells, faces = t.boundary_faces()
        flux = np.sum(-2.0 * h[cells] * phi[cells])
    print(f"periodic={periodic}: sum vol L phi {total:.6e}, boundary flux {flux:.6e}, scale {scale:.3e}", flush=True)
    assert abs(total - flux) <= 1e-12 * scale
