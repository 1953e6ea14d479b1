"""GPU path vs the reference solver, element by element, on identical seeded inputs.

FP64 bar: after the same fixed sequence of cycles the GPU leaf phi matches the
reference to 1e-11 relative max-norm (the iterates differ only by rounding order and
fused multiply-adds).  Cases span several blocks and levels, refinement boundaries,
variable coefficients, Neumann and non-zero Dirichlet values, small block sizes and a
forest of independent domains.
"""
import numpy as np
import pytest

from helpers import gpu_tree, inputs, oracle_trees, rel_err, split
from paper_1901_11370_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-11


def _run(w, script, tol=TOL, remove_mean=False, **params):
    t = gpu_tree(w, **params)
    refs = oracle_trees(w)
    for o in refs:
        if params.get("smoother", 0) == 1:
            o.set_smoother(o.JACOBI, params.get("jacobi_weight", 2.0 / 3.0))
        if "n_down" in params or "n_up" in params:
            o.set_params(n_down=params.get("n_down", 2), n_up=params.get("n_up", 2))
        if "helmholtz_lambda" in params:
            o.set_lambda(params["helmholtz_lambda"])
        if params.get("axisymmetric", 0):
            o.set_axisymmetric()
    f, e = inputs(w, t)
    if w.variable_eps:
        t.set_eps(np.concatenate(e))
        for o, ei in zip(refs, e):
            o.set_eps(ei)
    t.set_rhs(np.concatenate(f))
    for o, fi in zip(refs, f):
        o.set_rhs(fi)
    for op in script:
        if op == "v":
            t.vcycle()
            for o in refs:
                o.vcycle()
        elif op == "f":
            t.fmg()
            for o in refs:
                o.fmg()
        elif op == "n":
            g_norms = t.domain_residual_norms()[0]
            o_norms = np.array([o.residual_norm()[0] for o in refs])
            assert np.allclose(g_norms, o_norms, rtol=1e-6, atol=1e-14)
    phis = split(t, t.get_phi())
    errs = [rel_err(p, o.get_phi(), remove_mean) for p, o in zip(phis, refs)]
    print(w.name, script, "rel err per domain", errs, flush=True)
    assert max(errs) <= tol
    return t, refs


def test_config1_ten_vcycles():
    _run(W.config1(), "v" * 10)


def test_config1_with_norms_between_cycles():
    _run(W.config1(), "vnvnvn")


def test_periodic_3d_fmg_then_vcycles():
    _run(W.config2(n=64), "fvvn", remove_mean=True)


def test_periodic_3d_multi_block_tail():
    # 96^3: three blocks per axis on the lowest block level, a 3^3 coarsest grid
    w = W.config2(n=96)
    _run(w, "fvv", remove_mean=True)


def test_amr_literal_rule_3d():
    w = W.config3(nested=False, base=32)
    _run(w, "fvvnv")


def test_amr_nested_small():
    w = W.config3(nested=True, base=16)
    w.bs = 8
    _run(w, "fvv")


def test_variable_eps_amr():
    w = W.config4(nested=False)
    w.domains[0].base_cells = [32, 32, 32]
    _run(w, "fvv")


def test_forest_three_domains():
    w = W.config5(sizes=(32, 48, 80))
    _run(w, "fvvn")


@pytest.mark.parametrize("bs", [4, 8])
def test_small_blocks_2d_refined(bs):
    dom = W.Domain(2, [32, 32], [0, 0], [1, 1], [W.DIRICHLET] * 4, [0.5, -1.0, 0.0, 2.0])
    g = W.Gaussians(np.array([[0.3, 0.6]]), np.array([1.0]), np.array([0.1]))

    def ref(d, lev, o, b):
        return lev < 2 and 8 * 2 ** lev <= o[0] < 20 * 2 ** lev and 12 * 2 ** lev <= o[1] < 24 * 2 ** lev

    w = W.Workload("amr2d", [dom], bs=bs, max_refine=2, refine=ref,
                   rhs=lambda i, lay: g(W.cell_centres(lay, dom)))
    _run(w, "fvvv")


def test_neumann_and_periodic_mix_3d():
    dom = W.Domain(3, [32, 32, 32], [0, 0, 0], [1, 2, 1], [W.NEUMANN, W.NEUMANN, W.PERIODIC, W.PERIODIC,
                                                           W.DIRICHLET, W.DIRICHLET],
                   [0.3, -0.2, 0.0, 0.0, 1.0, 0.0])
    g = W.Gaussians(np.array([[0.5, 1.0, 0.5]]), np.array([3.0]), np.array([0.2]))
    w = W.Workload("mixbc", [dom], bs=8, rhs=lambda i, lay: g(W.cell_centres(lay, dom)))
    _run(w, "vvfv")


def _smooth_eps(dom, lay, amp=0.6):
    x = W.cell_centres(lay, dom)
    return np.exp(amp * np.prod(np.sin(2 * np.pi * x / (np.array(dom.hi) - np.array(dom.lo))), axis=1))


def test_large_tail_grids_2d_mixed_bc_variable_eps():
    # 240 x 144 cells in 16^2 blocks: (15, 9) blocks on the lowest block level, so the
    # grid below it (120 x 72) runs as multi-workgroup launches
    dom = W.Domain(2, [240, 144], [0, 0], [1.0, 0.6], [W.NEUMANN, W.DIRICHLET, W.DIRICHLET, W.NEUMANN],
                   [0.4, 1.0, -0.5, 0.0])
    g = W.Gaussians(np.array([[0.3, 0.2], [0.7, 0.4]]), np.array([2.0, -1.0]), np.array([0.08, 0.05]))
    w = W.Workload("bigtail2d", [dom], bs=16, variable_eps=True,
                   rhs=lambda i, lay: g(W.cell_centres(lay, dom)), eps=lambda i, lay: _smooth_eps(dom, lay))
    _run(w, "fvvn")


def test_large_tail_grids_3d_periodic_neumann():
    # 96 x 96 x 64 cells in 16^3 blocks: a 24 x 24 x 16 grid below the block levels
    dom = W.Domain(3, [96, 96, 64], [0, 0, 0], [1.5, 1.5, 1.0], [W.PERIODIC, W.PERIODIC, W.NEUMANN, W.NEUMANN,
                                                                  W.DIRICHLET, W.DIRICHLET],
                   [0.0, 0.0, 0.2, -0.1, 1.0, 0.5])
    g = W.Gaussians(np.array([[0.7, 0.5, 0.4]]), np.array([5.0]), np.array([0.15]))
    w = W.Workload("bigtail3d", [dom], bs=16, variable_eps=True,
                   rhs=lambda i, lay: g(W.cell_centres(lay, dom)), eps=lambda i, lay: _smooth_eps(dom, lay, 0.4))
    _run(w, "vfvv")


def _wide_level_workload():
    # 128 x 128 x 96 cells in 16^3 blocks: 384 blocks on the finest level, which the
    # sweep runs with 512-thread workgroups; variable eps and all three boundary kinds
    dom = W.Domain(3, [128, 128, 96], [0, 0, 0], [1.0, 1.0, 0.75],
                   [W.DIRICHLET, W.NEUMANN, W.PERIODIC, W.PERIODIC, W.DIRICHLET, W.DIRICHLET],
                   [0.5, -0.2, 0.0, 0.0, 0.0, 1.0])
    g = W.Gaussians(np.array([[0.4, 0.6, 0.3]]), np.array([8.0]), np.array([0.1]))
    return W.Workload("widelevel3d", [dom], bs=16, variable_eps=True,
                      rhs=lambda i, lay: g(W.cell_centres(lay, dom)), eps=lambda i, lay: _smooth_eps(dom, lay))


def test_wide_sweep_level_variable_eps():
    _run(_wide_level_workload(), "fvv")


def test_wide_sweep_level_variable_eps_mixed():
    # the FP32 forms of the same level (zero-start and ordinary 512-thread sweeps)
    w = _wide_level_workload()
    t = gpu_tree(w, precision=1)
    o = oracle_trees(w)[0]
    f, e = inputs(w, t)
    t.set_eps(np.concatenate(e))
    t.set_rhs(np.concatenate(f))
    cycles, rc = t.solve(rel_tol=1e-10, max_cycles=40)
    o.set_eps(e[0])
    o.set_rhs(f[0])
    o.solve(rel_tol=1e-11, max_cycles=40)
    err = rel_err(t.get_phi(), o.get_phi())
    print("wide level mixed", cycles, err, flush=True)
    assert rc == 0 and err <= 1e-8


def test_face_gradient_matches_reference():
    w = W.config5(sizes=(32, 48))
    t = gpu_tree(w)
    refs = oracle_trees(w)
    lay = t.leaf_layout()
    rng = np.random.default_rng(9)
    _, e = inputs(w, t)
    t.set_eps(np.concatenate(e))
    phi = rng.normal(size=t.n_leaf)
    lam = rng.normal(size=t.n_leaf)
    g = split(t, t.face_gradient(phi, lam))
    for i, o in enumerate(refs):
        o.set_eps(e[i])
        sel = lay[:, 0] == i
        want = o.face_gradient(phi[sel], lam[sel])
        assert rel_err(g[i], want) <= 1e-13


def _mixed_vs_reference(w, tol):
    t = gpu_tree(w, precision=1)
    refs = oracle_trees(w)
    f, e = inputs(w, t)
    if w.variable_eps:
        t.set_eps(np.concatenate(e))
        for o, ei in zip(refs, e):
            o.set_eps(ei)
    t.set_rhs(np.concatenate(f))
    for o, fi in zip(refs, f):
        o.set_rhs(fi)
    cycles, rc = t.solve(rel_tol=1e-10, max_cycles=40)
    r, _ = t.solve_stats()
    print(w.name, "mixed IR steps", cycles, "history", r, flush=True)
    assert r[-1] <= 1e-10
    per_dom = t.domain_residual_norms()[0]
    assert per_dom.max() <= 1e-10
    errs = []
    for p, o in zip(split(t, t.get_phi()), refs):
        hist = o.solve(rel_tol=1e-13, max_cycles=80)
        errs.append(rel_err(p, o.get_phi()))
    print("mixed vs FP64 reference solution: rel err per domain", errs, flush=True)
    assert max(errs) < tol


def test_mixed_precision_forest_variable_eps():
    _mixed_vs_reference(W.config5(sizes=(32, 48)), 1e-8)


def test_mixed_precision_amr():
    _mixed_vs_reference(W.config3(nested=False, base=32), 1e-8)


@pytest.mark.parametrize("bs", [8, 16])
def test_mixed_precision_uniform_mixed_bc(bs):
    # without refinement the correction and the next residual run as one launch, which
    # rebuilds the Neumann and Dirichlet ghosts from the corrected boundary cells
    dom = W.Domain(3, [32, 32, 48], [0, 0, 0], [1, 2, 1.5], [W.NEUMANN, W.DIRICHLET, W.PERIODIC, W.PERIODIC,
                                                             W.DIRICHLET, W.NEUMANN],
                   [0.3, -0.2, 0.0, 0.0, 1.0, 0.5])
    g = W.Gaussians(np.array([[0.5, 1.0, 0.5]]), np.array([3.0]), np.array([0.2]))
    w = W.Workload("mixbcmix", [dom], bs=bs, rhs=lambda i, lay: g(W.cell_centres(lay, dom)))
    _mixed_vs_reference(w, 1e-8)


def test_fp64_solve_reaches_tolerance_and_reference_agrees():
    w = W.config2(n=64)
    t = gpu_tree(w)
    f, _ = inputs(w, t)
    t.set_rhs(f[0])
    cycles, rc = t.solve(rel_tol=1e-10, max_cycles=30)
    r, s = t.solve_stats()
    assert r[-1] <= 1e-10
    # the reference's composite residual of the GPU solution
    o = oracle_trees(w)[0]
    o.set_rhs(f[0])
    o.set_phi(t.get_phi())
    assert o.residual_norm()[0] <= 1.5e-10


# ------------------------------------------------ weighted Jacobi smoother
@pytest.mark.parametrize("case", ["dirichlet3d", "periodic_forest", "amr_var", "amr2d_odd_steps", "big_tail"])
def test_jacobi_smoother(case):
    if case == "dirichlet3d":
        w = W.Workload("jac3d", [W.Domain(3, [64] * 3, [0] * 3, [1] * 3, [W.DIRICHLET] * 6)],
                       rhs=lambda i, lay: np.ones(len(lay)))
        _run(w, "fvvv", smoother=1)
    elif case == "periodic_forest":
        w = W.config5(sizes=(32, 48))
        _run(w, "vvfv", smoother=1, jacobi_weight=0.8)
    elif case == "amr_var":
        w = W.config4(nested=False)
        w.domains[0].base_cells = [32, 32, 32]
        _run(w, "fvv", smoother=1)
    elif case == "amr2d_odd_steps":
        # odd step counts exercise the copy back; refined 2D tree with coarse-fine faces
        dom = W.Domain(2, [32, 32], [0, 0], [1, 1], [W.DIRICHLET] * 4, [0.5, -1.0, 0.0, 2.0])
        g = W.Gaussians(np.array([[0.3, 0.6]]), np.array([1.0]), np.array([0.1]))

        def ref(d, lev, o, b):
            return lev < 2 and 8 * 2 ** lev <= o[0] < 20 * 2 ** lev and 12 * 2 ** lev <= o[1] < 24 * 2 ** lev
        w = W.Workload("jacamr2d", [dom], bs=8, max_refine=2, refine=ref,
                       rhs=lambda i, lay: g(W.cell_centres(lay, dom)))
        t = gpu_tree(w, smoother=1, n_down=3, n_up=1)
        refs = oracle_trees(w)
        refs[0].set_smoother(refs[0].JACOBI, 2.0 / 3.0)
        refs[0].set_params(n_down=3, n_up=1)
        f, _ = inputs(w, t)
        t.set_rhs(f[0])
        refs[0].set_rhs(f[0])
        t.fmg(); refs[0].fmg()
        t.vcycle(3); refs[0].vcycle(3)
        err = rel_err(t.get_phi(), refs[0].get_phi())
        print("odd steps rel err", err, flush=True)
        assert err <= TOL
    else:
        # odd block counts: large coarse grids run by the grid-wide kernels
        dom = W.Domain(3, [96, 96, 64], [0, 0, 0], [1.5, 1.5, 1.0], [W.PERIODIC, W.PERIODIC, W.NEUMANN, W.NEUMANN,
                                                                      W.DIRICHLET, W.DIRICHLET],
                       [0.0, 0.0, 0.2, -0.1, 1.0, 0.5])
        g = W.Gaussians(np.array([[0.7, 0.5, 0.4]]), np.array([5.0]), np.array([0.15]))
        w = W.Workload("jacbig", [dom], bs=16, rhs=lambda i, lay: g(W.cell_centres(lay, dom)))
        _run(w, "vfv", smoother=1, n_down=1, n_up=2)


# ------------------------------------------------------------ Helmholtz term
@pytest.mark.parametrize("case", ["periodic3d", "amr_var", "forest_jacobi", "mixed_amr"])
def test_helmholtz(case):
    if case == "periodic3d":
        # regular operator: the constant part of f is kept (no mean removal)
        w = W.config2(n=64)
        f0 = w.rhs
        w.rhs = lambda i, lay: f0(i, lay) + 0.3
        _run(w, "fvv", helmholtz_lambda=40.0)
    elif case == "amr_var":
        w = W.config4(nested=False)
        w.domains[0].base_cells = [32, 32, 32]
        _run(w, "fvv", helmholtz_lambda=500.0)
    elif case == "forest_jacobi":
        w = W.config5(sizes=(32, 48))
        _run(w, "vfv", helmholtz_lambda=100.0, smoother=1)
    else:
        _mixed_vs_reference_l(W.config3(nested=False, base=32), 1e-8, 250.0)


def _mixed_vs_reference_l(w, tol, lam, axisymmetric=0):
    import torch
    t = gpu_tree(w, precision=1, helmholtz_lambda=lam, axisymmetric=axisymmetric)
    refs = oracle_trees(w)
    f, e = inputs(w, t)
    t.set_rhs(torch.from_numpy(np.concatenate(f)).cuda())
    cycles, rc = t.solve(rel_tol=1e-10, max_cycles=40)
    for o, fi in zip(refs, f):
        o.set_lambda(lam)
        if axisymmetric:
            o.set_axisymmetric()
        o.set_rhs(fi)
        o.solve(rel_tol=1e-12, max_cycles=60)
    errs = [rel_err(p, o.get_phi()) for p, o in zip(split(t, t.get_phi()), refs)]
    print("mixed helmholtz", cycles, errs, flush=True)
    assert rc == 0 and max(errs) <= tol


# ------------------------------------------------------- 2D axisymmetric form
def _axi_domain(n=(64, 128), lo=(0.0, -1.0), hi=(1.0, 1.0), kinds=None, values=None):
    # x is the radius: the face at r = 0 has weight 0, so its kind does not matter
    kinds = kinds or [W.NEUMANN, W.DIRICHLET, W.DIRICHLET, W.DIRICHLET]
    values = values or [0.0, 0.5, -0.25, 1.0]
    return W.Domain(2, list(n), list(lo), list(hi), kinds, values)


def _axi_workload(name, doms, bs=16, **kw):
    srcs = [W.Gaussians(np.array([[d.lo[0] + 0.3 * (d.hi[0] - d.lo[0]), 0.5 * (d.lo[1] + d.hi[1])]]),
                        np.array([4.0]), np.array([0.12])) for d in doms]
    return W.Workload(name, doms, bs=bs, rhs=lambda i, lay: srcs[i](W.cell_centres(lay, doms[i])), **kw)


@pytest.mark.parametrize("case", ["axis_dirichlet", "annulus_neumann", "amr_axis", "var_jacobi", "forest_helmholtz",
                                  "large_coarse", "mixed"])
def test_axisymmetric(case):
    if case == "axis_dirichlet":
        _run(_axi_workload("axi", [_axi_domain()]), "fvvnv", axisymmetric=1)
    elif case == "annulus_neumann":
        # r in [0.5, 1.5], periodic in z, a Neumann flux at the outer radius
        d = _axi_domain((64, 64), (0.5, 0.0), (1.5, 1.0), [W.DIRICHLET, W.NEUMANN, W.PERIODIC, W.PERIODIC],
                        [1.0, -0.5, 0.0, 0.0])
        _run(_axi_workload("axiann", [d]), "vfvn", axisymmetric=1)
    elif case == "amr_axis":
        # refinement around a source on the axis: coarse-fine faces next to r = 0
        d = _axi_domain((32, 64))
        g = W.Gaussians(np.array([[0.05, 0.1]]), np.array([6.0]), np.array([0.08]))

        def refine(dom, level, origin, bs, dm=d):
            h = (dm.hi[0] - dm.lo[0]) / (dm.base_cells[0] << level)
            cx = dm.lo[0] + (origin[0] + bs / 2) * h
            cy = dm.lo[1] + (origin[1] + bs / 2) * h
            return level < 2 and (cx - 0.05) ** 2 + (cy - 0.1) ** 2 < (0.3 / (level + 1)) ** 2

        w = W.Workload("axiamr", [d], bs=8, max_refine=2, refine=refine,
                       rhs=lambda i, lay: g(W.cell_centres(lay, d)))
        _run(w, "fvvnv", axisymmetric=1)
    elif case == "var_jacobi":
        d = _axi_domain((64, 64), (0.0, 0.0), (1.0, 1.0))
        w = _axi_workload("axivar", [d], variable_eps=True, eps=lambda i, lay: _smooth_eps(d, lay))
        _run(w, "vfv", axisymmetric=1, smoother=1)
        _run(w, "fvv", axisymmetric=1)
    elif case == "forest_helmholtz":
        doms = [_axi_domain((32, 64)), _axi_domain((48, 48), (2.0, 0.0), (3.0, 1.0))]
        _run(_axi_workload("axiforest", doms), "fvvn", axisymmetric=1, helmholtz_lambda=30.0)
    elif case == "large_coarse":
        # 768^2: coarse grids above 4096 cells run as grid-wide launches
        d = _axi_domain((768, 768), (0.0, 0.0), (1.0, 1.0))
        _run(_axi_workload("axibig", [d]), "fvv", axisymmetric=1)
    else:
        _mixed_vs_reference_l(_axi_workload("aximix", [_axi_domain()]), 1e-8, 0.0, axisymmetric=1)


# ------------------------------------------- mixed-form iterates, cycle by cycle
@pytest.mark.parametrize("case", ["dirichlet_neumann_2d", "periodic_3d", "forest_equal", "forest_unequal", "amr"])
def test_mixed_iterates_follow_fp64_cycles(case):
    # a refinement step (FP32 cycle on the residual equation from e = 0, added to phi)
    # equals one FAS cycle on phi up to FP32 rounding, so after FMG + 3 cycles the
    # mixed iterate stays within ~1e-6 of the reference's FP64 iterate; an FP32 cycle
    # that started from stale values instead of zero would leave the previous step's
    # correction in it and miss that by orders of magnitude
    if case == "dirichlet_neumann_2d":
        dom = W.Domain(2, [128, 96], [0, 0], [1, 0.75], [W.DIRICHLET, W.NEUMANN, W.NEUMANN, W.DIRICHLET],
                       [0.5, 0.2, -0.3, 1.0])
        g = W.Gaussians(np.array([[0.4, 0.3]]), np.array([5.0]), np.array([0.1]))
        w = W.Workload(case, [dom], bs=16, rhs=lambda i, lay: g(W.cell_centres(lay, dom)))
    elif case == "periodic_3d":
        w = W.config2(n=64)
    elif case == "forest_equal":
        w = W.config5(sizes=(48, 48))
    elif case == "forest_unequal":
        w = W.config5(sizes=(32, 64))
    else:
        w = W.config3(nested=False, base=32)
    t = gpu_tree(w, precision=1, ir_vcycles=1)   # one FP32 V-cycle per refinement step
    refs = oracle_trees(w)
    f, e = inputs(w, t)
    if w.variable_eps:
        t.set_eps(np.concatenate(e))
        for o, ei in zip(refs, e):
            o.set_eps(ei)
    t.set_rhs(np.concatenate(f))
    for o, fi in zip(refs, f):
        o.set_rhs(fi)
    t.fmg()
    t.vcycle(3)
    for o in refs:
        o.fmg()
        o.vcycle(3)
    errs = [rel_err(p, o.get_phi(), case == "periodic_3d") for p, o in zip(split(t, t.get_phi()), refs)]
    print(case, "mixed vs FP64 iterates", errs, flush=True)
    assert max(errs) < 2e-6
