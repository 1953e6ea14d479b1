"""Parity at the benchmark sizes, in the configuration bench.py times (FMG then
V(2,2) cycles, captured graphs): every leaf value of the 256^3 periodic grid and of
the literal-rule AMR tree against the reference solver after the same cycles."""
import numpy as np
import pytest

from helpers import gpu_tree, inputs, oracle_trees, rel_err
from paper_1901_11370_amd import workloads as W

pytestmark = pytest.mark.gpu


def _fmg_v(w, n_v, remove_mean=False, setup=None, **params):
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
    if setup:
        setup(o)
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
    # mixed form: an FP32 FMG refinement step and two FP32 V-cycle steps (one V-cycle
    # each) against the FP64 reference after FMG + 2 V-cycles: a refinement step equals
    # one FAS cycle up to FP32 rounding of the correction (measured 1.4e-9)
    err, g, o = _fmg_v(W.config2(n=256), 2, remove_mean=True, precision=1, ir_vcycles=1)
    assert err <= 1e-7


def test_dirichlet_box_mixed_against_fp64_reference():
    # a 256 x 256 x 128 box (cubic cells) with phi = 0 on every face: its 128 x 128 x 64
    # level holds 256 parent blocks, so the FP32 cycles compute the FAS right-hand side
    # there with the LDS-staged kernel, next to physical-boundary ghosts; the mixed form's
    # FMG step and two one-V-cycle steps against the FP64 reference's FMG + 2 V-cycles
    rng = np.random.default_rng(21)
    g = W.Gaussians(rng.uniform(0.1, 0.9, (8, 3)) * np.array([1.0, 1.0, 0.5]),
                    np.where(rng.random(8) < 0.5, -1.0, 1.0), np.full(8, 0.03))
    dom = W.Domain(3, [256, 256, 128], [0.0, 0.0, 0.0], [1.0, 1.0, 0.5], [W.DIRICHLET] * 6)
    w = W.Workload("dirichlet_box_256x256x128", [dom], rhs=lambda i, lay: g(W.cell_centres(lay, dom)))
    err, g_norm, o_norm = _fmg_v(w, 2, precision=1, ir_vcycles=1)
    assert err <= 1e-7


def test_amr_literal_full_size():
    err, g, o = _fmg_v(W.config3(nested=False), 1)
    assert err <= 1e-11 and abs(g - o) <= 1e-6 * o


def test_helmholtz_256_full_size():
    # the Helmholtz form on the benchmark grid (lambda = 100, the helmholtz report line)
    err, g, o = _fmg_v(W.config2(n=256), 1, setup=lambda o: o.set_lambda(100.0), helmholtz_lambda=100.0)
    assert err <= 1e-11 and abs(g - o) <= 1e-6 * o


def test_divb_clean_256_full_size():
    # the divergence-cleaning report line's configuration: 256^3 periodic field, fourth-
    # order div B, FMG + 1 V-cycle, projection with the energy fix
    import torch
    from oracle import divb
    w = W.divb_periodic(256)
    d = w.domains[0]
    t = gpu_tree(w)
    B = W.field_loop_B(d, W.cell_centres(t.leaf_layout()[:, 1:], d))
    e = 1.0 + 0.5 * np.sum(B * B, axis=0)
    Bd, ed = torch.from_numpy(B.copy()).cuda(), torch.from_numpy(e.copy()).cuda()
    t.set_phi(np.zeros(t.n_leaf))
    t.divb_rhs(Bd, 4)
    t.fmg()
    t.vcycle(1)
    t.divb_project(Bd, ed)
    phi = t.get_phi()
    Bg, eg = Bd.cpu().numpy(), ed.cpu().numpy()
    del t, Bd, ed
    o = oracle_trees(w)[0]
    o.set_rhs(divb.divergence(o, B, 4))
    o.fmg()
    o.vcycle(1)
    po = o.get_phi()
    Bn, en = divb.project(o, B, po, e)
    corr = np.abs(Bn - B).max()
    err = rel_err(phi, po, True)
    print("divb 256^3: phi", err, "B", np.abs(Bg - Bn).max() / corr, flush=True)
    assert err <= 1e-11
    assert np.abs(Bg - Bn).max() <= 1e-9 * corr
    assert np.abs(eg - en).max() <= 1e-9 * corr * np.abs(B).max() + 4e-16 * np.abs(e).max()


def test_amr_nested_full_size_residual_by_reference():
    # the nested AMR tree of the amr-nested report line (115,867,648 leaf cells) solved to
    # 1e-10 on the GPU; the reference solver builds the same tree, takes the GPU's phi and
    # evaluates the composite residual itself (too large for the reference to run cycles)
    import torch
    w = W.config3(nested=True)
    t = gpu_tree(w)
    f, _ = inputs(w, t)
    t.set_rhs(torch.from_numpy(f[0]).cuda())
    cycles, rc = t.solve(rel_tol=1e-10, max_cycles=20)
    g_rel, g_l2 = t.residual_norm()
    phi = t.get_phi()
    del t
    o = oracle_trees(w)[0]
    o.set_rhs(f[0])
    o.set_phi(phi)
    o_rel, o_l2 = o.residual_norm()
    print("nested full size: cycles", cycles, "GPU residual", g_rel, g_l2, "reference on the GPU's phi", o_rel, o_l2,
          flush=True)
    assert rc == 0 and cycles <= 12
    assert o_rel <= 1e-10 * 1.01 and abs(o_rel - g_rel) <= 1e-3 * g_rel and abs(o_l2 - g_l2) <= 1e-3 * g_l2
