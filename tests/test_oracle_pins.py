"""Pins of the reference solver's arithmetic against what the mathematics fixes.

Each test is chosen so that a plausible slip in the oracle (a dropped term, a wrong
sign, index or weight, a transposed operand) fails it:

- closed forms: the sine eigenvector with the Dirichlet reflection ghost (2D, config 1
  of the benchmark), periodic cosines in 2D/3D, anisotropic spacing, exact second
  differences of quadratics (operator of eq. poisson-2d and its 3D form);
- O(h^2) convergence of the discrete solution to the continuum one;
- dense direct solves of the composite operator on tiny uniform and refined trees: the
  multigrid fixed point must equal the direct solution;
- V-cycle contraction;
- the coarse-fine flux identity (Sec. 2.6, corrected form: the sum over the fine faces
  of (c - g) equals 2^(d-2) (D - B)) and global conservation on periodic refined trees;
- exactness of the coarse-fine ghost rule, the restriction and the prolongation
  (eq. interp_2d / interp_3d) for linear functions;
- adjoint gradients against central finite differences.
"""
import itertools

import numpy as np
import pytest

from oracle import DIRICHLET, NEUMANN, PERIODIC, OracleTree
from paper_1901_11370_amd import workloads as W


def _centres(t, dom):
    return W.cell_centres(t.leaf_layout(), dom)


def _dom(dim, n, bc, lo=None, hi=None):
    lo = lo or [0.0] * dim
    hi = hi or [1.0] * dim
    return W.Domain(dim, list(n), list(lo), list(hi), [bc] * (2 * dim))


def _tree(dom, bs, **kw):
    return OracleTree(dom.dim, dom.base_cells, dom.lo, dom.hi, dom.bc_kind, bs=bs, **kw)


# ------------------------------------------------------------- closed forms
def test_config1_sine_closed_form_and_order():
    errs = {}
    for n in (64, 128):
        dom = _dom(2, (n, n), DIRICHLET)
        t = _tree(dom, 16)
        x = _centres(t, dom)
        t.set_rhs(W.sine_rhs_2d(x))
        for _ in range(16):
            t.vcycle()
        h = 1.0 / n
        s = np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1])
        # sin(pi x) sin(pi y) is an eigenvector of the discrete operator with the
        # reflection ghost, eigenvalue -8 sin^2(pi h/2)/h^2
        phi_h = (np.pi ** 2 * h ** 2 / (4.0 * np.sin(np.pi * h / 2) ** 2)) * s
        phi = t.get_phi()
        assert np.abs(phi - phi_h).max() <= 1e-12 * np.abs(phi_h).max()
        errs[n] = np.abs(phi - s).max()
    ratio = errs[64] / errs[128]
    assert 3.9 < ratio < 4.1
    assert errs[128] == pytest.approx(np.pi ** 2 / (12 * 128 ** 2), rel=0.01)


@pytest.mark.parametrize("dim,n,k,hi", [
    (2, (32, 32), (1, 2), (1.0, 1.0)),
    (2, (64, 32), (2, 1), (2.0, 1.0)),      # anisotropic h: hx = 1/32, hy = 1/32 -> use (2,1)
    (2, (64, 64), (3, 1), (2.0, 1.0)),      # anisotropic: hx = 1/32, hy = 1/64
    (3, (32, 32, 32), (1, 2, 3), (1.0, 1.0, 1.0)),
    (3, (32, 16, 32), (1, 1, 2), (1.0, 1.0, 2.0)),
])
def test_periodic_cosine_closed_form(dim, n, k, hi):
    dom = _dom(dim, n, PERIODIC, hi=list(hi))
    bs = 8
    t = _tree(dom, bs)
    x = _centres(t, dom)
    arg = sum(k[d] * x[:, d] / hi[d] for d in range(dim))
    f = np.cos(2 * np.pi * arg)
    t.set_rhs(f)
    t.solve(rel_tol=1e-13, max_cycles=40)
    h = [hi[d] / n[d] for d in range(dim)]
    lam = -sum(4.0 / h[d] ** 2 * np.sin(np.pi * k[d] * h[d] / hi[d]) ** 2 for d in range(dim))
    phi = t.get_phi()
    phi -= phi.mean()
    assert np.abs(phi - f / lam).max() <= 1e-11 * np.abs(f / lam).max()


@pytest.mark.parametrize("var_eps", [False, True])
def test_operator_exact_on_quadratics(var_eps):
    dom = _dom(3, (16, 16, 16), DIRICHLET, hi=[1.0, 2.0, 1.0])
    t = _tree(dom, 8, variable_eps=var_eps)
    lay = t.leaf_layout()
    x = W.cell_centres(lay, dom)
    if var_eps:
        t.set_eps(np.full(t.n_leaf, 3.0))
    phi = x[:, 0] ** 2 + 2 * x[:, 1] ** 2 + 3 * x[:, 2] ** 2 - x[:, 0] * x[:, 1]
    out = t.apply(phi)
    interior = np.all((lay[:, 1:] > 0) & (lay[:, 1:] < 15), axis=1)
    want = (2 + 4 + 6) * (3.0 if var_eps else 1.0)
    assert np.abs(out[interior] - want).max() < 1e-9 * want


def test_neumann_closed_form_1d_profile():
    # phi'' = f in x with phi'(0) = b0, phi'(1) = b1 and periodic y: the discrete
    # solution of a quadratic is exact up to a constant (second differences of
    # quadratics are exact, the Neumann ghost reproduces a linear slope at the face)
    n = 32
    dom = W.Domain(2, [n, 8], [0.0, 0.0], [1.0, 0.25], [NEUMANN, NEUMANN, PERIODIC, PERIODIC],
                   [-1.0, 1.0, 0.0, 0.0])
    t = OracleTree(2, dom.base_cells, dom.lo, dom.hi, dom.bc_kind, bc_value=dom.bc_value, bs=8)
    x = _centres(t, dom)
    t.set_rhs(np.full(t.n_leaf, 2.0))      # phi = x^2 - x + c: phi'' = 2, phi'(0) = -1, phi'(1) = 1
    hist = t.solve(rel_tol=1e-13, max_cycles=80)
    assert hist[-1] <= 1e-12
    phi = t.get_phi()
    exact = x[:, 0] ** 2 - x[:, 0]
    d = phi - exact
    # the ghost phi_g = phi_i - h b is the one-sided difference at the face; for a
    # quadratic the cell-centred scheme is exact up to a constant shift
    assert np.ptp(d) < 1e-9


# ------------------------------------------------------- dense direct solves
def _dense(t):
    n = t.n_leaf
    A = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        A[:, j] = t.apply(e)
    return A


def _refine_one(target):
    def pred(dom, level, origin, bs):
        return level == 0 and tuple(origin[:len(target)]) == target
    return pred


@pytest.mark.parametrize("case", ["uniform2d", "amr2d", "amr2d_periodic", "amr3d", "uniform3d_var"])
def test_dense_direct_solve_matches_fixed_point(case):
    rng = np.random.default_rng(7)
    if case == "uniform2d":
        dom, bs, kw = _dom(2, (8, 8), DIRICHLET), 4, {}
    elif case == "amr2d":
        dom, bs, kw = _dom(2, (8, 8), DIRICHLET), 4, dict(max_refine=1, refine=_refine_one((4, 0)))
    elif case == "amr2d_periodic":
        dom, bs, kw = _dom(2, (12, 8), PERIODIC), 4, dict(max_refine=1, refine=_refine_one((4, 4)))
    elif case == "amr3d":
        dom, bs, kw = _dom(3, (4, 4, 4), DIRICHLET), 2, dict(max_refine=1, refine=_refine_one((2, 0, 2)))
    else:
        dom, bs, kw = _dom(3, (4, 4, 4), DIRICHLET), 2, dict(variable_eps=True)
    t = _tree(dom, bs, **kw)
    if case == "uniform3d_var":
        t.set_eps(np.exp(rng.normal(size=t.n_leaf)))
    A = _dense(t)
    f = rng.normal(size=t.n_leaf)
    if case == "amr2d_periodic":
        vol = np.prod(W.cell_widths(t.leaf_layout(), dom), axis=1)
        f -= np.sum(vol * f) / np.sum(vol)
        phi_d = np.linalg.lstsq(A, f, rcond=None)[0]
    else:
        phi_d = np.linalg.solve(A, f)
    t.set_phi(np.zeros(t.n_leaf))
    t.set_rhs(f)
    for _ in range(60):
        t.vcycle()
    phi = t.get_phi()
    if case == "amr2d_periodic":
        vol = np.prod(W.cell_widths(t.leaf_layout(), dom), axis=1)
        phi -= np.sum(vol * phi) / np.sum(vol)
        phi_d -= np.sum(vol * phi_d) / np.sum(vol)
    assert np.abs(phi - phi_d).max() <= 1e-12 * np.abs(phi_d).max()
    if case.startswith("uniform"):
        assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()   # symmetric without refinement


def test_dense_operator_is_conservative_on_periodic_refined_tree():
    # sum over leaves of vol_i (L v)_i = 0 for every v: the columns of A weighted by
    # the cell volumes vanish (divergence theorem with matching fluxes, Sec. 2.6)
    dom = _dom(2, (12, 8), PERIODIC)
    t = _tree(dom, 4, max_refine=2, refine=lambda d, lev, o, bs: (lev == 0 and o[0] == 4 and o[1] == 4) or
              (lev == 1 and o[0] == 8 and o[1] == 8))
    A = _dense(t)
    vol = np.prod(W.cell_widths(t.leaf_layout(), dom), axis=1)
    assert np.abs(vol @ A).max() <= 1e-12 * np.abs(A).max() * vol.max()


# ---------------------------------------------------------- contraction
@pytest.mark.parametrize("case", ["config1", "periodic3d", "amr3d"])
def test_vcycle_contraction(case):
    if case == "config1":
        dom = _dom(2, (128, 128), DIRICHLET)
        t = _tree(dom, 16)
        t.set_rhs(W.sine_rhs_2d(_centres(t, dom)))
        bound = 0.15
    elif case == "periodic3d":
        w = W.config2(n=32)
        dom = w.domains[0]
        t = _tree(dom, 8)
        t.set_rhs(w.rhs(0, t.leaf_layout()))
        bound = 0.15
    else:
        dom = _dom(3, (16, 16, 16), DIRICHLET)
        t = _tree(dom, 8, max_refine=2,
                  refine=lambda d, lev, o, bs: all(4 * 2 ** lev <= oi < 12 * 2 ** lev for oi in o))
        g = W.Gaussians(np.array([[0.5, 0.5, 0.5]]), np.array([1.0]), np.array([0.05]))
        t.set_rhs(g(_centres(t, dom)))
        bound = 0.25
    res = [t.residual_norm()[0]]
    for _ in range(8):
        t.vcycle()
        res.append(t.residual_norm()[0])
    rates = [res[i + 1] / res[i] for i in range(3, 8)]
    assert max(rates) < bound


# ---------------------------------------------- refinement boundary identities
def _level_maps(t):
    maps = []
    for l in range(t.num_levels):
        bs = t.level_info(l)[0]
        m = {}
        for ib in range(t.level_nblocks(l)):
            org, _ = t.block_meta(l, ib)
            m[tuple(o // bs if (i < t.dim) else 0 for i, o in enumerate(org))] = ib
        maps.append(m)
    return maps


def _amr_tree(dim, periodic=False):
    bc = PERIODIC if periodic else DIRICHLET
    if dim == 2:
        dom = _dom(2, (16, 16), bc)
        pred = lambda d, lev, o, bs: (lev == 0 and 4 <= o[0] < 12 and 4 <= o[1] < 8) or (lev == 1 and o[0] == 12 and o[1] == 8)
        return dom, _tree(dom, 4, max_refine=2, refine=pred)
    dom = _dom(3, (8, 8, 8), bc)
    pred = lambda d, lev, o, bs: (lev == 0 and o[0] == 4 and o[1] == 0 and o[2] == 4) or (lev == 1 and o == (8, 0, 8))
    return dom, _tree(dom, 4, max_refine=2, refine=pred)


def _fine_faces(t):
    """(level, block, d, side, coarse block) for every refinement-boundary face."""
    maps = _level_maps(t)
    out = []
    dim = t.dim
    for l in range(t.base_level + 1, t.num_levels):
        bs, ncell, _ = t.level_info(l)
        nb = [ncell[d] // bs for d in range(dim)]
        for key, ib in maps[l].items():
            for d in range(dim):
                for side in (0, 1):
                    nbk = list(key)
                    nbk[d] += 1 if side else -1
                    if nbk[d] < 0 or nbk[d] >= nb[d]:
                        continue
                    if tuple(nbk) in maps[l]:
                        continue
                    ck = tuple(x // 2 for x in nbk[:dim]) + (0,) * (3 - dim)
                    ck = ck if dim == 3 else ck[:2] + (0,)
                    out.append((l, ib, d, side, maps[l - 1][tuple(ck[:3]) if dim == 3 else ck[:2] + (0,)]))
    return out


def _take(arr, dim, d, layer, tang):
    """arr is padded, indexed [k][j][i] (3D) or [j][i] (2D); layer is the padded index
    along d, tang the padded indices along the other axes in increasing axis order."""
    idx = [None] * dim
    others = [a for a in range(dim) if a != d]
    idx[d] = layer
    for a, v in zip(others, tang):
        idx[a] = v
    return arr[tuple(reversed(idx))]


@pytest.mark.parametrize("dim", [2, 3])
def test_flux_identity_at_refinement_faces(dim):
    dom, t = _amr_tree(dim)
    rng = np.random.default_rng(11)
    t.set_phi(rng.normal(size=t.n_leaf))          # parents become the mean of children
    faces = _fine_faces(t)
    assert faces
    checked = 0
    for l, ib, d, side, qb in faces:
        bs = t.level_info(l)[0]
        v = t.block_field(l, ib, "v")
        org, _ = t.block_meta(l, ib)
        qorg, _ = t.block_meta(l - 1, qb)
        vq = t.block_field(l - 1, qb, "v")
        others = [a for a in range(dim) if a != d]
        gl, cl, c2l = (bs + 1, bs, bs - 1) if side else (0, 1, 2)
        # coarse cells along the face: pairs of fine cells in each tangential axis
        for tc in itertools.product(range(bs // 2), repeat=dim - 1):
            s_cg, s_D = 0.0, 0.0
            for sub in itertools.product((0, 1), repeat=dim - 1):
                tang = [1 + 2 * a + b for a, b in zip(tc, sub)]
                c = _take(v, dim, d, cl, tang)
                g = _take(v, dim, d, gl, tang)
                c2 = _take(v, dim, d, c2l, tang)
                s_cg += c - g
                s_D += c + c2
            D = s_D / 2 ** dim
            # coarse cell B across the face
            gidx = [0] * 3
            gidx[d] = (org[d] + (bs if side else -1)) // 2
            for a, v0 in zip(others, tc):
                gidx[a] = (org[a] + 2 * v0) // 2
            loc = [gidx[a] - qorg[a] + 1 for a in range(dim)]
            B = vq[tuple(reversed(loc))]
            # orientation: with the fine side at larger x_d, (D - B) is the coarse
            # difference across the face and (c - g) the fine ones
            assert s_cg == pytest.approx(2 ** (dim - 2) * (D - B), abs=1e-12)
            checked += 1
    assert checked > 0


@pytest.mark.parametrize("dim", [2, 3])
def test_global_conservation_periodic_refined(dim):
    dom, t = _amr_tree(dim, periodic=True)
    rng = np.random.default_rng(5)
    out = t.apply(rng.normal(size=t.n_leaf))
    vol = np.prod(W.cell_widths(t.leaf_layout(), dom), axis=1)
    assert abs(np.sum(vol * out)) <= 1e-12 * np.sum(vol * np.abs(out))


@pytest.mark.parametrize("dim", [2, 3])
def test_linear_exactness_of_ghosts_restriction(dim):
    dom, t = _amr_tree(dim)
    coef = np.array([0.3, -1.2, 0.7][:dim])
    lay = t.leaf_layout()
    x = W.cell_centres(lay, dom)
    t.set_phi(1.5 + x @ coef)
    maps = _level_maps(t)
    nchecked = ncf = 0
    for l in range(t.num_levels):
        bs, ncell, nb = t.level_info(l)
        h = 1.0 / ncell[0]
        for ib in range(nb):
            org, _ = t.block_meta(l, ib)
            v = t.block_field(l, ib, "v")
            for idx in itertools.product(range(-1, bs + 1), repeat=dim):
                nout = sum(1 for i in idx if i < 0 or i >= bs)
                if nout > 1:
                    continue                      # corners are never filled
                g = [org[a] + idx[a] for a in range(dim)]
                if any(gi < 2 or gi >= ncell[a] - 2 for a, gi in enumerate(g)):
                    continue                      # reflection ghosts enter near the boundary
                want = 1.5 + sum(coef[a] * (g[a] + 0.5) * h for a in range(dim))
                got = v[tuple(reversed([i + 1 for i in idx]))]
                assert got == pytest.approx(want, abs=1e-12)
                nchecked += 1
                key = tuple(gi // bs for gi in g) + (0,) * (3 - dim)
                ncf += nout == 1 and key[:3] not in maps[l]
    assert nchecked > 300 and ncf > 20


@pytest.mark.parametrize("dim", [2, 3])
def test_prolongation_linear_exactness(dim):
    dom = _dom(dim, (8,) * dim, DIRICHLET)
    t = _tree(dom, 4)
    lt = t.num_levels - 1
    coef = np.array([0.9, -0.4, 0.25][:dim])
    bsc, ncc, nbc = t.level_info(lt - 1)
    hc = 1.0 / ncc[0]
    for ib in range(nbc):
        org, _ = t.block_meta(lt - 1, ib)
        shape = (bsc + 2,) * dim
        vals = np.zeros(shape)
        for idx in itertools.product(range(-1, bsc + 1), repeat=dim):
            g = [org[a] + idx[a] for a in range(dim)]
            vals[tuple(reversed([i + 1 for i in idx]))] = 2.0 + sum(coef[a] * (g[a] + 0.5) * hc for a in range(dim))
        t.set_block_field(lt - 1, ib, "v", vals)
        t.set_block_field(lt - 1, ib, "vold", np.zeros(shape))
    bs, nc, nb = t.level_info(lt)
    for ib in range(nb):
        t.set_block_field(lt, ib, "v", np.zeros((bs + 2,) * dim))
    t.correct_level(lt)
    x = W.cell_centres(t.leaf_layout(), dom)
    want = 2.0 + x @ coef
    assert np.abs(t.get_phi() - want).max() < 1e-13


# ------------------------------------------------------------------ adjoint
def test_adjoint_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    dom = _dom(3, (16, 16, 16), DIRICHLET)
    t = _tree(dom, 8, variable_eps=True)
    lay = t.leaf_layout()
    x = W.cell_centres(lay, dom)
    eps = np.exp(0.5 * np.sin(2 * np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1]) + 0.3 * x[:, 2])
    f = W.Gaussians(np.array([[0.4, 0.5, 0.6], [0.7, 0.3, 0.4]]), np.array([1.0, -0.7]),
                    np.array([0.15, 0.1]))(x)
    tgt = 1e-3 * np.prod(np.sin(np.pi * x), axis=1)

    def solve(e, ff):
        t.set_eps(e)
        t.set_rhs(ff)
        t.set_phi(np.zeros(t.n_leaf))
        hist = t.solve(rel_tol=1e-14, max_cycles=40)
        for _ in range(2):
            t.vcycle()
        return t.get_phi()

    phi = solve(eps, f)
    lam = solve(eps, phi - tgt)
    g_eps = t.face_gradient(phi, lam)
    g_f = lam

    def J_diff(pp, pm):
        return 0.5 * np.sum((pp - pm) * (pp + pm - 2 * tgt))

    delta = 1e-6
    big = np.flatnonzero(np.abs(g_eps) >= 1e-2 * np.abs(g_eps).max())
    for k in rng.choice(big, 4, replace=False):
        e = eps.copy(); e[k] += delta
        pp = solve(e, f)
        e[k] -= 2 * delta
        pm = solve(e, f)
        fd = J_diff(pp, pm) / (2 * delta)
        assert fd == pytest.approx(g_eps[k], rel=2e-6)
    bigf = np.flatnonzero(np.abs(g_f) >= 1e-2 * np.abs(g_f).max())
    for k in rng.choice(bigf, 3, replace=False):
        ff = f.copy(); ff[k] += delta
        pp = solve(eps, ff)
        ff[k] -= 2 * delta
        pm = solve(eps, ff)
        fd = J_diff(pp, pm) / (2 * delta)
        assert fd == pytest.approx(g_f[k], rel=2e-6)


def test_dirichlet_nonzero_values_linear_solution():
    # phi = 1 + 2x solves phi'' = 0 with phi(0) = 1, phi(1) = 3; the reflection ghost
    # 2a - phi_i puts the face value exactly at the face, so the discrete solution is
    # the linear function at cell centres (y periodic).
    dom = W.Domain(2, [32, 16], [0.0, 0.0], [1.0, 0.5], [DIRICHLET, DIRICHLET, PERIODIC, PERIODIC],
                   [1.0, 3.0, 0.0, 0.0])
    t = OracleTree(2, dom.base_cells, dom.lo, dom.hi, dom.bc_kind, bc_value=dom.bc_value, bs=8)
    x = _centres(t, dom)
    t.set_rhs(np.zeros(t.n_leaf))
    t.solve(rel_tol=1e-14, max_cycles=60)
    assert np.abs(t.get_phi() - (1 + 2 * x[:, 0])).max() < 1e-12


def test_conservation_with_coefficient_jump_on_refinement_face():
    # eps = 4 on the refined patch and 1 elsewhere, the jump on the refinement
    # boundary.  Flux matching across the coarse-fine faces needs the same face
    # coefficient on both sides; with the ghost carrying the coarse cell's eps both
    # sides use the harmonic mean of 1 and 4, and sum vol (L v) vanishes.
    dom = _dom(2, (16, 16), PERIODIC)
    t = _tree(dom, 4, max_refine=1, variable_eps=True,
              refine=lambda d, lev, o, bs: lev == 0 and 4 <= o[0] < 12 and 4 <= o[1] < 8)
    lay = t.leaf_layout()
    t.set_eps(np.where(lay[:, 0] == 1, 4.0, 1.0))
    out = t.apply(np.random.default_rng(2).normal(size=t.n_leaf))
    vol = np.prod(W.cell_widths(lay, dom), axis=1)
    assert abs(np.sum(vol * out)) <= 1e-12 * np.sum(vol * np.abs(out))


def test_adjoint_gradient_boundary_cells():
    # cells next to the Dirichlet boundary carry the one-sided boundary term
    dom = _dom(3, (16, 16, 16), DIRICHLET)
    t = _tree(dom, 8, variable_eps=True)
    lay = t.leaf_layout()
    x = W.cell_centres(lay, dom)
    eps = 1.0 + 0.5 * x[:, 0] + 0.25 * x[:, 1] * x[:, 2]
    f = np.ones(t.n_leaf)
    tgt = np.zeros(t.n_leaf)

    def solve(e, ff):
        t.set_eps(e)
        t.set_rhs(ff)
        t.set_phi(np.zeros(t.n_leaf))
        t.solve(rel_tol=1e-14, max_cycles=40)
        t.vcycle(2)
        return t.get_phi()

    phi = solve(eps, f)
    lam = solve(eps, phi - tgt)
    g = t.face_gradient(phi, lam)
    edge = np.flatnonzero(np.any((lay[:, 1:] == 0) | (lay[:, 1:] == 15), axis=1))
    delta = 1e-6
    for k in edge[np.argsort(-np.abs(g[edge]))[:3]]:
        e = eps.copy(); e[k] += delta
        pp = solve(e, f)
        e[k] -= 2 * delta
        pm = solve(e, f)
        fd = 0.5 * np.sum((pp - pm) * (pp + pm - 2 * tgt)) / (2 * delta)
        assert fd == pytest.approx(g[k], rel=2e-6)


def _global_gsrb_2d(n, h, f, steps, a=0.0):
    """Red-black Gauss-Seidel on one whole n x n grid with reflection ghosts (brute
    force, tiny sizes): red = even i + j first, ghosts refreshed after each colour."""
    v = np.zeros((n + 2, n + 2))
    for _ in range(steps):
        for colour in (0, 1):
            v[0, :] = 2 * a - v[1, :]; v[-1, :] = 2 * a - v[-2, :]
            v[:, 0] = 2 * a - v[:, 1]; v[:, -1] = 2 * a - v[:, -2]
            old = v.copy()
            for j in range(n):
                for i in range(n):
                    if (i + j) % 2 != colour:
                        continue
                    s = old[j + 1, i] + old[j + 1, i + 2] + old[j, i + 1] + old[j + 2, i + 1]
                    v[j + 1, i + 1] = (s / h ** 2 - f[j, i]) / (4 / h ** 2)
    return v[1:-1, 1:-1]


@pytest.mark.parametrize("n", [5, 7])
def test_blocked_gsrb_equals_global_sweep(n):
    # An odd base grid of 1-cell blocks has a single level, so a V-cycle is only the
    # coarsest-grid smoother; the colour must follow global, not block-local, indices.
    bs = 1
    dom = _dom(2, (n, n), DIRICHLET)
    t = _tree(dom, bs)
    assert t.num_levels == 1
    steps = 5
    t.set_params(n_down=0, n_up=0, n_max=steps, abs_tol=0.0, rel_tol=0.0)
    rng = np.random.default_rng(1)
    f = rng.normal(size=(n, n))
    lay = t.leaf_layout()
    t.set_rhs(f[lay[:, 2], lay[:, 1]])
    t.vcycle()
    want = _global_gsrb_2d(n, 1.0 / n, f, steps)
    got = np.zeros((n, n))
    got[lay[:, 2], lay[:, 1]] = t.get_phi()
    assert t.last_coarse_steps == steps
    assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()
