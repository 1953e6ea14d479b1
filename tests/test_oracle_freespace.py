"""Pins of the reference free-space boundary conditions (Sec. 2.8) against what the paper
and the mathematics fix: the closed-form solution of the Sec. 3.2 test (eq. gauss-sol),
the total charge of its source, exactness of linear interpolation on linear data, the
equivalence of a folded right-hand side with the solver's own constant Dirichlet
faces, and the second-order convergence the paper reports for this test."""
import numpy as np
import pytest

from oracle import OracleTree, DIRICHLET
from oracle import freespace as FS
from paper_1901_11370_amd import workloads as W


def _tree(n, bs=16, bc_value=0.0):
    return OracleTree(3, (n, n, n), (-0.5,) * 3, (0.5,) * 3, [DIRICHLET] * 6, bc_value=[bc_value] * 6, bs=bs)


def _rhs(t, w):
    return w.rhs(0, t.leaf_layout())


def test_charges_sum_to_the_source_integral():
    # the Gaussian of eq. gauss-rhs integrates to -1; it is negligible at the faces
    w = W.freespace_gauss((32,))
    t = _tree(32)
    for k in (0, 1, 2, 3):
        q, hc = FS.coarse_charges(t, _rhs(t, w), k)
        assert q.shape == (32 >> k,) * 3
        assert np.allclose(hc, 1.0 / (32 >> k))
        assert abs(q.sum() + 1.0) < 1e-9


def _plane_error(t, f, k, r0=(0.0, 0.0, 0.0)):
    pl, hc = FS.planes(t, f, k)
    err = 0.0
    for face in range(6):
        pts, shp = FS.plane_points(t, hc, face)
        exact = FS.gauss_sol(pts[:, 0], pts[:, 1], pts[:, 2], r0=r0).reshape(shp)
        err = max(err, np.max(np.abs(pl[face] - exact)) / np.max(np.abs(exact)))
    return err


def test_planes_match_the_closed_form_solution():
    # the potential of the charges on the boundary planes (ghost positions included)
    # against eq. gauss-sol.  Leaf samples as charges (k = 0) form a midpoint sum of a
    # smooth source, exact to rounding; coarse charges (mean of the leaf samples at the
    # coarse centre) converge fast with the coarse spacing.  A wrong constant, sign,
    # distance or position fails at once.
    w = W.freespace_gauss((32,))
    t = _tree(32)
    f = _rhs(t, w)
    assert _plane_error(t, f, 0) < 1e-10
    e1 = _plane_error(t, f, 1)
    assert e1 < 1e-5
    w64 = W.freespace_gauss((64,))
    t64 = _tree(64)
    assert _plane_error(t64, _rhs(t64, w64), 1) < e1 / 10


def test_plane_orientation_with_an_off_centre_source():
    # a source off the centre makes the six faces differ; each face must see its own
    # side (a swapped face or a transposed plane fails)
    r0 = (0.12, -0.07, 0.05)
    w = W.freespace_gauss((32,), offsets=[r0])
    t = _tree(32)
    f = _rhs(t, w)
    assert _plane_error(t, f, 0, r0) < 1e-6   # the source tail cut at the nearest face
    assert _plane_error(t, f, 1, r0) < 3e-5


def test_interpolation_is_exact_on_linear_planes():
    t = _tree(32)
    h = 1.0 / 32
    for k in (1, 2, 3):
        hc = np.full(3, h * (1 << k))
        for face in range(6):
            a, t1, t2 = FS._inplane(face)
            pts, shp = FS.plane_points(t, hc, face)
            lin = lambda p1, p2: 0.3 + 1.7 * p1 - 0.9 * p2
            plane = lin(pts[:, t1], pts[:, t2]).reshape(shp)
            got = FS.interpolate(t, plane, hc, face)
            c = -0.5 + (np.arange(32) + 0.5) * h
            C2, C1 = np.meshgrid(c, c, indexing="ij")
            assert np.max(np.abs(got - lin(C1, C2))) < 1e-13


def test_fold_equals_the_solver_dirichlet_faces():
    # a different constant value on every face: folding them into f and solving with
    # homogeneous faces gives the solution of the solver's own Dirichlet faces
    vals, n = [0.3, -0.2, 0.5, 0.1, -0.4, 0.25], 32
    rng = np.random.default_rng(5)
    t_ref = OracleTree(3, (n, n, n), (-0.5,) * 3, (0.5,) * 3, [DIRICHLET] * 6, bc_value=vals, bs=16)
    f = rng.standard_normal(t_ref.n_leaf)
    t_ref.set_rhs(f)
    t_ref.solve(rel_tol=1e-13, max_cycles=40)
    ref = t_ref.get_phi()
    t0 = _tree(n)
    bv = [np.full((n, n), a) for a in vals]
    t0.set_rhs(FS.fold(t0, f, bv))
    t0.solve(rel_tol=1e-13, max_cycles=40)
    assert np.max(np.abs(t0.get_phi() - ref)) < 1e-11 * np.max(np.abs(ref))


def test_boundary_values_at_the_leaf_faces():
    # the values of every face at its leaf face centres, placed here from the grid alone,
    # against eq. gauss-sol for an off-centre source (a face computed on the opposite
    # side or a transposed face fails)
    r0 = (0.12, -0.07, 0.05)
    n = 32
    w = W.freespace_gauss((n,), offsets=[r0])
    t = _tree(n)
    f = _rhs(t, w)
    c = -0.5 + (np.arange(n) + 0.5) / n
    C2, C1 = np.meshgrid(c, c, indexing="ij")   # [j2, j1]: lower in-plane axis fastest
    for k, tol in ((0, 1e-6), (1, 1e-2)):   # k = 1: linear interpolation between 1/16 planes
        bv = FS.boundary_values(t, f, k)
        for face in range(6):
            a = face // 2
            t1, t2 = [b for b in range(3) if b != a]
            P = [None] * 3
            P[a] = np.full_like(C1, 0.5 if face & 1 else -0.5)
            P[t1], P[t2] = C1, C2
            exact = FS.gauss_sol(P[0], P[1], P[2], r0=r0)
            assert np.max(np.abs(bv[face] - exact)) < tol * np.max(np.abs(exact)), (k, face)


def _error(n, k):
    w = W.freespace_gauss((n,))
    t = _tree(n)
    lay = t.leaf_layout()
    f = w.rhs(0, lay)
    ff, _ = FS.freespace_rhs(t, f, k)
    t.set_rhs(ff)
    t.solve(rel_tol=1e-10, max_cycles=40)
    x = W.cell_centres(lay, w.domains[0])
    e = t.get_phi() - FS.gauss_sol(x[:, 0], x[:, 1], x[:, 2])
    return np.sqrt(np.mean(e * e)), np.max(np.abs(e))


def test_second_order_convergence_to_the_free_space_solution():
    # the paper's Fig. free-space-error: second-order convergence of the error
    l2a, maxa = _error(32, 1)
    l2b, maxb = _error(64, 1)
    assert 3.3 < l2a / l2b < 4.7
    assert 3.3 < maxa / maxb < 4.7
    assert maxb < 3e-3 * np.max(np.abs(FS.gauss_sol(np.zeros(1), np.zeros(1), np.zeros(1))))


def test_checks():
    t = OracleTree(3, (32,) * 3, (0,) * 3, (1,) * 3, [DIRICHLET] * 4 + [2, 2])
    with pytest.raises(ValueError):
        FS.coarse_charges(t, np.zeros(t.n_leaf), 1)
    t = _tree(32, bc_value=1.0)
    with pytest.raises(ValueError):
        FS.coarse_charges(t, np.zeros(t.n_leaf), 1)
    t = _tree(48)
    with pytest.raises(ValueError):
        FS.coarse_charges(t, np.zeros(t.n_leaf), 5)


def test_far_field_guess_matches_the_far_solution():
    # outside the source the Gaussian's potential is that of its total charge at its
    # centre (eq. gauss-sol with erf -> 1), so the guess matches it there, for a centred
    # and an off-centre source (the centroid); a neutral source gives zero
    for r0 in ((0.0, 0.0, 0.0), (0.12, -0.07, 0.05)):
        w = W.freespace_gauss((32,), offsets=[r0])
        t = _tree(32)
        lay = t.leaf_layout()
        g = FS.far_field_guess(t, w.rhs(0, lay), 1)
        x = W.cell_centres(lay, w.domains[0])
        r = np.sqrt(((x - np.asarray(r0)) ** 2).sum(axis=1))
        far = r > 0.35
        exact = FS.gauss_sol(x[:, 0], x[:, 1], x[:, 2], r0=r0)
        assert np.max(np.abs(g[far] - exact[far])) < 1e-5 * np.max(np.abs(exact[far]))
        assert np.all(np.isfinite(g))
    t = _tree(32)
    lay = t.leaf_layout()
    x = W.cell_centres(lay, W.freespace_gauss((32,)).domains[0])
    pos = np.exp(-((x - 0.1) ** 2).sum(axis=1) / 0.01)
    neg = np.exp(-((x + 0.1) ** 2).sum(axis=1) / 0.01)
    assert np.all(FS.far_field_guess(t, pos - neg, 1) == 0.0)
