"""Pins of the reference solver's coarsest-grid solve, residual norms and face-varying
Dirichlet values against closed forms, brute force and hand-worked values.

Coarsest grid (Sec. 2.4: smoothing steps until the residual has fallen by the
relative tolerance, at most n_max = 1000).  On a one-cell grid Gauss-Seidel with the
boundary ghosts held at their last values is v <- rho v + c, with rho fixed by the
boundary kinds: each Dirichlet face contributes -1 and each zero-flux Neumann face +1
to sum_f w g_f (w the face weight), so rho = (2d - 2 n_D) / (2d + lambda h^2) for n_D
Dirichlet faces.  The residual then falls exactly as |rho|^k, and the paper's rule
stops after the first k with |rho|^k <= 1e-8.  With rho = -1 (every face Dirichlet)
the iteration only alternates; the reference's stall window ends it after 8 steps, and
because the alternation has period two the state equals that after the paper's 1000
steps.  On a slowly converging 8 x 1 grid the step count equals that of a brute-force
red-black Gauss-Seidel written here with numpy, with the window on or off.  The window's
known limit is pinned too: where the residual rises for more than 8 steps before it falls,
the window stops the coarsest solve too early and the cycles crawl.

Norms (Sec. 3.1; the L2 norm weighted by cell volume): phi = 1 in one cell of a
refined tree, f = c everywhere, gives hand-computable residuals.

Fully periodic problems: the mean of f is removed on the coarsest grid, so an
inconsistent f = g + c solves, up to a constant, to the closed-form solution for g."""
import math

import numpy as np
import pytest

from oracle import OracleTree
from paper_1901_11370_amd import workloads as W

D, N, P = W.DIRICHLET, W.NEUMANN, W.PERIODIC


def _one_cell(dim, kinds, lam=0.0, values=None):
    n = [16] * dim
    o = OracleTree(dim, n, [0.0] * dim, [1.0 * 16] * dim, kinds, bc_value=values, bs=16)
    if lam:
        o.set_lambda(lam)
    assert o.level_info(0)[1][:dim] == (1,) * dim   # the coarsest grid is a single cell
    return o


def _coarse_from(o, v0, f0):
    """Set the single coarsest cell, fill its ghosts, run the coarsest solve."""
    dim = o.dim
    shape = (3,) * dim
    v = np.zeros(shape)
    v[(1,) * dim] = v0
    f = np.zeros(shape)
    f[(1,) * dim] = f0
    o.set_block_field(0, 0, "v", v)
    o.set_block_field(0, 0, "f", f)
    o.fill_ghosts_level(0)
    o.coarse_solve()
    return o.block_field(0, 0, "v")[(1,) * dim]


def _expected_steps(rho, rel=1e-8):
    if rho == 0.0:
        return 1
    return math.ceil(math.log(rel) / math.log(abs(rho)))


@pytest.mark.parametrize("dim,n_dir,lam", [(2, 1, 0.0), (2, 2, 0.0), (2, 3, 0.0), (2, 4, 4.0),
                                           (3, 1, 0.0), (3, 2, 0.0), (3, 3, 0.0), (3, 4, 0.0),
                                           (3, 5, 0.0), (3, 6, 3.0)])
def test_one_cell_step_count_is_the_papers_rule(dim, n_dir, lam):
    # the domain [0,16]^d of 16^d cells: the one coarsest cell has h = 16, weight 1/256
    kinds = [D] * n_dir + [N] * (2 * dim - n_dir)
    o = _one_cell(dim, kinds, lam)
    h2 = 16.0 ** 2
    rho = (2 * dim - 2 * n_dir) / (2 * dim + lam * h2)
    for stall in (8, 0):
        o.set_coarse_stall(stall)
        _coarse_from(o, 0.37, 1.3)
        assert o.last_coarse_steps == _expected_steps(rho), (rho, stall)
        assert o.last_coarse_exit == OracleTree.EXIT_TARGET


@pytest.mark.parametrize("dim", [2, 3])
def test_alternating_one_cell_dirichlet_grid(dim):
    # rho = -1: the residual never falls.  The window stops after 8 steps; the paper's
    # rule alone runs n_max = 1000 steps; both even, so both end where they started
    o = _one_cell(dim, [D] * (2 * dim))
    o.set_coarse_stall(8)
    a = _coarse_from(o, 0.37, 1.3)
    assert o.last_coarse_steps == 8 and o.last_coarse_exit == OracleTree.EXIT_STALL
    o.set_coarse_stall(0)
    b = _coarse_from(o, 0.37, 1.3)
    assert o.last_coarse_steps == 1000 and o.last_coarse_exit == OracleTree.EXIT_NMAX
    # to rounding of the alternation's larger value, -v - f/sum(w) = -0.37 - 83.2 (2D)
    amp = 0.37 + 1.3 * 256 / (2 * dim)
    assert abs(a - 0.37) <= 1e-15 * amp and abs(b - 0.37) <= 1e-15 * amp


def _brute_force_line(v, f, h, a_left, b_right, b_y, rel=1e-8, n_max=1000):
    """Red-black Gauss-Seidel on a row of cells, one cell high: Dirichlet value a_left at
    x = 0, Neumann derivative b_right at the right end, Neumann derivative b_y on both
    y faces (ghosts v -+ h b_y, whose terms cancel in the operator but which hold the
    cell's value from the last fill during its update), every ghost refilled after each
    colour.  Returns (steps, v) under the paper's rule."""
    v = v.astype(float).copy()
    n = len(v)
    w = 1.0 / (h * h)

    def ghosts(v):
        return 2.0 * a_left - v[0], v[-1] + h * b_right, v - h * b_y, v + h * b_y

    def resid(v):
        gl, gr, ys, yn = ghosts(v)
        ext = np.concatenate([[gl], v, [gr]])
        return np.abs(f - w * (ext[:-2] - 2 * v + ext[2:] + (ys - v) + (yn - v))).max()

    r0 = resid(v)
    for k in range(1, n_max + 1):
        for colour in (0, 1):
            gl, gr, ys, yn = ghosts(v)
            ext = np.concatenate([[gl], v, [gr]])
            for i in range(colour, n, 2):
                v[i] = (w * (ext[i] + ext[i + 2] + ys[i] + yn[i]) - f[i]) / (4 * w)
        if resid(v) <= rel * r0:
            return k, v
    return n_max, v


@pytest.mark.parametrize("n", [4, 8])
def test_slow_line_grid_matches_brute_force(n):
    # (16 n) x 16 cells in 16^2 blocks: the coarsest grid is n x 1 cells (h = 16); one
    # Dirichlet end, Neumann elsewhere.  Gauss-Seidel with ghosts held during a colour
    # needs a few hundred steps on 4 x 1 (the residual rising on the way) and more than
    # n_max = 1000 on 8 x 1; the step count and the values are those of the brute force
    o = OracleTree(2, [16 * n, 16], [0.0, 0.0], [16.0 * n, 16.0], [D, N, N, N], bc_value=[0.3, -0.01, 0.02, 0.02],
                   bs=16)
    bs, nc, nb = o.level_info(0)
    assert (bs, nc[:2], nb) == (1, (n, 1), n)
    rng = np.random.default_rng(3)
    v0 = rng.standard_normal(n)
    f0 = rng.standard_normal(n) * 1e-3
    order = [o.block_meta(0, ib)[0][0] for ib in range(nb)]
    res = {}
    for stall in (8, 0):
        o.set_coarse_stall(stall)
        for ib in range(nb):
            x = order[ib]
            vb = np.zeros((3, 3))
            vb[1, 1] = v0[x]
            fb = np.zeros((3, 3))
            fb[1, 1] = f0[x]
            o.set_block_field(0, ib, "v", vb)
            o.set_block_field(0, ib, "f", fb)
        o.fill_ghosts_level(0)
        o.coarse_solve()
        v = np.zeros(n)
        for ib in range(nb):
            v[order[ib]] = o.block_field(0, ib, "v")[1, 1]
        res[stall] = (o.last_coarse_steps, o.last_coarse_exit, v)
    k, vb = _brute_force_line(v0, f0, 16.0, 0.3, -0.01, 0.02)
    print("steps", k, res[8][0], res[0][0])
    want = OracleTree.EXIT_TARGET if n == 4 else OracleTree.EXIT_NMAX
    assert (100 < k < 1000) if n == 4 else k == 1000
    for stall in (8, 0):
        steps, ex, v = res[stall]
        assert steps == k and ex == want
        assert np.abs(v - vb).max() <= 1e-12 * np.abs(vb).max()
    assert np.array_equal(res[8][2], res[0][2])


def _cycles(w, stall, fmg=1, vc=3):
    from helpers import oracle_trees
    o = oracle_trees(w)[0]
    o.set_coarse_stall(stall)
    lay = o.leaf_layout()
    o.set_rhs(w.rhs(0, lay))
    exits = []
    for _ in range(fmg):
        o.fmg()
        exits.append(o.last_coarse_exit)
    for _ in range(vc):
        o.vcycle()
        exits.append(o.last_coarse_exit)
    return o.get_phi(), exits


@pytest.mark.parametrize("case", ["config1", "odd3", "odd5"])
def test_window_leaves_cycles_unchanged(case):
    # before the rounding floor the window does not fire on the configurations' grids
    # (or, on the one-cell Dirichlet grid of config 1, ends an even alternation): the
    # cycles are the same with and without it
    if case == "config1":
        w = W.config1(n=64)
    else:
        n = 48 if case == "odd3" else 80
        dom = W.Domain(3, [n] * 3, [0, 0, 0], [1, 1, 1], [D] * 6)
        g = W.Gaussians(np.array([[0.3, 0.6, 0.5], [0.7, 0.3, 0.4]]), np.array([1.0, -0.5]), np.array([0.1, 0.15]))
        w = W.Workload(case, [dom], rhs=lambda i, lay: g(W.cell_centres(lay, dom)))
    a, ea = _cycles(w, 8)
    b, eb = _cycles(w, 0)
    print(case, ea, eb)
    if case == "config1":
        assert all(e == OracleTree.EXIT_STALL for e in ea) and all(e == OracleTree.EXIT_NMAX for e in eb)
        assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()
    else:
        assert all(e == OracleTree.EXIT_TARGET for e in ea + eb)
        assert np.array_equal(a, b)


def test_window_at_the_rounding_floor():
    # once the fine problem is solved to its rounding floor the coarse residual cannot
    # fall by 1e-8 any more: the paper's rule then takes all 1000 steps, the window
    # stops after a few, and the solutions agree to rounding
    dom = W.Domain(3, [48] * 3, [0, 0, 0], [1, 1, 1], [D] * 6)
    g = W.Gaussians(np.array([[0.3, 0.6, 0.5]]), np.array([1.0]), np.array([0.1]))
    w = W.Workload("floor", [dom], rhs=lambda i, lay: g(W.cell_centres(lay, dom)))
    a, ea = _cycles(w, 8, vc=16)
    b, eb = _cycles(w, 0, vc=16)
    print(ea, eb)
    assert OracleTree.EXIT_STALL in ea and OracleTree.EXIT_NMAX in eb
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()


def test_window_stops_early_while_the_residual_rises():
    # the window's known limit: on this coarsest grid (Dirichlet x-, Neumann x+, periodic
    # y, eps varying along x) the max-norm residual rises for more than 8 steps before it
    # falls, so the window ends every coarsest solve too early and the V-cycles crawl at
    # about 0.94 per cycle; with the paper's rule alone they contract by about 0.1 and
    # reach 1e-10 in 9 cycles
    from helpers import oracle_trees
    lo, hi = [-0.3279, -0.1514], [0.4321, 0.3236]
    dom = W.Domain(2, [32, 20], lo, hi, [D, N, P, P])
    g = W.Gaussians(np.array([[(lo[0] + hi[0]) / 2, (lo[1] + hi[1]) / 2]]), np.array([1.0]), np.array([0.1]))
    w = W.Workload("rising", [dom], bs=4, variable_eps=True, rhs=lambda i, lay: g(W.cell_centres(lay, dom)),
                   eps=lambda i, lay: np.exp(np.sin(3 * W.cell_centres(lay, dom)[:, 0])))
    out = {}
    for stall in (8, 0):
        o = oracle_trees(w)[0]
        o.set_coarse_stall(stall)
        lay = o.leaf_layout()
        o.set_rhs(w.rhs(0, lay))
        o.set_eps(w.eps(0, lay))
        out[stall] = (o.solve(rel_tol=1e-10, max_cycles=20), o.last_coarse_exit)
    (h8, exit8), (h0, _) = out[8], out[0]
    print(len(h8), h8[-1], exit8, len(h0), h0[-1])
    assert exit8 == OracleTree.EXIT_STALL and h8[-1] > 1e-3 and (h8[-1] / h8[1]) ** (1 / (len(h8) - 2)) > 0.9
    assert len(h0) <= 10 and h0[-1] <= 1e-10


def test_l2_norm_hand_worked_on_a_refined_tree():
    # 2D, base 32^2 on [0,1]^2, the lower-left quarter refined once (h = 1/64 there);
    # phi = 1 in one fine cell away from every block edge, f = c everywhere.  Then
    # (L phi) = -4/h^2 in that cell and +1/h^2 in its four neighbours, zero elsewhere,
    # so r = c + 4/h^2, c - 1/h^2 (four cells), c elsewhere, and
    #   sum vol r^2 = c^2 (area) + h^2 [(c + 4/h^2)^2 - c^2 + 4 ((c - 1/h^2)^2 - c^2)],
    #   sum vol f^2 = c^2 (area = 1).
    def refine(d, level, origin, bs):
        return level == 0 and origin[0] < 16 and origin[1] < 16

    o = OracleTree(2, [32, 32], [0, 0], [1, 1], [D] * 4, bs=16, max_refine=1, refine=refine)
    lay = o.leaf_layout()
    fine = lay[:, 0] == 1
    assert fine.sum() == 32 * 32
    k = np.flatnonzero(fine & (lay[:, 1] == 9) & (lay[:, 2] == 6))[0]
    phi = np.zeros(o.n_leaf)
    phi[k] = 1.0
    c = 3.0
    h = 1.0 / 64
    o.set_rhs(np.full(o.n_leaf, c))
    o.set_phi(phi)
    mx, l2 = o.residual_norm()
    s_r = c * c + h * h * ((c + 4 / h ** 2) ** 2 - c * c + 4 * ((c - 1 / h ** 2) ** 2 - c * c))
    assert abs(l2 - math.sqrt(s_r / (c * c))) <= 1e-12 * l2
    assert abs(mx - (c + 4 / h ** 2) / c) <= 1e-12 * mx


def _periodic_laplacian(n, h):
    """Dense 5-point periodic Laplacian on an n x n grid of spacing h (x fastest)."""
    A = np.zeros((n * n, n * n))
    for j in range(n):
        for i in range(n):
            r = j * n + i
            A[r, r] = -4.0 / h ** 2
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                A[r, ((j + dj) % n) * n + (i + di) % n] += 1.0 / h ** 2
    return A


def test_periodic_coarsest_grid_solves_the_zero_mean_system():
    # 48^2 cells in 16^2 blocks, fully periodic: the coarsest grid is 3 x 3 cells.  Its
    # solve first subtracts the mean of f (the singular system is only solvable for
    # zero-mean f), then smooths: v - mean(v) is the pseudo-inverse solution of the
    # dense periodic system for f - mean(f), to the coarse tolerance
    o = OracleTree(2, [48, 48], [0, 0], [1, 1], [P] * 4, bs=16)
    bs, nc, nb = o.level_info(0)
    assert (bs, nc[:2], nb) == (1, (3, 3), 9)
    h = 1.0 / 3
    rng = np.random.default_rng(9)
    f = rng.standard_normal(9) + 0.7          # mean far from zero
    v0 = rng.standard_normal(9)
    pos = {}
    for ib in range(nb):
        org = o.block_meta(0, ib)[0]
        pos[ib] = org[1] * 3 + org[0]
        vb = np.zeros((3, 3))
        vb[1, 1] = v0[pos[ib]]
        fb = np.zeros((3, 3))
        fb[1, 1] = f[pos[ib]]
        o.set_block_field(0, ib, "v", vb)
        o.set_block_field(0, ib, "f", fb)
    o.fill_ghosts_level(0)
    o.coarse_solve()
    assert o.last_coarse_exit == OracleTree.EXIT_TARGET
    v = np.zeros(9)
    for ib in range(nb):
        v[pos[ib]] = o.block_field(0, ib, "v")[1, 1]
    A = _periodic_laplacian(3, h)
    Ap = np.linalg.pinv(A)
    fc = f - f.mean()
    ref = Ap @ fc
    assert abs(ref.mean()) <= 1e-14
    # the rule: max-norm residual of the projected system reduced by 1e-8 ...
    r0 = np.abs(fc - A @ v0).max()
    assert np.abs(fc - A @ v).max() <= 1e-8 * r0
    # ... so the zero-mean part of v is within |A^+|_inf 1e-8 r0 of the solution
    err = np.abs((v - v.mean()) - ref).max()
    bound = np.abs(Ap).sum(axis=1).max() * 1e-8 * r0
    print("coarse steps", o.last_coarse_steps, "err", err, "bound", bound)
    assert err <= bound
    # without the mean removal no v could bring the residual below |mean(f)|
    r = f - A @ v
    assert abs(r.mean() - f.mean()) <= 1e-12


def test_face_values_reproduce_a_linear_solution():
    # phi = 1 + 2x - 3y + 0.5z is discretely harmonic; with its values at the face
    # centres as Dirichlet data (varying along every face) the solve returns it exactly,
    # also across a refinement boundary that meets the domain boundary
    dom = W.Domain(3, [32] * 3, [0, 0, 0], [1, 1, 1], [D] * 6)

    def refine(d, level, origin, bs):
        return level == 0 and origin[0] < 16 and origin[1] < 16

    lin = lambda x: 1 + 2 * x[:, 0] - 3 * x[:, 1] + 0.5 * x[:, 2]
    w = W.Workload("lin", [dom], max_refine=1, refine=refine, rhs=lambda i, lay: np.zeros(len(lay)),
                   dirichlet=lambda i, x: lin(x))
    from helpers import oracle_trees
    o = oracle_trees(w)[0]
    lay = o.leaf_layout()
    o.set_rhs(np.zeros(o.n_leaf))
    o.solve(rel_tol=0, max_cycles=24, fmg_first=True)
    exact = lin(W.cell_centres(lay, dom))
    assert np.abs(o.get_phi() - exact).max() <= 1e-12


def test_constant_face_values_equal_the_constant_boundary():
    # per-face values that equal each face's constant give the same cycles bit for bit
    vals = [0.7, -0.2, 0.4, 1.1]
    dom = W.Domain(2, [64, 64], [0, 0], [1, 1], [D] * 4, vals)

    def refine(d, level, origin, bs):
        return level == 0 and origin[0] >= 32

    g = W.Gaussians(np.array([[0.3, 0.6]]), np.array([1.0]), np.array([0.1]))
    from helpers import oracle_trees
    base = W.Workload("c", [dom], max_refine=1, refine=refine, rhs=lambda i, lay: g(W.cell_centres(lay, dom)))
    a = oracle_trees(base)[0]
    per = oracle_trees(base)[0]
    x, faces = per.boundary_faces()
    per.set_boundary_values(np.asarray(vals)[faces])
    for o in (a, per):
        o.set_rhs(base.rhs(0, o.leaf_layout()))
        o.fmg()
        o.vcycle(2)
    assert np.array_equal(a.get_phi(), per.get_phi())


def test_threads_do_not_change_results():
    # the block loops of a level run in parallel (OpenMP); each block writes only its own
    # cells and ghosts, so any thread count gives the same bits
    import oracle
    from helpers import oracle_trees
    dom = W.Domain(3, [32, 32, 48], [0, 0, 0], [1, 1, 1.5], [D, N, P, P, N, D], [0.3, -0.2, 0, 0, 0.1, 0.5])

    def refine(d, level, origin, bs):
        return level == 0 and origin[0] >= 16

    g = W.Gaussians(np.array([[0.6, 0.4, 0.7]]), np.array([1.0]), np.array([0.2]))
    w = W.Workload("thr", [dom], max_refine=1, refine=refine, variable_eps=True,
                   rhs=lambda i, lay: g(W.cell_centres(lay, dom)),
                   eps=lambda i, lay: np.exp(np.sin(4 * W.cell_centres(lay, dom)).sum(axis=1)))
    out = []
    for nt in (1, 4):
        oracle.set_threads(nt)
        o = oracle_trees(w)[0]
        lay = o.leaf_layout()
        o.set_eps(w.eps(0, lay))
        o.set_rhs(w.rhs(0, lay))
        o.fmg()
        o.vcycle(2)
        out.append((o.get_phi(), o.residual_norm()))
    oracle.set_threads(1)
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]
