"""The numpy FGMRES used to check the library's FGMRES refinement, pinned to
direct solves (not to itself)."""
import numpy as np

from helpers import oracle_trees
from oracle.krylov import fgmres
from paper_1901_11370_amd import workloads as W


def test_identity_preconditioner_matches_dense_solve():
    rng = np.random.default_rng(7)
    n = 60
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) / np.sqrt(n)    # nonsymmetric, well conditioned
    b = rng.standard_normal(n)
    x, hist = fgmres(lambda v: A @ v, lambda v: v, b, np.zeros(n), m=15, tol=1e-13)
    assert hist[-1] <= 1e-13
    assert np.allclose(x, np.linalg.solve(A, b), rtol=0, atol=1e-12 * np.abs(np.linalg.solve(A, b)).max())


def test_varying_preconditioner_still_converges():
    # a different (damped Jacobi) preconditioner at every step: only a flexible
    # method converges to the exact solution with it
    rng = np.random.default_rng(8)
    n = 50
    A = np.diag(rng.uniform(1, 10, n)) + rng.standard_normal((n, n)) * 0.3
    b = rng.standard_normal(n)
    d = np.diag(A)
    state = {"k": 0}

    def precond(v):
        state["k"] += 1
        return v / d * (0.5 + 0.5 * ((state["k"] * 0.37) % 1.0))
    x, hist = fgmres(lambda v: A @ v, precond, b, np.zeros(n), m=10, tol=1e-12, max_restarts=40)
    ref = np.linalg.solve(A, b)
    assert np.abs(x - ref).max() <= 1e-10 * np.abs(ref).max()


def test_multigrid_preconditioned_fgmres_matches_dense_composite_solve():
    # variable eps with a 1000:1 jump on a small refined 2D tree: the composite
    # operator is built column by column and solved by LU
    dom = W.Domain(2, [8, 8], [0, 0], [1, 1], [W.DIRICHLET] * 4)
    w = W.Workload("kry", [dom], bs=4, max_refine=1, variable_eps=True,
                   refine=lambda d, lev, o, bs: o[0] < 4 and o[1] < 4)
    A_t = oracle_trees(w, )[0]
    P_t = oracle_trees(w)[0]
    lay = A_t.leaf_layout()
    x = W.cell_centres(lay, dom)
    eps = np.where(np.hypot(x[:, 0] - 0.4, x[:, 1] - 0.4) < 0.25, 1000.0, 1.0)
    f = np.sin(3 * x[:, 0]) * np.cos(2 * x[:, 1]) + 0.1
    A_t.set_eps(eps)
    P_t.set_eps(eps)
    n = A_t.n_leaf
    Adense = np.column_stack([A_t.apply(np.eye(n)[i]) for i in range(n)])
    ref = np.linalg.solve(Adense, f)

    def M(v):
        P_t.set_rhs(v)
        P_t.set_phi(np.zeros_like(v))
        P_t.vcycle(1)
        return P_t.get_phi()
    # the rounding floor of the residual is ~eps_mach * 1000 h^-2 |phi| / |f| ~ 1e-12
    xs, hist = fgmres(A_t.apply, M, f, np.zeros(n), m=10, tol=1e-11)
    assert hist[-1] <= 1e-11 and len(hist) <= 4
    assert np.abs(xs - ref).max() <= 1e-9 * np.abs(ref).max()
