"""FGMRES refinement (mixed precision, krylov = m) on the eps-jump workload, where
the plain cycles stall: the GPU solution must satisfy the reference solver's FP64
composite equations to the requested tolerance, and agree with the reference
FGMRES solution (numpy FGMRES around the reference operator and V-cycle)."""
import numpy as np
import pytest

from helpers import gpu_tree, inputs, oracle_trees
from oracle.krylov import fgmres
from paper_1901_11370_amd import workloads as W

pytestmark = pytest.mark.gpu


def _config4_small(base=32):
    w = W.config4(nested=True)
    w.domains[0].base_cells = [base] * 3
    return w


def test_fgmres_refinement_solves_eps_jump_problem():
    import torch
    w = _config4_small()
    t = gpu_tree(w, precision=1, krylov=20)
    f, e = inputs(w, t)
    t.set_eps(torch.from_numpy(e[0]).cuda())
    t.set_rhs(torch.from_numpy(f[0]).cuda())
    cycles, rc = t.solve(rel_tol=1e-10, max_cycles=120)
    phi = t.get_phi()
    res, _ = t.solve_stats()
    print("cycles", cycles, "restart residuals", res, flush=True)
    assert rc == 0 and res[-1] <= 1e-10
    # the reference solver's FP64 operator applied to the GPU solution
    A_t, P_t = oracle_trees(w)[0], oracle_trees(w)[0]
    for o in (A_t, P_t):
        o.set_eps(e[0])
    r = f[0] - A_t.apply(phi)
    rel = np.abs(r).max() / np.abs(f[0]).max()
    print("reference residual of the GPU solution", rel, flush=True)
    assert rel <= 1.2e-10

    def M(v):
        P_t.set_rhs(v)
        P_t.set_phi(np.zeros_like(v))
        P_t.vcycle(1)
        return P_t.get_phi()
    ref, hist = fgmres(A_t.apply, M, f[0], np.zeros_like(f[0]), m=20, tol=1e-13)
    err = np.abs(phi - ref).max() / np.abs(ref).max()
    print("reference FGMRES residuals", hist, "relative difference", err, flush=True)
    assert err <= 1e-7


def test_plain_refinement_stalls_where_fgmres_converges():
    # the same problem with plain refinement steps: the paper's cycles alone contract
    # by less than 0.95 per cycle here (coefficient jump of 1000, no special treatment)
    import torch
    w = _config4_small(16)
    t = gpu_tree(w, precision=1, ir_vcycles=1)   # the contraction of single cycles
    f, e = inputs(w, t)
    t.set_eps(torch.from_numpy(e[0]).cuda())
    t.set_rhs(torch.from_numpy(f[0]).cuda())
    cycles, rc = t.solve(rel_tol=1e-10, max_cycles=25, raise_on_fail=False)
    res, _ = t.solve_stats()
    assert rc != 0 and res[-1] / res[-5] > 0.8   # slower than 0.95 per step
    tk = gpu_tree(w, precision=1, krylov=10)
    tk.set_eps(torch.from_numpy(e[0]).cuda())
    tk.set_rhs(torch.from_numpy(f[0]).cuda())
    cycles, rc = tk.solve(rel_tol=1e-10, max_cycles=60)
    assert rc == 0
