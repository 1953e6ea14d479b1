"""Differentiable solve: the adjoint backward against the reference solver's adjoint
and against central finite differences of the loss.

J = 1/2 sum (phi - phi_target)^2 over leaf cells; phi = L(eps)^-1 f on a forest of
independent uniform Dirichlet cubes with log-normal eps (the differentiable-solve
workload: six members of 64^3 to 256^3 cells).

Finite differences.  J(eps +- delta e_k) needs phi+- = L(eps +- delta e_k)^-1 f.  A
plain re-solve of phi+- carries rounding noise of relative size ~1e-16 in every cell,
uncorrelated between the two solves, while phi+ - phi- is only ~delta: at delta = 1e-6
the central difference is then wrong in its fourth digit.  Here phi+- = phi0 + D+-,
with phi0 the FP64 solution at eps and D+- the solution of the defect equation
L(eps +- delta e_k) D = L(eps) phi0 - L(eps +- delta e_k) phi0 (homogeneous boundary
values).  Both operator applications are the library's, with identical inputs away
from cell k, so the defect is exactly zero there and accurate to rounding near k; D is
solved to 1e-13 relative to its own size.  That is the same central difference
(J(phi0 + D+) - J(phi0 - ...)) / (2 delta), evaluated without the cancellation.  The
difference of J is summed as 1/2 sum (D+ - D-)(2 (phi0 - t) + D+ + D-).  For f the
defect is +-delta e_k itself (the solve is linear in f).  The residual of phi0 (at
the FP64 floor, ~1e-13 of f) changes the difference by that relative amount only.
"""
import numpy as np
import pytest

from helpers import gpu_tree, inputs, oracle_trees, rel_err, split
from paper_1901_11370_amd import workloads as W

pytestmark = pytest.mark.gpu

FD_DELTA = 1e-6        # the workload's central-difference step, for eps and for f
FD_TOL = 1e-6          # the bar: adjoint gradient within 1e-6 of the finite differences
# Entries are drawn uniformly, so some gradients are tiny.  The forward and adjoint
# solves stop at a relative residual of 1e-10, which leaves an absolute gradient error
# of order 1e-10 to 1e-8 of the member's largest entry; below 1e-2 of that entry the
# bar is therefore applied to the error relative to 1e-2 max|g| of the member.
FD_FLOOR = 1e-2


def _setup(sizes, precision=1):
    import torch
    w = W.config5(sizes=sizes)
    t = gpu_tree(w, precision=precision)
    f, e = inputs(w, t)
    lay = t.leaf_layout()
    tgt = np.concatenate([w.target(i, lay[lay[:, 0] == i][:, 1:]) for i in range(len(sizes))])
    dev = lambda a: torch.from_numpy(np.concatenate(a) if isinstance(a, list) else a).cuda()
    return w, t, dev(f), dev(e), dev(tgt), f, e


def _grads(t, f, e, tgt, rel_tol=1e-10, max_cycles=60):
    import torch
    from paper_1901_11370_amd.autograd import mg_solve
    f = f.clone().requires_grad_(True)
    e = e.clone().requires_grad_(True)
    phi = mg_solve(f, e, t, rel_tol, max_cycles)
    J = 0.5 * torch.sum((phi - tgt) ** 2)
    J.backward()
    return phi.detach(), f.grad.detach(), e.grad.detach()


def _oracle_adjoint(w, t, tgt, fl, el, rel_tol):
    """Per member: the reference solver's phi, lambda and dJ/deps (solves to rel_tol)."""
    lay = t.leaf_layout()
    tg = tgt.cpu().numpy()
    out = []
    for i, o in enumerate(oracle_trees(w)):
        sel = lay[:, 0] == i
        o.set_eps(el[i])
        o.set_rhs(fl[i])
        o.solve(rel_tol=rel_tol, max_cycles=80)
        p = o.get_phi()
        o.set_rhs(p - tg[sel])
        o.set_phi(np.zeros_like(p))
        o.solve(rel_tol=rel_tol, max_cycles=80)
        lam = o.get_phi()
        out.append((p, lam, o.face_gradient(p, lam)))
    return out


def _check_against_oracle(sizes, tol):
    # FP64 forward and adjoint on both sides: the GPU to 1e-11 (the FP64 floor of the
    # adjoint problem at 128^3 and above, with its smaller right-hand side, lies near
    # 1e-12), the reference to 1e-12
    w, t, f, e, tgt, fl, el = _setup(sizes, precision=0)
    phi, gf, ge = _grads(t, f, e, tgt, rel_tol=1e-11, max_cycles=40)
    ref = _oracle_adjoint(w, t, tgt, fl, el, 1e-12)
    gfs, ges = split(t, gf.cpu().numpy()), split(t, ge.cpu().numpy())
    phs = split(t, phi.cpu().numpy())
    worst = 0.0
    for i, (p, lam, g_eps) in enumerate(ref):
        ep, ef, ee = rel_err(phs[i], p), rel_err(gfs[i], lam), rel_err(ges[i], g_eps)
        print(f"{sizes[i]}^3: phi rel err {ep:.2e}, dJ/df rel err {ef:.2e}, dJ/deps rel err {ee:.2e}", flush=True)
        worst = max(worst, ef, ee)
    assert worst <= tol


def test_adjoint_matches_reference_adjoint_small():
    _check_against_oracle((32, 48), 1e-9)


def test_adjoint_matches_reference_adjoint_64_96_128():
    # the three smaller members of the differentiable-solve batch at full size
    _check_against_oracle((64, 96, 128), 1e-9)


def test_adjoint_matches_reference_adjoint_160():
    # an odd coarsest grid (5^3 cells below the block levels)
    _check_against_oracle((160,), 1e-9)


def _fd_check(sizes, n_eps=10, n_f=10, seed=0, precision=1):
    """20 seeded entries (10 of dJ/deps, 10 of dJ/df), drawn uniformly over all leaf
    cells of the forest, against central differences with step FD_DELTA."""
    import torch
    w, t, f, e, tgt, fl, el = _setup(sizes, precision=precision)
    phi, gf, ge = _grads(t, f, e, tgt)
    t64 = gpu_tree(w, precision=0)

    def solve(rhs, eps):
        t64.set_eps(eps)
        t64.set_rhs(rhs)
        t64.set_phi(torch.zeros_like(rhs))
        t64.solve(rel_tol=1e-13, max_cycles=40, raise_on_fail=False)
        t64.vcycle(2)
        out = torch.empty_like(rhs)
        t64.get_phi(out=out)
        return out

    phi0 = solve(f, e)
    t64.set_eps(e)
    L0 = t64.apply_operator(phi0)
    r0 = float(torch.max(torch.abs(L0 - f)) / torch.max(torch.abs(f)))
    print(f"FP64 reference phi0: relative residual {r0:.2e}", flush=True)
    res0 = 2.0 * (phi0 - tgt)

    def defect_solve(eps, d):
        t64.set_homogeneous_bc(True)
        try:
            return solve(d, eps)
        finally:
            t64.set_homogeneous_bc(False)

    def central(dp, dm):
        return float(0.5 * torch.sum((dp - dm) * (res0 + dp + dm))) / (2 * FD_DELTA)

    n = t.n_leaf
    bounds = np.cumsum(np.concatenate([[0], t.domain_leaf_cells()]))
    member = lambda k: int(np.searchsorted(bounds, k, side="right") - 1)
    ge_h, gf_h = ge.cpu().numpy(), gf.cpu().numpy()
    gmax = {(kind, i): np.abs(g[bounds[i]:bounds[i + 1]]).max()
            for kind, g in (("eps", ge_h), ("f", gf_h)) for i in range(len(sizes))}
    rng = np.random.default_rng(seed)
    worst = 0.0
    for kind, grad, cnt in (("eps", ge_h, n_eps), ("f", gf_h, n_f)):
        for k in rng.choice(n, cnt, replace=False):
            k = int(k)
            if kind == "eps":
                ds = []
                for s in (1.0, -1.0):
                    ep = e.clone()
                    ep[k] += s * FD_DELTA
                    t64.set_eps(ep)
                    d = L0 - t64.apply_operator(phi0)
                    ds.append(defect_solve(ep, d))
            else:
                ds = []
                for s in (1.0, -1.0):
                    d = torch.zeros_like(f)
                    d[k] = s * FD_DELTA
                    ds.append(defect_solve(e, d))
            fd = central(ds[0], ds[1])
            scale = max(abs(grad[k]), FD_FLOOR * gmax[(kind, member(k))])
            r = abs(fd - grad[k]) / scale
            worst = max(worst, r)
            print(f"{kind}[{k}] ({sizes[member(k)]}^3): adjoint {grad[k]:.12e} fd {fd:.12e} "
                  f"|g|/max {abs(grad[k]) / gmax[(kind, member(k))]:.1e} err {r:.2e}", flush=True)
    assert worst <= FD_TOL
    return worst


def test_adjoint_matches_finite_differences_small():
    _fd_check((32, 48), n_eps=6, n_f=4)


def test_adjoint_finite_differences_full_batch():
    # the six members of the batch at full size (64^3 ... 256^3), mixed-precision
    # forward and adjoint as configured, 20 seeded entries
    _fd_check(W.CONFIG5_SIZES, n_eps=10, n_f=10)


def test_fp64_adjoint_finite_differences_full_batch():
    # the same entries with the FP64 forward and adjoint (a check of the difference
    # machinery itself: here the two agree far below the bar)
    _fd_check(W.CONFIG5_SIZES, n_eps=10, n_f=10, precision=0)
