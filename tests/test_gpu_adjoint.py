"""Differentiable solve: the adjoint backward against the reference solver's adjoint
and against central finite differences of the loss.

J = 1/2 sum (phi - phi_target)^2 over leaf cells; phi = L(eps)^-1 f on a forest of
independent uniform Dirichlet cubes with log-normal eps (the differentiable-solve
workload, at reduced sizes here and at full size in the last test).
"""
import numpy as np
import pytest

from helpers import gpu_tree, inputs, oracle_trees, rel_err, split
from paper_1901_11370_amd import workloads as W

pytestmark = pytest.mark.gpu


def _setup(sizes, precision=1):
    import torch
    w = W.config5(sizes=sizes)
    t = gpu_tree(w, precision=precision)
    f, e = inputs(w, t)
    lay = t.leaf_layout()
    tgt = np.concatenate([w.target(i, lay[lay[:, 0] == i][:, 1:]) for i in range(len(sizes))])
    dev = lambda a: torch.from_numpy(np.concatenate(a) if isinstance(a, list) else a).cuda()
    return w, t, dev(f), dev(e), dev(tgt), f, e


def _grads(t, f, e, tgt):
    import torch
    from paper_1901_11370_amd.autograd import mg_solve
    f = f.clone().requires_grad_(True)
    e = e.clone().requires_grad_(True)
    phi = mg_solve(f, e, t, 1e-10, 60)
    J = 0.5 * torch.sum((phi - tgt) ** 2)
    J.backward()
    return phi.detach(), f.grad.detach(), e.grad.detach()


def test_adjoint_matches_reference_adjoint():
    w, t, f, e, tgt, fl, el = _setup((32, 48))
    phi, gf, ge = _grads(t, f, e, tgt)
    refs = oracle_trees(w)
    lay = t.leaf_layout()
    gfs, ges = split(t, gf.cpu().numpy()), split(t, ge.cpu().numpy())
    tg = tgt.cpu().numpy()
    for i, o in enumerate(refs):
        sel = lay[:, 0] == i
        o.set_eps(el[i])
        o.set_rhs(fl[i])
        o.solve(rel_tol=1e-13, max_cycles=80)
        p = o.get_phi()
        o.set_rhs(p - tg[sel])
        o.set_phi(np.zeros_like(p))
        o.solve(rel_tol=1e-13, max_cycles=80)
        lam = o.get_phi()
        g_eps = o.face_gradient(p, lam)
        ef, ee = rel_err(gfs[i], lam), rel_err(ges[i], g_eps)
        print(f"domain {i}: dJ/df rel err {ef:.2e}, dJ/deps rel err {ee:.2e}", flush=True)
        assert ef < 1e-6 and ee < 1e-6


def _fd_check(sizes, n_eps=10, n_f=10, tol=2e-6, seed=0, delta_f=1e-6, delta_eps=1e-4):
    """Central differences of J with FP64 solves run to the rounding floor, the J
    difference summed in cancellation-free form.

    dJ/deps entries are ~1e-8 while J ~ 50: at delta = 1e-6 the J difference (~6e-14)
    sits at the FP64 resolution of the sum over ~1e6 cells, and a delta sweep shows
    the FD error falling from ~1e-4 (delta 1e-6) to ~5e-7 (delta 1e-4) before
    truncation sets in near 1e-3.  The eps entries are therefore differenced with
    delta 1e-4, the larger dJ/df entries with delta 1e-6.  The remaining FD error
    depends on the rounding of the individual solves (5e-7 to 1e-6 on the 64^3 and
    96^3 members), hence the bound of 2e-6."""
    import torch
    w, t, f, e, tgt, fl, el = _setup(sizes)
    phi, gf, ge = _grads(t, f, e, tgt)
    t64 = gpu_tree(w, precision=0)

    def solve(ff, ee):
        t64.set_eps(ee)
        t64.set_rhs(ff)
        t64.set_phi(torch.zeros_like(ff))
        t64.solve(rel_tol=1e-13, max_cycles=40, raise_on_fail=False)
        t64.vcycle(2)
        out = torch.empty_like(ff)
        t64.get_phi(out=out)
        return out

    def dJ(pp, pm):
        return float(0.5 * torch.sum((pp - pm) * (pp + pm - 2 * tgt)))

    rng = np.random.default_rng(seed)
    ge_h, gf_h = ge.cpu().numpy(), gf.cpu().numpy()
    worst = 0.0
    for grad, which, n in ((ge_h, "eps", n_eps), (gf_h, "f", n_f)):
        big = np.flatnonzero(np.abs(grad) >= 1e-2 * np.abs(grad).max())
        for k in rng.choice(big, n, replace=False):
            delta = delta_eps if which == "eps" else delta_f
            if which == "eps":
                ep, em = e.clone(), e.clone()
                ep[k] += delta
                em[k] -= delta
                fd = dJ(solve(f, ep), solve(f, em)) / (2 * delta)
            else:
                fp, fm = f.clone(), f.clone()
                fp[k] += delta
                fm[k] -= delta
                fd = dJ(solve(fp, e), solve(fm, e)) / (2 * delta)
            r = abs(fd - grad[k]) / abs(grad[k])
            worst = max(worst, r)
            print(f"{which}[{k}]: adjoint {grad[k]:.9e} fd {fd:.9e} rel {r:.2e}", flush=True)
    assert worst < tol
    return worst


def test_adjoint_matches_finite_differences_small():
    _fd_check((32, 48), n_eps=6, n_f=4)


def test_adjoint_finite_differences_full_size_members():
    # the 64^3 and 96^3 members of the full-size batch, 20 seeded entries
    _fd_check((64, 96), n_eps=10, n_f=10)
