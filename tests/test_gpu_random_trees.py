"""Seeded random trees, GPU against the reference solver after FMG + 2 V-cycles (the FP64
bar, 1e-11 relative): 2D and 3D, block sizes 4, 8 and 16, forests of one to three
domains, random boundary kinds and values (periodic axes in pairs), random refinement
up to two levels (a hash of the block's position decides, so both builders see the same
predicate), and in some trees variable eps, the Jacobi smoother or a Helmholtz term."""
import numpy as np
import pytest

from helpers import gpu_tree, inputs, oracle_trees, rel_err, split
from paper_1901_11370_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(seed):
    rng = np.random.default_rng(1000 + seed)
    dim = 2 if seed % 2 == 0 else 3
    bs = int(rng.choice([4, 8, 16]))
    ndom = int(rng.integers(1, 4))
    doms = []
    for _ in range(ndom):
        mult = rng.integers(1, 5 if dim == 3 else 9, size=dim)
        if bs == 16 and dim == 3:
            mult = np.minimum(mult, 3)
        n = [int(bs * m) for m in mult]
        lo = rng.uniform(-1, 1, size=dim)
        hi = lo + np.array(n) * rng.uniform(0.5, 1.5) / 32.0
        kinds, vals = [], []
        for a in range(dim):
            k = int(rng.integers(0, 3))
            kinds += [W.PERIODIC, W.PERIODIC] if k == 2 else [int(rng.integers(0, 2)), int(rng.integers(0, 2))]
            vals += list(rng.uniform(-1, 1, size=2))
        if W.DIRICHLET not in kinds:
            kinds[0] = W.DIRICHLET      # keep the problem regular (no constant null space)
            if kinds[1] == W.PERIODIC:
                kinds[1] = W.NEUMANN
        doms.append(W.Domain(dim, n, list(lo), list(hi), kinds, vals))
    max_ref = int(rng.integers(0, 3))
    salt = int(rng.integers(1, 1 << 30))

    def refine(d, level, origin, b):
        h = hash((salt, d, level) + tuple(int(x) for x in origin[:dim])) & 0xFFFF
        return h < 0x4000

    srcs = [W.Gaussians(rng.uniform(np.array(d.lo), np.array(d.hi), size=(2, dim)), rng.normal(size=2),
                        np.full(2, 0.2 * float(np.min(np.array(d.hi) - np.array(d.lo))))) for d in doms]
    var = bool(rng.random() < 0.3) or seed % 3 == 1
    params = {}
    if rng.random() < 0.2 or seed % 5 == 3:
        params["smoother"] = 1
    if rng.random() < 0.2:
        params["helmholtz_lambda"] = float(rng.uniform(1, 50))
    w = W.Workload(f"rand{seed}", doms, bs=bs, max_refine=max_ref, refine=refine if max_ref else None,
                   variable_eps=var, rhs=lambda i, lay: srcs[i](W.cell_centres(lay, doms[i])),
                   eps=(lambda i, lay: np.exp(0.5 * np.sin(3 * W.cell_centres(lay, doms[i])).sum(axis=1))) if var else None)
    return w, params


@pytest.mark.parametrize("seed", range(48))
def test_random_tree_matches_reference(seed):
    w, params = _case(seed)
    t = gpu_tree(w, **params)
    refs = oracle_trees(w)
    for o in refs:
        if params.get("smoother") == 1:
            o.set_smoother(o.JACOBI)
        if "helmholtz_lambda" in params:
            o.set_lambda(params["helmholtz_lambda"])
    f, e = inputs(w, t)
    if w.variable_eps:
        t.set_eps(np.concatenate(e))
        for o, ei in zip(refs, e):
            o.set_eps(ei)
    t.set_rhs(np.concatenate(f))
    for o, fi in zip(refs, f):
        o.set_rhs(fi)
    t.fmg()
    t.vcycle(2)
    for o in refs:
        o.fmg()
        o.vcycle(2)
    errs = [rel_err(p, o.get_phi()) for p, o in zip(split(t, t.get_phi()), refs)]
    print(w.name, "dim", w.domains[0].dim, "bs", w.bs, "doms", len(w.domains), "leaf", t.n_leaf, params,
          "var", w.variable_eps, "err", max(errs), flush=True)
    assert max(errs) <= 1e-11


@pytest.mark.parametrize("seed", range(0, 48, 2))
def test_random_tree_mixed_solve_reaches_reference_solution(seed):
    # the same trees in the mixed form, solved to 1e-10: FP64 refinement removes the FP32
    # rounding of the corrections, so the solution is the reference's converged one
    import torch
    w, params = _case(seed)
    t = gpu_tree(w, precision=1, **params)
    refs = oracle_trees(w)
    for o in refs:
        if params.get("smoother") == 1:
            o.set_smoother(o.JACOBI)
        if "helmholtz_lambda" in params:
            o.set_lambda(params["helmholtz_lambda"])
    f, e = inputs(w, t)
    if w.variable_eps:
        t.set_eps(np.concatenate(e))
        for o, ei in zip(refs, e):
            o.set_eps(ei)
    t.set_rhs(torch.from_numpy(np.concatenate(f)).cuda())
    cycles, rc = t.solve(rel_tol=1e-10, max_cycles=60)
    for o, fi in zip(refs, f):
        o.set_rhs(fi)
        o.solve(rel_tol=1e-12, max_cycles=120)
    errs = [rel_err(p, o.get_phi()) for p, o in zip(split(t, t.get_phi()), refs)]
    print(w.name, "mixed solve", cycles, "err", max(errs), flush=True)
    assert rc == 0 and max(errs) <= 1e-8
