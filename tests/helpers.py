"""Shared test helpers: build the GPU tree and the reference trees of one workload
from the same seeded inputs, and compare leaf arrays."""
import numpy as np

from paper_1901_11370_amd import workloads as W


def gpu_domain(mg, d):
    return mg.Domain(d.dim, d.base_cells, d.lo, d.hi, d.bc_kind, list(d.bc_value))


def oracle_trees(w, **kw):
    """Reference trees of a workload; face-varying Dirichlet values (w.dirichlet) go into
    the reference's ghost cells on every level."""
    from oracle import OracleTree
    out = []
    for i, d in enumerate(w.domains):
        o = OracleTree(d.dim, d.base_cells, d.lo, d.hi, d.bc_kind, bc_value=list(d.bc_value), bs=w.bs,
                       max_refine=w.max_refine, refine=w.refine, domain_id=i,
                       variable_eps=w.variable_eps, **kw)
        if w.dirichlet is not None:
            o.set_boundary_function(lambda x, f, i=i: w.dirichlet(i, x))
        out.append(o)
    return out


def fold_dirichlet(w, t):
    """Face-varying Dirichlet values of a workload into the GPU tree's current
    right-hand side (mg_fold_dirichlet), evaluated at the leaf face centres."""
    cells, faces = t.boundary_faces()
    lay = t.leaf_layout()
    vals = np.empty(len(cells))
    for i, d in enumerate(w.domains):
        on = lay[cells, 0] == i
        xf = W.face_centres(lay[cells[on], 1:], d, faces[on])
        vals[on] = w.dirichlet(i, xf)
    t.fold_dirichlet(vals)


def gpu_tree(w, bind=True, **params):
    from paper_1901_11370_amd import mg
    p = mg.default_params(variable_eps=1 if w.variable_eps else 0, **params)
    return mg.Tree([gpu_domain(mg, d) for d in w.domains], bs=w.bs, max_refine=w.max_refine,
                   refine=w.refine, params=p, bind=bind)


def split(t, arr):
    """Split a GPU leaf array into per-domain pieces."""
    n = t.domain_leaf_cells()
    return np.split(np.asarray(arr), np.cumsum(n)[:-1])


def inputs(w, t):
    """Per-domain (f, eps) arrays evaluated on the GPU tree's layout."""
    lay = t.leaf_layout()
    f, e = [], []
    for i in range(len(w.domains)):
        li = lay[lay[:, 0] == i][:, 1:]
        f.append(w.rhs(i, li))
        e.append(w.eps(i, li) if w.eps else None)
    return f, e


def rel_err(a, b, remove_mean=False):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if remove_mean:
        a = a - a.mean()
        b = b - b.mean()
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
