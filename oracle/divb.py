"""Elliptic divergence cleaning (Sec. 4.1: eq. poisson-divb, poisson-divb-cleaning,
divb-central-diff, divb-4th-order, divb-pressure-fix) on a tree without refinement.

Test infrastructure only, like the rest of this package: the plain numpy statement of
the projection that the paper couples to its MHD code.  A magnetic field B given at
cell centres is cleaned by solving lap(phi) = div(B) with the multigrid solver and
setting B <- B - grad(phi); the energy density keeps its thermal part,
e <- e + (|B_new|^2 - |B_old|^2) / 2.  div(B) uses second- or fourth-order central
differences, grad(phi) second-order central differences.

Arrays are leaf-ordered as the trees use them (component-major for B); each function
places them on the domain's uniform grid, numpy axis order (z, y, x) / (y, x), and
works there.  Readings where the paper defers to the MHD code:
  - outside a non-periodic face B repeats its boundary cell (zero gradient), for both
    layers the fourth-order stencil reaches;
  - grad(phi) takes phi's ghost values from the solver's boundary conditions (Sec. 2.6):
    Dirichlet 2a - phi_b, Neumann phi_b -/+ h b on the lower/upper face, periodic wrap.
"""
from __future__ import annotations

import numpy as np

from . import DIRICHLET, NEUMANN, PERIODIC


def _grid_of(tree):
    lay = tree.leaf_layout()
    if np.any(lay[:, 0] != 0):
        raise ValueError("divergence cleaning needs a tree without refinement")
    dim = tree.dim
    shape = tuple(int(tree.base[a]) for a in reversed(range(dim)))
    idx = tuple(lay[:, 1 + a] for a in reversed(range(dim)))
    h = (tree.hi - tree.lo)[:dim] / tree.base[:dim]
    return shape, idx, h


def _to_grid(leaf, shape, idx):
    g = np.zeros(shape)
    g[idx] = leaf
    return g


def _shift(p, ax, w, o):
    """View of the padded array p (w layers on axis ax) shifted by o cells."""
    n = p.shape[ax] - 2 * w
    sl = [slice(None)] * p.ndim
    sl[ax] = slice(w + o, w + o + n)
    return p[tuple(sl)]


def divergence(tree, B, order=2):
    """div(B) on the leaf cells (eq. divb-central-diff for order 2, eq. divb-4th-order
    for order 4), B of shape (dim, n_leaf)."""
    if order not in (2, 4):
        raise ValueError("order is 2 or 4")
    shape, idx, h = _grid_of(tree)
    dim = tree.dim
    out = np.zeros(shape)
    w = order // 2
    for d in range(dim):
        g = _to_grid(np.asarray(B[d], dtype=np.float64), shape, idx)
        ax = dim - 1 - d
        periodic = tree.bc_kind[2 * d] == PERIODIC
        p = np.pad(g, [(w, w) if a == ax else (0, 0) for a in range(dim)], mode="wrap" if periodic else "edge")
        s = lambda o: _shift(p, ax, w, o)
        if order == 2:
            out += (s(1) - s(-1)) / (2.0 * h[d])
        else:
            out += (-s(2) + 8.0 * s(1) - 8.0 * s(-1) + s(-2)) / (12.0 * h[d])
    return out[idx]


def gradient(tree, phi):
    """grad(phi) on the leaf cells, second-order central differences with phi's
    boundary ghosts; shape (dim, n_leaf)."""
    shape, idx, h = _grid_of(tree)
    dim = tree.dim
    g = _to_grid(np.asarray(phi, dtype=np.float64), shape, idx)
    out = []
    for d in range(dim):
        ax = dim - 1 - d
        kind_lo, kind_hi = tree.bc_kind[2 * d], tree.bc_kind[2 * d + 1]
        if kind_lo == PERIODIC:
            p = np.pad(g, [(1, 1) if a == ax else (0, 0) for a in range(dim)], mode="wrap")
        else:
            first = np.take(g, [0], axis=ax)
            last = np.take(g, [g.shape[ax] - 1], axis=ax)
            ghosts = []
            for kind, val, inner, sign in ((kind_lo, tree.bc_value[2 * d], first, -1.0),
                                           (kind_hi, tree.bc_value[2 * d + 1], last, 1.0)):
                if kind == DIRICHLET:
                    ghosts.append(2.0 * val - inner)
                elif kind == NEUMANN:
                    ghosts.append(inner + sign * h[d] * val)
                else:
                    raise ValueError("unpaired periodic face")
            p = np.concatenate([ghosts[0], g, ghosts[1]], axis=ax)
        out.append(((_shift(p, ax, 1, 1) - _shift(p, ax, 1, -1)) / (2.0 * h[d]))[idx])
    return np.array(out)


def project(tree, B, phi, e=None):
    """B - grad(phi) (eq. poisson-divb-cleaning) and, if e is given, the energy density
    with the magnetic change added (eq. divb-pressure-fix)."""
    B = np.asarray(B, dtype=np.float64)
    Bn = B - gradient(tree, phi)
    if e is None:
        return Bn, None
    en = np.asarray(e, dtype=np.float64) + 0.5 * (np.sum(Bn * Bn, axis=0) - np.sum(B * B, axis=0))
    return Bn, en


def clean(tree, B, e=None, order=2, rel_tol=1e-12, max_cycles=60):
    """The whole projection: f = div(B), FMG + V-cycles on lap(phi) = f from phi = 0,
    then project.  Returns (B_new, e_new, phi, residual history)."""
    f = divergence(tree, B, order)
    tree.set_phi(np.zeros(tree.n_leaf))
    tree.set_rhs(f)
    hist = tree.solve(rel_tol=rel_tol, max_cycles=max_cycles)
    phi = tree.get_phi()
    Bn, en = project(tree, B, phi, e)
    return Bn, en, phi, hist
