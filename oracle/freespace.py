"""Free-space boundary conditions (Sec. 2.8) on a 3D tree without refinement, and the
Gaussian test problem of Sec. 3.2 (eq. gauss-rhs, gauss-sol).

Test infrastructure only, like the rest of this package: the plain numpy statement of
the coupling the paper describes, in its order:
  1. the right-hand side is restricted to a uniform level k levels below the leaf level
     (the mean of the 8^k leaf cells of each coarse cell, Sec. 2.3);
  2. the free-space potential of that coarse grid is found on the six boundary planes of
     the domain, at the coarse grid's face centres plus one ghost position on each side
     of every row (the paper's uniform grid carries a ghost layer);
  3. the planes are interpolated linearly to the leaf faces, which gives the Dirichlet
     values;
  4. multigrid cycles solve the problem with these values.
Readings where the paper leaves a choice:
  - step 2: the paper calls an external interpolating-scaling-function FFT solver; here
    the potential of the coarse cells, each a point charge q = f_c h_c^3 at its centre,
    is summed directly: phi(x) = -(1/4 pi) sum_c q_c / |x - x_c|;
  - step 4: face values that vary along a face enter through the right-hand side: with
    the Dirichlet ghost 2a - phi_b (Sec. 2.6) the boundary cell's equation is
    L_0 phi = f - 2 a / h_a^2 per boundary face, L_0 the operator with homogeneous
    Dirichlet faces, which the solver then uses.

Boundary values are returned face by face (x-, x+, y-, y+, z-, z+), each over the face's
leaf cells with the lower in-plane axis fastest (face x: y fastest, then z; faces y and
z: x fastest, then z or y).
"""
from __future__ import annotations

import numpy as np

from . import DIRICHLET
from .divb import _grid_of, _to_grid

FOUR_PI = 4.0 * np.pi


def _check(tree, k):
    if tree.dim != 3:
        raise ValueError("free-space boundaries are three-dimensional")
    if any(int(c) != DIRICHLET for c in tree.bc_kind[:6]) or np.any(tree.bc_value[:6] != 0.0):
        raise ValueError("free-space boundaries need homogeneous Dirichlet faces")
    n = [int(tree.base[a]) for a in range(3)]
    if k < 0 or any(x % (1 << k) for x in n):
        raise ValueError("the coarse level must divide the leaf grid")


def coarse_charges(tree, f, k):
    """Charges q_c = mean(f over the 8^k leaf cells) * h_c^3 on the level k below the
    leaf level, numpy order (z, y, x), and the coarse spacing h_c (x, y, z)."""
    _check(tree, k)
    shape, idx, h = _grid_of(tree)
    g = _to_grid(np.asarray(f, dtype=np.float64), shape, idx)
    c = 1 << k
    nz, ny, nx = shape
    fc = g.reshape(nz // c, c, ny // c, c, nx // c, c).mean(axis=(1, 3, 5))
    hc = h * c
    return fc * (hc[0] * hc[1] * hc[2]), hc


def _centres(tree, hc, n):
    """Coordinates (x, y, z) of the coarse cell centres, numpy order (z, y, x)."""
    ax = [tree.lo[a] + (np.arange(n[a]) + 0.5) * hc[a] for a in range(3)]
    z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def potential(q, centres, points):
    """phi(p) = -(1/4 pi) sum_c q_c / |p - x_c| at each point p (free-space Green's
    function of the Laplacian, the potential vanishing at infinity)."""
    q = np.asarray(q, dtype=np.float64).ravel()
    out = np.empty(len(points))
    chunk = max(1, (1 << 21) // max(1, len(centres)))
    for s in range(0, len(points), chunk):
        p = points[s:s + chunk]
        d = np.sqrt(((p[:, None, :] - centres[None, :, :]) ** 2).sum(axis=2))
        out[s:s + chunk] = -(q[None, :] / d).sum(axis=1) / FOUR_PI
    return out


def _inplane(face):
    a = face // 2
    t1, t2 = [b for b in range(3) if b != a]
    return a, t1, t2


def plane_points(tree, hc, face):
    """Points of boundary plane `face`: the coarse face centres with one ghost position
    on each side, shape ((n2 + 2) * (n1 + 2), 3), in-plane axis t1 fastest."""
    a, t1, t2 = _inplane(face)
    n = [int(round((tree.hi[b] - tree.lo[b]) / hc[b])) for b in range(3)]
    u1 = tree.lo[t1] + (np.arange(-1, n[t1] + 1) + 0.5) * hc[t1]
    u2 = tree.lo[t2] + (np.arange(-1, n[t2] + 1) + 0.5) * hc[t2]
    P2, P1 = np.meshgrid(u2, u1, indexing="ij")
    pts = np.zeros((P1.size, 3))
    pts[:, t1] = P1.ravel()
    pts[:, t2] = P2.ravel()
    pts[:, a] = tree.hi[a] if face & 1 else tree.lo[a]
    return pts, (n[t2] + 2, n[t1] + 2)


def planes(tree, f, k):
    """The free-space potential on the six boundary planes (list of 2D arrays, index
    [t2 + 1, t1 + 1] for coarse face cell (t1, t2), ghosts at -1 and n)."""
    q, hc = coarse_charges(tree, f, k)
    n = [q.shape[2], q.shape[1], q.shape[0]]
    cen = _centres(tree, hc, n)
    out = []
    for face in range(6):
        pts, shp = plane_points(tree, hc, face)
        out.append(potential(q, cen, pts).reshape(shp))
    return out, hc


def interpolate(tree, plane, hc, face):
    """Linear interpolation (in both in-plane directions) of a boundary plane to the
    centres of the leaf faces, array [j2, j1]."""
    _, t1, t2 = _inplane(face)
    h = (tree.hi - tree.lo) / tree.base
    n1, n2 = int(tree.base[t1]), int(tree.base[t2])

    def coords(n, hh, hcc):
        u = (np.arange(n) + 0.5) * hh / hcc - 0.5    # position in coarse cell units
        i = np.floor(u).astype(int)
        return i + 1, u - i                           # plane index (ghost at 0), weight

    i1, w1 = coords(n1, h[t1], hc[t1])
    i2, w2 = coords(n2, h[t2], hc[t2])
    I2, I1 = np.meshgrid(i2, i1, indexing="ij")
    W2, W1 = np.meshgrid(w2, w1, indexing="ij")
    return ((1 - W2) * ((1 - W1) * plane[I2, I1] + W1 * plane[I2, I1 + 1])
            + W2 * ((1 - W1) * plane[I2 + 1, I1] + W1 * plane[I2 + 1, I1 + 1]))


def boundary_values(tree, f, k):
    """Dirichlet values on the leaf faces of the six boundary faces (list of arrays
    [j2, j1]) from the free-space potential of the right-hand side restricted k levels."""
    pl, hc = planes(tree, f, k)
    return [interpolate(tree, pl[face], hc, face) for face in range(6)]


def flatten(bvals):
    """The face-by-face order of the library's boundary-value output."""
    return np.concatenate([b.ravel() for b in bvals])


def fold(tree, f, bvals):
    """f - 2 a / h_a^2 on the boundary cells of every face (leaf order): the right-hand
    side that carries Dirichlet values a into a solve with homogeneous faces."""
    shape, idx, h = _grid_of(tree)
    g = _to_grid(np.asarray(f, dtype=np.float64), shape, idx)
    for face in range(6):
        a = face // 2
        ax = 2 - a                                   # numpy axis of x_a
        sl = [slice(None)] * 3
        sl[ax] = -1 if face & 1 else 0
        # bvals[face] is [j2, j1] with t1 < t2, i.e. numpy order of the remaining axes
        g[tuple(sl)] -= 2.0 * bvals[face] / (h[a] * h[a])
    return g[idx]


def freespace_rhs(tree, f, k):
    """(folded right-hand side, boundary values) for the free-space problem."""
    bv = boundary_values(tree, f, k)
    return fold(tree, f, bv), bv


def far_field_guess(tree, f, k):
    """Initial guess for the cycles: the potential -Q / (4 pi r) of the
    coarse charges' total Q placed at their centroid, r at least one coarse spacing, on
    the leaf cells (leaf order); zero for a neutral source (|Q| <= 1e-12 sum |q|).  The
    paper starts from its uniform-grid free-space solution instead."""
    q, hc = coarse_charges(tree, f, k)
    qq = q.ravel()
    cen = _centres(tree, hc, [q.shape[2], q.shape[1], q.shape[0]])
    lay = tree.leaf_layout()
    Q = qq.sum()
    if not abs(Q) > 1e-12 * np.abs(qq).sum():
        return np.zeros(len(lay))
    xbar = (qq[:, None] * cen).sum(axis=0) / Q
    h = (tree.hi - tree.lo) / tree.base
    x = np.stack([tree.lo[a] + (lay[:, 1 + a] + 0.5) * h[a] for a in range(3)], axis=1)
    r = np.maximum(np.sqrt(((x - xbar) ** 2).sum(axis=1)), hc.min())
    return -Q / (FOUR_PI * r)


# ------------------------------------------------------------ Sec. 3.2 test problem
def gauss_rhs(x, y, z, sigma=0.1, r0=(0.0, 0.0, 0.0)):
    """eq. gauss-rhs: -exp(-|r - r0|^2 / sigma^2) / (sigma^3 pi^(3/2))."""
    r2 = (x - r0[0]) ** 2 + (y - r0[1]) ** 2 + (z - r0[2]) ** 2
    return -np.exp(-r2 / sigma ** 2) / (sigma ** 3 * np.pi ** 1.5)


def gauss_sol(x, y, z, sigma=0.1, r0=(0.0, 0.0, 0.0)):
    """eq. gauss-sol: erf(|r - r0| / sigma) / (4 pi |r - r0|), with its limit
    1 / (2 pi^(3/2) sigma) at the centre."""
    from scipy.special import erf
    r = np.sqrt((x - r0[0]) ** 2 + (y - r0[1]) ** 2 + (z - r0[2]) ** 2)
    out = np.empty_like(r)
    small = r < 1e-12
    out[small] = 1.0 / (2.0 * np.pi ** 1.5 * sigma)
    out[~small] = erf(r[~small] / sigma) / (FOUR_PI * r[~small])
    return out
