"""Seeded synthetic inputs for the multigrid workloads.

This module holds no part of the solver's arithmetic: it only describes domains and
evaluates right-hand sides, coefficients, targets and refinement predicates at cell
centres that it computes from the integer leaf layout (level above base, I, J, K) each
library reports.  Both the GPU library's tests/benchmark and the reference solver read
their inputs from here, so the two always see identical arrays.

Shapes follow the paper's test problems (Sec. 3): unit cubes/squares, 16^d blocks,
Dirichlet or periodic boundaries, Gaussian sources.  Random parameters come from
``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional, Sequence

import numpy as np

DIRICHLET, NEUMANN, PERIODIC = 0, 1, 2


@dataclass
class Domain:
    dim: int
    base_cells: Sequence[int]
    lo: Sequence[float]
    hi: Sequence[float]
    bc_kind: Sequence[int]
    bc_value: Sequence[float] = field(default_factory=lambda: [0.0] * 6)

    def h_base(self):
        return [(self.hi[d] - self.lo[d]) / self.base_cells[d] for d in range(self.dim)]


def cell_centres(layout: np.ndarray, dom: Domain) -> np.ndarray:
    """(n, dim) centres of the cells listed in an integer layout (level, I, J, K)."""
    layout = np.asarray(layout)
    out = np.empty((layout.shape[0], dom.dim))
    scale = 2.0 ** layout[:, 0].astype(np.float64)
    for d in range(dom.dim):
        h = (dom.hi[d] - dom.lo[d]) / dom.base_cells[d] / scale
        out[:, d] = dom.lo[d] + (layout[:, d + 1] + 0.5) * h
    return out


def cell_widths(layout: np.ndarray, dom: Domain) -> np.ndarray:
    scale = 2.0 ** np.asarray(layout)[:, 0].astype(np.float64)
    return np.stack([(dom.hi[d] - dom.lo[d]) / dom.base_cells[d] / scale for d in range(dom.dim)], axis=1)


def face_centres(layout: np.ndarray, dom: Domain, faces: np.ndarray) -> np.ndarray:
    """(n, dim) centres of face `faces[i]` (0..2 dim - 1: -x, +x, -y, ...) of the cells
    listed in an integer layout (level, I, J, K)."""
    x = cell_centres(layout, dom)
    w = cell_widths(layout, dom)
    faces = np.asarray(faces)
    for a in range(dom.dim):
        on = faces // 2 == a
        sgn = np.where(faces[on] % 2 == 1, 0.5, -0.5)
        x[on, a] += sgn * w[on, a]
    return x


def block_centres(dom: Domain, level: int, origin, bs: int) -> np.ndarray:
    """Centres of the bs^d cells of a block given its level (above base) and origin."""
    ax = []
    for d in range(dom.dim):
        h = (dom.hi[d] - dom.lo[d]) / dom.base_cells[d] / 2.0 ** level
        ax.append(dom.lo[d] + (origin[d] + 0.5 + np.arange(bs)) * h)
    g = np.meshgrid(*ax, indexing="ij")
    return np.stack([x.ravel() for x in g], axis=1)


# ----------------------------------------------------------------- sources
@dataclass
class Gaussians:
    centres: np.ndarray     # (k, dim)
    amps: np.ndarray        # (k,)
    sigmas: np.ndarray      # (k,)
    periodic: bool = False

    def __call__(self, x: np.ndarray) -> np.ndarray:
        out = np.zeros(x.shape[0])
        for c, a, s in zip(self.centres, self.amps, self.sigmas):
            d = x - c
            if self.periodic:
                d = d - np.round(d)
            out += a * np.exp(-np.sum(d * d, axis=1) / (s * s))
        return out


def sine_rhs_2d(x):
    """f = -2 pi^2 sin(pi x) sin(pi y), whose solution is sin(pi x) sin(pi y)."""
    return -2.0 * np.pi ** 2 * np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1])


# --------------------------------------------------------------- workloads
@dataclass
class Workload:
    name: str
    domains: list
    bs: int = 16
    max_refine: int = 0
    refine: Optional[Callable] = None   # refine(domain, level, origin, bs) -> bool
    variable_eps: bool = False
    rhs: Optional[Callable] = None      # rhs(domain_index, layout) -> f
    eps: Optional[Callable] = None      # eps(domain_index, layout) -> eps
    target: Optional[Callable] = None
    # dirichlet(domain_index, face centres (n, dim)) -> values of a Dirichlet boundary
    # that varies along the faces (None: the domains' constant face values)
    dirichlet: Optional[Callable] = None
    note: str = ""


def _unit(dim, n, bc):
    return Domain(dim, [n] * dim, [0.0] * dim, [1.0] * dim, [bc] * (2 * dim))


def config1(n: int = 128) -> Workload:
    """2D Poisson on the unit square, 128^2 cells in 16^2 blocks, phi = 0 on the
    boundary, f from the manufactured phi = sin(pi x) sin(pi y)."""
    dom = _unit(2, n, DIRICHLET)
    return Workload("poisson2d_128_dirichlet_sine", [dom],
                    rhs=lambda i, lay: sine_rhs_2d(cell_centres(lay, dom)))


def config2(n: int = 256, seed: int = 2) -> Workload:
    """3D periodic Poisson, n^3 cells in 16^3 blocks; f = sum of 32 Gaussians
    (sigma 0.02, centres uniform, amplitudes +-1, minimum-image distance), with the
    discrete mean removed."""
    rng = np.random.default_rng(seed)
    centres = rng.random((32, 3))
    amps = np.where(rng.random(32) < 0.5, -1.0, 1.0)
    g = Gaussians(centres, amps, np.full(32, 0.02), periodic=True)
    dom = _unit(3, n, PERIODIC)

    def rhs(i, lay):
        f = g(cell_centres(lay, dom))
        return f - f.mean()
    return Workload(f"poisson3d_{n}_periodic_32gauss", [dom], rhs=rhs)


def _config3_sources(seed=3):
    rng = np.random.default_rng(seed)
    sig = rng.uniform(0.005, 0.02, 4)
    centres = rng.uniform(0.1, 0.9, (4, 3))
    amps = np.where(rng.random(4) < 0.5, -1.0, 1.0)
    return Gaussians(centres, amps, sig)


def config3(nested: bool = True, base: int = 128, seed: int = 3) -> Workload:
    """3D AMR octree, base 128^3 in 16^3 blocks, 3 refinement levels, phi = 0 on the
    boundary, f = 4 Gaussians (sigma 0.005-0.02).

    nested=False: the literal rule, a block is refined where |f| > 0.05 max|a_k| at
    one of its cell centres.  nested=True: the paper-shaped nested layout of about
    1.16e8 leaf cells (level 1 everywhere, level 2 on [0.125,0.875]^3, level 3 on
    [0.3125,0.6875]^3) with the same f."""
    g = _config3_sources(seed)
    dom = _unit(3, base, DIRICHLET)
    thr = 0.05 * np.max(np.abs(g.amps))

    def literal(d, level, origin, bs):
        x = block_centres(dom, level, origin, bs)
        return bool(np.any(np.abs(g(x)) > thr))

    boxes = {0: (0.0, 1.0), 1: (0.125, 0.875), 2: (0.3125, 0.6875)}

    def nested_rule(d, level, origin, bs):
        if level not in boxes:
            return False
        lo, hi = boxes[level]
        h = 1.0 / (base * 2 ** level)
        for k in range(3):
            a, b = origin[k] * h, (origin[k] + bs) * h
            if a < lo - 1e-12 or b > hi + 1e-12:
                return False
        return True

    return Workload("poisson3d_amr_" + ("nested" if nested else "literal"), [dom], max_refine=3,
                    refine=nested_rule if nested else literal,
                    rhs=lambda i, lay: g(cell_centres(lay, dom)))


def config4(nested: bool = True, seed: int = 4) -> Workload:
    """Config-3 tree and f with eps = 1 + 999 s, s a linear ramp over two leaf cells
    around three spheres of radius 0.1 (centres uniform in [0.1,0.9]^3)."""
    w = config3(nested)
    dom = w.domains[0]
    rng = np.random.default_rng(seed)
    C = rng.uniform(0.1, 0.9, (3, 3))

    def eps(i, lay):
        x = cell_centres(lay, dom)
        hl = cell_widths(lay, dom)[:, 0]
        s = np.zeros(x.shape[0])
        for c in C:
            r = np.sqrt(np.sum((x - c) ** 2, axis=1))
            s = np.maximum(s, np.clip(0.5 - (r - 0.1) / (2.0 * hl), 0.0, 1.0))
        return 1.0 + 999.0 * s
    w.name = w.name.replace("poisson3d", "varcoef3d")
    w.variable_eps = True
    w.eps = eps
    return w


CONFIG5_SIZES = (64, 96, 128, 160, 192, 256)


def _lognormal_field(n, seed, corr=8.0):
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n, n))
    k = np.fft.fftfreq(n)
    kk = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    kern = np.exp(-2.0 * np.pi ** 2 * corr ** 2 * kk)   # Gaussian of std `corr` cells
    g = np.real(np.fft.ifftn(np.fft.fftn(w) * kern))
    g = (g - g.mean()) / g.std()
    return g  # indexed [I, J, K]


def config5(sizes: Sequence[int] = CONFIG5_SIZES) -> Workload:
    """Batch of independent unit cubes (64^3 ... 256^3, 16^3 blocks, phi = 0 on the
    boundary); eps = exp(0.5 g), g unit-variance noise with 8-cell Gaussian
    correlation; f = 8 Gaussians (width 0.05, amplitudes +-1); target
    1e-3 sin(pi x) sin(pi y) sin(pi z)."""
    doms = [_unit(3, n, DIRICHLET) for n in sizes]
    srcs = []
    for i, n in enumerate(sizes):
        rng = np.random.default_rng(510 + i)
        c = rng.uniform(0.2, 0.8, (8, 3))
        a = np.where(rng.random(8) < 0.5, -1.0, 1.0)
        srcs.append(Gaussians(c, a, np.full(8, 0.05)))

    def rhs(i, lay):
        return srcs[i](cell_centres(lay, doms[i]))

    def eps(i, lay):
        g = _lognormal_field(sizes[i], 500 + i)
        return np.exp(0.5 * g[lay[:, 1], lay[:, 2], lay[:, 3]])

    def target(i, lay):
        x = cell_centres(lay, doms[i])
        return 1e-3 * np.prod(np.sin(np.pi * x), axis=1)

    return Workload("diffsolve3d_batch6", doms, variable_eps=True, rhs=rhs, eps=eps, target=target)


# ------------------------------------------------------- convergence test (Sec. 3.1)
X1_N = np.array([1.0, 2.0, 3.0])


def x1_solution(x: np.ndarray) -> np.ndarray:
    """phi_sol = cos(pi n.x) + 10 exp(-100 |x|^2), n = (1, 2, 3) (eq. poisson-conv)."""
    return np.cos(np.pi * x @ X1_N) + 10.0 * np.exp(-100.0 * np.sum(x * x, axis=1))


def x1_laplacian(x: np.ndarray) -> np.ndarray:
    """Analytic Laplacian of x1_solution."""
    r2 = np.sum(x * x, axis=1)
    return (-np.pi ** 2 * np.dot(X1_N, X1_N) * np.cos(np.pi * x @ X1_N)
            + 10.0 * np.exp(-100.0 * r2) * (-600.0 + 40000.0 * r2))


def x1(grid: str = "uniform", base: int = 64) -> Workload:
    """The paper's convergence test (Sec. 3.1): unit cube centred at the origin,
    lap(phi) = f with f the analytic Laplacian of x1_solution and Dirichlet values
    from the solution at the boundary face centres (``dirichlet``).  grid: 'uniform'
    (base^3), 'center' or 'corner' (two extra levels covering 0.5^3 and 0.25^3, each
    again base^3 cells, centred at the origin or around (-0.25, -0.25, -0.25))."""
    dom = Domain(3, [base] * 3, [-0.5] * 3, [0.5] * 3, [DIRICHLET] * 6)
    if grid == "center":
        boxes = {0: (-0.25, 0.25), 1: (-0.125, 0.125)}
    elif grid == "corner":
        boxes = {0: (-0.5, 0.0), 1: (-0.375, -0.125)}
    else:
        boxes = {}

    def rule(d, level, origin, bs):
        if level not in boxes:
            return False
        lo, hi = boxes[level]
        h = 1.0 / (base * 2 ** level)
        return all(lo - 1e-12 <= -0.5 + origin[q] * h and -0.5 + (origin[q] + bs) * h <= hi + 1e-12
                   for q in range(3))

    return Workload(f"convergence_{grid}_{base}", [dom], max_refine=len(boxes), refine=rule if boxes else None,
                    rhs=lambda i, lay: x1_laplacian(cell_centres(lay, dom)),
                    dirichlet=lambda i, xf: x1_solution(xf),
                    note="phi_sol = cos(pi n.x) + 10 exp(-100|x|^2), n = (1,2,3)")


# ------------------------------------------------ divergence cleaning (Sec. 4)
def field_loop_B(dom: Domain, x: np.ndarray, seed: int = 11, amp: float = 2e-4) -> np.ndarray:
    """Cell-centred magnetic field of shape (dim, n): the field loop of Sec. 4.2
    (vector potential A_z = A0 (R0 - r) for r <= R0 around the z axis, A0 = 1e-3,
    R0 = 0.3; B_x = dA_z/dy, B_y = -dA_z/dx by central differences on the cell
    centres, as the paper sets it up), plus a seeded sum of Gaussian bumps in every
    component (width^2 0.05, amplitude amp) that gives B a divergence to clean."""
    dim = dom.dim
    h = (np.array(dom.hi, dtype=float) - np.array(dom.lo, dtype=float)) / np.array(dom.base_cells, dtype=float)
    A0, R0 = 1e-3, 0.3

    def Az(p):
        r = np.sqrt(p[:, 0] ** 2 + p[:, 1] ** 2)
        return np.where(r <= R0, A0 * (R0 - r), 0.0)

    B = np.zeros((dim, len(x)))
    ex = np.zeros(dim)
    ex[0] = h[0]
    ey = np.zeros(dim)
    ey[1] = h[1]
    B[0] = (Az(x + ey) - Az(x - ey)) / (2 * h[1])
    B[1] = -(Az(x + ex) - Az(x - ex)) / (2 * h[0])
    rng = np.random.default_rng(seed)
    c = rng.uniform(np.array(dom.lo) + 0.2, np.array(dom.hi) - 0.2, size=(4, dim))
    for a in range(dim):
        for ck in c:
            B[a] += amp * rng.normal() * np.exp(-np.sum((x - ck) ** 2, axis=1) / 0.05)
    return B


def divb_periodic(n: int, dim: int = 3) -> Workload:
    """Periodic box [-1,1]^dim of n^dim cells in 16^dim blocks for the cleaning runs."""
    dom = Domain(dim, [n] * dim, [-1.0] * dim, [1.0] * dim, [PERIODIC] * (2 * dim))
    return Workload(f"divb_periodic{dim}d_{n}", [dom], bs=16)


def freespace_gauss(sizes: Sequence[int] = (64,), sigma: float = 0.1, bs: int = 16,
                    offsets: Optional[Sequence[Sequence[float]]] = None) -> Workload:
    """The free-space test of Sec. 3.2: unit cubes centred at the origin, each of n^3
    cells in bs^3 blocks, homogeneous Dirichlet faces (the free-space values are folded
    into the right-hand side), f = -exp(-|r - r0|^2 / sigma^2) / (sigma^3 pi^(3/2)) with
    r0 = 0 or the given per-domain offsets.  Several sizes make a forest of independent
    problems."""
    doms = [Domain(3, [n] * 3, [-0.5] * 3, [0.5] * 3, [DIRICHLET] * 6) for n in sizes]
    r0s = [tuple(o) for o in offsets] if offsets is not None else [(0.0, 0.0, 0.0)] * len(doms)

    def rhs(i, lay):
        x = cell_centres(lay, doms[i]) - np.asarray(r0s[i])
        return -np.exp(-np.sum(x * x, axis=1) / sigma ** 2) / (sigma ** 3 * np.pi ** 1.5)

    def target(i, lay):
        # the closed-form free-space solution erf(r / sigma) / (4 pi r)
        from scipy.special import erf
        x = cell_centres(lay, doms[i]) - np.asarray(r0s[i])
        r = np.sqrt(np.sum(x * x, axis=1))
        out = np.full(r.shape, 1.0 / (2.0 * np.pi ** 1.5 * sigma))
        nz = r > 1e-12
        out[nz] = erf(r[nz] / sigma) / (4.0 * np.pi * r[nz])
        return out
    name = "freespace_gauss_" + "_".join(str(n) for n in sizes)
    return Workload(name, doms, bs=bs, rhs=rhs, target=target, note=f"sigma={sigma}; centres {r0s}")
