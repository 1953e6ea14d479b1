"""Divergence cleaning in the reference solver (Sec. 4.1), pinned to closed forms.

On a periodic grid every difference operator is diagonal in Fourier modes, so one mode
of B goes through the whole projection in closed form: for B_x = sin(kx) the
second-order divergence is (sin(kh)/h) cos(kx), the fourth-order one
((8 sin(kh) - sin(2kh))/(6h)) cos(kx), the compact Laplacian has the symbol
-4 sin^2(kh/2)/h^2, and the central gradient of cos(kx) is -(sin(kh)/h) sin(kx).
With the second-order divergence the cleaned field is sin^2(kh/2) sin(kx).  Central
differences along different axes commute, so the central curl of any periodic A is
exactly divergence-free and passes through unchanged.
"""
import numpy as np
import pytest

from oracle import DIRICHLET, NEUMANN, PERIODIC, OracleTree
from oracle import divb
from paper_1901_11370_amd import workloads as W


def _tree(dim, n, lo, hi, kinds, values=None, bs=8):
    t = OracleTree(dim, n, lo, hi, kinds, bc_value=values, bs=bs)
    t.set_params(rel_tol=1e-12)
    return t


def _centres(t):
    dom = W.Domain(t.dim, list(t.base[:t.dim]), list(t.lo[:t.dim]), list(t.hi[:t.dim]), [0] * (2 * t.dim))
    return W.cell_centres(t.leaf_layout(), dom)


def _symbols(k, h, order):
    d = np.sin(k * h) / h if order == 2 else (8 * np.sin(k * h) - np.sin(2 * k * h)) / (6 * h)
    phi = -d / (4 * np.sin(k * h / 2) ** 2 / h ** 2)       # phi amplitude of cos(kx)
    return d, 1.0 + phi * np.sin(k * h) / h                # div amplitude, cleaned amplitude


@pytest.mark.parametrize("order", [2, 4])
def test_single_modes_in_closed_form(order):
    # the field-loop domain of Sec. 4.2, [-1,1] x [-1/2,1/2], periodic, h = 1/32
    t = _tree(2, [64, 32], [-1, -0.5], [1, 0.5], [PERIODIC] * 4)
    x = _centres(t)
    h = 1.0 / 32
    kx, ky = 2 * np.pi * 3 / 2.0, 2 * np.pi * 2 / 1.0
    B = np.array([np.sin(kx * x[:, 0]), 0.5 * np.cos(ky * x[:, 1])])
    dx, cx = _symbols(kx, h, order)
    dy, cy = _symbols(ky, h, order)
    f = divb.divergence(t, B, order)
    assert np.abs(f - (dx * np.cos(kx * x[:, 0]) - 0.5 * dy * np.sin(ky * x[:, 1]))).max() < 1e-11
    Bn, _, _, hist = divb.clean(t, B, order=order)
    assert hist[-1] <= 1e-12
    assert np.abs(Bn[0] - cx * np.sin(kx * x[:, 0])).max() < 1e-9
    assert np.abs(Bn[1] - 0.5 * cy * np.cos(ky * x[:, 1])).max() < 1e-9
    if order == 2:
        assert abs(cx - np.sin(kx * h / 2) ** 2) < 1e-14


def test_central_curl_passes_unchanged():
    # the curl built with the same central differences as the divergence (order 2 or
    # 4) is exactly divergence-free: differences along different axes commute
    t = _tree(3, [16, 16, 32], [0, 0, 0], [1, 1, 2], [PERIODIC] * 6, bs=8)
    rng = np.random.default_rng(7)
    n = (32, 16, 16)        # (z, y, x)
    A = rng.normal(size=(3,) + n)
    h = 1.0 / 16
    lay = t.leaf_layout()
    idx = (lay[:, 3], lay[:, 2], lay[:, 1])
    e = rng.uniform(1, 2, size=t.n_leaf)
    for order in (2, 4):
        def dc(a, d):
            ax = 2 - d
            s = lambda o: np.roll(a, -o, axis=ax)
            if order == 2:
                return (s(1) - s(-1)) / (2 * h)
            return (-s(2) + 8 * s(1) - 8 * s(-1) + s(-2)) / (12 * h)

        curl = np.array([dc(A[2], 1) - dc(A[1], 2), dc(A[0], 2) - dc(A[2], 0), dc(A[1], 0) - dc(A[0], 1)])
        B = np.array([c[idx] for c in curl])
        assert np.abs(divb.divergence(t, B, order)).max() < 1e-12 * np.abs(B).max() / h
        Bn, en, _, _ = divb.clean(t, B, e, order=order)
        assert np.abs(Bn - B).max() < 1e-11 * np.abs(B).max()
        assert np.abs(en - e).max() < 1e-11 * np.abs(B).max() ** 2


def test_divergence_orders_of_accuracy():
    errs = {2: [], 4: []}
    for n in (32, 64, 128):
        t = _tree(2, [n, n], [0, 0], [1, 1], [PERIODIC] * 4, bs=16)
        x = _centres(t)
        B = np.array([np.sin(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1]),
                      np.cos(4 * np.pi * x[:, 1]) * np.sin(2 * np.pi * x[:, 0])])
        exact = (2 * np.pi * np.cos(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1])
                 - 4 * np.pi * np.sin(4 * np.pi * x[:, 1]) * np.sin(2 * np.pi * x[:, 0]))
        for order in (2, 4):
            errs[order].append(np.abs(divb.divergence(t, B, order) - exact).max())
    for order, expect in ((2, 4.0), (4, 16.0)):
        ratios = np.array(errs[order][:-1]) / np.array(errs[order][1:])
        assert np.all(np.abs(ratios - expect) < 0.1 * expect), (order, ratios)


def test_zero_gradient_boundary_layers():
    # B_x = x on a Dirichlet box: interior divergence 1; the repeated boundary cell
    # gives 1/2 in the first cell (both orders) and 13/12 in the second (order 4)
    t = _tree(2, [32, 16], [0, 0], [2, 1], [DIRICHLET] * 4)
    x = _centres(t)
    lay = t.leaf_layout()
    i = lay[:, 1]
    B = np.array([x[:, 0], np.zeros(t.n_leaf)])
    f2, f4 = divb.divergence(t, B, 2), divb.divergence(t, B, 4)
    edge = (i == 0) | (i == 31)
    assert np.allclose(f2[~edge], 1.0, atol=1e-12) and np.allclose(f2[edge], 0.5, atol=1e-12)
    second = (i == 1) | (i == 30)
    assert np.allclose(f4[edge], 0.5, atol=1e-12) and np.allclose(f4[second], 13 / 12, atol=1e-12)
    assert np.allclose(f4[~(edge | second)], 1.0, atol=1e-12)


@pytest.mark.parametrize("kind", [DIRICHLET, NEUMANN])
def test_gradient_uses_solver_ghosts(kind):
    # phi linear: the Dirichlet ghost 2a - phi_b (a the value on the face) and the
    # Neumann ghost phi_b -/+ h b (b = d phi / d x_d) both extend phi linearly, so the
    # central gradient is exact in the boundary cells too; e follows eq. divb-pressure-fix
    lo, hi = np.array([0.0, 0.0]), np.array([1.0, 0.5])
    t0 = _tree(2, [16, 8], lo, hi, [PERIODIC] * 4)
    x = _centres(t0)
    phi = 2 * x[:, 0] + 3 * x[:, 1]
    if kind == NEUMANN:
        t = _tree(2, [16, 8], lo, hi, [NEUMANN] * 4, [2.0, 2.0, 3.0, 3.0])
        g = divb.gradient(t, phi)
        assert np.allclose(g[0], 2.0, atol=1e-12) and np.allclose(g[1], 3.0, atol=1e-12)
    else:
        # a Dirichlet value is one number per face, so phi = 2x with phi = 0 and 2 on
        # the x faces (periodic in y)
        phi = 2 * x[:, 0]
        t = _tree(2, [16, 8], lo, hi, [DIRICHLET, DIRICHLET, PERIODIC, PERIODIC], [0.0, 2.0, 0, 0])
        g = divb.gradient(t, phi)
        assert np.allclose(g[0], 2.0, atol=1e-12) and np.allclose(g[1], 0.0, atol=1e-12)
    B = np.array([np.full(t.n_leaf, 2.5), np.full(t.n_leaf, -1.0)])
    e = np.full(t.n_leaf, 10.0)
    Bn, en = divb.project(t, B, phi, e)
    assert np.allclose(Bn[0], 2.5 - (2.0 if kind == DIRICHLET else 2.0), atol=1e-12)
    assert np.allclose(Bn[1], -1.0 - (0.0 if kind == DIRICHLET else 3.0), atol=1e-12)
    # the thermal part e - |B|^2 / 2 is what the energy fix keeps
    assert np.allclose(en - 0.5 * (Bn ** 2).sum(axis=0), e - 0.5 * (B ** 2).sum(axis=0), atol=1e-12)
