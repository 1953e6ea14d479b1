"""Differentiable multigrid solve: phi = L(eps)^-1 f as a torch.autograd.Function.

Forward solves div(eps grad phi) = f on the tree (FP64, or FP32 cycles inside FP64
iterative refinement) to a relative residual tolerance.  Only phi, f and eps are
saved -- no cycle history.  Backward, given g = dJ/dphi, solves the adjoint problem
L lambda = g with the same multigrid and homogeneous boundary values (the discrete
operator of a tree without refinement is symmetric: harmonic-mean face coefficients
and reflection ghosts), then

    dJ/df   = lambda,
    dJ/deps = face-gradient kernel: for each cell, over its faces,
              interior: h^-2 * 2 eps_j^2 / (eps_i + eps_j)^2 * (lambda_j - lambda_i)(phi_j - phi_i)
              boundary: -h^-2 * lambda_i * (phi_g - phi_i).

The formulas follow from differentiating the discrete operator of the paper's
eq. poisson-2d-vcoeff: for L phi = f, dJ/deps_k = -lambda^T (dL/deps_k) phi.
"""
from __future__ import annotations

import torch

from . import mg


class MGSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, eps, tree, rel_tol=1e-10, max_cycles=60):
        if tree.store is None:
            raise RuntimeError("tree is not bound to a device store")
        f = f.detach().to(torch.float64).contiguous()
        eps = eps.detach().to(torch.float64).contiguous()
        tree.set_eps(eps)
        tree.set_rhs(f)
        tree.set_phi(torch.zeros_like(f))
        tree.solve(rel_tol=rel_tol, max_cycles=max_cycles, fmg_first=True)
        phi = torch.empty_like(f)
        tree.get_phi(out=phi)
        ctx.save_for_backward(phi, f, eps)
        ctx.tree = tree
        ctx.rel_tol = rel_tol
        ctx.max_cycles = max_cycles
        return phi

    @staticmethod
    def backward(ctx, g):
        phi, f, eps = ctx.saved_tensors
        tree = ctx.tree
        g = g.detach().to(torch.float64).contiguous()
        tree.set_eps(eps)
        tree.set_homogeneous_bc(True)
        try:
            tree.set_rhs(g)
            tree.set_phi(torch.zeros_like(g))
            tree.solve(rel_tol=ctx.rel_tol, max_cycles=ctx.max_cycles, fmg_first=True)
            lam = torch.empty_like(g)
            tree.get_phi(out=lam)
        finally:
            tree.set_homogeneous_bc(False)
        g_eps = tree.face_gradient(phi, lam)
        # the tree's state is phi again (the face gradient leaves phi in it)
        return lam, g_eps, None, None, None


def mg_solve(f, eps, tree, rel_tol=1e-10, max_cycles=60):
    """phi = L(eps)^-1 f, differentiable in f and eps."""
    return MGSolve.apply(f, eps, tree, rel_tol, max_cycles)
