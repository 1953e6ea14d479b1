"""Restarted flexible GMRES (Saad, "A flexible inner-outer preconditioned GMRES
algorithm", 1993) in plain numpy, for checking the library's FGMRES refinement.

Test infrastructure, like the rest of this package: only the tests, the smoke check
and the benchmark's CPU baseline use it.

fgmres(apply, precond, b, x0, m, tol, max_restarts) solves apply(x) = b.  Each
restart forms r = b - apply(x), runs at most m Arnoldi steps on the preconditioned
directions z_j = precond(v_j) (modified Gram-Schmidt), stops early once the
least-squares residual estimate is below 1e-6 ||r||, and sets x += Z y with y the
minimiser of ||beta e_1 - H y||.  Returns x and the list of true residual norms
(max norm relative to max |b|) at the start of each restart.
"""
import numpy as np


def fgmres(apply, precond, b, x0, m=20, tol=1e-10, max_restarts=50, inner_tol=1e-6):
    x = np.array(x0, dtype=np.float64, copy=True)
    bmax = np.abs(b).max()
    hist = []
    for _ in range(max_restarts):
        r = b - apply(x)
        hist.append(np.abs(r).max() / bmax)
        if hist[-1] <= tol:
            break
        beta = np.linalg.norm(r)
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        k = 0
        for j in range(m):
            z = precond(V[j])
            Z.append(z)
            w = apply(z)
            for i in range(j + 1):
                H[i, j] = V[i] @ w
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            k = j + 1
            e1 = np.zeros(k + 1)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(H[:k + 1, :k], e1, rcond=None)
            est = np.linalg.norm(e1 - H[:k + 1, :k] @ y)
            if H[j + 1, j] == 0.0 or est <= inner_tol * beta:
                break
            V.append(w / H[j + 1, j])
        e1 = np.zeros(k + 1)
        e1[0] = beta
        y, *_ = np.linalg.lstsq(H[:k + 1, :k], e1, rcond=None)
        x = x + sum(yi * zi for yi, zi in zip(y, Z))
    return x, hist
