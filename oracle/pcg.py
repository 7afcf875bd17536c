"""Preconditioned conjugate gradients with a Lanczos condition estimate
(oracle).

TEST INFRASTRUCTURE: the FP64 CPU oracle (see oracle/__init__.py).

CG on T = BA (Sec. 3.1, Sec. 4.1) from x0 = 0, stopped when the residual
2-norm falls to rtol times ||b||_2 (Sec. 4.1 uses rtol = 1e-8). The CG step
lengths alpha_k and ratios beta_k define the Lanczos tridiagonal matrix of
BA, T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1}, T_{j,j+1} = sqrt(beta_j)/alpha_j,
whose extreme eigenvalues estimate lambda_min(T), lambda_max(T) and the
iterative condition number kappa(T) of Sec. 3.1.
"""
from __future__ import annotations

import numpy as np


def lanczos_extremes(alphas, betas):
    n = len(alphas)
    if n == 0:
        return float("nan"), float("nan")
    T = np.zeros((n, n))
    for j in range(n):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < n:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    ev = np.linalg.eigvalsh(T)
    return float(ev[0]), float(ev[-1])


def pcg(A, B, b, rtol=1e-8, maxit=1000, x0=None):
    """A, B: callables v -> A v, v -> B v. Returns (x, info dict)."""
    b = np.asarray(b, dtype=float)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=float)
    r = b - A(x)
    bnorm = np.linalg.norm(b)
    z = B(r)
    p = z.copy()
    rz = float(r @ z)
    alphas, betas = [], []
    it = 0
    converged = np.linalg.norm(r) <= rtol * bnorm
    while not converged and it < maxit:
        Ap = A(p)
        pAp = float(p @ Ap)
        if pAp <= 0 or rz <= 0:
            raise FloatingPointError("CG breakdown: operator or preconditioner not SPD")
        alpha = rz / pAp
        x += alpha * p
        r -= alpha * Ap
        alphas.append(alpha)
        it += 1
        if np.linalg.norm(r) <= rtol * bnorm:
            converged = True
            break
        z = B(r)
        rz_new = float(r @ z)
        beta = rz_new / rz
        betas.append(beta)
        p = z + beta * p
        rz = rz_new
    lmin, lmax = lanczos_extremes(alphas, betas)
    return x, dict(iters=it, converged=converged,
                   rel_res=float(np.linalg.norm(r) / bnorm) if bnorm > 0 else 0.0,
                   lambda_min=lmin, lambda_max=lmax, cond=lmax / lmin,
                   alphas=alphas, betas=betas)
