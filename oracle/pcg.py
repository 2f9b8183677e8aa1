"""Oracle: BDDC-PCG on the reduced problem and the Lanczos condition estimate.

PCG is applied to the reduced problem (eq. (reduced-problem)) with the
preconditioner M_BDDC (eq. (s-BDDC)).  Following the Remark after Lemma 1 the
initial approximation is zero on the interface with interior Dirichlet solves,
so every residual vanishes in the interiors and (I - P)^T can be omitted.
Stopping: ||r_k||_2 <= rtol ||r_0||_2 with rtol = 1e-8 (Sec. 7: relative
residual tolerance 10^-8).  The condition number is estimated from the
Lanczos tridiagonal matrix built from the CG coefficients (Sec. 7, captions of
the result tables): diagonal 1/a_j + b_{j-1}/a_{j-1}, off-diagonal
sqrt(b_j)/a_j (the standard CG-Lanczos relation; the paper does not print
it).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def lanczos_tridiagonal(alphas, betas):
    """T_k from CG coefficients: diag_j = 1/a_j + b_{j-1}/a_{j-1},
    offdiag_j = sqrt(b_j)/a_j."""
    k = len(alphas)
    d = np.empty(k)
    e = np.empty(max(k - 1, 0))
    for j in range(k):
        d[j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j < k - 1:
            e[j] = np.sqrt(betas[j]) / alphas[j]
    return d, e


def lanczos_extremes(alphas, betas):
    if len(alphas) == 0:
        return np.nan, np.nan
    d, e = lanczos_tridiagonal(alphas, betas)
    ev = sla.eigvalsh_tridiagonal(d, e) if len(d) > 1 else d
    return float(ev.min()), float(ev.max())


def pcg(Aop, f, Mop, u0, rtol=1e-8, maxit=1000):
    """Preconditioned CG.  Returns dict(u, iters, relres, kappa, lmin, lmax,
    alphas, betas, resid)."""
    u = u0.copy()
    r = f - Aop(u)
    r0 = np.linalg.norm(r)
    res = [1.0]
    alphas, betas = [], []
    if r0 == 0.0:
        return dict(u=u, iters=0, relres=0.0, kappa=1.0, lmin=1.0, lmax=1.0,
                    alphas=alphas, betas=betas, resid=res)
    z = Mop(r)
    p = z.copy()
    rz = float(r @ z)
    it = 0
    converged = False
    for it in range(1, maxit + 1):
        q = Aop(p)
        alpha = rz / float(p @ q)
        alphas.append(alpha)
        u += alpha * p
        r -= alpha * q
        rel = np.linalg.norm(r) / r0
        res.append(rel)
        if rel <= rtol:
            converged = True
            break
        z = Mop(r)
        rz_new = float(r @ z)
        beta = rz_new / rz
        betas.append(beta)
        rz = rz_new
        p = z + beta * p
    lmin, lmax = lanczos_extremes(alphas, betas)
    return dict(u=u, iters=it, relres=res[-1], kappa=lmax / lmin, lmin=lmin, lmax=lmax,
                alphas=alphas, betas=betas, resid=res, converged=converged)
