"""Displacement-based linear CG of Algorithm 1 and a dense reference solve.

Reading of Algorithm 1 (its printed signs mix u += alpha d with f -= alpha z and
compute alpha from <z, d> with z = r(d)): with the residual map of eq.
resVector, f = b - A u, z = A d (the residual map with zero macro strain), and
standard preconditioned CG on A u = b.

Stopping criterion (eq. stoppingCriterion): res_k <= tol ||<sigma(u_k)>||, where
res_k = sqrt(f^T P^-1 f / |Y|) -- the preconditioned residual norm of eq.
convergence normalised by the cell volume so that it is a stress-like quantity
independent of the grid size -- and ||.|| is the Euclidean norm of the Mandel
6-vector.
"""

import numpy as np


def pcg(apply_A, b, apply_P, avg_stress, volume, tol, maxit, u0=None):
    """Returns (u, info) with info = dict(iters, res, sigma, history).

    ``avg_stress(u)`` returns <sigma(u)> for the current iterate.
    """
    u = np.zeros_like(b) if u0 is None else u0.copy()
    f = b - apply_A(u) if u0 is not None else b.copy()
    d = apply_P(f)
    res2 = float(f @ d)
    res = np.sqrt(max(res2, 0.0) / volume)
    sig = avg_stress(u)
    hist = [res]
    k = 0
    while k < maxit and res > tol * np.linalg.norm(sig):
        k += 1
        z = apply_A(d)
        dz = float(z @ d)
        if not dz > 0.0:
            raise FloatingPointError("CG breakdown: d^T A d <= 0")
        alpha = res2 / dz
        u += alpha * d
        f -= alpha * z
        y = apply_P(f)
        res2_new = float(f @ y)
        beta = res2_new / res2
        d = y + beta * d
        res2 = res2_new
        res = np.sqrt(max(res2, 0.0) / volume)
        sig = avg_stress(u)
        hist.append(res)
    return u, dict(iters=k, res=res, sigma=sig, history=hist)


def dense_solve(A, b, nfe):
    """Minimum-norm least-squares solution of the singular system A u = b.

    The null space of A is spanned by the constant FE translations, so the
    minimum-norm solution has a mean-free FE part.
    """
    A = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    u, *_ = np.linalg.lstsq(A, b, rcond=None)
    return u
