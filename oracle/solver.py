"""Displacement-based linear CG of Algorithm 1, the other solution schemes of
Sec. 3 (basic, Barzilai-Borwein, nonlinear CG) and a dense reference solve.

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


def step_size(lame):
    """Step size s0 = 2 / (C_- + C_+) of eq. stepsize.

    C_- and C_+ are the smallest and largest eigenvalue of the stiffness of all
    phases.  An isotropic stiffness lambda 1 (x) 1 + 2 mu I (Mandel form) has
    the eigenvalues 3 lambda + 2 mu (once) and 2 mu (five times).
    """
    lame = np.asarray(lame, dtype=np.float64).reshape(-1, 2)
    eig = np.concatenate([3.0 * lame[:, 0] + 2.0 * lame[:, 1], 2.0 * lame[:, 1]])
    return 2.0 / (eig.min() + eig.max())


SCHEMES = ("lcg", "nlcg", "bb", "basic")


def fft_scheme(apply_A, b, apply_P, avg_stress, volume, tol, maxit, scheme, s0):
    """The solution schemes the paper lists beside Algorithm 1 (Sec. 3, solvers).

    All four work on the same residual f = b - A u, preconditioned residual
    y = P^-1 f and direction d, and stop by eq. stoppingCriterion; they differ
    in the step alpha and the direction weight beta of each iteration:

    * ``lcg``   linear CG (Algorithm 1): alpha = res^2 / <A d, d>,
                beta = res_new^2 / res^2.
    * ``basic`` the basic scheme (a Richardson iteration with the step size of
                eq. stepsize): alpha = s0, beta = 0, i.e. u += s0 P^-1 f.
    * ``bb``    Barzilai-Borwein: the basic scheme with the step
                <s, P s> / <s, A s> of the previous update s = u_k - u_{k-1};
                with d = P^-1 f that is the previous iteration's
                res^2 / <A d, d>.  The first step is s0.
    * ``nlcg``  nonlinear CG with the Fletcher-Reeves weight
                beta = res_new^2 / res^2 and the fixed step s0 of the basic
                scheme in place of a line search.
    The paper gives only the step size of eq. stepsize for the last three; the
    step rules are the readings stated above.  Returns (u, info) as pcg does.
    """
    if scheme not in SCHEMES:
        raise ValueError(f"unknown scheme {scheme!r}")
    u = np.zeros_like(b)
    f = b.copy()
    d = apply_P(f)
    res2 = float(f @ d)
    res = np.sqrt(max(res2, 0.0) / volume)
    sig = avg_stress(u)
    hist = [res]
    alpha_lag = None
    k = 0
    while k < maxit and res > tol * np.linalg.norm(sig):
        k += 1
        z = apply_A(d)
        dz = float(z @ d)
        if not dz > 0.0:
            raise FloatingPointError("breakdown: d^T A d <= 0")
        if scheme == "lcg":
            alpha = res2 / dz
        elif scheme == "bb":
            alpha = s0 if alpha_lag is None else alpha_lag
            alpha_lag = res2 / dz
        else:
            alpha = s0
        u += alpha * d
        f -= alpha * z
        y = apply_P(f)
        res2_new = float(f @ y)
        beta = res2_new / res2 if scheme in ("lcg", "nlcg") else 0.0
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
