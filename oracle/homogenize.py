"""Effective stiffness, energy form and its Lame-parameter derivative.

* ``effective_stiffness``: column k of C_eff is the average stress
  <sigma(u_k)> (eq. average stress, volume-weighted) for the unit Mandel macro
  strain e_k, with u_k the solution of the scaled system.
* ``energy_stiffness``: C^E_kl = |Y|^-1 int eps_k : C : eps_l with
  eps_k = eps_bar_k + grad^s u_k, by quadrature over all elements.  At the
  Galerkin solution it equals C_eff (the orthogonality used in App. A).
* ``lame_gradient``: derivative of C^E with respect to the Lame pair of each
  phase.  Galerkin orthogonality (int grad^s v : C : eps_l = 0 for every v in
  the discrete space, App. A) removes the derivative of u_k, leaving
  dC^E_kl/dlambda_p = |Y|^-1 int_p tr eps_k tr eps_l and
  dC^E_kl/dmu_p = 2 |Y|^-1 int_p eps_k . eps_l.
"""

import numpy as np

from .system import System
from .green import GreenOperator
from .solver import pcg, dense_solve, fft_scheme, step_size, SCHEMES


def solve_loads(disc, loads, tol=1e-12, maxit=5000, method="pcg"):
    """Solve the scaled system for every macro strain; returns (U, infos).

    method: "pcg" (Algorithm 1), "dense", or one of the schemes of
    solver.fft_scheme ("lcg", "nlcg", "bb", "basic") with the step size of
    eq. stepsize.
    """
    sysm = System(disc)
    loads = np.atleast_2d(np.asarray(loads, dtype=np.float64))
    U, infos = [], []
    if method == "dense":
        A = sysm.assemble()
        for eb in loads:
            u = dense_solve(A, sysm.rhs(eb), 3 * disc.N)
            U.append(u)
            infos.append(dict(iters=0, sigma=sysm.average_stress(u, eb)))
        return np.array(U), infos
    green = GreenOperator(disc.n)
    if method in SCHEMES:
        s0 = step_size(disc.lame)
        for eb in loads:
            u, info = fft_scheme(sysm.apply, sysm.rhs(eb), lambda f: green.apply(f, disc.nX),
                                 lambda x: sysm.average_stress(x, eb), disc.volume, tol, maxit, method, s0)
            U.append(u)
            infos.append(info)
        return np.array(U), infos
    for eb in loads:
        u, info = pcg(sysm.apply, sysm.rhs(eb), lambda f: green.apply(f, disc.nX),
                      lambda x: sysm.average_stress(x, eb), disc.volume, tol, maxit)
        U.append(u)
        infos.append(info)
    return np.array(U), infos


def effective_stiffness(disc, tol=1e-12, maxit=5000, method="pcg"):
    """C_eff (6 x 6, Mandel) from the six unit macro strains; also returns U."""
    loads = np.eye(6)
    U, infos = solve_loads(disc, loads, tol, maxit, method)
    sysm = System(disc)
    C = np.stack([sysm.average_stress(U[k], loads[k]) for k in range(6)], axis=1)
    return C, U, infos


def _qp_strains(disc, U, loads):
    """Yield (w, label, eps[k, 6]) blocks over all quadrature points."""
    sysm = System(disc)
    for t in range(6):
        m, dofs, _, _ = sysm._uncut(t)
        lab = disc.tet_label[m, t]
        eps = np.stack([loads[k][None, :] + U[k][dofs] @ disc.B_fe[t].T for k in range(len(loads))], axis=1)
        yield np.full(len(lab), disc.tet_vol[t]), lab, eps
    dc = sysm.dofs_cut
    for e, qps in enumerate(disc.cut_qp):
        for (w, B, lab) in qps:
            eps = np.stack([loads[k] + B @ U[k][dc[e]] for k in range(len(loads))], axis=0)
            yield np.array([w]), np.array([lab]), eps[None]


def energy_stiffness(disc, U, loads):
    """C^E_kl = |Y|^-1 sum_q w eps_k . C eps_l."""
    nl = len(loads)
    CE = np.zeros((nl, nl))
    one = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])
    for w, lab, eps in _qp_strains(disc, U, loads):
        lam = disc.lame[lab, 0]
        mu = disc.lame[lab, 1]
        tr = eps @ one                                  # (m, k)
        CE += np.einsum("m,mk,ml->kl", w * lam, tr, tr)
        CE += 2.0 * np.einsum("m,mki,mli->kl", w * mu, eps, eps)
    return CE / disc.volume


def lame_gradient(disc, U, loads):
    """dC^E/d(lambda_p, mu_p): array (nphase, 2, nl, nl)."""
    nl = len(loads)
    nph = len(disc.lame)
    g = np.zeros((nph, 2, nl, nl))
    one = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])
    for w, lab, eps in _qp_strains(disc, U, loads):
        tr = eps @ one
        tl = np.einsum("m,mk,ml->mkl", w, tr, tr)
        tm = 2.0 * np.einsum("m,mki,mli->mkl", w, eps, eps)
        np.add.at(g[:, 0], lab, tl)
        np.add.at(g[:, 1], lab, tm)
    return g / disc.volume
