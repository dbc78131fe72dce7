"""Pins of the oracle's basic, Barzilai-Borwein and nonlinear CG schemes (Sec. 3,
solution schemes; step size of eq. stepsize).

* the step size against the eigenvalues of the phase stiffness, written from
  Young's modulus and Poisson's ratio and from a numerical eigensolver;
* the basic scheme against the closed form of a Richardson iteration, built
  from dense matrices;
* the Barzilai-Borwein steps against <s, P s> / <s, A s> of consecutive
  iterates, with the reference stiffness P assembled as a matrix;
* every scheme converging in one step when P^-1 A = c I and s0 = 1 / c;
* every scheme converging to the dense Galerkin solution, with the iteration
  counts ordered as in the paper's Hashin study (basic > Barzilai-Borwein,
  basic > nonlinear CG >= linear CG).
"""

import numpy as np
import pytest

import microstructure as ms
from oracle.xfem import Discretization, iso_C
from oracle.system import System
from oracle.green import GreenOperator
from oracle.solver import fft_scheme, step_size, SCHEMES
from oracle.homogenize import solve_loads

LAME2 = np.array([[0.5769231, 0.3846154], [4.0, 4.0]])            # E = 1, nu = 0.3 / E = 10, nu = 0.25


def _sphere(N, r, lame=LAME2):
    n = (N, N, N)
    c = np.array([N / 2.0 + 0.13, N / 2.0 - 0.07, N / 2.0 + 0.21])
    L, ph = ms.spheres_levelset(n, [c], [r])
    return Discretization(n, (float(N),) * 3, L, ph, lame)


def _dense(d):
    """Dense A, dense P^-1 (columns of the Green operator) and dense P (reference
    stiffness: FE stiffness of the identity material, identity on the enriched block)."""
    A = System(d).assemble().toarray()
    n = A.shape[0]
    g = GreenOperator(d.n)
    Pinv = np.stack([g.apply(e, d.nX) for e in np.eye(n)], axis=1)
    ref = Discretization(d.n, tuple(float(v) for v in d.n), np.ones(d.N), np.zeros(d.N, dtype=int), np.array([[0.0, 0.5]]))
    P = np.eye(n)
    P[:3 * d.N, :3 * d.N] = System(ref).assemble().toarray()
    return A, Pinv, P


def _run(d, eb, scheme, k, s0=None):
    s = System(d)
    g = GreenOperator(d.n)
    s0 = step_size(d.lame) if s0 is None else s0
    u, info = fft_scheme(s.apply, s.rhs(eb), lambda f: g.apply(f, d.nX), lambda x: s.average_stress(x, eb),
                         d.volume, 0.0, k, scheme, s0)
    return u, info


@pytest.fixture(scope="module")
def sphere4():
    d = _sphere(4, 1.2)
    assert d.nX > 0
    return d, _dense(d)


def test_step_size_from_young_poisson_and_eigensolver():
    E = np.array([1.0, 10.0, 3.0])
    nu = np.array([0.3, 0.25, 0.45])
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    lame = np.stack([lam, mu], axis=1)
    # 3 lambda + 2 mu = E / (1 - 2 nu) (three times the bulk modulus), 2 mu = E / (1 + nu)
    cmin = (E / (1 + nu)).min()
    cmax = (E / (1 - 2 * nu)).max()
    assert abs(step_size(lame) - 2.0 / (cmin + cmax)) < 1e-14
    eig = np.concatenate([np.linalg.eigvalsh(iso_C(l, m)) for l, m in lame])
    assert abs(step_size(lame) - 2.0 / (eig.min() + eig.max())) < 1e-13


def test_basic_scheme_is_richardson_closed_form(sphere4):
    d, (A, Pinv, _) = sphere4
    eb = np.array([1.0, 0.0, 0.0, 0.0, 0.0, 0.3])
    b = System(d).rhs(eb)
    s0 = step_size(d.lame)
    M = np.eye(A.shape[0]) - s0 * Pinv @ A
    term = s0 * Pinv @ b
    u_ref = np.zeros_like(b)
    for k in range(1, 7):
        u_ref = u_ref + term                    # u_k = sum_{j<k} (I - s0 P^-1 A)^j s0 P^-1 b
        term = M @ term
        u, info = _run(d, eb, "basic", k)
        assert info["iters"] == k
        assert np.abs(u - u_ref).max() < 1e-12 * np.abs(u_ref).max()


def test_bb_steps_from_consecutive_iterates(sphere4):
    d, (A, Pinv, P) = sphere4
    eb = np.array([0.0, 1.0, 0.0, 0.2, 0.0, 0.0])
    b = System(d).rhs(eb)
    s0 = step_size(d.lame)
    us = [np.zeros_like(b)] + [_run(d, eb, "bb", k)[0] for k in range(1, 6)]
    assert np.abs(us[1] - s0 * Pinv @ b).max() < 1e-13 * np.abs(us[1]).max()
    for k in range(1, 5):
        s = us[k] - us[k - 1]
        step = (s @ P @ s) / (s @ A @ s)
        f = b - A @ us[k]
        expect = us[k] + step * (Pinv @ f)
        assert np.abs(us[k + 1] - expect).max() < 1e-11 * np.abs(expect).max()


@pytest.mark.parametrize("scheme", SCHEMES)
def test_one_step_when_preconditioner_is_exact(scheme):
    rng = np.random.default_rng(7)
    n = 12
    B = rng.standard_normal((n, n))
    Pm = B @ B.T + n * np.eye(n)
    c = 2.5
    b = rng.standard_normal(n)
    u, info = fft_scheme(lambda x: c * (Pm @ x), b, lambda f: np.linalg.solve(Pm, f), lambda x: np.ones(6),
                         1.0, 1e-12, 50, scheme, 1.0 / c)
    assert info["iters"] == 1
    assert np.abs(u - np.linalg.solve(c * Pm, b)).max() < 1e-12 * np.abs(u).max()


def test_schemes_converge_to_dense_solution_with_paper_ordering():
    d = _sphere(6, 1.9)
    eb = np.eye(6)[0]
    A = System(d).assemble()
    from oracle.solver import dense_solve
    u_ref = dense_solve(A, System(d).rhs(eb), 3 * d.N)
    its = {}
    for scheme in SCHEMES:
        U, infos = solve_loads(d, eb, tol=1e-11, maxit=5000, method=scheme)
        its[scheme] = infos[0]["iters"]
        assert np.abs(U[0] - u_ref).max() < 1e-8 * np.abs(u_ref).max(), scheme
    assert its["basic"] > its["bb"]
    assert its["basic"] > its["nlcg"] >= its["lcg"]
