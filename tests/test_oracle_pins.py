"""Pins of the oracle's discretisation, preconditioner, solver and outputs.

Each test compares the oracle with a result fixed independently of it:
textbook closed forms (homogeneous material, rank-one laminate, composite
sphere of the Hashin study, dilute Eshelby estimate), exact properties of a
conforming Galerkin method (symmetry, bounds, invariances; App. A), brute-force
dense solves and central finite differences.
"""

import numpy as np
import pytest

import microstructure as ms
from oracle.xfem import Discretization, iso_C
from oracle.system import System
from oracle.green import GreenOperator
from oracle.homogenize import effective_stiffness, solve_loads, energy_stiffness, lame_gradient
from closed_forms import (laminate_stiffness, composite_sphere_bulk, eshelby_dilute, voigt_reuss,
                          isotropic_projection)

LAME2 = np.array([[0.5769231, 0.3846154], [4.0, 4.0]])            # E = 1, nu = 0.3 / E = 10, nu = 0.25


def _sphere(N, r, lame=LAME2, center=None):
    n = (N, N, N)
    c = np.array([N / 2.0 + 0.13, N / 2.0 - 0.07, N / 2.0 + 0.21]) if center is None else center
    L, ph = ms.spheres_levelset(n, [c], [r])
    return Discretization(n, (float(N),) * 3, L, ph, lame)


# --------------------------------------------------------------------------- special cases
def test_homogeneous_material_gives_C_and_zero_rhs():
    n = (5, 6, 4)
    N = 120
    lame = np.array([[1.3, 0.7]])
    d = Discretization(n, (5.0, 6.0, 4.0), np.ones(N), np.zeros(N, dtype=int), lame)
    assert d.nX == 0
    s = System(d)
    for k in range(6):
        assert np.abs(s.rhs(np.eye(6)[k])).max() < 1e-14
    C, _, _ = effective_stiffness(d, method="dense")
    np.testing.assert_allclose(C, iso_C(1.3, 0.7), atol=1e-14)


def test_equal_moduli_sphere_has_zero_rhs_and_solution():
    d = _sphere(8, 2.6, lame=np.array([[1.0, 0.5], [1.0, 0.5]]))
    assert d.nX > 0
    s = System(d)
    for k in range(6):
        assert np.abs(s.rhs(np.eye(6)[k])).max() < 1e-14
    C, U, _ = effective_stiffness(d, tol=1e-13)
    assert np.abs(U).max() < 1e-14
    np.testing.assert_allclose(C, iso_C(1.0, 0.5), atol=1e-14)


LAMINATES = [
    ((1, 0, 0), 8, 1.37, 4.0),
    ((1, 1, 0), 12, 2.31, 6.0),
    ((1, 1, 1), 18, 3.17, 9.0),
]


@pytest.mark.parametrize("m,N,s1,w", LAMINATES)
def test_laminate_matches_rank_one_closed_form(m, N, s1, w):
    # the exact periodic laminate solution is piecewise linear with planar kinks;
    # the modified abs enrichment reproduces the kink exactly, so the X-FEM
    # solution and its C_eff are exact (up to the solver tolerance)
    if m == (1, 1, 1):
        pytest.importorskip("scipy")
    n = (N, N, N)
    lame = np.array([[0.5769231, 0.3846154], [27.77778, 41.66667]])
    L, ph = ms.laminate_levelset(n, m, s1, s1 + w)
    d = Discretization(n, (float(N),) * 3, L, ph, lame, keep_qp=False)
    assert d.nX > 0
    C, _, _ = effective_stiffness(d, tol=1e-13)
    f1 = w / N
    Cl = laminate_stiffness(m, [1.0 - f1, f1], lame)
    assert np.abs(C - Cl).max() / np.abs(Cl).max() < 1e-10


def test_dense_solve_matches_pcg_on_4cube():
    d = _sphere(4, 1.2, center=np.array([2.1, 1.9, 2.05]))
    assert d.nX > 0
    Cd, Ud, _ = effective_stiffness(d, method="dense")
    Cp, Up, infos = effective_stiffness(d, tol=1e-14)
    assert np.abs(Cd - Cp).max() / np.abs(Cd).max() < 1e-12
    # FE part of the dense min-norm solution is mean free
    N = d.N
    for u in Ud:
        assert np.abs(u[:3 * N].reshape(3, N).mean(axis=1)).max() < 1e-13


# --------------------------------------------------------------------------- C_eff structure
@pytest.fixture(scope="module")
def sphere8():
    d = _sphere(8, 2.5)
    C, U, infos = effective_stiffness(d, tol=1e-13)
    return d, C, U


def test_ceff_symmetric_positive_definite(sphere8):
    _, C, _ = sphere8
    assert np.abs(C - C.T).max() < 1e-10 * np.abs(C).max()
    assert np.linalg.eigvalsh(0.5 * (C + C.T)).min() > 0.0


def test_ceff_between_reuss_and_voigt(sphere8):
    d, C, U = sphere8
    # discrete phase volume fractions from the quadrature weights of the partition
    vol = np.zeros(len(d.lame))
    for t in range(6):
        np.add.at(vol, d.tet_label[~d.cut[:, t], t], d.tet_vol[t])
    for qps in d.cut_qp:
        for (w, _, lab) in qps:
            vol[lab] += w
    assert abs(vol.sum() - d.volume) < 1e-9
    V, R = voigt_reuss(vol / d.volume, d.lame)
    Cs = 0.5 * (C + C.T)
    assert np.linalg.eigvalsh(V - Cs).min() > -1e-10
    assert np.linalg.eigvalsh(Cs - R).min() > -1e-10


def test_energy_form_equals_average_stress_form(sphere8):
    # at the Galerkin solution <eps_k : C : eps_l> = <sigma_k> . e_l
    d, C, U = sphere8
    CE = energy_stiffness(d, U, np.eye(6))
    assert np.abs(CE - C).max() < 1e-9 * np.abs(C).max()


def test_ceff_scales_with_moduli_and_ignores_d0_scaling(sphere8):
    d, C, _ = sphere8
    L = d.Ls * d.h
    d2 = Discretization(d.n, (float(d.n[0]),) * 3, L, d.phase, 3.5 * d.lame, d0_scale=2.0)
    C2, _, _ = effective_stiffness(d2, tol=1e-13)
    assert np.abs(C2 - 3.5 * C).max() < 1e-10 * np.abs(C2).max()


def test_ceff_invariant_under_integer_roll_and_physical_units(sphere8):
    d, C, _ = sphere8
    n = d.n
    L3 = (d.Ls * d.h).reshape(n[2], n[1], n[0])
    P3 = d.phase.reshape(n[2], n[1], n[0])
    Lr = np.roll(L3, (1, 3, 2), axis=(0, 1, 2)).ravel()
    Pr = np.roll(P3, (1, 3, 2), axis=(0, 1, 2)).ravel()
    h = 0.37
    d2 = Discretization(n, (n[0] * h,) * 3, Lr * h, Pr, d.lame)
    C2, _, _ = effective_stiffness(d2, tol=1e-13)
    assert np.abs(C2 - C).max() < 1e-10 * np.abs(C).max()


def test_ceff_covariant_under_axis_permutation(sphere8):
    # swapping x and y maps the Kuhn mesh onto itself; C_eff permutes accordingly
    d, C, _ = sphere8
    n = d.n
    L3 = (d.Ls * d.h).reshape(n[2], n[1], n[0])
    P3 = d.phase.reshape(n[2], n[1], n[0])
    Lp = np.transpose(L3, (0, 2, 1)).ravel()          # (z, x, y) -> new x is old y
    Pp = np.transpose(P3, (0, 2, 1)).ravel()
    d2 = Discretization(n, (float(n[0]),) * 3, Lp, Pp, d.lame)
    C2, _, _ = effective_stiffness(d2, tol=1e-13)
    perm = [1, 0, 2, 4, 3, 5]                         # Mandel (11,22,33,23,13,12) under x<->y
    assert np.abs(C2 - C[np.ix_(perm, perm)]).max() < 1e-10 * np.abs(C).max()


# --------------------------------------------------------------------------- Green operator
@pytest.mark.parametrize("n", [(6, 6, 6), (8, 8, 8), (12, 12, 12), (8, 6, 10)])
def test_green_symbol_closed_forms(n):
    g = GreenOperator(n)
    S = g.symbol
    assert np.abs(S.imag).max() < 1e-13                     # real symmetric symbol
    Sm = np.moveaxis(S.real, (0, 1), (-2, -1)).reshape(-1, 3, 3)
    assert np.abs(Sm - np.swapaxes(Sm, 1, 2)).max() < 1e-13
    ev = np.linalg.eigvalsh(Sm[1:])
    Nmax = max(n)
    assert abs(ev.min() - 2.0 * np.sin(np.pi / Nmax) ** 2) < 1e-13
    # axial mode xi = (k, 0, 0): longitudinal 4 sin^2, transverse 2 sin^2
    for k in range(1, n[0]):
        s2 = np.sin(np.pi * k / n[0]) ** 2
        np.testing.assert_allclose(np.moveaxis(S.real[:, :, 0, 0, k], 0, 0),
                                   np.diag([4 * s2, 2 * s2, 2 * s2]), atol=1e-13)


def test_green_inverts_reference_stiffness():
    n = (6, 8, 4)
    N = 192
    A0 = System(Discretization(n, (6.0, 8.0, 4.0), np.ones(N), np.zeros(N, dtype=int),
                               np.array([[0.0, 0.5]]))).assemble()
    x = np.random.default_rng(1).standard_normal(3 * N)
    y = GreenOperator(n).apply_fe(A0 @ x)
    xm = x.reshape(3, N)
    xm = xm - xm.mean(axis=1, keepdims=True)
    assert np.abs(y - xm.ravel()).max() < 1e-12


# --------------------------------------------------------------------------- paper's own case
def test_hashin_table_moduli_from_composite_sphere_formula():
    # coating/inclusion bulk moduli of the neutral inclusion table follow from
    # K_eff = K_matrix = 1 with K_inclusion = 10 K_coating, nu = 0.25
    f = (6.0 / 5.0 * np.e / (2.0 * np.pi)) ** 3
    Kc = (6.0 - 5.0 * f) / (6.0 + 4.0 * f)
    assert abs(Kc - 0.808024) < 5e-7
    assert abs(10 * Kc - 8.080240) < 5e-6
    Gc = 0.6 * Kc
    assert abs(composite_sphere_bulk(Kc, Gc, 10 * Kc, f) - 1.0) < 1e-14


def _hashin(N):
    n = (N, N, N)
    h = 16.0 / N
    c = np.array([8.0, 8.0, 8.0]) / h
    from microstructure.shapes import coated_sphere_levelset
    L, ph = coated_sphere_levelset(n, c, 6.0 / 5.0 * np.e / h, 2.0 * np.pi / h)
    f = (6.0 / 5.0 * np.e / (2.0 * np.pi)) ** 3
    Kc = (6.0 - 5.0 * f) / (6.0 + 4.0 * f)
    K = np.array([1.0, Kc, 10.0 * Kc])
    lame = np.stack([0.6 * K, 0.6 * K], axis=1)
    d = Discretization(n, (16.0,) * 3, L * h, ph, lame, keep_qp=False)
    eb = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])
    U, infos = solve_loads(d, eb[None], tol=1e-10)
    sig = System(d).average_stress(U[0], eb)
    return sig[:3].sum() / 9.0, infos[0]["iters"]


@pytest.mark.slow
def test_hashin_neutral_inclusion_converges_quadratically():
    K8, _ = _hashin(8)
    K16, it16 = _hashin(16)
    e8, e16 = abs(K8 - 1.0), abs(K16 - 1.0)
    assert e16 < 5e-3
    assert e8 / e16 > 2.5          # O(h^2) (ratio 4 asymptotically)


@pytest.mark.slow
def test_dilute_sphere_close_to_eshelby():
    N = 24
    r = 0.15 * N
    lam, mu = ms.lame_from_E_nu(np.array([1.0, 10.0]), np.array([0.3, 0.25]))
    lame = np.stack([lam, mu], axis=1)
    d = _sphere(N, r, lame=lame)
    C, _, _ = effective_stiffness(d, tol=1e-9)
    K, G = isotropic_projection(C)
    f = 4.0 / 3.0 * np.pi * r ** 3 / N ** 3
    Km, Gm = lam[0] + 2 * mu[0] / 3, mu[0]
    Ki, Gi = lam[1] + 2 * mu[1] / 3, mu[1]
    Ke, Ge = eshelby_dilute(Km, Gm, Ki, Gi, f)
    assert abs((K - Km) - (Ke - Km)) < 0.1 * (Ke - Km)
    assert abs((G - Gm) - (Ge - Gm)) < 0.1 * (Ge - Gm)


# --------------------------------------------------------------------------- gradient
def test_lame_gradient_matches_central_differences():
    d = _sphere(6, 1.9)
    C, U, _ = effective_stiffness(d, method="dense")
    g = lame_gradient(d, U, np.eye(6))
    L = d.Ls * d.h
    for (p, q) in [(0, 0), (0, 1), (1, 0), (1, 1)]:
        dl = 1e-5 * d.lame[p, q]
        Cs = []
        for s in (+1, -1):
            lm = d.lame.copy()
            lm[p, q] += s * dl
            dd = Discretization(d.n, (6.0,) * 3, L, d.phase, lm)
            Cs.append(effective_stiffness(dd, method="dense")[0])
        fd = (Cs[0] - Cs[1]) / (2 * dl)
        assert np.abs(fd - g[p, q]).max() < 1e-6 * np.abs(g[p, q]).max() + 1e-9


# --------------------------------------------------------------------------- voxel stresses (eq. Sapp_q per voxel)
def test_voxel_stress_of_a_linear_field_in_homogeneous_material():
    # u = A x on the nodes: every voxel that does not straddle the periodic
    # seam sees the uniform strain sym(A), so its average stress is
    # C (eps_bar + sym A); u = 0 and u = const give C eps_bar everywhere
    n = (5, 6, 4)
    N = 120
    lam, mu = 1.3, 0.7
    d = Discretization(n, (5.0, 6.0, 4.0), np.ones(N), np.zeros(N, dtype=int), np.array([[lam, mu]]))
    s = System(d)
    C = iso_C(lam, mu)
    rng = np.random.default_rng(4)
    eb = rng.standard_normal(6)
    for u in (np.zeros(d.ndof), np.repeat(rng.standard_normal(3), N)):
        vs = s.voxel_stress(u, eb)
        np.testing.assert_allclose(vs, np.tile((C @ eb)[:, None], (1, N)), rtol=0, atol=1e-14)
    A = rng.standard_normal((3, 3))
    i, j, k = np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij")
    xyz = np.stack([i.transpose(2, 1, 0).ravel(), j.transpose(2, 1, 0).ravel(), k.transpose(2, 1, 0).ravel()])
    u = (A @ xyz).reshape(-1)                        # component-major, node index x fastest
    vs = s.voxel_stress(u, eb)
    E = 0.5 * (A + A.T)
    e_lin = np.array([E[0, 0], E[1, 1], E[2, 2], np.sqrt(2) * E[1, 2], np.sqrt(2) * E[0, 2], np.sqrt(2) * E[0, 1]])
    inner = ((xyz[0] < n[0] - 1) & (xyz[1] < n[1] - 1) & (xyz[2] < n[2] - 1))
    assert inner.sum() == 4 * 5 * 3
    np.testing.assert_allclose(vs[:, inner], np.tile((C @ (eb + e_lin))[:, None], (1, inner.sum())),
                               rtol=0, atol=1e-13 * np.abs(C @ (eb + e_lin)).max())
    assert np.abs(vs[:, ~inner] - (C @ (eb + e_lin))[:, None]).max() > 1e-3


@pytest.mark.parametrize("load", [0, 5])
def test_voxel_stress_of_laminate_matches_phase_stresses(load):
    # face-aligned laminate, layer 1 at x in [1.37, 5.37): voxels wholly inside a
    # layer carry that phase's closed-form stress, the two cut voxel columns the
    # volume-weighted mix of both (fractions 0.63 / 0.37)
    from closed_forms import laminate_phase_stresses
    N, s1, w = 8, 1.37, 4.0
    n = (N, N, N)
    lame = np.array([[0.5769231, 0.3846154], [27.77778, 41.66667]])
    L, ph = ms.laminate_levelset(n, (1, 0, 0), s1, s1 + w)
    d = Discretization(n, (float(N),) * 3, L, ph, lame, keep_qp=False)
    eb = np.eye(6)[load]
    U, _ = solve_loads(d, eb, tol=1e-13)
    vs = System(d).voxel_stress(U[0], eb)
    sig0, sig1 = laminate_phase_stresses((1, 0, 0), [1.0 - w / N, w / N], lame, eb)
    ix = np.arange(N ** 3) % N
    frac1 = np.clip(np.minimum(ix + 1.0, s1 + w) - np.maximum(ix * 1.0, s1), 0.0, 1.0)
    expect = np.outer(sig1, frac1) + np.outer(sig0, 1.0 - frac1)
    assert sorted(set(np.round(frac1, 6))) == [0.0, 0.37, 0.63, 1.0]
    np.testing.assert_allclose(vs, expect, rtol=0, atol=1e-10 * np.abs(expect).max())


def test_voxel_stresses_average_to_the_average_stress(sphere8):
    d = sphere8[0]
    s = System(d)
    rng = np.random.default_rng(9)
    x = rng.standard_normal(d.ndof)
    eb = rng.standard_normal(6)
    np.testing.assert_allclose(s.voxel_stress(x, eb).mean(axis=1), s.average_stress(x, eb), rtol=1e-13, atol=1e-14)
