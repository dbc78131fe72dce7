"""Local-field accuracy machinery of Sec. 4.1 (eqs. relError, L2NormGauss) and its
use in the paper's Hashin study (Sec. 4.2, accuracy).

Pins, each independent of the machinery itself:
* the textbook composite-sphere field: continuity of displacement and radial
  traction at both interfaces, and the neutral condition for the paper's moduli;
* a rank-one laminate, where the X-FEM solution is exact: the L^2 errors of the
  local strain and stress against the closed-form phase fields vanish;
* the energy identity behind eqs. upperBoundOnEffStiffnessError and
  upperBoundOnLocalStrainError: for the Galerkin solution u_h and any admissible
  v, W(v) - W(u_h) = |Y|^-1 int (eps_v - eps_h) : C : (eps_v - eps_h), hence
  C_- |e|^2 <= W(v) - W(u_h) <= C_+ |e|^2 with |e|^2 the volume-normalised
  squared L^2 norm by the same quadrature;
* Hashin's neutral inclusion at N = 16 and 32: the relative L^2 error of the
  local strain and stress falls at first order in h (the paper observes O(h)).
"""

import numpy as np
import pytest

import microstructure as ms
from microstructure.shapes import coated_sphere_levelset
from oracle.xfem import Discretization, iso_C
from oracle.homogenize import solve_loads, energy_stiffness
from oracle.accuracy import quadrature_fields, stresses, local_errors, l2_norm, relative_error
from closed_forms import CoatedSphereField, laminate_phase_strains, laminate_phase_stresses


def _hashin_moduli():
    f = (6.0 / 5.0 * np.e / (2.0 * np.pi)) ** 3
    Kc = (6.0 - 5.0 * f) / (6.0 + 4.0 * f)
    K = np.array([1.0, Kc, 10.0 * Kc])
    return K, 0.6 * K                      # nu = 0.25


def test_relative_error_definition():
    assert relative_error(1.1, 1.0) == pytest.approx(0.1)
    assert relative_error(-2.0, -4.0) == pytest.approx(0.5)


def test_coated_sphere_field_is_the_textbook_solution():
    K, G = _hashin_moduli()
    ri, rc = 6.0 / 5.0 * np.e, 2.0 * np.pi
    ex = CoatedSphereField(K, G, ri, rc)
    # neutral inclusion: the matrix traction needs no disturbance field
    assert abs(ex.traction_jump()) < 1e-12
    # displacement and radial traction continuous at both interfaces
    n = np.array([0.48, -0.6, 0.64])
    for r0 in (ri, rc):
        a, b = ex.displacement((r0 * (1 - 1e-12)) * n[None]), ex.displacement((r0 * (1 + 1e-12)) * n[None])
        assert np.abs(a - b).max() < 1e-9
        ea, pa = ex.strain((r0 * (1 - 1e-12)) * n[None])
        eb, pb = ex.strain((r0 * (1 + 1e-12)) * n[None])
        sa = iso_C(0.6 * K[pa[0]], 0.6 * K[pa[0]]) @ ea[0]
        sb = iso_C(0.6 * K[pb[0]], 0.6 * K[pb[0]]) @ eb[0]
        N = np.outer(n, n)
        nm = np.array([N[0, 0], N[1, 1], N[2, 2], np.sqrt(2) * N[1, 2], np.sqrt(2) * N[0, 2], np.sqrt(2) * N[0, 1]])
        assert abs(sa @ nm - sb @ nm) < 1e-9            # radial traction n . sigma . n
    # uniform macro strain in the matrix, uniform dilatation in the core
    e_out, _ = ex.strain(np.array([[9.0, 1.0, 0.5]]))
    assert np.abs(e_out[0] - [1, 1, 1, 0, 0, 0]).max() < 1e-15
    e_in, _ = ex.strain(np.array([[0.3, -0.2, 0.1], [1.0, 2.0, -0.5]]))
    assert np.abs(e_in[0] - e_in[1]).max() < 1e-15 and abs(e_in[0][3:]).max() < 1e-15


@pytest.mark.parametrize("load", [0, 3])
def test_local_error_vanishes_for_laminate(load):
    # the laminate solution lies in the X-FEM space: its strain at every
    # quadrature point equals the closed-form phase strain
    N, s1, w = 8, 1.37, 4.0
    n = (N, N, N)
    lame = np.array([[0.5769231, 0.3846154], [27.77778, 41.66667]])
    L, ph = ms.laminate_levelset(n, (1, 0, 0), s1, s1 + w)
    d = Discretization(n, (float(N),) * 3, L, ph, lame, keep_qp=True)
    eb = np.eye(6)[load]
    U, _ = solve_loads(d, eb, tol=1e-13)
    wq, x, lab, eps = quadrature_fields(d, U[0], eb)
    assert wq.sum() == pytest.approx(N ** 3, rel=1e-13)
    fr = [1.0 - w / N, w / N]
    e0, e1 = laminate_phase_strains((1, 0, 0), fr, lame, eb)
    s0, s1_ = laminate_phase_stresses((1, 0, 0), fr, lame, eb)
    inside = ((x[:, 0] - s1) % N) < w                      # exact phase at the point
    eps_ref = np.where(inside[:, None], e1[None], e0[None])
    sig_ref = np.where(inside[:, None], s1_[None], s0[None])
    es, ss = local_errors(wq, eps, stresses(lame, lab, eps), eps_ref, sig_ref)
    assert es < 1e-10 and ss < 1e-10


def test_energy_identity_bounds_the_local_error():
    # eqs. upperBoundOnEffStiffnessError / upperBoundOnLocalStrainError for the
    # discrete problem: u_h is the Galerkin optimum, v = u_h + perturbation
    n = (8, 8, 8)
    lame = np.array([[0.5769231, 0.3846154], [4.0, 4.0]])
    L, ph = ms.spheres_levelset(n, [np.array([4.13, 3.93, 4.21])], [2.6])
    d = Discretization(n, (8.0,) * 3, L, ph, lame, keep_qp=True)
    eb = np.array([0.3, -0.2, 1.0, 0.0, 0.4, 0.0])
    U, _ = solve_loads(d, eb, tol=1e-13)
    uh = U[0]
    rng = np.random.default_rng(7)
    V = float(np.prod(n))
    Cm = [iso_C(*lp) for lp in lame]
    eig = np.concatenate([np.linalg.eigvalsh(C) for C in Cm])
    c_minus, c_plus = eig.min(), eig.max()
    W_h = energy_stiffness(d, uh[None], eb[None])[0, 0]
    w, _, lab, eps_h = quadrature_fields(d, uh, eb)
    for scale in (1e-3, 0.1, 1.0):
        v = uh + scale * rng.standard_normal(d.ndof)
        W_v = energy_stiffness(d, v[None], eb[None])[0, 0]
        _, _, _, eps_v = quadrature_fields(d, v, eb)
        de = eps_v - eps_h
        err2 = l2_norm(w, de) ** 2 / V
        energy_err = float(np.sum(w * np.sum(de * stresses(lame, lab, de), axis=1))) / V
        gap = W_v - W_h
        assert gap == pytest.approx(energy_err, rel=1e-9)        # Pythagoras (Galerkin orthogonality)
        assert c_minus * err2 * (1 - 1e-12) <= gap <= c_plus * err2 * (1 + 1e-12)


@pytest.mark.slow
def test_hashin_local_errors_are_first_order():
    # Sec. 4.2 (accuracy): relative L^2 errors of the local strain and stress of
    # the X-FEM solution against the textbook field fall at O(h)
    K, G = _hashin_moduli()
    lame = np.stack([0.6 * K, 0.6 * K], axis=1)
    eb = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])
    errs = {}
    for N in (16, 32):
        h = 16.0 / N
        c = np.full(3, 8.0 / h)
        ri, rc = 6.0 / 5.0 * np.e / h, 2.0 * np.pi / h
        L, ph = coated_sphere_levelset((N,) * 3, c, ri, rc)
        d = Discretization((N,) * 3, (float(N),) * 3, L, ph, lame, keep_qp=True)
        U, _ = solve_loads(d, eb, tol=1e-11)
        w, x, lab, eps = quadrature_fields(d, U[0], eb)
        off = x - c
        off -= N * np.round(off / N)
        eps_ref, ph_ref = CoatedSphereField(K, G, ri, rc).strain(off)
        errs[N] = local_errors(w, eps, stresses(lame, lab, eps), eps_ref, stresses(lame, ph_ref, eps_ref))
    rate_e = np.log(errs[16][0] / errs[32][0]) / np.log(2.0)
    rate_s = np.log(errs[16][1] / errs[32][1]) / np.log(2.0)
    print(f"strain errors {errs[16][0]:.3e} {errs[32][0]:.3e} (rate {rate_e:.2f}); "
          f"stress {errs[16][1]:.3e} {errs[32][1]:.3e} (rate {rate_s:.2f})")
    assert 0.02 < errs[16][0] < 0.2
    assert 0.8 < rate_e < 1.5 and 0.8 < rate_s < 1.5
