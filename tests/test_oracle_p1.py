"""Pins of the oracle's voxel-segmented P1 discretisation (the paper's P1
comparison discretisation, Sec. 4.1, Tab. discretizations): no enrichment,
one material per voxel.

* A laminate whose interfaces the voxel centres resolve into whole voxel
  layers: the exact solution is piecewise linear with kinks on element faces, so
  the conforming P1 space contains it and C_eff equals the rank-one laminate
  formula with the voxel-layer volume fraction.
* A sphere: C_eff is symmetric positive definite and lies between the Reuss and
  Voigt averages taken with the voxel volume fractions (exact for a conforming
  Galerkin method on this mesh).
* Voxels whose eight corners carry one phase take that phase, as in the X-FEM
  discretisation's uncut elements.
"""

import numpy as np
import pytest

import microstructure as ms
from oracle.xfem import Discretization
from oracle.homogenize import effective_stiffness
from closed_forms import laminate_stiffness, voigt_reuss

LAMEL = np.array([[0.5769231, 0.3846154], [27.77778, 41.66667]])


@pytest.mark.parametrize("m,N,s1,s2,layers", [((1, 0, 0), 12, 2.3, 6.3, 4), ((0, 1, 0), 8, 0.7, 3.6, 3),
                                              ((0, 0, 1), 10, 5.2, 9.4, 4)])
def test_p1_face_aligned_laminate_matches_closed_form(m, N, s1, s2, layers):
    n = (N, N, N)
    L, ph = ms.laminate_levelset(n, m, s1, s2)
    d = Discretization(n, (float(N),) * 3, L, ph, LAMEL, discretization="p1")
    assert d.nX == 0 and not d.cut.any()
    assert np.sum(d.tet_label[:, 0] == 1) == layers * N * N
    C, _, _ = effective_stiffness(d, tol=1e-13)
    Cl = laminate_stiffness(m, [1.0 - layers / N, layers / N], LAMEL)
    assert np.abs(C - Cl).max() < 1e-10 * np.abs(Cl).max()


@pytest.fixture(scope="module")
def sphere_p1():
    n = (8, 8, 8)
    L, ph = ms.spheres_levelset(n, [np.array([4.13, 3.93, 4.21])], [2.6])
    lame = np.array([[0.5769231, 0.3846154], [4.0, 4.0]])
    dp = Discretization(n, (8.0,) * 3, L, ph, lame, discretization="p1")
    dx = Discretization(n, (8.0,) * 3, L, ph, lame, keep_qp=False)
    return dp, dx, lame


def test_p1_sphere_bounds_and_symmetry(sphere_p1):
    d, _, lame = sphere_p1
    C, _, _ = effective_stiffness(d, tol=1e-13)
    nrm = np.linalg.norm(C)
    assert np.abs(C - C.T).max() < 1e-11 * nrm
    assert np.linalg.eigvalsh(0.5 * (C + C.T)).min() > 0.0
    f = np.bincount(d.tet_label[:, 0], minlength=2) / d.N
    V, R = voigt_reuss(f, lame)
    assert np.linalg.eigvalsh(V - C).min() > -1e-10 * nrm
    assert np.linalg.eigvalsh(C - R).min() > -1e-10 * nrm


def test_p1_single_phase_voxels_keep_their_phase(sphere_p1):
    d, dx, _ = sphere_p1
    vn = d.vert_nodes.reshape(d.N, -1)
    same = np.all(d.phase[vn] == d.phase[vn][:, :1], axis=1)
    assert same.sum() > 0
    np.testing.assert_array_equal(d.tet_label[same, 0], d.phase[vn][same, 0])
    uncut = ~dx.cut.any(axis=1) & same
    np.testing.assert_array_equal(d.tet_label[uncut], dx.tet_label[uncut])
