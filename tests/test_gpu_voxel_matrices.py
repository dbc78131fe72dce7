"""Cached voxel matrices (Sec. 3, caching strategy; Sec. 4.2, numerical
efficiency) on the GPU against the oracle.

With the option "always" the irregular voxels are applied through their cached
scaled 48 x 48 matrices (read once for all loads of a launch) instead of the
moment form.  Checked element by element against the oracle's assembled
element loop (FP64 1e-12, FP32 2e-5 relative), with and without the stress
integral; end to end (C_eff, FP64 1e-10, mixed 1e-8) with 1, 2, 3 and 6 loads
in one launch (every load-count variant of the kernel); after a change of the
moduli (the matrices are rebuilt); and the automatic choice gives the same
C_eff as the moment form.
"""

import numpy as np
import pytest

import microstructure as ms
from microstructure.shapes import coated_sphere_levelset
from oracle.xfem import Discretization
from oracle.system import System
from oracle.homogenize import effective_stiffness, solve_loads

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "two_spheres_36x24x18":
        n = (36, 24, 18)
        L, ph = ms.spheres_levelset(n, [np.array([9.3, 11.2, 8.7]), np.array([27.1, 6.4, 12.9])], [5.1, 3.7])
        return n, L, ph, np.array([[0.5769231, 0.3846154], [27.77778, 41.66667], [4.0, 4.0]])
    if name == "coated12":
        n = (12, 12, 12)
        L, ph = coated_sphere_levelset(n, np.array([6.1, 5.8, 6.05]), 2.1, 4.4)
        return n, L, ph, np.array([[0.6, 0.6], [0.48, 0.48], [4.8, 4.8]])
    if name == "snapped8":
        n = (8, 8, 8)
        L, ph = ms.spheres_levelset(n, [np.array([4.0, 4.0, 4.0])], [3.0 + 4e-7])
        return n, L, ph, np.array([[0.5769231, 0.3846154], [4.0, 4.0]])
    if name == "spheres_128x128x16":
        n = (128, 128, 16)
        centers = [(20.3, 30.1, 8.2), (70.7, 90.4, 7.9), (110.2, 15.6, 4.1), (55.5, 55.5, 12.3)]
        L, ph = ms.spheres_levelset(n, [np.array(c) for c in centers], [5.6, 6.1, 3.7, 4.4])
        lame = np.array([[0.5769231, 0.3846154]] + [[4.0, 4.0], [27.77778, 41.66667]] * 2)
        return n, L, ph, lame
    raise KeyError(name)


_OR = {}


def _oracle(name):
    if name not in _OR:
        n, L, ph, lame = _case(name)
        d = Discretization(n, tuple(float(v) for v in n), L, ph, lame, keep_qp=False)
        _OR[name] = (d, System(d))
    return _OR[name]


def _gpu(name, **kw):
    from paper_2601_02172_amd import Problem
    n, L, ph, lame = _case(name)
    return Problem(n, [float(v) for v in n], L, ph, lame, **kw)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("name", ["two_spheres_36x24x18", "coated12", "snapped8", "spheres_128x128x16"])
def test_cached_operator_matches_oracle(name):
    d, s = _oracle(name)
    rng = np.random.default_rng(41)
    x = rng.standard_normal(d.ndof)
    y_or = s.apply(x)
    sig_or = s.average_stress(x, np.zeros(6))
    with _gpu(name, voxel_matrices="always") as p:
        assert p.layout(with_arrays=False)["n_irregular_voxels"] > 0
        y64, sig64 = p.apply_operator(x)
        y64n, _ = p.apply_operator(x, with_stress=False)
        y32, sig32 = p.apply_operator(x, precision="fp32")
        y32n, _ = p.apply_operator(x, precision="fp32", with_stress=False)
    assert _rel(y64, y_or) < 1e-12
    assert _rel(y64n, y_or) < 1e-12
    assert _rel(y32, y_or) < 2e-5
    assert _rel(y32n, y_or) < 2e-5
    np.testing.assert_allclose(sig64, sig_or, rtol=0, atol=1e-12 * np.abs(sig_or).max())
    np.testing.assert_allclose(sig32, sig_or, rtol=0, atol=2e-5 * np.abs(sig_or).max())


@pytest.mark.parametrize("nload", [1, 2, 3, 6])
@pytest.mark.parametrize("precision,rtol,tol", [("fp64", 1e-12, 1e-10), ("mixed", 1e-11, 1e-8)])
def test_cached_solve_matches_oracle(nload, precision, rtol, tol):
    name = "two_spheres_36x24x18"
    d, s = _oracle(name)
    E = np.eye(6)[:nload] if nload < 6 else np.eye(6)
    if nload == 2:
        E = np.array([[1.0, 0.0, 0.3, 0.0, 0.0, 0.0], [0.0, 0.0, 0.0, 0.5, 0.0, 1.0]])
    U, _ = solve_loads(d, E, tol=1e-13)
    sig_or = np.array([s.average_stress(U[k], E[k]) for k in range(nload)])
    with _gpu(name, rtol=rtol, precision=precision, voxel_matrices="always") as p:
        r = p.solve(E)
    assert r["converged"] and r["voxel_matrices"]
    assert _rel(r["avg_stress"], sig_or) < tol


def test_cached_matrices_follow_new_moduli():
    from paper_2601_02172_amd import Problem
    name = "coated12"
    n, L, ph, lame = _case(name)
    lame2 = lame * np.array([[1.4, 0.9], [0.6, 1.7], [1.1, 1.3]])
    with _gpu(name, rtol=1e-12, voxel_matrices="always") as p:
        C1, _ = p.effective_stiffness()
        p.set_lame(lame2)
        C2, info = p.effective_stiffness()
    assert info["voxel_matrices"]
    with Problem(n, [float(v) for v in n], L, ph, lame2, rtol=1e-12, voxel_matrices="never") as q:
        C2_ref, _ = q.effective_stiffness()
    assert _rel(C1, C2) > 1e-3
    assert _rel(C2, C2_ref) < 1e-10


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_automatic_choice_gives_the_moment_form_result(precision):
    name = "spheres_128x128x16"
    rtol = 1e-12 if precision == "fp64" else 1e-11
    with _gpu(name, rtol=rtol, precision=precision, voxel_matrices="auto") as p:
        Ca, ia = p.effective_stiffness()
    with _gpu(name, rtol=rtol, precision=precision, voxel_matrices="never") as p:
        Cn, inn = p.effective_stiffness()
    assert not inn["voxel_matrices"]
    print(f"{precision}: automatic choice uses cached matrices: {ia['voxel_matrices']}")
    assert _rel(Ca, Cn) < (1e-10 if precision == "fp64" else 1e-8)
