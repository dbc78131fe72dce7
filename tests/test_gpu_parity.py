"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle.

Step level (operator, right-hand side, preconditioner, enriched layout) on
grids that span several operator tiles with ragged tails, and end to end
(effective stiffness) for FP64 and mixed precision.  Bars: bit-exact for the
enriched node numbering, 1e-12 relative for FP64 step-level results, 1e-10
relative for FP64 C_eff, 1e-8 relative for mixed-precision C_eff, 2e-5 relative
for FP32 step-level results (single-precision rounding of O(10) terms).
"""

import json
import os

import numpy as np
import pytest

import microstructure as ms
from microstructure.shapes import coated_sphere_levelset
from oracle.xfem import Discretization
from oracle.system import System
from oracle.green import GreenOperator
from oracle.homogenize import effective_stiffness, solve_loads
from closed_forms import laminate_stiffness

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
LAME2 = np.array([[0.5769231, 0.3846154], [4.0, 4.0]])


def _case(name):
    if name == "sphere8":
        n = (8, 8, 8)
        L, ph = ms.spheres_levelset(n, [np.array([4.13, 3.93, 4.21])], [2.6])
        return n, L, ph, LAME2
    if name == "two_spheres_36x24x18":
        n = (36, 24, 18)
        L, ph = ms.spheres_levelset(n, [np.array([9.3, 11.2, 8.7]), np.array([27.1, 6.4, 12.9])], [5.1, 3.7])
        lame = np.array([[0.5769231, 0.3846154], [27.77778, 41.66667], [4.0, 4.0]])
        return n, L, ph, lame
    if name == "snapped8":
        # nodes exactly on (and within 1e-6 of) the sphere: zero-vertex subdivisions
        n = (8, 8, 8)
        L, ph = ms.spheres_levelset(n, [np.array([4.0, 4.0, 4.0])], [3.0 + 4e-7])
        return n, L, ph, LAME2
    if name == "coated12":
        n = (12, 12, 12)
        L, ph = coated_sphere_levelset(n, np.array([6.1, 5.8, 6.05]), 2.1, 4.4)
        lame = np.array([[0.6, 0.6], [0.48, 0.48], [4.8, 4.8]])
        return n, L, ph, lame
    if name == "laminate110_12":
        n = (12, 12, 12)
        L, ph = ms.laminate_levelset(n, (1, 1, 0), 2.31, 8.31)
        return n, L, ph, np.array([[0.5769231, 0.3846154], [27.77778, 41.66667]])
    if name == "homogeneous6":
        n = (6, 6, 6)
        return n, np.ones(216), np.zeros(216, dtype=np.int32), np.array([[1.3, 0.7]])
    if name == "spheres_32x16x48":
        # n0 != n1: compile-time x, y and z passes instead of the xy-plane kernels
        n = (32, 16, 48)
        L, ph = ms.spheres_levelset(n, [np.array([9.3, 8.2, 14.7]), np.array([24.1, 7.4, 33.9])], [5.1, 4.3])
        return n, L, ph, np.array([[0.5769231, 0.3846154], [27.77778, 41.66667], [4.0, 4.0]])
    if name == "spheres_256x16x16":
        # length-256 x lines (the radix-16 x 16 plan), periodic images along x
        n = (256, 16, 16)
        L, ph = ms.spheres_levelset(n, [np.array([37.2, 8.1, 7.6]), np.array([250.3, 7.7, 9.2])], [4.6, 5.2])
        return n, L, ph, np.array([[0.5769231, 0.3846154], [4.0, 4.0], [27.77778, 41.66667]])
    if name == "tiny4":
        n = (4, 4, 4)
        L, ph = ms.spheres_levelset(n, [np.array([2.1, 1.9, 2.05])], [1.2])
        return n, L, ph, LAME2
    raise KeyError(name)


STEP_CASES = ["sphere8", "two_spheres_36x24x18", "snapped8", "coated12", "laminate110_12", "homogeneous6", "tiny4",
              "spheres_32x16x48", "spheres_256x16x16"]

_ORACLE = {}


def oracle_of(name):
    if name not in _ORACLE:
        n, L, ph, lame = _case(name)
        d = Discretization(n, tuple(float(v) for v in n), L, ph, lame, keep_qp=False)
        _ORACLE[name] = (d, System(d))
    return _ORACLE[name]


def gpu_of(name, **kw):
    from paper_2601_02172_amd import Problem
    n, L, ph, lame = _case(name)
    return Problem(n, [float(v) for v in n], L, ph, lame, **kw)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("name", STEP_CASES)
def test_enriched_layout_matches_oracle(name):
    d, _ = oracle_of(name)
    with gpu_of(name) as p:
        lay = p.layout()
    assert lay["nX"] == d.nX
    assert lay["n_cut_elements"] == len(d.cut_voxel)
    if d.nX:
        assert np.array_equal(lay["jlist"], d.J)
        assert _rel(lay["d0"], d.D0) < 1e-12


@pytest.mark.parametrize("name", STEP_CASES)
def test_operator_matches_oracle(name):
    d, s = oracle_of(name)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(d.ndof)
    with gpu_of(name) as p:
        y, _ = p.apply_operator(x)
        y32, _ = p.apply_operator(x, precision="fp32")
        eb = rng.standard_normal(6)
        r, sig = p.apply_operator(x, macro_strain=eb)
        r0, sig0 = p.apply_operator(np.zeros(d.ndof), macro_strain=eb)
    y_or = s.apply(x)
    assert _rel(y, y_or) < 1e-12
    assert _rel(y32, y_or) < 2e-5
    assert _rel(r, s.residual(x, eb)) < 1e-12
    np.testing.assert_allclose(sig, s.average_stress(x, eb), rtol=0, atol=1e-12 * np.abs(sig).max())
    # right-hand side: r(0) = -b
    assert _rel(r0, -s.rhs(eb)) < 1e-12 or np.abs(s.rhs(eb)).max() < 1e-14
    np.testing.assert_allclose(sig0, s.average_stress(np.zeros(d.ndof), eb), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("name", STEP_CASES)
def test_preconditioner_matches_oracle(name):
    d, _ = oracle_of(name)
    g = GreenOperator(d.n)
    rng = np.random.default_rng(5)
    f = rng.standard_normal(d.ndof)
    with gpu_of(name) as p:
        y, r2 = p.apply_precond(f)
        y32, r232 = p.apply_precond(f, precision="fp32")
    y_or = g.apply(f, d.nX)
    assert _rel(y, y_or) < 1e-12
    assert abs(r2 - f @ y_or) < 1e-12 * abs(f @ y_or)
    assert _rel(y32, y_or) < 2e-5
    assert abs(r232 - f @ y_or) < 2e-5 * abs(f @ y_or)


SOLVE_CASES = ["sphere8", "coated12", "snapped8", "tiny4"]
_CEFF = {}


def oracle_ceff(name):
    if name not in _CEFF:
        d, _ = oracle_of(name)
        C, _, _ = effective_stiffness(d, tol=1e-13)
        _CEFF[name] = C
    return _CEFF[name]


@pytest.mark.parametrize("name", SOLVE_CASES)
def test_ceff_fp64_matches_oracle(name):
    C_or = oracle_ceff(name)
    with gpu_of(name, rtol=1e-12) as p:
        C, info = p.effective_stiffness()
    assert info["converged"]
    assert _rel(C, C_or) < 1e-10


@pytest.mark.parametrize("name", SOLVE_CASES)
def test_ceff_mixed_matches_oracle(name):
    C_or = oracle_ceff(name)
    with gpu_of(name, rtol=1e-11, precision="mixed") as p:
        C, info = p.effective_stiffness()
    assert info["converged"]
    assert _rel(C, C_or) < 1e-8


def test_one_load_at_a_time_equals_batched():
    with gpu_of("sphere8", rtol=1e-12) as p:
        Cb, _ = p.effective_stiffness()
    with gpu_of("sphere8", rtol=1e-12, batch=False) as p:
        Cs, _ = p.effective_stiffness()
    assert _rel(Cs, Cb) < 1e-11


def test_homogeneous_gives_stiffness_exactly():
    with gpu_of("homogeneous6") as p:
        C, info = p.effective_stiffness()
    lam, mu = 1.3, 0.7
    C_ex = lam * np.outer([1, 1, 1, 0, 0, 0], [1, 1, 1, 0, 0, 0]) + 2 * mu * np.eye(6)
    assert np.abs(C - C_ex).max() < 1e-13
    assert np.all(info["iters"] == 0)


@pytest.mark.parametrize("m,N,s1,w", [((1, 0, 0), 8, 1.37, 4.0), ((1, 1, 1), 18, 3.17, 9.0)])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-8)])
def test_laminate_closed_form_on_gpu(m, N, s1, w, precision, tol):
    from paper_2601_02172_amd import Problem
    n = (N, N, N)
    lame = np.array([[0.5769231, 0.3846154], [27.77778, 41.66667]])
    L, ph = ms.laminate_levelset(n, m, s1, s1 + w)
    with Problem(n, [float(N)] * 3, L, ph, lame, rtol=1e-12 if precision == "fp64" else 1e-11,
                 precision=precision) as p:
        C, _ = p.effective_stiffness()
    Cl = laminate_stiffness(m, [1 - w / N, w / N], lame)
    assert _rel(C, Cl) < tol


def test_displacement_and_stress_outputs_consistent():
    # voxel stresses average to <sigma>; displacements scale with h
    from paper_2601_02172_amd import Problem
    n, L, ph, lame = _case("sphere8")
    h = 0.25
    with Problem(n, [8 * h] * 3, L * h, ph, lame, rtol=1e-12) as p:
        r = p.solve(np.eye(6)[:2], disp=True, stress=True)
    with gpu_of("sphere8", rtol=1e-12) as p:
        r1 = p.solve(np.eye(6)[:2], disp=True)
    np.testing.assert_allclose(r["stress"].mean(axis=2), r["avg_stress"], atol=1e-13)
    np.testing.assert_allclose(r["disp"], h * r1["disp"], atol=1e-12 * np.abs(r1["disp"]).max())
    np.testing.assert_allclose(r["avg_stress"], r1["avg_stress"], atol=1e-12)
    # mean-free FE displacement
    assert np.abs(r["disp"].mean(axis=2)).max() < 1e-13


def test_device_buffer_solve_matches_host_solve():
    # xfft_solve_device (torch device buffers) returns what xfft_solve returns,
    # displacements in units of len (h != 1 here)
    import torch
    from paper_2601_02172_amd import Problem
    n, L, ph, lame = _case("two_spheres_36x24x18")
    h = 0.5
    E = np.eye(6)[[0, 3, 5]]
    with Problem(n, [v * h for v in n], L * h, ph, lame, rtol=1e-11) as p:
        r = p.solve(E, disp=True)
        dev = torch.device("cuda:0")
        strain = torch.tensor(E, dtype=torch.float64, device=dev).contiguous()
        disp = torch.full((3, 3, p.N), float("nan"), dtype=torch.float64, device=dev)
        avg = torch.full((3, 6), float("nan"), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        p.solve_device(strain.data_ptr(), 3, disp.data_ptr(), avg.data_ptr())
        d_dev, a_dev = disp.cpu().numpy(), avg.cpu().numpy()
    np.testing.assert_allclose(a_dev, r["avg_stress"], rtol=0, atol=1e-13 * np.abs(r["avg_stress"]).max())
    np.testing.assert_allclose(d_dev, r["disp"], rtol=0, atol=1e-13 * np.abs(r["disp"]).max())


def _golden(case):
    path = os.path.join(GOLDEN, f"oracle_{case}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    return json.load(open(path))


@pytest.mark.parametrize("precision,rtol,tol", [("fp64", 1e-12, 1e-10), ("mixed", 1e-11, 1e-8)])
def test_single_sphere16_against_golden(precision, rtol, tol):
    g = _golden("single_sphere16")
    cfg = ms.config_single_sphere()
    from paper_2601_02172_amd import Problem
    with Problem(cfg["n"], cfg["length"], cfg["L"], cfg["phase"], cfg["lame"], rtol=rtol, precision=precision) as p:
        C, _ = p.effective_stiffness()
    assert _rel(C, np.array(g["c_eff"])) < tol


@pytest.mark.parametrize("precision,rtol,tol", [("fp64", 1e-12, 1e-10), ("mixed", 1e-11, 1e-8)])
def test_spheres64_against_golden(precision, rtol, tol):
    g = _golden("spheres64")
    cfg = ms.config_spheres64()
    from paper_2601_02172_amd import Problem
    with Problem(cfg["n"], cfg["length"], cfg["L"], cfg["phase"], cfg["lame"], rtol=rtol, precision=precision) as p:
        C, info = p.effective_stiffness()
        lay = p.layout(with_arrays=False)
    assert lay["nX"] == g["stats"]["n_enriched"]
    assert _rel(C, np.array(g["c_eff"])) < tol


@pytest.mark.parametrize("name", STEP_CASES)
def test_voxel_stress_matches_oracle(name):
    # eq. Sapp_q per element, summed over each voxel: element by element
    d, s = oracle_of(name)
    rng = np.random.default_rng(17)
    x = rng.standard_normal(d.ndof)
    eb = rng.standard_normal(6)
    with gpu_of(name) as p:
        vs = p.voxel_stress(x, macro_strain=eb)
        vs0 = p.voxel_stress(x)
    ref = s.voxel_stress(x, eb)
    ref0 = s.voxel_stress(x, np.zeros(6))
    assert _rel(vs, ref) < 1e-12
    assert _rel(vs0, ref0) < 1e-12


def test_solve_stress_output_matches_oracle():
    # the stress output of xfft_solve at the converged solution (GPU rtol 1e-12,
    # oracle 1e-13), two loads, grid spacing h != 1 (stresses do not scale with h)
    from paper_2601_02172_amd import Problem
    name = "two_spheres_36x24x18"
    d, s = oracle_of(name)
    n, L, ph, lame = _case(name)
    E = np.eye(6)[[0, 4]]
    U, _ = solve_loads(d, E, tol=1e-13)
    h = 0.3
    with Problem(n, [v * h for v in n], L * h, ph, lame, rtol=1e-12) as p:
        r = p.solve(E, stress=True)
    for k in range(2):
        ref = s.voxel_stress(U[k], E[k])
        assert _rel(r["stress"][k], ref) < 1e-9
        np.testing.assert_allclose(r["avg_stress"][k], s.average_stress(U[k], E[k]), rtol=0,
                                   atol=1e-10 * np.abs(ref).max())


def test_device_buffer_solve_one_load_at_a_time():
    # batch = 0 with three loads that are not the unit basis: every load's
    # displacement and average stress equal the host solve's
    import torch
    from paper_2601_02172_amd import Problem
    n, L, ph, lame = _case("two_spheres_36x24x18")
    h = 0.5
    E = np.array([[1.0, 0.2, 0.0, 0.0, 0.0, 0.0], [0.0, 0.0, 0.0, 1.0, 0.0, 0.0], [0.1, 0.0, 0.7, 0.0, 0.3, 0.0]])
    with Problem(n, [v * h for v in n], L * h, ph, lame, rtol=1e-11, batch=False) as p:
        r = p.solve(E, disp=True)
        dev = torch.device("cuda:0")
        strain = torch.tensor(E, dtype=torch.float64, device=dev).contiguous()
        disp = torch.full((3, 3, p.N), float("nan"), dtype=torch.float64, device=dev)
        avg = torch.full((3, 6), float("nan"), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        p.solve_device(strain.data_ptr(), 3, disp.data_ptr(), avg.data_ptr())
        d_dev, a_dev = disp.cpu().numpy(), avg.cpu().numpy()
    assert np.abs(r["disp"][0] - r["disp"][1]).max() > 1e-3 * np.abs(r["disp"]).max()
    np.testing.assert_allclose(a_dev, r["avg_stress"], rtol=0, atol=1e-13 * np.abs(r["avg_stress"]).max())
    np.testing.assert_allclose(d_dev, r["disp"], rtol=0, atol=1e-13 * np.abs(r["disp"]).max())


@pytest.mark.parametrize("precision,rtol,tol", [("fp64", 1e-12, 1e-10), ("mixed", 1e-11, 1e-8)])
def test_spheres128_against_golden(precision, rtol, tol):
    # the benchmark workload (128^3, 40 spheres, six unit loads) against the oracle
    g = _golden("spheres128")
    cfg = ms.config_spheres128()
    from paper_2601_02172_amd import Problem
    with Problem(cfg["n"], cfg["length"], cfg["L"], cfg["phase"], cfg["lame"], rtol=rtol, precision=precision) as p:
        C, info = p.effective_stiffness()
        lay = p.layout(with_arrays=False)
    assert info["converged"]
    assert lay["nX"] == g["stats"]["n_enriched"]
    assert _rel(C, np.array(g["c_eff"])) < tol
