"""Full-size checks on the benchmark workloads (128^3 spheres, 256^3 ellipsoids),
in the launch configuration bench.py times.  The oracle cannot run at these
sizes, so the checks are properties that hold at any size: the mixed-precision
C_eff against the FP64 path (mixed-precision tolerance 1e-8 relative), symmetry and
positive definiteness of C_eff, the Voigt and Reuss bounds of a conforming
Galerkin method (Appendix A), symmetry of the operator and of the
preconditioner, and the gradient of the two precisions against each other.
"""

import numpy as np
import pytest

import microstructure as ms
from closed_forms import voigt_reuss

pytestmark = pytest.mark.gpu

_CFG = {}


def _cfg(name):
    if name not in _CFG:
        _CFG[name] = ms.config_spheres128() if name == "spheres128" else ms.config_ellipsoids()
    return _CFG[name]


def _problem(cfg, **kw):
    from paper_2601_02172_amd import Problem
    return Problem(cfg["n"], cfg["length"], cfg["L"], cfg["phase"], cfg["lame"], **kw)


def _phase_fractions(cfg):
    """Analytic phase volume fractions of the generator (matrix first)."""
    info = cfg["info"]
    nph = cfg["lame"].shape[0]
    if info.get("kind") == "ellipsoids":
        f = np.full(nph, info["vf"] / (nph - 1))
    else:
        r = np.asarray(info["radii"]) / cfg["n"][0]
        f = np.concatenate([[0.0], 4.0 / 3.0 * np.pi * r ** 3])
    f[0] = 1.0 - f[1:].sum()
    return f


@pytest.mark.parametrize("name", ["spheres128", "ellipsoids256"])
def test_fullsize_ceff_mixed_vs_fp64_and_bounds(name):
    cfg = _cfg(name)
    with _problem(cfg, rtol=1e-10, precision="mixed") as pm:
        Cm, im = pm.effective_stiffness()
        gm, _ = pm.grad_lame(np.eye(6))
    with _problem(cfg, rtol=1e-13, precision="fp64", batch=False) as p64:
        C64, i64 = p64.effective_stiffness()
        g64, _ = p64.grad_lame(np.eye(6))
    assert im["converged"] and i64["converged"]
    nrm = np.linalg.norm(C64)
    assert np.linalg.norm(Cm - C64) < 1e-8 * nrm
    assert np.abs(C64 - C64.T).max() < 1e-10 * nrm
    assert np.linalg.eigvalsh(0.5 * (C64 + C64.T)).min() > 0.0
    V, R = voigt_reuss(_phase_fractions(cfg), cfg["lame"])
    assert np.linalg.eigvalsh(V - C64).min() > -1e-9 * nrm
    assert np.linalg.eigvalsh(C64 - R).min() > -1e-9 * nrm
    # gradients from the stored unit-load solutions of the two paths
    assert np.abs(gm - g64).max() < 1e-6 * np.abs(g64).max()


def test_fullsize_operator_and_preconditioner_symmetric():
    cfg = _cfg("spheres128")
    rng = np.random.default_rng(17)
    with _problem(cfg) as p:
        n = 3 * (p.N + p.nX)
        x, y = rng.standard_normal(n), rng.standard_normal(n)
        Ax, _ = p.apply_operator(x)
        Ay, _ = p.apply_operator(y)
        assert abs(x @ Ay - y @ Ax) < 1e-11 * np.sqrt((x @ Ax) * (y @ Ay))
        assert x @ Ax > 0.0
        Px, r2x = p.apply_precond(x)
        Py, _ = p.apply_precond(y)
        assert abs(x @ Py - y @ Px) < 1e-11 * np.sqrt((x @ Px) * (y @ Py))
        assert abs(r2x - x @ Px) < 1e-10 * abs(x @ Px)
        # the FP32 kernels of the mixed path at the same size
        Ax32, _ = p.apply_operator(x, precision="fp32")
        Px32, _ = p.apply_precond(x, precision="fp32")
        assert np.abs(Ax32 - Ax).max() < 2e-5 * np.abs(Ax).max()
        assert np.abs(Px32 - Px).max() < 2e-5 * np.abs(Px).max()
