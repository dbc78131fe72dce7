"""Green-operator kernel variants (option fft_variant) and their autotuner.

Every variant -- the xy-plane kernels or separate x and y passes, and the two
z-pass tiles -- computes the same preconditioner (eqs. scaledPreconditioner,
GreenHermitian).  Each is forced in turn and compared element by element with
the oracle's Green operator, whose symbol is the FFT of the assembled reference
stencil (FP64 1e-12, or the oracle's own symbol rounding at n = 256; FP32 2e-5
relative), and the Parseval value f^T P^-1 f, at shapes that reach every
compile-time kernel the variants add: 128^3 (plane or separate passes of
length 128, z tiles of 16 / 8 columns in FP32), 16 x 16 x 256 (z tiles of 8 /
16 columns in FP32, 4 / 8 in FP64), 48 x 48 x 96 (z pass outside the fast
staging path) and 256 x 256 x 16.  End to end, the 64^3 benchmark RVE solved
with the autotuned choice and with every fixed variant matches the oracle's
stored C_eff.
"""

import json
import os

import numpy as np
import pytest

import microstructure as ms
from oracle.xfem import Discretization
from oracle.green import GreenOperator

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
LAME3 = np.array([[0.5769231, 0.3846154], [4.0, 4.0], [27.77778, 41.66667]])

SHAPES = {
    "128x128x128": ((128, 128, 128), [(40.3, 77.1, 61.7), (101.2, 20.6, 110.9)], [9.6, 6.3]),
    "16x16x256": ((16, 16, 256), [(8.1, 7.7, 40.2), (4.4, 10.9, 190.3)], [5.3, 4.1]),
    "48x48x96": ((48, 48, 96), [(20.2, 30.7, 41.3), (9.9, 12.1, 80.6)], [6.2, 4.4]),
    "256x256x16": ((256, 256, 16), [(37.2, 201.5, 7.6), (180.3, 60.7, 9.2)], [5.6, 4.9]),
}


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _green_tol_fp64(n):
    # the oracle's symbol is the DFT of the assembled stencil: at the lowest
    # frequency its entries cancel to 2 sin^2(pi / n_max), so it carries a
    # relative error of up to about 12 u / (2 sin^2(pi / n_max))
    lam_min = 2.0 * np.sin(np.pi / max(n)) ** 2
    return max(1e-12, 12.0 * 2.0 ** -53 / lam_min)


_OR = {}


def _oracle(shape):
    if shape not in _OR:
        n, centers, radii = SHAPES[shape]
        L, ph = ms.spheres_levelset(n, [np.asarray(c, dtype=float) for c in centers], radii)
        d = Discretization(n, tuple(float(v) for v in n), L, ph, LAME3, keep_qp=False)
        f = np.random.default_rng(23).standard_normal(d.ndof)
        y = GreenOperator(n).apply(f, d.nX)
        _OR[shape] = (L, ph, d.nX, f, y, float(f @ y))
    return _OR[shape]


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("shape", list(SHAPES))
def test_preconditioner_variant_matches_oracle(shape, variant):
    from paper_2601_02172_amd import Problem
    n = SHAPES[shape][0]
    L, ph, nX, f, y_or, r2_or = _oracle(shape)
    with Problem(n, [float(v) for v in n], L, ph, LAME3, fft_variant=variant) as p:
        assert p.nX == nX
        y64, r64 = p.apply_precond(f)
        y32, r32 = p.apply_precond(f, precision="fp32")
    tol = _green_tol_fp64(n)
    assert _rel(y64, y_or) < tol
    assert abs(r64 - r2_or) < tol * abs(r2_or)
    assert _rel(y32, y_or) < 2e-5
    assert abs(r32 - r2_or) < 2e-5 * abs(r2_or)


@pytest.mark.parametrize("precision,rtol,tol", [("fp64", 1e-12, 1e-10), ("mixed", 1e-11, 1e-8)])
def test_spheres64_every_variant_against_golden(precision, rtol, tol):
    from paper_2601_02172_amd import Problem
    path = os.path.join(GOLDEN, "oracle_spheres64.json")
    C_or = np.array(json.load(open(path))["c_eff"])
    cfg = ms.config_spheres64()
    chosen = None
    for variant in ["auto", 0, 1, 2, 3]:
        with Problem(cfg["n"], cfg["length"], cfg["L"], cfg["phase"], cfg["lame"], rtol=rtol,
                     precision=precision, fft_variant=variant) as p:
            C, info = p.effective_stiffness()
        assert info["converged"]
        assert _rel(C, C_or) < tol, variant
        if variant == "auto":
            chosen = info["fft_variant"]
        else:
            assert info["fft_variant"] == variant
    print(f"{precision}: autotuned FFT variant at 64^3: {chosen}")
    assert chosen in (0, 1, 2, 3)
