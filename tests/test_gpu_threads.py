"""Distinct problems used from several threads at once (the header allows it).

Two problems on grids no other test uses -- so that both threads run the
operator-depth and Green-operator autotuners at the same time, whose
process-wide caches are shared -- are solved concurrently from two Python
threads (the ctypes calls release the GIL), then again one after the other.
C_eff agrees between the two runs to the solver tolerance, and the FP64 one
with the oracle.
"""

import threading

import numpy as np
import pytest

import microstructure as ms

pytestmark = pytest.mark.gpu

CASES = {
    "sphere_18": ((18, 18, 18), [(8.7, 9.4, 9.1)], [4.8], "fp64", 1e-12),
    "two_spheres_24x18x16": ((24, 18, 16), [(6.3, 8.8, 7.1), (17.2, 9.4, 8.3)], [4.1, 3.6], "mixed", 1e-11),
}
LAME = np.array([[0.5769231, 0.3846154], [4.0, 4.0], [27.77778, 41.66667]])


def _solve(name):
    from paper_2601_02172_amd import Problem
    n, centers, radii, precision, rtol = CASES[name]
    L, ph = ms.spheres_levelset(n, [np.asarray(c, dtype=float) for c in centers], radii)
    with Problem(n, [float(v) for v in n], L, ph, LAME[: len(radii) + 1], rtol=rtol, precision=precision) as p:
        C, info = p.effective_stiffness()
    assert info["converged"]
    return C


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_distinct_problems_from_two_threads():
    out, errors = {}, []

    def run(name):
        try:
            out[name] = _solve(name)
        except Exception as e:             # re-raised below
            errors.append((name, e))

    threads = [threading.Thread(target=run, args=(name,)) for name in CASES]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=240)
    assert not any(t.is_alive() for t in threads), "a solve did not finish"
    assert not errors, errors
    for name in CASES:
        C_seq = _solve(name)
        assert _rel(out[name], C_seq) < 1e-9, name
    # the FP64 case against the oracle
    from oracle.xfem import Discretization
    from oracle.homogenize import effective_stiffness
    n, centers, radii, _, _ = CASES["sphere_18"]
    L, ph = ms.spheres_levelset(n, [np.asarray(c, dtype=float) for c in centers], radii)
    d = Discretization(n, tuple(float(v) for v in n), L, ph, LAME[:2], keep_qp=False)
    C_or = effective_stiffness(d, tol=1e-13)[0]
    assert _rel(out["sphere_18"], C_or) < 1e-10
