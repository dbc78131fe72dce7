"""Single cubic inclusion on the GPU (Sec. 4.5): the paper's non-smooth test case.

Cell edge 128, cube edge 82.7854 centred at 67.4142 (1, 1, 1), polyamide matrix
(E = 2.1, nu = 0.22) and E-glass cube (E = 72, nu = 0.22), macro strain
eps_11 = 0.1 %, in the orientation parallel to the grid and rotated by 15
degrees about x, y and z (R = Rz Ry Rx; the paper does not state the order,
which changes the result by less than 0.1 %).

* The effective stress converges in N: N = 256 and 512 agree to 5e-4 relative
  (measured: 2e-5 parallel, 1.1e-4 rotated; the corners make the rate
  sub-quadratic, as the paper observes).
* Oracle parity at N = 16 (straight and rotated): average stress and the
  voxel stress field against the CPU oracle.
* Soft pin of the printed value: the paper reports the parallel case converging
  to about 4.58 MPa; the converged GPU value (4.622 MPa) lies within 1.5 % of it.
  The rotated case (4.603 MPa here, about 4.49 MPa printed) is parity unpinned.
"""

import numpy as np
import pytest

from microstructure.shapes import cube_levelset, rotation_xyz

pytestmark = pytest.mark.gpu

EB = np.array([1e-3, 0.0, 0.0, 0.0, 0.0, 0.0])


def _lame(E, nu):
    return [E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))]


LAME = np.array([_lame(2.1, 0.22), _lame(72.0, 0.22)])       # GPa -> stresses in GPa


def _sigma_xx_mpa(N, rotated, precision="fp64"):
    from paper_2601_02172_amd import Problem
    h = 128.0 / N
    L, ph = cube_levelset((N, N, N), np.full(3, 67.4142 / h), 82.7854 / h, rotation_xyz(15.0) if rotated else None)
    with Problem((N, N, N), [128.0] * 3, L * h, ph, LAME, rtol=1e-8, precision=precision) as p:
        r = p.solve(EB)
    assert r["converged"]
    return 1000.0 * r["avg_stress"][0][0]


@pytest.mark.parametrize("rotated", [False, True])
def test_cube_effective_stress_converges(rotated):
    s256 = _sigma_xx_mpa(256, rotated, "mixed")
    s512 = _sigma_xx_mpa(512, rotated, "mixed")
    print(f"{'rotated' if rotated else 'parallel'}: sigma_xx {s256:.5f} (256), {s512:.5f} (512) MPa", flush=True)
    assert abs(s256 - s512) < 5e-4 * abs(s512)


def test_parallel_cube_near_printed_value():
    s = _sigma_xx_mpa(256, False)
    assert abs(s - 4.58) < 0.015 * 4.58


@pytest.mark.parametrize("rotated", [False, True])
def test_cube_fields_match_oracle_n16(rotated):
    # the cubic inclusion at N = 16 against the oracle: <sigma> and the voxel
    # stress field at convergence, straight and rotated (non-smooth interface,
    # edges and corners cutting elements in every configuration)
    from paper_2601_02172_amd import Problem
    from oracle.xfem import Discretization
    from oracle.homogenize import solve_loads
    from oracle.system import System
    N = 16
    h = 128.0 / N
    L, ph = cube_levelset((N, N, N), np.full(3, 67.4142 / h), 82.7854 / h, rotation_xyz(15.0) if rotated else None)
    d = Discretization((N,) * 3, (128.0,) * 3, L * h, ph, LAME, keep_qp=False)
    U, _ = solve_loads(d, EB, tol=1e-13)
    s = System(d)
    sig_or = s.average_stress(U[0], EB)
    vs_or = s.voxel_stress(U[0], EB)
    with Problem((N,) * 3, [128.0] * 3, L * h, ph, LAME, rtol=1e-12) as p:
        r = p.solve(EB, stress=True)
    assert r["converged"]
    assert np.abs(r["avg_stress"][0] - sig_or).max() < 1e-10 * np.abs(sig_or).max()
    assert np.abs(r["stress"][0] - vs_or).max() < 1e-9 * np.abs(vs_or).max()
