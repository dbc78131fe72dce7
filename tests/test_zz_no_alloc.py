"""xfft_apply_operator_noalloc (static work space, no device allocation) against
xfft_apply_operator on the same inputs: two calls in a row, the second on a
smaller grid, with and without a macro strain.  Bar: 1e-12 relative (FP64
step-level parity; the two run the same kernels and the same reduction order,
so they agree to the last bit in practice).  A grid whose work space exceeds
the static area is refused with XFFT_EINVAL."""

import numpy as np
import pytest

import microstructure as ms

pytestmark = pytest.mark.gpu

LAME = np.array([[0.5769231, 0.3846154], [27.77778, 41.66667], [4.0, 4.0]])


def _grid(name):
    if name == "two_spheres_36x24x18":
        n = (36, 24, 18)
        L, ph = ms.spheres_levelset(n, [np.array([9.3, 11.2, 8.7]), np.array([27.1, 6.4, 12.9])], [5.1, 3.7])
        return n, L, ph, LAME
    if name == "sphere8":
        n = (8, 8, 8)
        L, ph = ms.spheres_levelset(n, [np.array([4.13, 3.93, 4.21])], [2.6])
        return n, L, ph, LAME[[0, 2]]
    raise KeyError(name)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_noalloc_operator_matches_apply_operator_twice():
    import torch
    from paper_2601_02172_amd import Problem
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(31)
    for name in ("two_spheres_36x24x18", "sphere8"):          # second call: smaller grid
        n, L, ph, lame = _grid(name)
        with Problem(n, [float(v) for v in n], L, ph, lame) as p:
            ndof = 3 * (p.N + p.nX)
            x = rng.standard_normal(ndof)
            eb = rng.standard_normal(6)
            y_ref, avg_ref = p.apply_operator(x, macro_strain=eb)
            y0_ref, _ = p.apply_operator(x, with_stress=False)
            xd = torch.tensor(x, dtype=torch.float64, device=dev)
            ebd = torch.tensor(eb, dtype=torch.float64, device=dev)
            yd = torch.full((ndof,), float("nan"), dtype=torch.float64, device=dev)
            y0d = torch.full((ndof,), float("nan"), dtype=torch.float64, device=dev)
            avgd = torch.full((6,), float("nan"), dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            p.apply_operator_noalloc(xd.data_ptr(), yd.data_ptr(), ebd.data_ptr(), avgd.data_ptr())
            p.apply_operator_noalloc(xd.data_ptr(), y0d.data_ptr())
            torch.cuda.synchronize()
            y, y0, avg = yd.cpu().numpy(), y0d.cpu().numpy(), avgd.cpu().numpy()
        print(name, "max |diff| y", np.abs(y - y_ref).max(), "avg", np.abs(avg - avg_ref).max(), flush=True)
        assert np.all(np.isfinite(y)) and np.all(np.isfinite(y0))
        assert _rel(y, y_ref) < 1e-12
        assert _rel(y0, y0_ref) < 1e-12
        np.testing.assert_allclose(avg, avg_ref, rtol=0, atol=1e-12 * np.abs(avg_ref).max())


def test_noalloc_operator_refuses_work_space_beyond_the_static_area():
    # planar interfaces every two voxels along x: half of the 96^3 voxels are
    # irregular (442 k), more than the static area's corner-force buffer holds
    import torch
    from paper_2601_02172_amd import Problem, XfftError
    N = 96
    n = (N, N, N)
    x = np.arange(N ** 3) % N
    L = (4.0 / (2.0 * np.pi)) * np.sin(2.0 * np.pi * (x + 0.3) / 4.0)
    ph = (L < 0).astype(np.int32)
    with Problem(n, [float(N)] * 3, L, ph, LAME[:2]) as p:
        assert p.layout(with_arrays=False)["n_irregular_voxels"] > 160000
        ndof = 3 * (p.N + p.nX)
        xd = torch.zeros(ndof, dtype=torch.float64, device="cuda:0")
        yd = torch.zeros(ndof, dtype=torch.float64, device="cuda:0")
        with pytest.raises(XfftError) as e:
            p.apply_operator_noalloc(xd.data_ptr(), yd.data_ptr())
        assert e.value.code == -1
