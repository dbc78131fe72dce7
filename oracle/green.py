"""Green operator: inverse of the constant-coefficient preconditioner A11^0.

A11^0 (eq. constantCoefficientPreconditioner) is the FE stiffness of the
identity material (C = I in Mandel form, i.e. energy grad^s u : grad^s u) on
the periodic grid.  It is translation invariant, so it acts as a 3 x 3 matrix
Fourier multiplier (eq. GreenHermitian).  The oracle does not use the closed
form of that multiplier: it assembles A11^0 on a 4^3 grid with the same element
machinery as the full system, reads off the 27-point stencil of node 0 and
takes its discrete Fourier transform.  The multiplier is inverted at every
non-zero frequency; the zero frequency maps to zero, which removes the mean of
the FE field (the constraint sum u_FE = 0 of eq. X-FEM space).

The block preconditioner of eq. scaledPreconditioner is this Green operator on
the FE block and the identity on the scaled enriched block.
"""

import numpy as np

from .xfem import Discretization
from .system import System


def _stencil():
    """K[c, d][dz+1, dy+1, dx+1] = (A11^0)_{(c, node at offset), (d, node 0)}."""
    n = (4, 4, 4)
    N = 64
    disc = Discretization(n, (4.0, 4.0, 4.0), np.ones(N), np.zeros(N, dtype=np.int64),
                          np.array([[0.0, 0.5]]))
    A = System(disc).assemble().toarray()
    K = np.zeros((3, 3, 3, 3, 3))
    for c in range(3):
        for dcomp in range(3):
            col = A[c * N:(c + 1) * N, dcomp * N]
            for dz in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        node = (dx % 4) + 4 * ((dy % 4) + 4 * (dz % 4))
                        K[c, dcomp, dz + 1, dy + 1, dx + 1] = col[node]
    # everything outside the 27-point neighbourhood must vanish
    mask = np.zeros(N, dtype=bool)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                mask[(dx % 4) + 4 * ((dy % 4) + 4 * (dz % 4))] = True
    assert np.all(A[:3 * N, 0][np.tile(~mask, 3)] == 0.0)
    return K


_STENCIL = None


def stencil():
    global _STENCIL
    if _STENCIL is None:
        _STENCIL = _stencil()
    return _STENCIL


class GreenOperator:
    """P^-1 of eq. scaledPreconditioner on an n0 x n1 x n2 grid (voxel units)."""

    def __init__(self, n):
        self.n = tuple(int(v) for v in n)
        n0, n1, n2 = self.n
        K = stencil()
        grid = np.zeros((3, 3, n2, n1, n0))
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    grid[:, :, dz % n2, dy % n1, dx % n0] += K[:, :, dz + 1, dy + 1, dx + 1]
        # symbol: S(xi) = sum_m K(m) exp(-2 pi i xi . m / n)
        S = np.fft.fftn(grid, axes=(2, 3, 4))
        self.symbol = S
        Sm = np.moveaxis(S, (0, 1), (-2, -1))          # (..., 3, 3)
        Sm = Sm.copy()
        Sm[0, 0, 0] = np.eye(3)
        G = np.linalg.inv(Sm)
        G[0, 0, 0] = 0.0
        self.G = G                                      # (n2, n1, n0, 3, 3)

    def apply_fe(self, f):
        """Green operator on an FE field given as (3, N) or flat 3N (component-major)."""
        n0, n1, n2 = self.n
        F = np.fft.fftn(np.asarray(f, dtype=np.float64).reshape(3, n2, n1, n0), axes=(1, 2, 3))
        Y = np.einsum("zyxcd,dzyx->czyx", self.G, F)
        return np.real(np.fft.ifftn(Y, axes=(1, 2, 3))).reshape(-1)

    def apply(self, f, nX):
        """Block preconditioner: Green on the FE block, identity on the enriched block."""
        N = int(np.prod(self.n))
        out = np.empty_like(f)
        out[:3 * N] = self.apply_fe(f[:3 * N])
        out[3 * N:] = f[3 * N:]
        return out
