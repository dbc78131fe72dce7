"""Reference voxel and its six P1 tetrahedra (Sec. 3, Fig. "Division of the voxel").

The paper numbers the eight voxel corners by the matrix Y of eq. GreenHermitian
(rows = corners 1..8, columns = x, y, z).  The figure showing the six P1
elements is not available; the decomposition used here is the one forced by the
single reference voxel matrix of eq. A0Voxel (translation invariance and
conformity): the six tetrahedra sharing the main diagonal from corner 1 (0,0,0)
to corner 7 (1,1,1), one per monotone corner path (Kuhn / Freudenthal).
"""

import itertools

import numpy as np

# Corner coordinates in the paper's numbering (0-based here: corner c = Y row c).
CORNERS = np.array([
    [0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
    [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1],
], dtype=np.int64)


def _corner_index(xyz):
    for c, row in enumerate(CORNERS):
        if tuple(row) == tuple(xyz):
            return c
    raise KeyError(xyz)


def kuhn_tets():
    """The six tetrahedra as lists of four corner indices in path order.

    Each permutation (a, b, c) of the axes gives the path
    0 -> e_a -> e_a + e_b -> e_a + e_b + e_c; permutations are enumerated in
    lexicographic order.  The position along the path is the vertex order.
    """
    tets = []
    for perm in itertools.permutations(range(3)):
        p = np.zeros(3, dtype=np.int64)
        verts = [_corner_index(p)]
        for ax in perm:
            p = p.copy()
            p[ax] += 1
            verts.append(_corner_index(p))
        tets.append(verts)
    return tets


def bary_gradients(X):
    """Barycentric coordinates of a tetrahedron with vertices X (4 x 3).

    Returns (c, G) with lambda_a(x) = c[a] + G[a] . x, obtained by inverting the
    affine map [1, x] -> barycentric coordinates.
    """
    T = np.ones((4, 4))
    T[:, 1:] = X
    Tinv = np.linalg.inv(T)          # column a holds the coefficients of lambda_a
    return Tinv[0, :].copy(), Tinv[1:, :].T.copy()


def tet_volume(X):
    """Unsigned volume of a tetrahedron with vertices X (4 x 3)."""
    return abs(np.linalg.det(X[1:] - X[0])) / 6.0
