"""Quadrature rules on tetrahedra in barycentric form.

* ``degree2_rule``: the symmetric four-point rule of degree 2 that Sec. 3 uses
  on every subtetrahedron (Shunn and Ham, App. F): the four barycentric
  permutations of (alpha, beta, beta, beta), alpha = (5 + 3 sqrt 5)/20,
  beta = (5 - sqrt 5)/20, each with a quarter of the volume.
* ``degree3_rule``: the five-point degree-3 rule (centroid weight -4/5, points
  (1/2, 1/6, 1/6, 1/6) weight 9/20), used only to check exactness.
* ``centroid_rule``: one point, exact for the constant integrand of uncut P1
  elements (eq. A0Voxel).
"""

import numpy as np


def degree2_rule():
    a = (5.0 + 3.0 * np.sqrt(5.0)) / 20.0
    b = (5.0 - np.sqrt(5.0)) / 20.0
    pts = np.full((4, 4), b)
    np.fill_diagonal(pts, a)
    return pts, np.full(4, 0.25)


def degree3_rule():
    pts = np.full((5, 4), 1.0 / 6.0)
    pts[0, :] = 0.25
    for i in range(4):
        pts[i + 1, i] = 0.5
    w = np.array([-0.8, 0.45, 0.45, 0.45, 0.45])
    return pts, w


def centroid_rule():
    return np.full((1, 4), 0.25), np.ones(1)
