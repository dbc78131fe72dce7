"""Pins of the oracle's geometry: Kuhn voxel, quadrature, subdivision, D0.

Each check compares against something fixed by mathematics, not by the oracle
itself: exact polynomial integrals on the simplex, analytic volumes of the
pieces of a cut tetrahedron, and brute-force sampling of the pointwise
definitions of the enrichment (eqs. modified abs enrichment, enrichedN,
scaling factors).
"""

import math

import numpy as np
import pytest

from oracle.kuhn import CORNERS, kuhn_tets, bary_gradients, tet_volume
from oracle.quadrature import degree2_rule, degree3_rule
from oracle.xfem import subdivide, Discretization, mandel_B, mandel


def test_kuhn_tets_tile_the_voxel():
    tets = kuhn_tets()
    assert len(tets) == 6
    vols = [tet_volume(CORNERS[t].astype(float)) for t in tets]
    np.testing.assert_allclose(vols, 1.0 / 6.0, rtol=0, atol=1e-15)
    # every tet contains the main diagonal 1 -> 7 of the paper's numbering
    for t in tets:
        assert t[0] == 0 and t[-1] == 6
    # random points of the unit cube lie in exactly one tet (up to boundaries)
    rng = np.random.default_rng(0)
    pts = rng.uniform(size=(2000, 3))
    counts = np.zeros(len(pts), dtype=int)
    for t in tets:
        c, G = bary_gradients(CORNERS[t].astype(float))
        lam = c[None, :] + pts @ G.T
        counts += np.all(lam >= -1e-12, axis=1)
    assert np.all(counts == 1)


def test_kuhn_mesh_is_conforming_across_voxels():
    # every face of the 6 tets is either interior (shared by two tets of the same
    # voxel) or lies on a voxel face, and the boundary triangulation of opposite
    # voxel faces matches under the unit translation (periodic conformity)
    tets = kuhn_tets()
    faces = {}
    for t in tets:
        for drop in range(4):
            f = tuple(sorted(c for i, c in enumerate(t) if i != drop))
            faces[f] = faces.get(f, 0) + 1
    boundary = [f for f, k in faces.items() if k == 1]
    assert all(k in (1, 2) for k in faces.values())
    assert len(boundary) == 12                       # two triangles per cube face
    for axis in range(3):
        low = sorted(tuple(sorted(tuple(CORNERS[c]) for c in f)) for f in boundary
                     if all(CORNERS[c][axis] == 0 for c in f))
        high = []
        for f in boundary:
            if all(CORNERS[c][axis] == 1 for c in f):
                tri = []
                for c in f:
                    p = list(CORNERS[c])
                    p[axis] = 0
                    tri.append(tuple(p))
                high.append(tuple(sorted(tri)))
        assert sorted(high) == low


def _simplex_monomial_integral(a):
    # mean over a simplex of l1^a1 l2^a2 l3^a3 l4^a4 = 3! prod(a_i!) / (sum a + 3)!
    return 6.0 * np.prod([math.factorial(k) for k in a]) / math.factorial(sum(a) + 3)


@pytest.mark.parametrize("rule,deg", [(degree2_rule, 2), (degree3_rule, 3)])
def test_quadrature_exactness(rule, deg):
    pts, w = rule()
    np.testing.assert_allclose(np.sum(w), 1.0, atol=1e-15)
    import itertools
    for a in itertools.product(range(deg + 1), repeat=4):
        if sum(a) > deg:
            continue
        q = np.sum(w * np.prod(pts ** np.array(a)[None, :], axis=1))
        exact = _simplex_monomial_integral(a)   # mean value over the simplex (weights are volume fractions)
        assert abs(q - exact) < 1e-14, (a, q, exact)


def _random_cut_tet(rng, pattern):
    X = rng.uniform(size=(4, 3))
    while tet_volume(X) < 0.01:
        X = rng.uniform(size=(4, 3))
    L = np.array([rng.uniform(0.1, 1.0) * s if s != 0 else 0.0 for s in pattern])
    return X, L


PATTERNS = [(1, -1, -1, -1), (-1, 1, 1, 1), (1, 1, -1, -1), (1, -1, 1, -1),
            (1, -1, -1, 0), (-1, 1, 1, 0), (0, 1, -1, 0), (-1, 0, 0, 1)]


@pytest.mark.parametrize("pattern", PATTERNS)
def test_subdivision_tiles_each_side(pattern):
    rng = np.random.default_rng(hash(pattern) % 2**32)
    for _ in range(20):
        X, L = _random_cut_tet(rng, pattern)
        pieces = subdivide(X, L)
        c, G = bary_gradients(X)
        vol = {1: 0.0, -1: 0.0}
        for P, side in pieces:
            vol[side] += tet_volume(P)
            lam = c[None, :] + P @ G.T
            Lh = lam @ L
            assert np.all(side * Lh >= -1e-12)   # each piece lies on its side
        V = tet_volume(X)
        assert abs(vol[1] + vol[-1] - V) < 1e-14
        # analytic volume of the side with a lone vertex: product of the edge fractions
        npos = sum(1 for v in L if v > 0)
        nneg = sum(1 for v in L if v < 0)
        if npos == 1 or nneg == 1:
            lone_side = 1 if npos == 1 else -1
            lone = [a for a in range(4) if np.sign(L[a]) == lone_side][0]
            frac = 1.0
            for b in range(4):
                if b == lone:
                    continue
                if L[b] == 0:
                    continue
                frac *= L[lone] / (L[lone] - L[b])
            assert abs(vol[lone_side] - frac * V) < 1e-14


def _pointwise_NX(X, L, x):
    """N_X^a(x) = N^a(x) rho^m(x) straight from the definitions (barycentric by solve)."""
    T = np.ones((4, 4))
    T[:, 1:] = X
    lam = np.linalg.solve(T.T, np.concatenate([[1.0], x]))
    rho = lam @ np.abs(L) - abs(lam @ L)
    return lam * rho


def _brute_force_element(X, L, n_per_axis=60):
    """Midpoint sampling of int grad N_X^a . grad N_X^b with central differences."""
    lo, hi = X.min(axis=0), X.max(axis=0)
    hstep = (hi - lo) / n_per_axis
    # lattice offsets differ per axis so that no sample lands on the tet's faces
    # (Kuhn faces are the planes x = y, y = z, x = z)
    offs = (0.5, 0.27, 0.73)
    g = [lo[k] + (np.arange(n_per_axis) + offs[k]) * hstep[k] for k in range(3)]
    T = np.ones((4, 4))
    T[:, 1:] = X
    Tinv = np.linalg.inv(T)
    dV = np.prod(hstep)
    eps = 1e-6
    D = np.zeros(4)
    M = np.zeros((4, 4, 3, 3))
    for x0 in g[0]:
        for x1 in g[1]:
            pts = np.stack([np.full(n_per_axis, x0), np.full(n_per_axis, x1), g[2]], axis=1)
            lam = np.concatenate([np.ones((n_per_axis, 1)), pts], axis=1) @ Tinv
            inside = np.all(lam >= 0, axis=1)
            for p in pts[inside]:
                grad = np.zeros((4, 3))
                for k in range(3):
                    e = np.zeros(3)
                    e[k] = eps
                    grad[:, k] = (_pointwise_NX(X, L, p + e) - _pointwise_NX(X, L, p - e)) / (2 * eps)
                for a in range(4):
                    D[a] += dV * np.sum(grad[a] * grad[a])
                M += dV * np.einsum("ak,bl->abkl", grad, grad)
    return D, M


@pytest.mark.slow
@pytest.mark.parametrize("L", [np.array([0.7, -0.35, -0.55, 0.2]),      # (2, 2) split
                               np.array([-0.4, 0.3, 0.25, 0.6]),        # (3, 1) split
                               np.array([0.5, -0.45, 0.0, -0.3])])      # (1, 2, 1) split
def test_cut_element_quadrature_against_brute_force_sampling(L):
    # one cut Kuhn tetrahedron: the oracle's subdivision + degree-2 quadrature of
    # the enriched gradients vs midpoint sampling of the pointwise definitions
    # N_X = N rho^m with central-difference gradients
    from oracle.xfem import cut_element_qps, d0_contributions
    tet = kuhn_tets()[0]
    X = CORNERS[tet].astype(float)
    D_bf, M_bf = _brute_force_element(X, L, n_per_axis=48)
    pts, w = degree2_rule()
    qps = cut_element_qps(X, L, pts, w)
    D_or = d0_contributions(qps)
    M_or = sum(wq * np.einsum("ak,bl->abkl", gX, gX) for (wq, gX, _) in qps)
    np.testing.assert_allclose(D_or, D_bf, rtol=3e-2)   # O(h) sampling error, h = 1/48
    np.testing.assert_allclose(M_or, M_bf, atol=3e-2 * np.abs(M_bf).max())


def test_mandel_B_frobenius_is_twice_gradient_norm():
    # ||M(g (x) I3)||_F^2 = 2 |g|^2: the symmetrised gradient of the vector
    # fields N e_1, e_2, e_3 carries twice the gradient norm of N
    rng = np.random.default_rng(3)
    for _ in range(10):
        g = rng.standard_normal(3)
        B = mandel_B(g)
        assert abs(np.sum(B * B) - 2.0 * g @ g) < 1e-13
        # and B u is the Mandel vector of sym(u (x) g)
        u = rng.standard_normal(3)
        E = 0.5 * (np.outer(u, g) + np.outer(g, u))
        np.testing.assert_allclose(B @ u, mandel(E), atol=1e-14)


def test_element_matrices_independent_of_the_exact_rule():
    # the integrand is quadratic, so the degree-3 rule must reproduce the
    # degree-2 element matrices to rounding
    import microstructure as ms
    n = (6, 6, 6)
    L, ph = ms.spheres_levelset(n, [np.array([2.9, 3.1, 3.05])], [1.9])
    lame = np.array([[1.0, 0.5], [3.0, 2.0]])
    d2 = Discretization(n, (6.0,) * 3, L, ph, lame, rule="degree2")
    d3 = Discretization(n, (6.0,) * 3, L, ph, lame, rule="degree3")
    assert d2.nX > 0
    np.testing.assert_allclose(d2.D0, d3.D0, rtol=1e-12)
    np.testing.assert_allclose(d2.cut_K, d3.cut_K, atol=1e-12 * np.abs(d2.cut_K).max())
    np.testing.assert_allclose(d2.cut_S, d3.cut_S, atol=1e-12 * np.abs(d2.cut_S).max())
