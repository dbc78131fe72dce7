"""Accuracy measures of Sec. 4.1: relative error (eq. relError) and the L^2 norm
of a discretised field evaluated by quadrature (eq. L2NormGauss).

TEST INFRASTRUCTURE ONLY (part of the oracle).

The quadrature is the one the discretisation integrates with (Sec. 3): one
point at the centroid of every uncut element (weight = element volume; the
discrete strain is constant there) and the degree-2 four-point rule on every
piece of the subdivided cut elements.  ``quadrature_fields`` returns, for a
solution vector u and macro strain eps_bar, every point's weight, position
(voxel units, node i at x = i), element label and discrete strain
eps_h = eps_bar + B u (Mandel); the exact field of a test problem is then
evaluated at the same points.
"""

import numpy as np

from .kuhn import tet_volume
from .xfem import subdivide
from .quadrature import degree2_rule, degree3_rule
from .system import System


def relative_error(a, a_ref):
    """e(a, a_ref) = |(a - a_ref) / a_ref| (eq. relError)."""
    return abs((a - a_ref) / a_ref)


def l2_norm(w, values):
    """sqrt(sum_q w_q a(x_q) . a(x_q)) (eq. L2NormGauss); values (m, k)."""
    values = np.asarray(values, dtype=np.float64).reshape(len(w), -1)
    return float(np.sqrt(np.sum(np.asarray(w) * np.sum(values * values, axis=1))))


def _cut_points(X, Lv, pts, wts):
    """(weight, position) of every quadrature point of one cut element, in the
    order in which the discretisation built its quadrature data."""
    out = []
    for P, _side in subdivide(X, Lv):
        vol = tet_volume(P)
        for q in range(len(wts)):
            out.append((wts[q] * vol, pts[q] @ P))
    return out


def quadrature_fields(disc, u, ebar):
    """Arrays w (m,), x (m, 3), label (m,), eps (m, 6) over all quadrature points.

    Needs a discretisation built with keep_qp=True (per-point B of cut elements).
    """
    if len(disc.cut_voxel) and not disc.keep_qp:
        raise ValueError("quadrature_fields needs Discretization(..., keep_qp=True)")
    ebar = np.asarray(ebar, dtype=np.float64)
    n0, n1, _ = disc.n
    v = np.arange(disc.N)
    origin = np.stack([v % n0, (v // n0) % n1, v // (n0 * n1)], axis=1).astype(np.float64)
    W, Xs, Lab, Eps = [], [], [], []
    sysm = System(disc)
    for t in range(6):
        m, dofs, _, _ = sysm._uncut(t)
        centroid = disc.tet_X[t].mean(axis=0)
        W.append(np.full(int(m.sum()), disc.tet_vol[t]))
        Xs.append(origin[m] + centroid)
        Lab.append(disc.tet_label[m, t])
        Eps.append(ebar[None, :] + u[dofs] @ disc.B_fe[t].T)
    pts, wts = degree2_rule() if disc.rule == "degree2" else degree3_rule()
    dc = sysm.dofs_cut
    for e in range(len(disc.cut_voxel)):
        t = disc.cut_type[e]
        Lv = disc.Ls[disc.cut_nodes[e]]
        geo = _cut_points(disc.tet_X[t], Lv, pts, wts)
        qps = disc.cut_qp[e]
        assert len(geo) == len(qps)
        o = origin[disc.cut_voxel[e]]
        for (wg, x), (w, B, lab) in zip(geo, qps):
            assert wg == w
            W.append(np.array([w]))
            Xs.append((o + x)[None, :])
            Lab.append(np.array([lab]))
            Eps.append((ebar + B @ u[dc[e]])[None, :])
    return np.concatenate(W), np.concatenate(Xs), np.concatenate(Lab), np.concatenate(Eps)


def stresses(lame, labels, eps):
    """Mandel stress C(label) eps at every point."""
    lam = lame[labels, 0]
    mu = lame[labels, 1]
    tr = eps[:, 0] + eps[:, 1] + eps[:, 2]
    one = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])
    return lam[:, None] * tr[:, None] * one[None, :] + 2.0 * mu[:, None] * eps


def local_errors(w, eps_h, sig_h, eps_ref, sig_ref):
    """Relative L^2 errors of the local strain and stress (eqs. relError, L2NormGauss)."""
    es = l2_norm(w, eps_h - eps_ref) / l2_norm(w, eps_ref)
    ss = l2_norm(w, sig_h - sig_ref) / l2_norm(w, sig_ref)
    return es, ss
