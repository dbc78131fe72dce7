"""Textbook closed forms used as pins (none of them is the discretisation itself).

* rank-one laminate of isotropic phases (traction continuity + strain
  compatibility across planar interfaces): phase stresses and C_eff;
* composite-sphere bulk modulus (Hashin), the neutral-inclusion construction
  of the Hashin study;
* dilute Eshelby estimates for spherical inclusions;
* Voigt and Reuss bounds.
"""

import numpy as np

S2 = np.sqrt(2.0)


def mandel_to_tensor(v):
    return np.array([[v[0], v[5] / S2, v[4] / S2],
                     [v[5] / S2, v[1], v[3] / S2],
                     [v[4] / S2, v[3] / S2, v[2]]])


def tensor_to_mandel(E):
    return np.array([E[0, 0], E[1, 1], E[2, 2], S2 * E[1, 2], S2 * E[0, 2], S2 * E[0, 1]])


def iso_stiffness(lam, mu):
    one = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])
    return lam * np.outer(one, one) + 2.0 * mu * np.eye(6)


def laminate_phase_stresses(normal, fractions, lames, ebar):
    """Uniform stress (Mandel) in each phase of a rank-one laminate under the macro strain ebar.

    Each phase strain is ebar + sym(a_p (x) n) (compatibility across the
    planes); the traction sigma_p n is the same vector t in every phase and the
    jumps a_p average to zero over the fractions.
    """
    n = np.asarray(normal, dtype=np.float64)
    n = n / np.linalg.norm(n)
    eb = mandel_to_tensor(np.asarray(ebar, dtype=np.float64))
    Kinv, rhs = [], []
    for (lam, mu) in lames:
        K = mu * np.eye(3) + (lam + mu) * np.outer(n, n)
        sig = lam * np.trace(eb) * np.eye(3) + 2.0 * mu * eb
        Kinv.append(np.linalg.inv(K))
        rhs.append(np.linalg.inv(K) @ (sig @ n))
    Kavg = sum(f * Ki for f, Ki in zip(fractions, Kinv))
    t = np.linalg.solve(Kavg, sum(f * r for f, r in zip(fractions, rhs)))
    out = []
    for (lam, mu), Ki in zip(lames, Kinv):
        sig0 = lam * np.trace(eb) * np.eye(3) + 2.0 * mu * eb
        a = Ki @ (t - sig0 @ n)
        eps = eb + 0.5 * (np.outer(a, n) + np.outer(n, a))
        out.append(tensor_to_mandel(lam * np.trace(eps) * np.eye(3) + 2.0 * mu * eps))
    return out


def laminate_stiffness(normal, fractions, lames):
    """Effective Mandel stiffness of a rank-one laminate of isotropic phases."""
    C = np.zeros((6, 6))
    for k in range(6):
        sig = laminate_phase_stresses(normal, fractions, lames, np.eye(6)[k])
        C[:, k] = sum(f * s for f, s in zip(fractions, sig))
    return C


def composite_sphere_bulk(Kc, Gc, Ki, f):
    """Bulk modulus of a composite sphere: core Ki, coating (Kc, Gc), core fraction f."""
    return Kc + f * (Ki - Kc) / (1.0 + (1.0 - f) * (Ki - Kc) / (Kc + 4.0 * Gc / 3.0))


def eshelby_dilute(Km, Gm, Ki, Gi, f):
    """Dilute-sphere estimates of the effective bulk and shear moduli."""
    K = Km + f * (Ki - Km) * (3.0 * Km + 4.0 * Gm) / (3.0 * Ki + 4.0 * Gm)
    zeta = Gm * (9.0 * Km + 8.0 * Gm) / (6.0 * (Km + 2.0 * Gm))
    G = Gm + f * (Gi - Gm) * (Gm + zeta) / (Gi + zeta)
    return K, G


def voigt_reuss(fractions, lames):
    """Voigt (arithmetic) and Reuss (harmonic) averages of the phase stiffnesses."""
    Cs = [iso_stiffness(l, m) for (l, m) in lames]
    V = sum(f * C for f, C in zip(fractions, Cs))
    R = np.linalg.inv(sum(f * np.linalg.inv(C) for f, C in zip(fractions, Cs)))
    return V, R


def isotropic_projection(C):
    """Bulk and shear moduli of the isotropic projection of a Mandel stiffness."""
    one = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0]) / np.sqrt(3.0)
    Jp = np.outer(one, one)
    Kp = np.eye(6) - Jp
    K = np.trace(Jp @ C) / 3.0
    G = np.trace(Kp @ C) / 10.0
    return K, G


def laminate_phase_strains(normal, fractions, lames, ebar):
    """Uniform strain (Mandel) in each phase of a rank-one laminate (see laminate_phase_stresses)."""
    out = []
    for (lam, mu), sig in zip(lames, laminate_phase_stresses(normal, fractions, lames, ebar)):
        S = np.linalg.inv(iso_stiffness(lam, mu))
        out.append(S @ sig)
    return out


class CoatedSphereField:
    """Exact field of a composite sphere (core radius ri, coating radius rc) in an
    infinite matrix under the hydrostatic macro strain e I, all phases isotropic.

    The displacement is radial, u = (A r + B / r^2) x / r in every phase (B = 0
    in the core, and u = e x in the matrix when the sphere is neutral), so the
    strain is A I + (B / r^3)(I - 3 n (x) n).  A and B follow from continuity of
    u and of the radial traction 3 K A - 4 G B / r^3 at ri and continuity of u at
    rc.  The remaining condition -- continuity of the radial traction at rc --
    holds exactly when the matrix bulk modulus equals the composite-sphere bulk
    modulus (the neutral inclusion); ``traction_jump`` reports its residual.
    """

    def __init__(self, K, G, ri, rc, e=1.0):
        self.K = np.asarray(K, dtype=np.float64)       # (matrix, coating, core)
        self.G = np.asarray(G, dtype=np.float64)
        self.ri, self.rc, self.e = float(ri), float(rc), float(e)
        Kc, Gc, Ki = self.K[1], self.G[1], self.K[2]
        # unknowns (A_core, A_coat, B_coat)
        M = np.array([[self.ri, -self.ri, -1.0 / self.ri ** 2],          # u continuous at ri
                      [3.0 * Ki, -3.0 * Kc, 4.0 * Gc / self.ri ** 3],     # traction continuous at ri
                      [0.0, self.rc, 1.0 / self.rc ** 2]])                # u = e rc at rc
        self.Ai, self.Ac, self.Bc = np.linalg.solve(M, np.array([0.0, 0.0, self.e * self.rc]))

    def traction_jump(self):
        """Radial traction of the coating minus that of the matrix at rc."""
        return 3.0 * self.K[1] * self.Ac - 4.0 * self.G[1] * self.Bc / self.rc ** 3 - 3.0 * self.K[0] * self.e

    def phase_at(self, r):
        return np.where(r >= self.rc, 0, np.where(r >= self.ri, 1, 2))

    def strain(self, d):
        """Total strain (Mandel, (m, 6)) and phase (m,) at offsets d (m, 3) from the centre."""
        d = np.atleast_2d(d)
        r = np.sqrt(np.sum(d * d, axis=1))
        ph = self.phase_at(r)
        A = np.where(ph == 0, self.e, np.where(ph == 1, self.Ac, self.Ai))
        B = np.where(ph == 1, self.Bc, 0.0)
        rs = np.where(r > 0, r, 1.0)
        n = d / rs[:, None]
        b = B / rs ** 3
        E = A[:, None, None] * np.eye(3)[None] + b[:, None, None] * (np.eye(3)[None] - 3.0 * n[:, :, None] * n[:, None, :])
        eps = np.stack([E[:, 0, 0], E[:, 1, 1], E[:, 2, 2], S2 * E[:, 1, 2], S2 * E[:, 0, 2], S2 * E[:, 0, 1]], axis=1)
        return eps, ph

    def displacement(self, d):
        d = np.atleast_2d(d)
        r = np.sqrt(np.sum(d * d, axis=1))
        ph = self.phase_at(r)
        A = np.where(ph == 0, self.e, np.where(ph == 1, self.Ac, self.Ai))
        B = np.where(ph == 1, self.Bc, 0.0)
        rs = np.where(r > 0, r, 1.0)
        return (A + B / rs ** 3)[:, None] * d
