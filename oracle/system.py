"""Global scaled system of eq. linearSystem_element, assembled or applied element by element.

Layout of a global vector (component-major): FE dof (node i, component c) at
``c * N + i``; scaled enriched dof (enriched node j, component c) at
``3 N + c * nX + j``.

Sign reading of eqs. b, resVector and Algorithm 1: the discrete weak form with
strain eps = eps_bar + grad^s u requires sum_e Lambda_e^T int B^T C (eps_bar + B u)
= 0, so the right-hand side is b = -sum_e Lambda_e^T int B^T C eps_bar and the
residual map r(u) = A u - b is the gradient of the cell energy.
"""

import numpy as np
import scipy.sparse as sp

ONE = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])


def _iso_stress(eps, lam, mu):
    """Row-wise isotropic Hooke law in Mandel form."""
    tr = eps[:, 0] + eps[:, 1] + eps[:, 2]
    return lam[:, None] * tr[:, None] * ONE[None, :] + 2.0 * mu[:, None] * eps


class System:
    """Element-level operators of one discretisation."""

    def __init__(self, disc):
        self.d = disc
        self.dofs_cut = disc.element_dofs_cut()

    @property
    def ndof(self):
        return self.d.ndof

    # --------------------------------------------------------------- uncut element helpers
    def _uncut(self, t):
        d = self.d
        m = ~d.cut[:, t]
        dofs = d.element_dofs_uncut(t)[m]
        lm = d.uncut_lame(t)[m]
        return m, dofs, lm[:, 0], lm[:, 1]

    # --------------------------------------------------------------- operator and rhs
    def apply(self, x):
        """A x by the element loop sum_e Lambda_e^T A_e Lambda_e x."""
        d = self.d
        y = np.zeros(self.ndof)
        for t in range(6):
            _, dofs, lam, mu = self._uncut(t)
            B = d.B_fe[t]
            eps = x[dofs] @ B.T
            f = d.tet_vol[t] * _iso_stress(eps, lam, mu) @ B
            y += np.bincount(dofs.ravel(), f.ravel(), minlength=self.ndof)
        if len(self.dofs_cut):
            f = np.einsum("eij,ej->ei", d.cut_K, x[self.dofs_cut])
            y += np.bincount(self.dofs_cut.ravel(), f.ravel(), minlength=self.ndof)
        return y

    def rhs(self, ebar):
        """b = -sum_e Lambda_e^T int B^T C eps_bar."""
        d = self.d
        ebar = np.asarray(ebar, dtype=np.float64)
        y = np.zeros(self.ndof)
        for t in range(6):
            _, dofs, lam, mu = self._uncut(t)
            B = d.B_fe[t]
            sig = _iso_stress(np.broadcast_to(ebar, (len(lam), 6)), lam, mu)
            f = -d.tet_vol[t] * sig @ B
            y += np.bincount(dofs.ravel(), f.ravel(), minlength=self.ndof)
        if len(self.dofs_cut):
            f = -np.einsum("eki,k->ei", d.cut_S, ebar)
            y += np.bincount(self.dofs_cut.ravel(), f.ravel(), minlength=self.ndof)
        return y

    def residual(self, x, ebar):
        """r(u) = sum_e Lambda_e^T int B^T C (eps_bar + B u) (eq. resVector)."""
        return self.apply(x) - self.rhs(ebar)

    def average_stress(self, x, ebar):
        """<sigma> = |Y|^-1 sum_e int C (eps_bar + B u) (volume-weighted sum of element averages)."""
        d = self.d
        ebar = np.asarray(ebar, dtype=np.float64)
        s = np.zeros(6)
        for t in range(6):
            _, dofs, lam, mu = self._uncut(t)
            eps = ebar[None, :] + x[dofs] @ d.B_fe[t].T
            s += d.tet_vol[t] * _iso_stress(eps, lam, mu).sum(axis=0)
        if len(self.dofs_cut):
            s += np.einsum("eij,j->i", d.cut_Cbar, ebar)
            s += np.einsum("eij,ej->i", d.cut_S, x[self.dofs_cut])
        return s / d.volume

    def voxel_stress(self, x, ebar):
        """Average stress of every voxel (6 x N, Mandel), voxel volume 1."""
        d = self.d
        ebar = np.asarray(ebar, dtype=np.float64)
        out = np.zeros((d.N, 6))
        for t in range(6):
            m, dofs, lam, mu = self._uncut(t)
            eps = ebar[None, :] + x[dofs] @ d.B_fe[t].T
            out[np.nonzero(m)[0]] += d.tet_vol[t] * _iso_stress(eps, lam, mu)
        if len(self.dofs_cut):
            sc = np.einsum("eij,j->ei", d.cut_Cbar, ebar) + np.einsum("eij,ej->ei", d.cut_S, x[self.dofs_cut])
            np.add.at(out, d.cut_voxel, sc)
        return out.T.copy()

    # --------------------------------------------------------------- assembled matrix
    def assemble(self):
        """The scaled system matrix as scipy CSR (for small grids)."""
        d = self.d
        rows, cols, vals = [], [], []
        for t in range(6):
            _, dofs, lam, mu = self._uncut(t)
            B = d.B_fe[t]
            Kl = d.tet_vol[t] * (B.T @ np.outer(ONE, ONE) @ B)
            Km = d.tet_vol[t] * 2.0 * (B.T @ B)
            K = lam[:, None, None] * Kl[None] + mu[:, None, None] * Km[None]
            rows.append(np.repeat(dofs, 12, axis=1).ravel())
            cols.append(np.tile(dofs, (1, 12)).ravel())
            vals.append(K.ravel())
        if len(self.dofs_cut):
            dc = self.dofs_cut
            rows.append(np.repeat(dc, 24, axis=1).ravel())
            cols.append(np.tile(dc, (1, 24)).ravel())
            vals.append(d.cut_K.ravel())
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(self.ndof, self.ndof))
        return A.tocsr()
