"""Interpolated dense-mesh BSE Hamiltonian and its on-the-fly product.

Eq. (bse1) (TDA): H = (eps_ck - eps_vk) delta + K.
Eq. (interp1): the interpolated kernel on the dense mesh,
  K^i[(v c k), (v' c' k')] =
    sum_{k~ in N(k)} f(k,k~) sum_{n1 n2} d_{vk}^{n1 k~} conj(d_{ck}^{n2 k~})
    sum_{k~' in N(k')} f(k',k~') sum_{n3 n4} conj(d_{v'k'}^{n3 k~'}) d_{c'k'}^{n4 k~'}
    K_c[(n1 n2 k~), (n3 n4 k~')].
Eqs. (matmul1)-(matmul3): the same product applied to a vector p in three
steps: restrict p to per-(cell, corner) coarse vectors q, contract with K_c
to get r, prolong r back onto the dense mesh.

Transition order on the dense mesh: t = (kd * nv + v) * nc + c.  Vectors are
[n_rhs, N] (or [n_rhs, N_k, nv, nc] internally).
"""

from __future__ import annotations

import numpy as np

from .grids import neighbour_table


def transition_energies(eps_dense: np.ndarray, nv: int, nc: int) -> np.ndarray:
    """Diagonal of Eq. (bse1): eps_{c k} - eps_{v k} in transition order -> [N]."""
    de = eps_dense[:, nv:nv + nc][:, None, :] - eps_dense[:, :nv][:, :, None]
    return de.reshape(-1)


class InterpOperator:
    """H^i = diag(delta) + K^i on the dense mesh, applied without storing K^i.

    Dv, Dc  overlaps from ``overlaps`` ([N_k, 8, nv, nv], [N_k, 8, nc, nc])
    f       prefactors [n_div^3, 8] (trilinear or one-neighbour)
    Kc      coarse kernel [N_coarse, N_coarse]
    delta   transition energies [N]
    """

    def __init__(self, Dv, Dc, f, Kc, delta, n_c, n_div, nv, nc):
        self.Dv, self.Dc, self.f, self.Kc = Dv, Dc, f, Kc
        self.delta = np.asarray(delta, dtype=np.float64)
        self.n_c, self.n_div, self.nv, self.nc = n_c, n_div, nv, nc
        self.ndiv3 = n_div ** 3
        self.nk = Dv.shape[0]
        self.nkc = n_c ** 3
        self.N = self.nk * nv * nc
        self.Nc = self.nkc * nv * nc
        self.nbr = neighbour_table(n_c)
        kd = np.arange(self.nk)
        self.cell = kd // self.ndiv3
        self.sub = kd % self.ndiv3
        self.fk = f[self.sub]                               # [N_k, 8]
        self.corner_k = self.nbr[self.cell]                 # [N_k, 8] coarse index

    # ---- Eq. (matmul1): per (cell, corner) coarse vectors ----------------------
    def restrict_partials(self, x):
        """q^{z}_{cell}[n3, n4] = sum_{k in S(cell)} f(k, z) sum_{v'c'}
        conj(d_{v'k}^{n3 k~z}) d_{c'k}^{n4 k~z} p_{v'c'k}  ->  [n_rhs, cells, 8, nv, nc]."""
        x = x.reshape(-1, self.nk, self.nv, self.nc)
        # X[r, k, z] = Dv[k, z]^H  x[r, k]  Dc[k, z]
        X = np.matmul(np.matmul(np.conj(self.Dv).swapaxes(-1, -2)[None], x[:, :, None]),
                      self.Dc[None])
        X = X * self.fk[None, :, :, None, None]
        return X.reshape(x.shape[0], self.nkc, self.ndiv3, 8, self.nv, self.nc).sum(axis=2)

    def restrict(self, x):
        """Collapse the partials onto coarse points: qbar [n_rhs, N_coarse].

        Every (cell, corner) contribution is added to the coarse point
        k~ = corner z of that cell; this regroups the sums over k~'' and uvw
        of Eq. (matmul2) ahead of the product with K_c.
        """
        q = self.restrict_partials(x)
        out = np.zeros((q.shape[0], self.nkc, self.nv, self.nc), dtype=np.complex128)
        for z in range(8):
            np.add.at(out, (slice(None), self.nbr[:, z]), q[:, :, z])
        return out.reshape(q.shape[0], -1)

    # ---- Eq. (matmul3) ---------------------------------------------------------
    def prolong(self, r):
        """s_{vck} = sum_z f(k, z) sum_{n1 n2} d_{vk}^{n1 k~z} conj(d_{ck}^{n2 k~z}) r_{n1 n2 k~z}."""
        r = r.reshape(-1, self.nkc, self.nv, self.nc)
        rk = r[:, self.corner_k]                             # [n_rhs, N_k, 8, nv, nc]
        # s[r, k] = sum_z f[k, z] Dv[k, z]  r[r, k~z]  Dc[k, z]^H
        t = np.matmul(np.matmul(self.Dv[None], rk), np.conj(self.Dc).swapaxes(-1, -2)[None])
        s = np.sum(t * self.fk[None, :, :, None, None], axis=2)
        return s.reshape(r.shape[0], -1)

    def coarse_product(self, qbar):
        """Eq. (matmul2) with the corner sum collapsed: r = K_c qbar."""
        return (self.Kc @ qbar.T).T

    def apply_kernel(self, x):
        x = np.atleast_2d(x)
        return self.prolong(self.coarse_product(self.restrict(x)))

    def apply(self, x):
        """H^i x = delta * x + K^i x (fast three-step form)."""
        x = np.atleast_2d(x)
        return self.delta[None, :] * x + self.apply_kernel(x)

    def apply_literal(self, x):
        """H^i x with Eq. (matmul2) evaluated as printed: one coarse product per
        corner uvw on the uncollapsed partials q^{uvw}, summed afterwards."""
        x = np.atleast_2d(x)
        q = self.restrict_partials(x)                        # [r, cells, 8, nv, nc]
        Kb = self.Kc.reshape(self.Nc, self.nkc, self.nv * self.nc)
        r = np.zeros((x.shape[0], self.Nc), dtype=np.complex128)
        for z in range(8):
            cols = Kb[:, self.nbr[:, z], :].reshape(self.Nc, -1)     # K[:, (n3 n4 k~''^z)]
            r += (cols @ q[:, :, z].reshape(x.shape[0], -1).T).T
        return self.delta[None, :] * x + self.prolong(r)

    # ---- Eq. (interp1): explicit matrices (small meshes only) --------------------
    def expansion_matrix(self):
        """B[(v c k), (n1 n2 k~)] = sum_{z: k~z = k~} f(k,z) d_{vk}^{n1 k~z} conj(d_{ck}^{n2 k~z}).

        Built entry block by entry block, so that K^i = B K_c B^H.
        """
        nv, nc = self.nv, self.nc
        npair = nv * nc
        B = np.zeros((self.N, self.Nc), dtype=np.complex128)
        for k in range(self.nk):
            for z in range(8):
                kc = self.corner_k[k, z]
                # blk[v, c, n1, n2] = f d_v^{n1} conj(d_c^{n2})
                blk = (self.fk[k, z] * self.Dv[k, z][:, None, :, None]
                       * np.conj(self.Dc[k, z])[None, :, None, :])
                B[k * npair:(k + 1) * npair, kc * npair:(kc + 1) * npair] += blk.reshape(npair, npair)
        return B

    def explicit_kernel(self):
        B = self.expansion_matrix()
        return B @ self.Kc @ B.conj().T

    def explicit_hamiltonian(self):
        return np.diag(self.delta).astype(np.complex128) + self.explicit_kernel()
