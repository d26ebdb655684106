"""Selected outputs of H x and S x for cells too large to assemble densely.

Each output (G, i) is the same sum of matrix elements as a row of the dense
operator of ``operators.Problem`` (Sec. II.B.1), evaluated directly:

  (S x)(G,i) = sum_j S_z[i,j] x(G,j)
  (T x)(G,i) = 1/2 sum_j (D_z[i,j] + |k+G|^2 S_z[i,j]) x(G,j)
  (V x)(G,i) = sum_q w_q B_i(z_q) sum_G' Vt(G - G', z_q) sum_j B_j(z_q) x(G',j)
  (N x)(G,i) = sum_p E_p F_p(G) Z_p(i) sum_{G',j} conj(F_p(G') Z_p(j)) x(G',j)
  ultrasoft overlap: (S x)(G,i) gains the same sum with q_p in place of E_p

with Vt the grid-consistent transform of the sampled potential.  The potential
is sampled only on the z-planes that the requested rows touch (Gaussian wells
through the in-plane x z factorisation of operators.py, pinned against the
direct sum).
"""
from __future__ import annotations

import numpy as np

from .bspline import ZBasis
from .lattice import gset
from .operators import (gaussian_potential_on_grid_separable, potential_on_grid, projector_augmentation,
                        projector_factors, vtilde_grid)


class RowOracle:
    def __init__(self, desc, ik: int = 0, vfunc=None):
        self.desc = desc
        self.ik = ik
        self.zb = ZBasis(desc["breakpoints"], desc["order"], desc["nq"])
        self.m, self.kg = gset(desc, ik)
        self.ng = len(self.m)
        self.nb = self.zb.nb
        self.Sz = self.zb.overlap()
        self.Dz = self.zb.deriv_overlap()
        self.kg2 = np.sum(self.kg * self.kg, axis=1)
        self.F, self.Z, self.E = projector_factors(desc, ik, self.zb)
        self.Q = projector_augmentation(desc)
        self.vfunc = vfunc
        self._vt = {}

    def _vtilde(self, qs):
        need = [q for q in qs if q not in self._vt]
        if need:
            has_v = self.vfunc is not None or bool(self.desc["atoms"])
            if has_v:
                if self.vfunc is None:
                    vg = gaussian_potential_on_grid_separable(self.desc, self.zb.zq[need])
                else:
                    vg = potential_on_grid(self.desc, self.zb.zq[need], self.vfunc)
                vt = vtilde_grid(self.desc, vg)
            else:
                N1, N2 = self.desc["grid"]
                vt = np.zeros((len(need), N1, N2), dtype=np.complex128)
            for n, q in enumerate(need):
                self._vt[q] = vt[n]
        return [self._vt[q] for q in qs]

    def apply_rows(self, x: np.ndarray, rows):
        """x in library layout [band][i][G] (complex); rows = list of (i, g).

        Returns (Hx, Sx) of shape (nbands, len(rows)).
        """
        N1, N2 = self.desc["grid"]
        nbands = x.shape[0]
        rows = list(rows)
        Hx = np.zeros((nbands, len(rows)), dtype=np.complex128)
        Sx = np.zeros((nbands, len(rows)), dtype=np.complex128)
        B = self.zb.B
        wq = self.zb.wq
        # projections <beta_p | x_b> for all p, b
        if len(self.E):
            proj = np.einsum("pg,pi,big->pb", self.F.conj(), self.Z.conj(), x)
        psis = {}  # psi(G', z_q) of every band, per touched plane
        for r, (i, g) in enumerate(rows):
            Sx[:, r] = x[:, :, g] @ self.Sz[i, :]
            Hx[:, r] = 0.5 * (x[:, :, g] @ (self.Dz[i, :] + self.kg2[g] * self.Sz[i, :]))
            qs = [int(q) for q in np.nonzero(B[:, i])[0]]
            vts = self._vtilde(qs)
            d1 = (self.m[g, 0] - self.m[:, 0]) % N1
            d2 = (self.m[g, 1] - self.m[:, 1]) % N2
            for q, vt in zip(qs, vts):
                if q not in psis:
                    psis[q] = np.einsum("j,bjG->bG", B[q, :], x)  # psi(G', z_q)
                Hx[:, r] += wq[q] * B[q, i] * (psis[q] @ vt[d1, d2])
            if len(self.E):
                coef = self.E * self.F[:, g] * self.Z[:, i]
                Hx[:, r] += coef @ proj
                if np.any(self.Q != 0):
                    Sx[:, r] += (self.Q * self.F[:, g] * self.Z[:, i]) @ proj
        return Hx, Sx
