"""Matrix-free FP64 application of S and H for cells too large for dense
assembly, and their lowest eigenpairs by a library block eigensolver.

H x is the same sum of matrix elements as the dense operator of
``operators.Problem`` (Sec. II.B.1), regrouped without forming H:
  kinetic / overlap: banded products with S_z, D_z per G;
  local potential: psi(G', z_q) = sum_j B_j(z_q) x(G', j), then for every Gauss
    plane the dense in-plane sum sum_G' Vt(G - G', z_q) psi(G', z_q), then
    sum_q w_q B_i(z_q) (...);
  nonlocal: sum_p E_p F_p(G) Z_p(i) <beta_p|x>.
The lowest eigenpairs come from scipy's LOBPCG (a library routine) for the
generalized problem H c = eps S c, with the per-G kinetic solve as
preconditioner; convergence is to a stated residual, and the result is checked
against the dense oracle on small cells by the tests.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse.linalg

from .bspline import ZBasis
from .lattice import gset
from .operators import potential_on_grid, projector_factors, vtilde_grid


class MatFree:
    def __init__(self, desc, ik: int = 0, vfunc=None):
        self.desc = desc
        self.zb = ZBasis(desc["breakpoints"], desc["order"], desc["nq"])
        self.m, self.kg = gset(desc, ik)
        self.ng, self.nb = len(self.m), self.zb.nb
        self.n = self.ng * self.nb
        self.Sz = self.zb.overlap()
        self.Dz = self.zb.deriv_overlap()
        self.kg2 = np.sum(self.kg * self.kg, axis=1)
        N1, N2 = desc["grid"]
        has_v = vfunc is not None or bool(desc["atoms"])
        if has_v:
            vt = vtilde_grid(desc, potential_on_grid(desc, self.zb.zq, vfunc))
            d1 = (self.m[:, None, 0] - self.m[None, :, 0]) % N1
            d2 = (self.m[:, None, 1] - self.m[None, :, 1]) % N2
            self.Vpl = vt[:, d1, d2]  # (Nq, NG, NG): Vt(G - G', z_q)
        else:
            self.Vpl = None
        self.F, self.Z, self.E = projector_factors(desc, ik, self.zb)

    # vectors as [nvec][G][i]
    def apply(self, x: np.ndarray):
        """(H x, S x) for x of shape (nvec, NG, Nb)."""
        Sx = x @ self.Sz
        Hx = 0.5 * (x @ self.Dz) + 0.5 * self.kg2[None, :, None] * Sx
        if self.Vpl is not None:
            psi = np.einsum("qj,vgj->qgv", self.zb.B, x)          # (Nq, NG, nvec)
            vpsi = np.matmul(self.Vpl, psi)                      # per plane: Vt @ psi
            Hx = Hx + np.einsum("qi,qgv->vgi", self.zb.B * self.zb.wq[:, None], vpsi)
        if len(self.E):
            proj = np.einsum("pg,pi,vgi->pv", self.F.conj(), self.Z, x)
            Hx = Hx + np.einsum("p,pg,pi,pv->vgi", self.E, self.F, self.Z, proj)
        return Hx, Sx

    def _linop(self, which: str):
        n, ng, nb = self.n, self.ng, self.nb

        def mv(v):
            v2 = np.asarray(v).reshape(n, -1)
            x = v2.T.reshape(-1, ng, nb)
            h, s = self.apply(x)
            out = h if which == "H" else s
            return out.reshape(x.shape[0], n).T

        return scipy.sparse.linalg.LinearOperator((n, n), matvec=mv, matmat=mv, dtype=np.complex128)

    def _precond(self, sigma: float = 1.0):
        facs = []
        for g in range(self.ng):
            A = 0.5 * self.Dz + (0.5 * self.kg2[g] + sigma) * self.Sz
            facs.append(scipy.linalg.cho_factor(A))
        ng, nb, n = self.ng, self.nb, self.n

        def mv(v):
            v2 = np.asarray(v).reshape(n, -1)
            x = v2.T.reshape(-1, ng, nb)
            out = np.empty_like(x)
            for g in range(ng):
                out[:, g, :] = scipy.linalg.cho_solve(facs[g], x[:, g, :].T).T
            return out.reshape(x.shape[0], n).T

        return scipy.sparse.linalg.LinearOperator((n, n), matvec=mv, matmat=mv, dtype=np.complex128)

    def lowest(self, nev: int, extra: int = 8, tol: float = 1e-10, maxiter: int = 2000, seed: int = 0):
        """Lowest nev eigenpairs: (eps, C [nev][NG][Nb] S-orthonormal, residual norms)."""
        rng = np.random.default_rng(seed)
        k = nev + extra
        X0 = rng.standard_normal((self.n, k)) + 1j * rng.standard_normal((self.n, k))
        w, V = scipy.sparse.linalg.lobpcg(self._linop("H"), X0, B=self._linop("S"), M=self._precond(),
                                          tol=tol, maxiter=maxiter, largest=False)
        order = np.argsort(w)[:nev]
        w, V = w[order], V[:, order]
        C = V.T.reshape(nev, self.ng, self.nb)
        h, s = self.apply(C)
        nrm = np.sqrt(np.real(np.sum(C.conj() * s, axis=(1, 2))))
        C = C / nrm[:, None, None]
        h, s = self.apply(C)
        eps = np.real(np.sum(C.conj() * h, axis=(1, 2)))
        r = np.linalg.norm((h - eps[:, None, None] * s).reshape(nev, -1), axis=1)
        return eps, C, r
