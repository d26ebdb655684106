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
            self.Vpl = np.ascontiguousarray(vt[:, d1, d2])  # (Nq, NG, NG): Vt(G - G', z_q)
        else:
            self.Vpl = None
        self.F, self.Z, self.E = projector_factors(desc, ik, self.zb)

    # vectors as [nvec][G][i]
    def apply_s(self, x: np.ndarray) -> np.ndarray:
        return x @ self.Sz

    def apply(self, x: np.ndarray):
        """(H x, S x) for x of shape (nvec, NG, Nb)."""
        nv = x.shape[0]
        Sx = x @ self.Sz
        Hx = 0.5 * (x @ self.Dz) + 0.5 * self.kg2[None, :, None] * Sx
        if self.Vpl is not None:
            # psi(G', z_q) = sum_j B_j(z_q) x(G', j), as (Nq, NG, nvec)
            psi = (x.reshape(nv * self.ng, self.nb) @ self.zb.B.T).reshape(nv, self.ng, -1)
            psi = np.ascontiguousarray(np.transpose(psi, (2, 1, 0)))
            vpsi = np.matmul(self.Vpl, psi)                      # per plane: Vt(G - G') psi(G')
            wb = self.zb.B * self.zb.wq[:, None]                 # (Nq, Nb)
            out = np.transpose(vpsi, (2, 1, 0)).reshape(nv * self.ng, -1) @ wb
            Hx = Hx + out.reshape(nv, self.ng, self.nb)
        if len(self.E):
            FZ = (self.F[:, :, None] * self.Z[:, None, :]).reshape(len(self.E), -1)  # <G,i|beta_p>
            proj = FZ.conj() @ x.reshape(nv, -1).T               # (Np, nvec)
            Hx = Hx + ((FZ.T * self.E[None, :]) @ proj).T.reshape(nv, self.ng, self.nb)
        return Hx, Sx

    def _linop(self, which: str):
        n, ng, nb = self.n, self.ng, self.nb

        def mv(v):
            v2 = np.asarray(v).reshape(n, -1)
            x = v2.T.reshape(-1, ng, nb)
            out = self.apply(x)[0] if which == "H" else self.apply_s(x)
            return out.reshape(x.shape[0], n).T

        return scipy.sparse.linalg.LinearOperator((n, n), matvec=mv, matmat=mv, dtype=np.complex128)

    def _precond(self, sigma: float = 1.0):
        # (T + sigma S)^{-1} per G, as explicit inverses applied in one batched product
        inv = np.empty((self.ng, self.nb, self.nb))
        for g in range(self.ng):
            A = 0.5 * self.Dz + (0.5 * self.kg2[g] + sigma) * self.Sz
            inv[g] = scipy.linalg.cho_solve(scipy.linalg.cho_factor(A), np.eye(self.nb))
        ng, nb, n = self.ng, self.nb, self.n

        def mv(v):
            v2 = np.asarray(v).reshape(n, -1)
            x = v2.T.reshape(-1, ng, nb)
            out = np.matmul(inv[None, :, :, :], x[:, :, :, None])[..., 0]
            return out.reshape(x.shape[0], n).T

        return scipy.sparse.linalg.LinearOperator((n, n), matvec=mv, matmat=mv, dtype=np.complex128)

    def lowest(self, nev: int, extra: int = 8, tol: float = 1e-9, maxiter: int = 200, seed: int = 0):
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
