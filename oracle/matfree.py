"""Matrix-free FP64 application of S and H for cells too large for dense
assembly, and their lowest eigenpairs by a library block eigensolver.

H x is the same sum of matrix elements as the dense operator of
``operators.Problem`` (Sec. II.B.1), regrouped without forming H:
  kinetic / overlap: banded products with S_z, D_z per G;
  local potential: psi(G', z_q) = sum_j B_j(z_q) x(G', j), then on every Gauss
    plane the in-plane sum sum_G' Vt(G - G', z_q) psi(G', z_q), then
    sum_q w_q B_i(z_q) (...).  Two ways of taking the in-plane sum:
      ``local="dense"``: the explicit pair table Vt(G - G', z_q) (index
        differences reduced modulo the grid), one dense product per plane;
      ``local="fft"``: the same circular convolution through the grid,
        N1 N2 * ifft2 of the scattered psi, times V(rho_j, z_q), then
        fft2 / (N1 N2), gathered back on the G set (numpy's FFT is the
        library step; the identity is the convolution theorem of the DFT);
  nonlocal: sum_p E_p F_p(G) Z_p(i) <beta_p|x>, with <beta_p|x> =
    sum_G conj(F_p(G)) sum_i Z_p(i) x(G, i);
  ultrasoft overlap (Sec. II.B.2): S x gains sum_p q_p F_p(G) Z_p(i) <beta_p|x>.
The lowest eigenpairs come from scipy's LOBPCG (a library routine) for the
generalized problem H c = eps S c, with the per-G kinetic solve
(T + sigma S)^{-1} as preconditioner, to a stated residual.

Pins (CPU tests): both local modes against the dense H and S of
``operators.Problem`` on the tiny cell and two small cells with projectors
(1e-13 relative), and ``lowest`` against LAPACK's eigenvalues of the dense
problem on a small cell.
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg

from .bspline import ZBasis
from .lattice import gset
from .operators import potential_on_grid, projector_augmentation, projector_factors, vtilde_grid


class MatFree:
    def __init__(self, desc, ik: int = 0, vfunc=None, local: str = "dense", vgrid=None, workers: int = -1):
        """local: "dense" or "fft" (see the module docstring).  vgrid: optional
        precomputed V(rho_j, z_q) of shape (Nq, N1, N2) (the sampled potential
        at this description's Gauss points)."""
        if local not in ("dense", "fft"):
            raise ValueError(local)
        self.desc = desc
        self.local = local
        self.workers = workers
        self.zb = ZBasis(desc["breakpoints"], desc["order"], desc["nq"])
        self.m, self.kg = gset(desc, ik)
        self.ng, self.nb = len(self.m), self.zb.nb
        self.n = self.ng * self.nb
        self.Sz = self.zb.overlap()
        self.Dz = self.zb.deriv_overlap()
        self.kg2 = np.sum(self.kg * self.kg, axis=1)
        self.N1, self.N2 = desc["grid"]
        self.j1 = self.m[:, 0] % self.N1
        self.j2 = self.m[:, 1] % self.N2
        self.has_v = vfunc is not None or bool(desc["atoms"]) or vgrid is not None
        self.Vpl = None
        self.Vgrid = None
        if self.has_v:
            vg = vgrid if vgrid is not None else potential_on_grid(desc, self.zb.zq, vfunc)
            if local == "dense":
                vt = vtilde_grid(desc, vg)
                d1 = (self.m[:, None, 0] - self.m[None, :, 0]) % self.N1
                d2 = (self.m[:, None, 1] - self.m[None, :, 1]) % self.N2
                self.Vpl = np.ascontiguousarray(vt[:, d1, d2])  # (Nq, NG, NG): Vt(G - G', z_q)
            else:
                self.Vgrid = np.ascontiguousarray(vg, dtype=np.float64)
        # sparse B(z_q, j) and w_q B(z_q, i): kappa non-zeros per Gauss point
        self.Bsp = scipy.sparse.csr_matrix(self.zb.B)
        self.WBsp = scipy.sparse.csr_matrix(self.zb.B * self.zb.wq[:, None])
        self.F, self.Z, self.E = projector_factors(desc, ik, self.zb)
        self.Q = projector_augmentation(desc)
        self.uspp = bool(len(self.Q)) and bool(np.any(self.Q != 0))

    def _expand(self, x: np.ndarray, coef: np.ndarray) -> np.ndarray:
        """sum_p coef_p |beta_p><beta_p|x> for x of shape (nvec, NG, Nb)."""
        xz = x @ self.Z.T                                   # (nvec, NG, Np)
        proj = np.einsum("pg,bgp->pb", self.F.conj(), xz)   # <beta_p|x_b>
        fz = np.einsum("pg,pb->bgp", self.F, coef[:, None] * proj)
        return fz @ self.Z

    # vectors as [nvec][G][i]
    def apply_s(self, x: np.ndarray) -> np.ndarray:
        Sx = x @ self.Sz
        if self.uspp:
            Sx = Sx + self._expand(x, self.Q)
        return Sx

    def _local_dense(self, psi):
        # psi (Nq, NG, nvec) -> per plane Vt(G - G') psi(G')
        return np.matmul(self.Vpl, psi)

    def _local_fft(self, psi):
        # psi (Nq, NG, nvec) -> the same circular convolution through the grid
        # grids are held as (N1, N2, planes x vectors) so that scatter and gather move
        # whole rows of the trailing batch axis
        nq, ng, nv = psi.shape
        N1, N2 = self.N1, self.N2
        flat = self.j1 * N2 + self.j2
        out = np.empty_like(psi)
        step = max(1, (1 << 22) // (N1 * N2 * max(nv, 1)))  # planes per chunk (~64 MB grids)
        for q0 in range(0, nq, step):
            q1 = min(nq, q0 + step)
            c = q1 - q0
            grid = np.zeros((N1 * N2, c, nv), dtype=np.complex128)
            grid[flat] = np.transpose(psi[q0:q1], (1, 0, 2))
            grid = grid.reshape(N1, N2, c, nv)
            real = scipy.fft.ifft2(grid, axes=(0, 1), workers=self.workers) * (N1 * N2)
            real *= np.transpose(self.Vgrid[q0:q1], (1, 2, 0))[:, :, :, None]
            back = scipy.fft.fft2(real, axes=(0, 1), workers=self.workers) / (N1 * N2)
            out[q0:q1] = np.transpose(back.reshape(N1 * N2, c, nv)[flat], (1, 0, 2))
        return out

    def apply(self, x: np.ndarray):
        """(H x, S x) for x of shape (nvec, NG, Nb)."""
        nv = x.shape[0]
        Sz_x = x @ self.Sz
        Hx = 0.5 * (x @ self.Dz) + 0.5 * self.kg2[None, :, None] * Sz_x
        Sx = Sz_x + self._expand(x, self.Q) if self.uspp else Sz_x
        if self.has_v:
            # psi(G', z_q) = sum_j B_j(z_q) x(G', j), as (Nq, NG, nvec)
            xt = np.ascontiguousarray(np.transpose(x, (2, 1, 0))).reshape(self.nb, -1)  # (Nb, NG*nvec)
            psi = np.asarray(self.Bsp @ xt).reshape(-1, self.ng, nv)
            vpsi = self._local_dense(psi) if self.local == "dense" else self._local_fft(psi)
            out = np.asarray(self.WBsp.T @ vpsi.reshape(vpsi.shape[0], -1))  # (Nb, NG*nvec)
            Hx = Hx + np.transpose(out.reshape(self.nb, self.ng, nv), (2, 1, 0))
        if len(self.E):
            # sum_p E_p |beta_p><beta_p|x>, <beta_p|x_b> = sum_G conj(F_p(G)) sum_i Z_p(i) x_b(G, i)
            Hx = Hx + self._expand(x, self.E)
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
        # (T + sigma S)^{-1} per G, by the banded Cholesky factor of each G block
        nb, ng, n = self.nb, self.ng, self.n
        bw = 3
        facs = []
        for g in range(ng):
            A = 0.5 * self.Dz + (0.5 * self.kg2[g] + sigma) * self.Sz
            ab = np.zeros((bw + 1, nb))
            for d in range(bw + 1):
                ab[bw - d, d:] = np.diagonal(A, d)
            facs.append(scipy.linalg.cholesky_banded(ab))

        def mv(v):
            v2 = np.asarray(v).reshape(n, -1)
            x = v2.T.reshape(-1, ng, nb)
            out = np.empty_like(x)
            for g in range(ng):
                out[:, g, :] = scipy.linalg.cho_solve_banded((facs[g], False), x[:, g, :].T).T
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
