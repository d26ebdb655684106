"""1D-periodic form of the mixed basis: B-splines along the two non-periodic
directions x and z, plane waves along the periodic axis y (the extension stated at
the end of Sec. II.B.2, used for the ribbon of Sec. III.C).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Basis:  chi_{G,i,j}(x, y, z) = L^{-1/2} e^{i(k+G) y} B_i(x) B_j(z),
        G = 2 pi m / L,  1/2 (k+G)^2 <= E_cut,  k = f 2 pi / L.
Both spline sets are the hard-wall sets of ``bspline.ZBasis`` (eqs. 1-3), each with
its own breakpoints and the same order and Gauss points per interval.
Index of a basis function in the oracle: (G * N_x + i) * N_z + j.

Matrix elements (the Sec. II.B.1 elements with one more spline direction):
  S = I_G (x) S_x (x) S_z
  T = 1/2 [D_x (x) S_z + S_x (x) D_z + (k+G)^2 S_x (x) S_z]          per G
  V_loc: sum_{q,p} w_q w_p B_i(x_q) B_i'(x_q) B_j(z_p) B_j'(z_p) Vt(m - m'; x_q, z_p)
     with the grid transform along y, Vt(d; x, z) = 1/N_y sum_n V(x, y_n, z)
     e^{-2 pi i d n / N_y}, y_n = n L / N_y (the index difference taken modulo N_y:
     the circular convolution an N_y-point FFT realises), or its closed form for the
     Gaussian wells (``vmode="analytic"``); the two differ only by aliasing.
  V_NL = sum_p E_p |beta_p><beta_p|, the s and real p_x, p_y, p_z projectors of
     ``operators`` with Gaussian radial parts; the overlap with a basis function
     factorises into three one-dimensional integrals,
        <G,i,j|beta_p> = F_p(G) X_p(i) Z_p(j),
        F_p(G) = C L^{-1/2} e^{-i q Y} sqrt(pi/a) e^{-q^2/4a} (times -i q / 2a for p_y),
        X_p(i) = int B_i(x) e^{-a (x-X)^2} dx (times (x-X) for p_x), Z_p likewise,
     q = k + G; the y integral runs over the whole line (the images of the atom
     along y tile it).
The local potential is the Gaussian part of the species (Gaussians summed over the
images of each atom along y).

Pins (tests/test_oracle_wire.py): separable potentials (none; V(y) = V0 cos(2 pi y/L);
V(x); V(z)) against sums of one-dimensional spectra; the grid and analytic local
transforms; the projector factors against direct quadrature in three dimensions;
the matrix-free and row forms against the dense matrices; hard-wall convergence of
the particle in a box.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from .bspline import ZBasis
from .operators import PROJ_NAMES, projector_norms


def basis_x(desc) -> ZBasis:
    return ZBasis(desc["breakpoints_x"], desc["order"], desc["nq"])


def basis_z(desc) -> ZBasis:
    return ZBasis(desc["breakpoints_z"], desc["order"], desc["nq"])


def gset(desc, ik: int):
    """Integers m (ascending) and k + G of the plane-wave set of k-point ik."""
    L = float(desc["period"])
    k = 2.0 * math.pi * float(desc["kpts"][ik]) / L
    ecut = float(desc["ecut"])
    r = math.sqrt(2.0 * ecut)
    n = int(math.ceil(r * L / (2.0 * math.pi))) + 2
    ms = [m for m in range(-n, n + 1) if 0.5 * (k + 2.0 * math.pi * m / L) ** 2 <= ecut]
    m = np.array(ms, dtype=np.int64)
    return m, k + 2.0 * math.pi * m / L


def image_range(desc, width: float) -> int:
    """Images along y so that every image within sqrt(45) w of the cell is summed."""
    return int(math.ceil(math.sqrt(45.0) * width / float(desc["period"]))) + 1


def potential_grid(desc, xq, zq, vfunc=None) -> np.ndarray:
    """Real V(x_q, y_n, z_p) on the Gauss points and the y grid, shape (Nxq, Nzq, Ny)."""
    L = float(desc["period"])
    ny = int(desc["ny"])
    x = np.asarray(xq, float)[:, None, None]
    z = np.asarray(zq, float)[None, :, None]
    y = (np.arange(ny) * L / ny)[None, None, :]
    if vfunc is not None:
        return np.broadcast_to(vfunc(x, y, z), (x.shape[0], z.shape[1], ny)).astype(np.float64)
    V = np.zeros((x.shape[0], z.shape[1], ny))
    for at in desc["atoms"]:
        sp = desc["species"][at["species"]]
        X, Y, Z = at["pos"]
        for A, w in sp["gauss"]:
            nimg = image_range(desc, w)
            fy = np.zeros(ny)
            for n in range(-nimg, nimg + 1):
                fy = fy + np.exp(-((y[0, 0] - Y - n * L) ** 2) / (w * w))
            V = V + A * np.exp(-((x - X) ** 2) / (w * w)) * np.exp(-((z - Z) ** 2) / (w * w)) * fy[None, None, :]
    return V


def vtilde_grid(V: np.ndarray) -> np.ndarray:
    """Vt[q, p, d] = 1/N_y sum_n V[q, p, n] e^{-2 pi i d n / N_y} (explicit DFT matrix)."""
    ny = V.shape[-1]
    n = np.arange(ny)
    F = np.exp(-2j * math.pi * np.outer(n, n) / ny)
    return (V.astype(np.complex128) @ F.T) / ny


def vtilde_analytic(desc, xq, zq, d: np.ndarray) -> np.ndarray:
    """Closed-form y transform of the Gaussian wells for integer differences d:
    (1/L) int dy e^{-i g y} A e^{-(y-Y)^2/w^2} = (A/L) sqrt(pi) w e^{-g^2 w^2/4} e^{-i g Y},
    g = 2 pi d / L, times the x and z Gaussians.  Shape (Nxq, Nzq, len(d))."""
    L = float(desc["period"])
    g = 2.0 * math.pi * np.asarray(d, float) / L
    x = np.asarray(xq, float)[:, None, None]
    z = np.asarray(zq, float)[None, :, None]
    out = np.zeros((x.shape[0], z.shape[1], len(g)), dtype=np.complex128)
    for at in desc["atoms"]:
        sp = desc["species"][at["species"]]
        X, Y, Z = at["pos"]
        for A, w in sp["gauss"]:
            fy = (A / L) * math.sqrt(math.pi) * w * np.exp(-(g * w) ** 2 / 4.0) * np.exp(-1j * g * Y)
            out += np.exp(-((x - X) ** 2 + (z - Z) ** 2) / (w * w)) * fy[None, None, :]
    return out


def projector_factors(desc, ik: int, xb: ZBasis, zb: ZBasis):
    """(F (Np, NG) complex, X (Np, Nx), Z (Np, Nz), E (Np,)) with
    <G,i,j|beta_p> = F[p, G] X[p, i] Z[p, j]."""
    L = float(desc["period"])
    _, q = gset(desc, ik)
    Fs, Xs, Zs, Es = [], [], [], []
    for at in desc["atoms"]:
        sp = desc["species"][at["species"]]
        if not sp.get("nonlocal", False):
            continue
        X0, Y0, Z0 = at["pos"]
        cs, cp = projector_norms(sp["alpha_s"], sp["alpha_p"])
        dx = xb.zq - X0
        dz = zb.zq - Z0
        for kind in PROJ_NAMES:
            a = sp["alpha_s"] if kind == "s" else sp["alpha_p"]
            c = cs if kind == "s" else cp
            fy = c / math.sqrt(L) * np.exp(-1j * q * Y0) * math.sqrt(math.pi / a) * np.exp(-q * q / (4.0 * a))
            if kind == "py":
                fy = fy * (-1j * q / (2.0 * a))
            fx = np.exp(-a * dx * dx) * (dx if kind == "px" else 1.0)
            fz = np.exp(-a * dz * dz) * (dz if kind == "pz" else 1.0)
            Fs.append(fy)
            Xs.append(xb.weighted(fx))
            Zs.append(zb.weighted(fz))
            Es.append(sp["E_s"] if kind == "s" else sp["E_p"])
    if not Fs:
        return (np.zeros((0, len(q)), dtype=np.complex128), np.zeros((0, xb.nb)), np.zeros((0, zb.nb)), np.zeros(0))
    return np.array(Fs), np.array(Xs), np.array(Zs), np.array(Es, dtype=np.float64)


class WireProblem:
    """Dense S and H of one k-point of the 1D-periodic form."""

    def __init__(self, desc, ik: int = 0, vmode: str = "grid", vfunc=None, with_local: bool = True,
                 with_nonlocal: bool = True):
        self.desc = desc
        self.ik = ik
        self.xb, self.zb = basis_x(desc), basis_z(desc)
        self.m, self.kg = gset(desc, ik)
        self.ng, self.nx, self.nz = len(self.m), self.xb.nb, self.zb.nb
        self.n = self.ng * self.nx * self.nz
        self.Sx, self.Dx = self.xb.overlap(), self.xb.deriv_overlap()
        self.Sz, self.Dz = self.zb.overlap(), self.zb.deriv_overlap()
        self.vmode, self.vfunc = vmode, vfunc
        self.with_local, self.with_nonlocal = with_local, with_nonlocal

    def overlap(self) -> np.ndarray:
        return np.kron(np.eye(self.ng), np.kron(self.Sx, self.Sz)).astype(np.complex128)

    def kinetic(self) -> np.ndarray:
        a = 0.5 * (np.kron(self.Dx, self.Sz) + np.kron(self.Sx, self.Dz))
        b = np.kron(self.Sx, self.Sz)
        T = np.zeros((self.n, self.n), dtype=np.complex128)
        blk = self.nx * self.nz
        for g in range(self.ng):
            s = slice(g * blk, (g + 1) * blk)
            T[s, s] = a + 0.5 * self.kg[g] ** 2 * b
        return T

    def vt_pairs(self) -> np.ndarray:
        """Vt(m_G - m_G'; x_q, z_p) for every pair, shape (NG, NG, Nxq, Nzq)."""
        dm = self.m[:, None] - self.m[None, :]
        if self.vmode == "grid":
            vt = vtilde_grid(potential_grid(self.desc, self.xb.zq, self.zb.zq, self.vfunc))
            return np.transpose(vt[:, :, dm % int(self.desc["ny"])], (2, 3, 0, 1))
        if self.vmode == "analytic":
            d = np.unique(dm)
            vt = vtilde_analytic(self.desc, self.xb.zq, self.zb.zq, d)
            return np.transpose(vt[:, :, np.searchsorted(d, dm)], (2, 3, 0, 1))
        raise ValueError(self.vmode)

    def local(self) -> np.ndarray:
        xb, zb = self.xb, self.zb
        Wx = (xb.B[:, :, None] * xb.B[:, None, :]) * xb.wq[:, None, None]  # (Nxq, Nx, Nx)
        Wz = (zb.B[:, :, None] * zb.B[:, None, :]) * zb.wq[:, None, None]  # (Nzq, Nz, Nz)
        vt = self.vt_pairs()
        M = np.einsum("abqp,qik,pjl->aijbkl", vt, Wx, Wz, optimize=True)
        return M.reshape(self.n, self.n)

    def projectors(self):
        F, X, Z, E = projector_factors(self.desc, self.ik, self.xb, self.zb)
        beta = F[:, :, None, None] * X[:, None, :, None] * Z[:, None, None, :]
        return beta.reshape(len(E), self.n), E

    def nonlocal_(self) -> np.ndarray:
        beta, E = self.projectors()
        return (beta.T * E[None, :]) @ beta.conj()

    def hamiltonian(self) -> np.ndarray:
        H = self.kinetic()
        if self.with_local and (self.vfunc is not None or self.desc["atoms"]):
            H = H + self.local()
        if self.with_nonlocal:
            H = H + self.nonlocal_()
        return H


def lowest(desc, ik: int, nev: int, **kw):
    """Lowest nev eigenvalues and S-orthonormal vectors of the dense problem (LAPACK)."""
    pr = WireProblem(desc, ik, **kw)
    w, C = scipy.linalg.eigh(pr.hamiltonian(), pr.overlap(), subset_by_index=[0, nev - 1])
    return w, C


class WireMatFree:
    """H x and S x without forming H: the same sums as ``WireProblem`` regrouped.
    Local part: psi(x_q, z_p, G') = sum_{i,j} B_i(x_q) B_j(z_p) x(G', i, j), then on
    every (x_q, z_p) the circular convolution along y through numpy's FFT (the
    convolution theorem of the DFT), N_y ifft of the scattered psi times V(x_q, y_n,
    z_p), fft / N_y, gathered on the G set, then sum_{q,p} w_q w_p B_i(x_q) B_j(z_p)."""

    def __init__(self, desc, ik: int = 0, vfunc=None):
        self.desc = desc
        self.xb, self.zb = basis_x(desc), basis_z(desc)
        self.m, self.kg = gset(desc, ik)
        self.ng, self.nx, self.nz = len(self.m), self.xb.nb, self.zb.nb
        self.ny = int(desc["ny"])
        self.Sx, self.Dx = self.xb.overlap(), self.xb.deriv_overlap()
        self.Sz, self.Dz = self.zb.overlap(), self.zb.deriv_overlap()
        has_v = vfunc is not None or bool(desc["atoms"])
        self.V = potential_grid(desc, self.xb.zq, self.zb.zq, vfunc) if has_v else None
        self.F, self.X, self.Z, self.E = projector_factors(desc, ik, self.xb, self.zb)
        self.pos = self.m % self.ny

    def _shape(self, x):
        return x.reshape(-1, self.ng, self.nx, self.nz)

    def apply_s(self, x):
        c = self._shape(x)
        return np.einsum("ik,jl,bgkl->bgij", self.Sx, self.Sz, c, optimize=True).reshape(x.shape)

    def apply(self, x):
        c = self._shape(x)
        y = 0.5 * (np.einsum("ik,jl,bgkl->bgij", self.Dx, self.Sz, c, optimize=True)
                   + np.einsum("ik,jl,bgkl->bgij", self.Sx, self.Dz, c, optimize=True))
        y += 0.5 * (self.kg ** 2)[None, :, None, None] * np.einsum("ik,jl,bgkl->bgij", self.Sx, self.Sz, c,
                                                                      optimize=True)
        if self.V is not None:
            xb, zb = self.xb, self.zb
            psi = np.einsum("qi,pj,bgij->bqpg", xb.B, zb.B, c, optimize=True)
            grid = np.zeros(psi.shape[:3] + (self.ny,), dtype=np.complex128)
            grid[..., self.pos] = psi
            u = np.fft.fft(np.fft.ifft(grid, axis=-1) * self.ny * self.V[None], axis=-1) / self.ny
            u = u[..., self.pos]
            y += np.einsum("q,p,qi,pj,bqpg->bgij", xb.wq, zb.wq, xb.B, zb.B, u, optimize=True)
        if len(self.E):
            P = np.einsum("pg,pi,pj,bgij->bp", self.F.conj(), self.X, self.Z, c, optimize=True)
            y += np.einsum("p,pg,pi,pj,bp->bgij", self.E, self.F, self.X, self.Z, P, optimize=True)
        return y.reshape(x.shape)


class WireRows:
    """Selected outputs (G, i, j) of H x and S x, each evaluated on its own: the local
    sum runs only over the Gauss points where B_i(x) B_j(z) is non-zero, with V
    sampled there."""

    def __init__(self, desc, ik: int = 0, vfunc=None):
        self.desc = desc
        self.xb, self.zb = basis_x(desc), basis_z(desc)
        self.m, self.kg = gset(desc, ik)
        self.ng, self.nx, self.nz = len(self.m), self.xb.nb, self.zb.nb
        self.ny = int(desc["ny"])
        self.Sx, self.Dx = self.xb.overlap(), self.xb.deriv_overlap()
        self.Sz, self.Dz = self.zb.overlap(), self.zb.deriv_overlap()
        self.vfunc = vfunc
        self.has_v = vfunc is not None or bool(desc["atoms"])
        self.F, self.X, self.Z, self.E = projector_factors(desc, ik, self.xb, self.zb)

    @staticmethod
    def _support(B, i):
        return np.nonzero(np.abs(B[:, i]) > 0)[0]

    def apply_rows(self, x, rows):
        """x: (NG, Nx, Nz) complex; rows: list of (g, i, j).  Returns (H x, S x) at the rows."""
        hs, ss = [], []
        P = np.einsum("pg,pi,pj,gij->p", self.F.conj(), self.X, self.Z, x) if len(self.E) else None
        for g, i, j in rows:
            sx = self.Sx[i] @ x[g] @ self.Sz[j]
            hx = 0.5 * (self.Dx[i] @ x[g] @ self.Sz[j] + self.Sx[i] @ x[g] @ self.Dz[j]) + 0.5 * self.kg[g] ** 2 * sx
            if self.has_v:
                qs, ps = self._support(self.xb.B, i), self._support(self.zb.B, j)
                V = potential_grid(self.desc, self.xb.zq[qs], self.zb.zq[ps], self.vfunc)
                vt = vtilde_grid(V)[:, :, (self.m[g] - self.m) % self.ny]  # (nq, np, NG)
                psi = np.einsum("qk,pl,gkl->qpg", self.xb.B[qs], self.zb.B[ps], x)
                u = np.sum(vt * psi, axis=-1)
                hx += np.einsum("q,p,q,p,qp->", self.xb.wq[qs], self.zb.wq[ps], self.xb.B[qs, i],
                                self.zb.B[ps, j], u)
            if P is not None:
                hx += np.sum(self.E * self.F[:, g] * self.X[:, i] * self.Z[:, j] * P)
            hs.append(hx)
            ss.append(sx)
        return np.array(hs), np.array(ss)
