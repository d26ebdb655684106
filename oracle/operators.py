"""Dense matrix elements of S and H in the mixed basis (Sec. II.B.1), and the
ultrasoft overlap of Sec. II.B.2.

Index of a basis function (G, i): G * N_b + i (the oracle's own order).

Readings of the paper used here:
* Hartree units: T = 1/2 (D_z + |k+G|^2 S_z) per G; the paper's -nabla^2 and
  cutoffs in Ry are the same operator in Rydberg.
* The kinetic block carries delta_{G,G'} (the printed delta_{G,G} is a typo).
* Local potential: sum over atoms of Gaussians A_t exp(-r^2 / w_t^2) (the
  Gaussian part of the paper's local pseudopotential; the erf core belongs to
  the self-consistent potential and is not part of this operator).
  Two forms of its in-plane transform are provided:
    - ``analytic``: the closed 2D Fourier transform of the paper,
      (A/A_c)(pi/a) exp(-|dG|^2 / 4a) exp(-i dG.R) with a = 1/w^2, times the
      z-Gaussian inside the integral I;
    - ``grid``: V sampled on the N1 x N2 in-plane grid (lattice images summed)
      and transformed with explicit DFT matrices, i.e. the circular
      convolution an FFT of the sampled potential realises.  This is the
      operator the library applies; the two differ only by aliasing.
* Nonlocal part: Kleinman-Bylander form sum_p E_p |beta_p><beta_p| per atom with
  one s and three real Cartesian p projectors,
      beta_s  = C_s exp(-alpha_s r^2),      C_s = (2 alpha_s / pi)^{3/4}
      beta_pc = C_p c exp(-alpha_p r^2),    C_p = (2 alpha_p / pi)^{3/4} 2 sqrt(alpha_p)
  (c = x, y, z; each normalised to one).  The real p_x, p_y, p_z span the same
  space as r Y_{1m}; with one energy per l the operator is the same.
  Their overlap with a basis function factorises into an in-plane factor Q and
  a z integral Z, as in the paper's S = Z Q factorisation; with the bra
  convention exp(-i(k+G).rho):
      <G,i|beta_s>  = A_c^{-1/2} e^{-i(k+G).R} C_s (pi/a) e^{-q^2/4a} Z_0(i)
      <G,i|beta_px> = A_c^{-1/2} e^{-i(k+G).R} C_p (-i q_x / 2a)(pi/a) e^{-q^2/4a} Z_0(i)
      <G,i|beta_pz> = A_c^{-1/2} e^{-i(k+G).R} C_p (pi/a) e^{-q^2/4a} Z_1(i)
  with q = k+G, Z_0(i) = int B_i e^{-a (z-R_z)^2}, Z_1(i) = int B_i (z-R_z) e^{-a (z-R_z)^2}.
"""
from __future__ import annotations

import math

import numpy as np

from .bspline import ZBasis
from .lattice import cell_area, gset, kvec, reciprocal


# ----------------------------------------------------------------------------
# local potential
# ----------------------------------------------------------------------------

def image_range(desc, width: float) -> int:
    """Number of lattice images per direction so that every image closer than
    sqrt(45) w to the cell is summed (exp(-45) < 3e-20)."""
    a1 = np.asarray(desc["a1"], float)
    a2 = np.asarray(desc["a2"], float)
    area = cell_area(a1, a2)
    h1 = area / np.linalg.norm(a2)  # distance between lines of a1-translates
    h2 = area / np.linalg.norm(a1)
    cut = math.sqrt(45.0) * width
    return int(math.ceil(cut / min(h1, h2))) + 1


def grid_points(desc) -> np.ndarray:
    """Cartesian in-plane grid rho_j = (j1/N1) a1 + (j2/N2) a2, shape (N1, N2, 2)."""
    N1, N2 = desc["grid"]
    a1 = np.asarray(desc["a1"], float)
    a2 = np.asarray(desc["a2"], float)
    f1 = np.arange(N1) / N1
    f2 = np.arange(N2) / N2
    return f1[:, None, None] * a1[None, None, :] + f2[None, :, None] * a2[None, None, :]


def gaussian_potential(desc, x: np.ndarray, y: np.ndarray, z: np.ndarray) -> np.ndarray:
    """V(r) = sum_atoms sum_t A_t sum_L exp(-|r - R - L|^2 / w_t^2), real space."""
    a1 = np.asarray(desc["a1"], float)
    a2 = np.asarray(desc["a2"], float)
    V = np.zeros(np.broadcast(x, y, z).shape)
    for at in desc["atoms"]:
        sp = desc["species"][at["species"]]
        X, Y, Z = at["pos"]
        for A, w in sp["gauss"]:
            nimg = image_range(desc, w)
            for n1 in range(-nimg, nimg + 1):
                for n2 in range(-nimg, nimg + 1):
                    Lx = n1 * a1[0] + n2 * a2[0]
                    Ly = n1 * a1[1] + n2 * a2[1]
                    r2 = (x - X - Lx) ** 2 + (y - Y - Ly) ** 2 + (z - Z) ** 2
                    V = V + A * np.exp(-r2 / (w * w))
    return V


def potential_on_grid(desc, zq: np.ndarray, vfunc=None) -> np.ndarray:
    """Real V(rho_j, z_q), shape (Nq, N1, N2)."""
    rho = grid_points(desc)
    x = rho[None, :, :, 0]
    y = rho[None, :, :, 1]
    z = np.asarray(zq, float)[:, None, None]
    if vfunc is None:
        return gaussian_potential(desc, x, y, z)
    return np.broadcast_to(vfunc(x, y, z), (len(zq),) + rho.shape[:2]).astype(np.float64)


def gaussian_potential_on_grid_separable(desc, zq: np.ndarray) -> np.ndarray:
    """The same V(rho_j, z_q) as ``potential_on_grid`` for the Gaussian wells,
    from the factorisation exp(-|r - R - L|^2 / w^2) =
    exp(-|rho - R_par - L|^2 / w^2) exp(-(z - R_z)^2 / w^2): in-plane maps of every
    (atom, term) once, combined plane by plane with their z factors (a matrix
    product).  Shape (Nq, N1, N2)."""
    a1 = np.asarray(desc["a1"], float)
    a2 = np.asarray(desc["a2"], float)
    rho = grid_points(desc)
    x, y = rho[..., 0], rho[..., 1]
    zq = np.asarray(zq, float)
    maps, zfac = [], []
    for at in desc["atoms"]:
        sp = desc["species"][at["species"]]
        X, Y, Z = at["pos"]
        for A, w in sp["gauss"]:
            nimg = image_range(desc, w)
            plane = np.zeros(x.shape)
            for n1 in range(-nimg, nimg + 1):
                for n2 in range(-nimg, nimg + 1):
                    Lx = n1 * a1[0] + n2 * a2[0]
                    Ly = n1 * a1[1] + n2 * a2[1]
                    plane += np.exp(-((x - X - Lx) ** 2 + (y - Y - Ly) ** 2) / (w * w))
            maps.append(A * plane.ravel())
            zfac.append(np.exp(-((zq - Z) ** 2) / (w * w)))
    if not maps:
        return np.zeros((len(zq),) + x.shape)
    out = np.array(zfac).T @ np.array(maps)
    return out.reshape((len(zq),) + x.shape)


def dft_matrix(N: int) -> np.ndarray:
    j = np.arange(N)
    return np.exp(-2j * math.pi * np.outer(j, j) / N)


def vtilde_grid(desc, vgrid: np.ndarray) -> np.ndarray:
    """Vt[q, d1, d2] = 1/(N1 N2) sum_j V(rho_j, z_q) exp(-2 pi i (d1 j1/N1 + d2 j2/N2))."""
    N1, N2 = desc["grid"]
    F1 = dft_matrix(N1)
    F2 = dft_matrix(N2)
    return np.einsum("ab,qbc,dc->qad", F1, vgrid.astype(np.complex128), F2, optimize=True) / (N1 * N2)


def vloc_pairs_grid(desc, ik: int, zq, vfunc=None) -> np.ndarray:
    """Vt(G - G', z_q) for all pairs of the G set, shape (NG, NG, Nq); the index
    difference is reduced modulo the grid (circular convolution)."""
    N1, N2 = desc["grid"]
    m, _ = gset(desc, ik)
    vt = vtilde_grid(desc, potential_on_grid(desc, zq, vfunc))
    d1 = (m[:, None, 0] - m[None, :, 0]) % N1
    d2 = (m[:, None, 1] - m[None, :, 1]) % N2
    return np.transpose(vt[:, d1, d2], (1, 2, 0))


def vloc_pairs_analytic(desc, ik: int, zq) -> np.ndarray:
    """Closed-form Vt(G - G', z_q) of the Gaussian potential, shape (NG, NG, Nq)."""
    b1, b2 = reciprocal(desc["a1"], desc["a2"])
    area = cell_area(desc["a1"], desc["a2"])
    m, _ = gset(desc, ik)
    dm = m[:, None, :] - m[None, :, :]
    dG = dm[..., 0:1] * b1 + dm[..., 1:2] * b2  # (NG, NG, 2)
    dG2 = np.sum(dG * dG, axis=-1)
    zq = np.asarray(zq, float)
    out = np.zeros(dG2.shape + (len(zq),), dtype=np.complex128)
    for at in desc["atoms"]:
        sp = desc["species"][at["species"]]
        X, Y, Z = at["pos"]
        phase = np.exp(-1j * (dG[..., 0] * X + dG[..., 1] * Y))
        for A, w in sp["gauss"]:
            a = 1.0 / (w * w)
            plane = (A / area) * (math.pi / a) * np.exp(-dG2 / (4.0 * a)) * phase
            out += plane[..., None] * np.exp(-a * (zq - Z) ** 2)[None, None, :]
    return out


# ----------------------------------------------------------------------------
# nonlocal projectors
# ----------------------------------------------------------------------------

PROJ_NAMES = ("s", "px", "py", "pz")


def projector_norms(alpha_s: float, alpha_p: float):
    cs = (2.0 * alpha_s / math.pi) ** 0.75
    cp = (2.0 * alpha_p / math.pi) ** 0.75 * 2.0 * math.sqrt(alpha_p)
    return cs, cp


def inplane_factor(kind: str, alpha: float, q: np.ndarray) -> np.ndarray:
    """Q(q) = int d^2 rho exp(-i q.rho) f(rho) exp(-alpha rho^2) for f = 1, x, y."""
    q2 = np.sum(q * q, axis=-1)
    g = (math.pi / alpha) * np.exp(-q2 / (4.0 * alpha))
    if kind in ("s", "pz"):
        return g.astype(np.complex128)
    if kind == "px":
        return -1j * q[..., 0] / (2.0 * alpha) * g
    if kind == "py":
        return -1j * q[..., 1] / (2.0 * alpha) * g
    raise ValueError(kind)


def projector_factors(desc, ik: int, zb: ZBasis):
    """Factored overlaps <G,i|beta_{a,p}> = F_p(G) Z_p(i) for every nonlocal
    atom and projector (the paper's Z Q factorisation with the phase and the
    normalisations folded into F).

    Returns (F, Z, energies) of shapes (Np, NG), (Np, Nb), (Np,).
    """
    area = cell_area(desc["a1"], desc["a2"])
    _, kg = gset(desc, ik)
    Fs, Zs, energies = [], [], []
    for at in desc["atoms"]:
        sp = desc["species"][at["species"]]
        if not sp.get("nonlocal", False):
            continue
        X, Y, Z = at["pos"]
        phase = np.exp(-1j * (kg[:, 0] * X + kg[:, 1] * Y)) / math.sqrt(area)
        cs, cp = projector_norms(sp["alpha_s"], sp["alpha_p"])
        dz = zb.zq - Z
        for kind in PROJ_NAMES:
            alpha = sp["alpha_s"] if kind == "s" else sp["alpha_p"]
            c = cs if kind == "s" else cp
            zf = np.exp(-alpha * dz * dz)
            if kind == "pz":
                zf = dz * zf
            Zs.append(zb.weighted(zf))
            Fs.append(c * phase * inplane_factor(kind, alpha, kg))
            energies.append(sp["E_s"] if kind == "s" else sp["E_p"])
    if not Fs:
        return (np.zeros((0, len(kg)), dtype=np.complex128), np.zeros((0, zb.nb)),
                np.zeros(0))
    return np.array(Fs), np.array(Zs), np.array(energies, dtype=np.float64)


def projector_augmentation(desc) -> np.ndarray:
    """Augmentation charge q_p of every projector, in the order of projector_factors
    (ultrasoft overlap S = I_G (x) S_z + sum_p q_p |beta_p><beta_p|, Sec. II.B.2; the
    paper's q_nm matrix taken diagonal, with one charge per projector channel)."""
    qs = []
    for at in desc["atoms"]:
        sp = desc["species"][at["species"]]
        if not sp.get("nonlocal", False):
            continue
        for kind in PROJ_NAMES:
            qs.append(float(sp.get("q_s" if kind == "s" else "q_p", 0.0)))
    return np.array(qs, dtype=np.float64)


def projectors(desc, ik: int, zb: ZBasis):
    """Dense overlaps <G,i|beta_{a,p}>, shape (Np, NG, Nb), and energies (Np,)."""
    F, Z, E = projector_factors(desc, ik, zb)
    return F[:, :, None] * Z[:, None, :], E


# ----------------------------------------------------------------------------
# assembly
# ----------------------------------------------------------------------------

class Problem:
    """Dense S and H of one k-point."""

    def __init__(self, desc, ik: int = 0, vmode: str = "grid", vfunc=None,
                 with_local: bool = True, with_nonlocal: bool = True):
        self.desc = desc
        self.ik = ik
        self.zb = ZBasis(desc["breakpoints"], desc["order"], desc["nq"])
        self.m, self.kg = gset(desc, ik)
        self.ng = len(self.m)
        self.nb = self.zb.nb
        self.n = self.ng * self.nb
        self.Sz = self.zb.overlap()
        self.Dz = self.zb.deriv_overlap()
        self.vmode = vmode
        self.vfunc = vfunc
        self.with_local = with_local
        self.with_nonlocal = with_nonlocal

    def overlap(self) -> np.ndarray:
        """S = I_G (x) S_z (+ sum_p q_p |beta_p><beta_p| in the ultrasoft form)."""
        S = np.kron(np.eye(self.ng), self.Sz).astype(np.complex128)
        q = projector_augmentation(self.desc)
        if np.any(q != 0):
            beta, _ = self.projectors()
            for p in range(len(q)):
                b = beta[p].reshape(-1)
                S += q[p] * np.outer(b, b.conj())
        return S

    def kinetic(self) -> np.ndarray:
        T = np.zeros((self.n, self.n), dtype=np.complex128)
        kg2 = np.sum(self.kg * self.kg, axis=1)
        for g in range(self.ng):
            s = slice(g * self.nb, (g + 1) * self.nb)
            T[s, s] = 0.5 * (self.Dz + kg2[g] * self.Sz)
        return T

    def local(self) -> np.ndarray:
        zb = self.zb
        if self.vmode == "grid":
            vt = vloc_pairs_grid(self.desc, self.ik, zb.zq, self.vfunc)
        elif self.vmode == "analytic":
            vt = vloc_pairs_analytic(self.desc, self.ik, zb.zq)
        else:
            raise ValueError(self.vmode)
        W = (zb.B[:, :, None] * zb.B[:, None, :]) * zb.wq[:, None, None]  # (Nq, Nb, Nb)
        M = vt.reshape(self.ng * self.ng, -1) @ W.reshape(W.shape[0], -1)
        M = M.reshape(self.ng, self.ng, self.nb, self.nb)
        return np.transpose(M, (0, 2, 1, 3)).reshape(self.n, self.n)

    def projectors(self):
        return projectors(self.desc, self.ik, self.zb)

    def nonlocal_(self) -> np.ndarray:
        beta, E = self.projectors()
        V = np.zeros((self.n, self.n), dtype=np.complex128)
        for p in range(len(E)):
            b = beta[p].reshape(-1)
            V += E[p] * np.outer(b, b.conj())
        return V

    def hamiltonian(self) -> np.ndarray:
        H = self.kinetic()
        if self.with_local and (self.vfunc is not None or self.desc["atoms"]):
            H = H + self.local()
        if self.with_nonlocal:
            H = H + self.nonlocal_()
        return H


def to_oracle_order(x_lib: np.ndarray) -> np.ndarray:
    """[band][i][G] -> [band][G*Nb + i] (vectors as columns are x.T)."""
    nbands, nb, ng = x_lib.shape
    return np.transpose(x_lib, (0, 2, 1)).reshape(nbands, ng * nb)


def from_oracle_order(x: np.ndarray, nb: int, ng: int) -> np.ndarray:
    nbands = x.shape[0]
    return np.transpose(x.reshape(nbands, ng, nb), (0, 2, 1))
