"""Electron density at the Gauss planes and the Hartree potential of a charge
distribution in the mixed (z, g) form (Sec. II.B.1), written out from their
definitions.  TEST INFRASTRUCTURE: used by tests/, the smoke check and the
benchmark's CPU baseline only; the library never calls it.

Density.  rho_e(r) = sum_b w_b |phi_b(r)|^2 with
  phi_b(rho, z) = A^{-1/2} sum_{G,i} c_b(G, i) e^{i(k+G).rho} B_i(z),
evaluated at the grid points rho_j = (j1/N1) a1 + (j2/N2) a2 and the Gauss points z_q
by explicit sums (no FFT).  The factor e^{ik.rho} has modulus one and drops out.

Hartree potential.  With the in-plane transform rho(z, g) = (1/A) int d^2rho rho(r)
e^{i g.rho}, taken on the grid as (1/(N1 N2)) sum_j rho(rho_j, z) e^{i g.rho_j}, and the
2D transform of 1/r,
  V(z, g) = int dz' rho(z', g) (2 pi / |g|) e^{-|g| |z - z'|}      (g != 0)
  V(z, 0) = -2 pi int dz' rho(z', 0) |z - z'|                      (g = 0)
  V(rho, z) = sum_g V(z, g) e^{-i g.rho}.
The g = 0 kernel is the finite part of (2 pi/|g|) e^{-|g||z - z'|} as g -> 0 (the
divergent constant 2 pi/|g| multiplies the net charge of the cell, zero for a neutral
system).  The z integral is the Gauss rule of the knot intervals, the same points and
weights as every other z integral of the method.  Each grid frequency
(m1 mod N1, m2 mod N2) is taken at its shortest alias
g = (m1 + n1 N1) b1 + (m2 + n2 N2) b2, n in {-1, 0, 1}^2, which keeps |g| even in g and
the potential real.

Pins (tests/test_oracle_density.py): the total charge equals sum_b w_b c_b^H S c_b
exactly; one basis function gives a constant in-plane density B_i(z)^2 / A; two plane
waves give the closed-form beat 2 B^2 (1 + cos(dG.rho)) / A; a Gaussian sheet with one
in-plane Fourier component against the closed form of its z integral (erfc form),
converging under knot refinement; the g = 0 potential of a neutral layer jumps by
4 pi times its dipole moment across it (exact for the Gauss sums); reciprocity
<rho1, V[rho2]> = <rho2, V[rho1]>; a real potential.
"""
from __future__ import annotations

import math

import numpy as np

from .bspline import ZBasis
from .lattice import cell_area, gset, reciprocal


def grid_g(desc):
    """Cartesian g and |g| of every grid frequency (j1, j2), shortest alias; shapes
    (N1, N2, 2) and (N1, N2)."""
    N1, N2 = desc["grid"]
    b1, b2 = reciprocal(desc["a1"], desc["a2"])
    best = np.full((N1, N2), np.inf)
    gvec = np.zeros((N1, N2, 2))
    j1 = np.arange(N1)[:, None]
    j2 = np.arange(N2)[None, :]
    for n1 in (-1, 0, 1):
        for n2 in (-1, 0, 1):
            m1 = j1 + n1 * N1
            m2 = j2 + n2 * N2
            g = m1[..., None] * b1[None, None, :] + m2[..., None] * b2[None, None, :]
            norm = np.sqrt(np.sum(g * g, axis=-1))
            take = norm < best - 1e-12
            best = np.where(take, norm, best)
            gvec = np.where(take[..., None], g, gvec)
    return gvec, best


def density_grid(desc, ik: int, C: np.ndarray, weights, planes=None) -> np.ndarray:
    """rho_e(rho_j, z_q) for vectors C of shape (nvec, NG, Nb) (oracle G order) with
    occupation weights w_b; returns (len(planes), N1, N2) (all Gauss planes by default)."""
    N1, N2 = desc["grid"]
    zb = ZBasis(desc["breakpoints"], desc["order"], desc["nq"])
    m, _ = gset(desc, ik)
    A = cell_area(desc["a1"], desc["a2"])
    qs = np.arange(len(zb.zq)) if planes is None else np.asarray(planes)
    j1 = np.repeat(np.arange(N1), N2)
    j2 = np.tile(np.arange(N2), N1)
    # e^{i G.rho_j} = e^{2 pi i (m1 j1 / N1 + m2 j2 / N2)}
    phase = np.exp(2j * math.pi * (np.outer(j1, m[:, 0]) / N1 + np.outer(j2, m[:, 1]) / N2))
    rho = np.zeros((len(qs), N1 * N2))
    Bq = zb.B[qs]                                   # (nplanes, Nb)
    for b in range(C.shape[0]):
        psi_g = C[b] @ Bq.T                         # (NG, nplanes): sum_i c(G, i) B_i(z_q)
        psi = phase @ psi_g                         # (N1 N2, nplanes)
        rho += float(weights[b]) * (np.abs(psi) ** 2).T / A
    return rho.reshape(len(qs), N1, N2)


def coulomb_zg(desc, rho_g: np.ndarray, gnorm: np.ndarray) -> np.ndarray:
    """V(z_q, g) = sum_q' w_q' rho(z_q', g) K_g(z_q - z_q') for rho_g of shape
    (Nq, ng) and |g| of shape (ng,): the Gauss-rule form of the z integral."""
    zb = ZBasis(desc["breakpoints"], desc["order"], desc["nq"])
    z, w = zb.zq, zb.wq
    dz = np.abs(z[:, None] - z[None, :])
    out = np.zeros_like(rho_g, dtype=np.complex128)
    for n, gn in enumerate(gnorm):
        if gn == 0.0:
            K = -2.0 * math.pi * dz
        else:
            K = (2.0 * math.pi / gn) * np.exp(-gn * dz)
        out[:, n] = K @ (w * rho_g[:, n])
    return out


def hartree_grid(desc, rho: np.ndarray, return_zg: bool = False):
    """Hartree potential V(rho_j, z_q) of a density rho (Nq, N1, N2) given at every
    Gauss plane; with return_zg also V(z_q, g) as (Nq, N1, N2) complex, indexed by the
    grid frequency (j1, j2)."""
    N1, N2 = desc["grid"]
    nq = rho.shape[0]
    j1 = np.arange(N1)
    j2 = np.arange(N2)
    # rho(z, g) = (1/N) sum_j rho(rho_j, z) e^{+2 pi i (m1 j1 / N1 + m2 j2 / N2)}
    E1 = np.exp(2j * math.pi * np.outer(j1, j1) / N1)
    E2 = np.exp(2j * math.pi * np.outer(j2, j2) / N2)
    rho_g = np.einsum("ma,qab,nb->qmn", E1, rho.astype(np.complex128), E2, optimize=True) / (N1 * N2)
    _, gnorm = grid_g(desc)
    vzg = coulomb_zg(desc, rho_g.reshape(nq, -1), gnorm.reshape(-1)).reshape(nq, N1, N2)
    # V(rho_j, z) = sum_g V(z, g) e^{-2 pi i (m1 j1 / N1 + m2 j2 / N2)}
    v = np.einsum("am,qmn,bn->qab", E1.conj(), vzg, E2.conj(), optimize=True)
    if return_zg:
        return v, vzg
    return v
