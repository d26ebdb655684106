"""B-splines along z (Sec. II.A, eqs. 1-3) and the z-integrals built from them.

Readings of the paper used here:
* eqs. 1-2 write ``x`` where ``z`` is meant; ``z`` is used.
* 0/0 := 0 in the recursion where knots coincide.
* The order-1 spline is the indicator of [tau_i, tau_{i+1}); the last
  non-empty interval is taken closed so the set sums to one at the right end.
* Hard walls: the knot sequence is clamped (multiplicity kappa at both ends) and
  the first and last spline are dropped, so every kept function vanishes at
  both ends.
* Integrals whose integrand is not a polynomial use a per-interval
  Gauss-Legendre rule with ``nq`` points; the same rule defines the discrete
  operator everywhere.
"""
from __future__ import annotations

import numpy as np


def clamped_knots(breakpoints, order: int) -> np.ndarray:
    """Full knot sequence tau: breakpoints with both ends repeated ``order`` times."""
    bp = np.asarray(breakpoints, dtype=np.float64)
    if np.any(np.diff(bp) <= 0):
        raise ValueError("breakpoints must be strictly increasing")
    return np.concatenate([np.full(order - 1, bp[0]), bp, np.full(order - 1, bp[-1])])


def n_full(tau: np.ndarray, order: int) -> int:
    return len(tau) - order


def bspline_values(tau: np.ndarray, order: int, z) -> np.ndarray:
    """All B_{i,order}(z) of the full set by the Cox-de Boor recursion (eqs. 1-2).

    Returns an array of shape (len(z), len(tau) - order).
    """
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    m = len(tau) - 1
    B = np.zeros((len(z), m))
    for i in range(m):
        B[:, i] = ((tau[i] <= z) & (z < tau[i + 1])).astype(np.float64)
    last = max(i for i in range(m) if tau[i] < tau[i + 1])
    B[z == tau[last + 1], last] = 1.0
    for k in range(2, order + 1):
        Bk = np.zeros((len(z), len(tau) - k))
        for i in range(len(tau) - k):
            d1 = tau[i + k - 1] - tau[i]
            d2 = tau[i + k] - tau[i + 1]
            left = (z - tau[i]) / d1 * B[:, i] if d1 > 0 else 0.0
            right = (tau[i + k] - z) / d2 * B[:, i + 1] if d2 > 0 else 0.0
            Bk[:, i] = left + right
        B = Bk
    return B


def bspline_derivs(tau: np.ndarray, order: int, z) -> np.ndarray:
    """d/dz B_{i,order}(z) from two order-1 lower splines (eq. 3)."""
    Bl = bspline_values(tau, order - 1, z)
    nz = Bl.shape[0]
    nf = len(tau) - order
    D = np.zeros((nz, nf))
    k = order
    for i in range(nf):
        d1 = tau[i + k - 1] - tau[i]
        d2 = tau[i + k] - tau[i + 1]
        if d1 > 0:
            D[:, i] += (k - 1) / d1 * Bl[:, i]
        if d2 > 0:
            D[:, i] -= (k - 1) / d2 * Bl[:, i + 1]
    return D


def gauss_rule(breakpoints, nq: int):
    """Gauss-Legendre nodes and weights, ``nq`` per interval, all intervals.

    Returns (zq, wq) ordered interval by interval.
    """
    bp = np.asarray(breakpoints, dtype=np.float64)
    x, w = np.polynomial.legendre.leggauss(nq)
    zs, ws = [], []
    for a, b in zip(bp[:-1], bp[1:]):
        h = 0.5 * (b - a)
        zs.append(0.5 * (a + b) + h * x)
        ws.append(h * w)
    return np.concatenate(zs), np.concatenate(ws)


class ZBasis:
    """The kept (hard-wall) B-spline basis and its tables at the Gauss points."""

    def __init__(self, breakpoints, order: int, nq: int):
        self.order = order
        self.breakpoints = np.asarray(breakpoints, dtype=np.float64)
        self.tau = clamped_knots(breakpoints, order)
        self.nfull = n_full(self.tau, order)
        self.nb = self.nfull - 2
        self.zq, self.wq = gauss_rule(breakpoints, nq)
        full = bspline_values(self.tau, order, self.zq)
        dfull = bspline_derivs(self.tau, order, self.zq)
        # drop the first and the last spline (hard walls)
        self.B = full[:, 1:-1]
        self.dB = dfull[:, 1:-1]

    def values(self, z):
        return bspline_values(self.tau, self.order, z)[:, 1:-1]

    def overlap(self) -> np.ndarray:
        """S_z[i, j] = int B_i B_j dz (symmetrised: the integral is symmetric)."""
        M = (self.B * self.wq[:, None]).T @ self.B
        return 0.5 * (M + M.T)

    def deriv_overlap(self) -> np.ndarray:
        """D_z[i, j] = int B'_i B'_j dz (equals -int B_i B_j'' with hard walls)."""
        M = (self.dB * self.wq[:, None]).T @ self.dB
        return 0.5 * (M + M.T)

    def weighted(self, f: np.ndarray) -> np.ndarray:
        """int B_i(z) f(z) dz for f sampled at the Gauss points."""
        return self.B.T @ (self.wq * f)

    def local(self, f: np.ndarray) -> np.ndarray:
        """int B_i(z) B_j(z) f(z) dz for f sampled at the Gauss points."""
        return (self.B * (self.wq * f)[:, None]).T @ self.B
