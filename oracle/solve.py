"""Lowest eigenpairs of the discrete generalized problem H c = eps S c.

The method's Lanczos-Krylov iteration (Sec. II.C) only reaches these exact
discrete eigenpairs faster; the oracle computes them directly with LAPACK's
generalized Hermitian solver.  The basis is non-orthogonal, so the NCPP
equation of Sec. II.B.1 is also read in the generalized form that Sec. II.B.2
writes for the ultrasoft case.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .operators import Problem


def lowest(H: np.ndarray, S: np.ndarray, nev: int):
    """(eps ascending, C with columns S-orthonormal)."""
    w, C = scipy.linalg.eigh(H, S, subset_by_index=[0, nev - 1])
    return w, C


def residuals(H: np.ndarray, S: np.ndarray, eps: np.ndarray, C: np.ndarray) -> np.ndarray:
    R = H @ C - (S @ C) * eps[None, :]
    return np.linalg.norm(R, axis=0)


def solve_problem(desc, ik: int = 0, nev=None, **kw):
    prob = Problem(desc, ik, **kw)
    H = prob.hamiltonian()
    S = prob.overlap()
    nev = nev or desc["nbands"]
    w, C = lowest(H, S, nev)
    return prob, H, S, w, C
