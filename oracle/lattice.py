"""In-plane lattice: reciprocal vectors, G sets and k-points.

The basis of Sec. II.B.1 is A^{-1/2} exp(i(k+G).rho) B_j(z) with G an in-plane
reciprocal lattice vector.  The paper selects G by an energy cutoff; in
Hartree units the sphere is 1/2 |k+G|^2 <= E_cut.  A plain index box
|m_1| <= M_1, |m_2| <= M_2 is also supported for the smallest cell.
"""
from __future__ import annotations

import math

import numpy as np


def cell_area(a1, a2) -> float:
    return abs(a1[0] * a2[1] - a1[1] * a2[0])


def reciprocal(a1, a2):
    """b1, b2 with a_i . b_j = 2 pi delta_ij."""
    A = np.array([a1, a2], dtype=np.float64)  # rows a1, a2
    Binv = 2.0 * math.pi * np.linalg.inv(A).T  # rows b1, b2
    return Binv[0], Binv[1]


def kvec(desc, ik: int) -> np.ndarray:
    b1, b2 = reciprocal(desc["a1"], desc["a2"])
    f = desc["kpts"][ik]
    return f[0] * b1 + f[1] * b2


def gset(desc, ik: int):
    """Integer pairs (m1, m2) and Cartesian k+G for the G set of k-point ik.

    Returned sorted by (m1, m2); the order is the oracle's own.
    """
    b1, b2 = reciprocal(desc["a1"], desc["a2"])
    k = kvec(desc, ik)
    rule = desc["gset"]
    ms = []
    if rule["kind"] == "box":
        M1, M2 = rule["mmax"]
        for m1 in range(-M1, M1 + 1):
            for m2 in range(-M2, M2 + 1):
                ms.append((m1, m2))
    elif rule["kind"] == "sphere":
        ecut = float(rule["ecut"])
        r = math.sqrt(2.0 * ecut)
        l1 = np.linalg.norm(desc["a1"])
        l2 = np.linalg.norm(desc["a2"])
        n1 = int(math.ceil(r * l1 / (2 * math.pi))) + 2
        n2 = int(math.ceil(r * l2 / (2 * math.pi))) + 2
        for m1 in range(-n1, n1 + 1):
            for m2 in range(-n2, n2 + 1):
                q = k + m1 * b1 + m2 * b2
                if 0.5 * float(q @ q) <= ecut:
                    ms.append((m1, m2))
    else:
        raise ValueError(rule["kind"])
    ms.sort()
    m = np.array(ms, dtype=np.int64)
    kg = k[None, :] + m[:, 0:1] * b1[None, :] + m[:, 1:2] * b2[None, :]
    return m, kg
