"""Pins of the Gamma-point reading used by hpsi_apply_gamma (oracle, CPU).

At k = 0 the G set is closed under G -> -G, and with a real local potential and
projectors whose in-plane factors satisfy beta(-G) = conj beta(G) (the s and p forms
of Sec. II.B.2), the dense H and S commute with the antiunitary map
K: c(G) -> conj c(-G).  Then the vectors with K c = c (wavefunctions real in space)
carry the whole spectrum: H and S written in a basis of such vectors are real, and
their generalized eigenvalues are those of the complex problem.  The same test at
k != 0 fails, which shows that the check can fail.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import operators
from paper_1406_4960_amd import workloads


def _dense(d):
    p = operators.Problem(d, 0)
    return p, p.hamiltonian(), p.overlap()


def _mirror(m):
    index = {(int(a), int(b)): g for g, (a, b) in enumerate(m)}
    return np.array([index[(-int(a), -int(b))] for a, b in m])


def _perm(mir, nb):
    # oracle order: row g * nb + i
    return (mir[:, None] * nb + np.arange(nb)[None, :]).reshape(-1)


CELLS = {
    "micro-gamma": lambda k: workloads.micro(seed=3, natoms=2, mmax=2, nint=9, grid=8, kfrac=k),
    "micro-gamma-odd-grid": lambda k: workloads.micro(seed=5, natoms=1, mmax=2, nint=8, grid=15, kfrac=k),
}


@pytest.mark.parametrize("cell", list(CELLS))
def test_h_and_s_commute_with_conjugate_mirror_at_gamma(cell):
    p, H, S = _dense(CELLS[cell]((0.0, 0.0)))
    P = _perm(_mirror(p.m), p.nb)
    for A in (H, S):
        assert np.max(np.abs(A[np.ix_(P, P)] - np.conj(A))) < 1e-12 * np.max(np.abs(A))


@pytest.mark.parametrize("cell", list(CELLS))
def test_conjugate_mirror_fails_away_from_gamma(cell):
    p, H, _ = _dense(CELLS[cell]((0.1, 0.2)))
    P = _perm(_mirror(p.m), p.nb)  # the box G set is symmetric at any k
    assert np.max(np.abs(H[np.ix_(P, P)] - np.conj(H))) > 1e-3 * np.max(np.abs(H))


@pytest.mark.parametrize("cell", list(CELLS))
def test_real_in_space_vectors_carry_the_whole_spectrum(cell):
    p, H, S = _dense(CELLS[cell]((0.0, 0.0)))
    mir = _mirror(p.m)
    nb, n = p.nb, p.n
    # unitary U whose columns satisfy K u = u: (e_G + e_-G)/sqrt2, i (e_G - e_-G)/sqrt2
    # for each pair G != -G, and e_0 for G = 0, one set per spline row i
    U = np.zeros((n, n), dtype=np.complex128)
    col = 0
    for g in range(p.ng):
        h = mir[g]
        if h < g:
            continue
        for i in range(nb):
            if h == g:
                U[g * nb + i, col] = 1.0
                col += 1
            else:
                r = 1.0 / np.sqrt(2.0)
                U[g * nb + i, col] = r
                U[h * nb + i, col] = r
                U[g * nb + i, col + 1] = 1j * r
                U[h * nb + i, col + 1] = -1j * r
                col += 2
    assert col == n
    assert np.allclose(U.conj().T @ U, np.eye(n), atol=1e-14)
    Hr = U.conj().T @ H @ U
    Sr = U.conj().T @ S @ U
    assert np.max(np.abs(Hr.imag)) < 1e-12 * np.max(np.abs(H))
    assert np.max(np.abs(Sr.imag)) < 1e-12 * np.max(np.abs(S))
    er = sla.eigh(Hr.real, Sr.real, eigvals_only=True)
    ec = sla.eigh(H, S, eigvals_only=True)
    assert np.max(np.abs(er - ec)) < 1e-10 * max(1.0, np.max(np.abs(ec)))
