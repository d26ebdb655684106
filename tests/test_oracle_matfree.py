"""Pins of the oracle's matrix-free operator (oracle/matfree.py) against the
dense matrices of oracle/operators.py (Sec. II.B.1), and of its eigensolver
against LAPACK's generalized Hermitian solver (the lowest roots of H c = eps S c,
Sec. II.C).  Each case would catch a dropped term (kinetic, local, nonlocal), a
wrong sign of the transform or a transposed operand in either local mode."""
import numpy as np
import pytest

from oracle import matfree, operators, solve
from paper_1406_4960_amd import workloads

CELLS = {
    "tiny": workloads.tiny,
    "micro-2": lambda: workloads.micro(seed=2, natoms=2, kfrac=(0.31, -0.17), mmax=2, nint=9, grid=8),
    "micro-odd": lambda: workloads.micro(seed=5, natoms=2, mmax=2, nint=8, grid=15, kfrac=(-0.4, 0.27)),
}


def _dense(d):
    p = operators.Problem(d, 0)
    return p, p.hamiltonian(), p.overlap()


@pytest.mark.parametrize("local", ["dense", "fft"])
@pytest.mark.parametrize("cell", list(CELLS))
def test_matfree_apply_matches_dense(cell, local):
    d = CELLS[cell]()
    p, H, S = _dense(d)
    mf = matfree.MatFree(d, 0, local=local)
    x = workloads.random_block(21, 4, p.nb, p.ng)         # [band][i][G]
    xg = np.transpose(x, (0, 2, 1))                        # [band][G][i]
    hx, sx = mf.apply(xg)
    xo = xg.reshape(4, -1)
    ref_h = (H @ xo.T).T.reshape(hx.shape)
    ref_s = (S @ xo.T).T.reshape(sx.shape)
    assert np.max(np.abs(hx - ref_h)) <= 1e-13 * np.max(np.abs(ref_h))
    assert np.max(np.abs(sx - ref_s)) <= 1e-13 * np.max(np.abs(ref_s))
    assert np.max(np.abs(mf.apply_s(xg) - ref_s)) <= 1e-13 * np.max(np.abs(ref_s))


def test_matfree_terms_are_all_present():
    # a cell where the kinetic, local and nonlocal parts each move H x by far more
    # than the bar above: dropping any one of them fails the dense comparison
    d = CELLS["micro-2"]()
    x = np.transpose(workloads.random_block(22, 2, 10, 25), (0, 2, 1))
    full = matfree.MatFree(d, 0, local="fft").apply(x)[0]
    no_nl = matfree.MatFree(dict(d, species=[{**s, "nonlocal": False} for s in d["species"]]), 0,
                            local="fft").apply(x)[0]
    no_v = matfree.MatFree(dict(d, species=[dict(s, gauss=[]) for s in d["species"]]), 0,
                           local="fft").apply(x)[0]
    scale = np.max(np.abs(full))
    assert np.max(np.abs(full - no_nl)) > 1e-3 * scale
    assert np.max(np.abs(full - no_v)) > 1e-3 * scale


def test_matfree_given_grid_equals_sampled_grid():
    d = CELLS["micro-odd"]()
    mf = matfree.MatFree(d, 0, local="fft")
    vg = operators.gaussian_potential_on_grid_separable(d, mf.zb.zq)
    mf2 = matfree.MatFree(d, 0, local="fft", vgrid=vg)
    x = np.transpose(workloads.random_block(23, 2, mf.nb, mf.ng), (0, 2, 1))
    a, b = mf.apply(x)[0], mf2.apply(x)[0]
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


@pytest.mark.parametrize("maker", [lambda: workloads.micro(seed=5, natoms=2),
                                   lambda: workloads.surface()])
def test_separable_potential_sampling_matches_direct(maker):
    # V(rho, z) sampled directly (3D Gaussians summed over lattice images) and
    # through the in-plane x z factorisation agree on a few planes
    d = maker()
    zq = np.array([-4.1, -0.3, 0.0, 0.8, 2.5])
    if len(d["atoms"]) > 8:
        d = dict(d, atoms=d["atoms"][::9])  # a subset of the surface slab's atoms keeps it quick
    direct = operators.potential_on_grid(d, zq)
    sep = operators.gaussian_potential_on_grid_separable(d, zq)
    assert np.max(np.abs(direct - sep)) <= 1e-14 * np.max(np.abs(direct))


@pytest.mark.parametrize("local", ["dense", "fft"])
def test_matfree_lowest_matches_lapack(local):
    d = workloads.micro(seed=3, natoms=2, mmax=2, nint=11, grid=8, kfrac=(0.23, -0.31))
    nev = 8
    w_ref = solve.solve_problem(d, 0, nev=nev)[3]
    mf = matfree.MatFree(d, 0, local=local)
    eps, C, r = mf.lowest(nev, extra=6, tol=1e-10, maxiter=2000, seed=1)
    assert np.max(np.abs(eps - w_ref)) < 1e-10
    assert np.max(r) < 1e-8
    # returned vectors are S-orthonormal
    s = mf.apply_s(C).reshape(nev, -1)
    g = C.reshape(nev, -1).conj() @ s.T
    assert np.max(np.abs(g - np.eye(nev))) < 1e-8
