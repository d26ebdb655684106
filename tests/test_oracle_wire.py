"""Pins of the 1D-periodic oracle (two B-spline directions x plane waves along y):
separable potentials against sums of one-dimensional spectra, the particle in a box,
the grid transform of the potential against its closed form, the projector factors
against direct quadrature, time reversal, and the matrix-free and row forms against
the dense matrices."""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.linalg

from oracle import wire
from oracle.bspline import ZBasis
from paper_1406_4960_amd import workloads


def _free(desc):
    return dict(desc, atoms=[], species=[])


def _spectrum(bp, nq, f=None):
    b = ZBasis(bp, 4, nq)
    A = 0.5 * b.deriv_overlap()
    if f is not None:
        A = A + b.local(f(b.zq))
    return scipy.linalg.eigh(A, b.overlap(), eigvals_only=True)


def _yspectrum(desc, ik, v0):
    # plane waves along y with V0 cos(2 pi y / L): couples m and m +- 1 by V0 / 2
    m, q = wire.gset(desc, ik)
    h = np.diag(0.5 * q * q).astype(complex)
    for a in range(len(m)):
        for b in range(len(m)):
            if abs(m[a] - m[b]) == 1:
                h[a, b] = 0.5 * v0
    return np.linalg.eigvalsh(h)


def _lowest_sums(parts, n):
    tot = parts[0]
    for p in parts[1:]:
        tot = (tot[:, None] + p[None, :]).ravel()
    return np.sort(tot)[:n]


def test_free_wire_is_a_sum_of_box_and_plane_wave_spectra():
    d = _free(workloads.wire_micro(seed=1, nint=7, ecut=8.0, kfrac=0.23))
    pr = wire.WireProblem(d, 0)
    w = scipy.linalg.eigh(pr.hamiltonian(), pr.overlap(), eigvals_only=True)[:20]
    ex = _spectrum(d["breakpoints_x"], d["nq"])
    ez = _spectrum(d["breakpoints_z"], d["nq"])
    _, q = wire.gset(d, 0)
    ref = _lowest_sums([ex, ez, 0.5 * q * q], 20)
    assert np.max(np.abs(w - ref)) < 1e-11


def test_particle_in_a_box_limit():
    # uniform fine splines: lowest level -> pi^2/2 (1/Lx^2 + 1/Lz^2) + 1/2 k^2
    d = _free(workloads.wire_micro(seed=1, nint=12, ecut=1.0, kfrac=0.0))
    d["breakpoints_z"] = workloads.uniform_breakpoints(-4.0, 4.0, 12)
    pr = wire.WireProblem(d, 0)
    w = scipy.linalg.eigh(pr.hamiltonian(), pr.overlap(), eigvals_only=True)[:3]
    Lx, Lz = 10.0, 8.0
    exact = sorted(0.5 * math.pi ** 2 * (a * a / Lx ** 2 + b * b / Lz ** 2) for a in (1, 2) for b in (1, 2))[:3]
    assert np.max(np.abs(w - exact) / exact) < 2e-5


def test_separable_potential_in_x_y_and_z():
    # V = f(x) + g(z) + V0 cos(2 pi y / L): the spectrum is every sum of three 1D spectra
    d = _free(workloads.wire_micro(seed=2, nint=7, ecut=9.0, ny=12, kfrac=-0.31))
    L = d["period"]
    v0 = 0.7
    f = lambda x: 0.15 * (x - 0.4) ** 2 - 1.0  # noqa: E731
    g = lambda z: -1.3 * np.exp(-((z + 0.6) ** 2) / 2.0)  # noqa: E731

    def vfunc(x, y, z):
        return f(x) + g(z) + v0 * np.cos(2.0 * math.pi * y / L)

    pr = wire.WireProblem(d, 0, vfunc=vfunc)
    H = pr.hamiltonian()
    assert np.max(np.abs(H - H.conj().T)) < 1e-13
    w = scipy.linalg.eigh(H, pr.overlap(), eigvals_only=True)[:25]
    ref = _lowest_sums([_spectrum(d["breakpoints_x"], d["nq"], f), _spectrum(d["breakpoints_z"], d["nq"], g),
                        _yspectrum(d, 0, v0)], 25)
    assert np.max(np.abs(w - ref)) < 1e-11


def test_grid_transform_matches_closed_form():
    # fine y grid: aliasing of the Gaussians' transform below 1e-12
    d = workloads.wire_micro(seed=3, nint=6, ecut=2.0, ny=48, nonlocal_=False, period=8.0)
    g = wire.WireProblem(d, 0, vmode="grid").local()
    a = wire.WireProblem(d, 0, vmode="analytic").local()
    assert np.max(np.abs(g - a)) < 1e-12 * np.max(np.abs(a))
    # coarse grid: the two differ (the grid form is the aliased one)
    d8 = dict(d, ny=8)
    g8 = wire.WireProblem(d8, 0, vmode="grid").local()
    assert np.max(np.abs(g8 - a)) > 1e-6 * np.max(np.abs(a))


def test_projector_factors_against_direct_quadrature():
    d = workloads.wire_micro(seed=4, nint=6, ecut=6.0, kfrac=0.19)
    d["nq"] = 14  # the Gauss rule of X and Z then integrates to ~1e-13
    xb, zb = wire.basis_x(d), wire.basis_z(d)
    F, X, Z, E = wire.projector_factors(d, 0, xb, zb)
    m, q = wire.gset(d, 0)
    L = d["period"]
    at = d["atoms"][1]
    sp = d["species"][at["species"]]
    X0, Y0, Z0 = at["pos"]
    # y: one image over the whole line (the Bloch phases of the other images cancel in
    # |beta><beta|, so the matrix element per period takes the full-line integral),
    # trapezoid rule on a wide window (spectrally accurate for the Gaussian)
    yy = np.linspace(Y0 - 14.0, Y0 + 14.0, 6001)
    for kind_idx, kind in enumerate(("s", "px", "py", "pz")):
        p = 4 + kind_idx  # second atom's projectors
        a = sp["alpha_s"] if kind == "s" else sp["alpha_p"]
        cs, cp = (2 * a / math.pi) ** 0.75, (2 * a / math.pi) ** 0.75 * 2 * math.sqrt(a)
        c = cs if kind == "s" else cp
        for gi in (0, len(m) // 2, len(m) - 1):
            dy = yy - Y0
            fy = np.exp(-a * dy * dy) * (dy if kind == "py" else 1.0)
            ypart = np.sum(np.exp(-1j * q[gi] * yy) * fy) * (yy[1] - yy[0]) / math.sqrt(L)
            for i, j in ((1, 2), (3, 3), (xb.nb - 2, 1)):
                def fx(x):
                    return xb.values([x])[0, i] * np.exp(-a * (x - X0) ** 2) * ((x - X0) if kind == "px" else 1.0)

                def fz(z):
                    return zb.values([z])[0, j] * np.exp(-a * (z - Z0) ** 2) * ((z - Z0) if kind == "pz" else 1.0)

                bx = d["breakpoints_x"]
                bz = d["breakpoints_z"]
                xpart = sum(scipy.integrate.quad(fx, lo, hi, epsabs=1e-14)[0] for lo, hi in zip(bx[:-1], bx[1:]))
                zpart = sum(scipy.integrate.quad(fz, lo, hi, epsabs=1e-14)[0] for lo, hi in zip(bz[:-1], bz[1:]))
                ref = c * ypart * xpart * zpart
                got = F[p, gi] * X[p, i] * Z[p, j]
                assert abs(got - ref) < 1e-10 * max(abs(ref), 1e-3 * c), (kind, gi, i, j, got, ref)


def test_time_reversal_pairs():
    d = workloads.wire_micro(seed=5, nint=6, ecut=7.0, kfrac=0.21)
    dm = dict(d, kpts=[-0.21])
    w1 = wire.lowest(d, 0, 10)[0]
    w2 = wire.lowest(dm, 0, 10)[0]
    assert np.max(np.abs(w1 - w2)) < 1e-11


@pytest.mark.parametrize("seed,ny", [(6, 8), (7, 12)])
def test_matrix_free_and_rows_match_dense(seed, ny):
    d = workloads.wire_micro(seed=seed, nint=6, ecut=7.0, ny=ny, kfrac=0.13)
    pr = wire.WireProblem(d, 0)
    H, S = pr.hamiltonian(), pr.overlap()
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((3, pr.n)) + 1j * rng.standard_normal((3, pr.n))
    mf = wire.WireMatFree(d, 0)
    ref_h = (H @ x.T).T
    ref_s = (S @ x.T).T
    assert np.max(np.abs(mf.apply(x) - ref_h)) < 1e-12 * np.max(np.abs(ref_h))
    assert np.max(np.abs(mf.apply_s(x) - ref_s)) < 1e-12 * np.max(np.abs(ref_s))
    rows = [(0, 0, 0), (pr.ng - 1, pr.nx - 1, pr.nz - 1), (pr.ng // 2, 3, 2), (1, pr.nx // 2, pr.nz - 2)]
    rr = wire.WireRows(d, 0)
    xh, xs = rr.apply_rows(x[0].reshape(pr.ng, pr.nx, pr.nz), rows)
    idx = [(g * pr.nx + i) * pr.nz + j for g, i, j in rows]
    assert np.max(np.abs(xh - ref_h[0, idx])) < 1e-12 * np.max(np.abs(ref_h))
    assert np.max(np.abs(xs - ref_s[0, idx])) < 1e-12 * np.max(np.abs(ref_s))


def test_overlap_positive_definite_and_hamiltonian_hermitian():
    d = workloads.wire_micro(seed=8, nint=5, ecut=6.0)
    pr = wire.WireProblem(d, 0)
    H, S = pr.hamiltonian(), pr.overlap()
    assert np.max(np.abs(H - H.conj().T)) < 1e-13 * np.max(np.abs(H))
    assert np.min(np.linalg.eigvalsh(S)) > 0
