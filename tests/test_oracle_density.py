"""Pins of the oracle's density and Hartree potential (Sec. II.B.1, charge density and
the Coulomb potential in the (z, g) form) against what the mathematics fixes."""
import math

import numpy as np
import pytest
import scipy.special

from oracle import density
from oracle.bspline import ZBasis
from oracle.lattice import cell_area, gset
from paper_1406_4960_amd import workloads


def _micro(**kw):
    base = dict(seed=4, nonlocal_=False, mmax=1, nint=9, grid=8, kfrac=(0.17, -0.29))
    base.update(kw)
    return workloads.micro(**base)


def test_total_charge_equals_overlap_norms():
    # int rho d^3r = sum_b w_b c_b^H S c_b: the Gauss rule is exact for B_i B_j and the
    # grid sum is exact for e^{i(G - G').rho} (distinct G differ by less than the grid)
    d = _micro(mmax=2, grid=8)
    zb = ZBasis(d["breakpoints"], d["order"], d["nq"])
    m, _ = gset(d, 0)
    ng, nb = len(m), zb.nb
    C = np.transpose(workloads.random_block(70, 3, nb, ng), (0, 2, 1))
    w = np.array([2.0, 1.0, 0.5])
    rho = density.density_grid(d, 0, C, w)
    N1, N2 = d["grid"]
    A = cell_area(d["a1"], d["a2"])
    total = float(np.sum(zb.wq[:, None, None] * rho) * A / (N1 * N2))
    S = np.kron(np.eye(ng), zb.overlap())
    ref = sum(w[b] * np.real(np.vdot(C[b].reshape(-1), S @ C[b].reshape(-1))) for b in range(3))
    assert abs(total - ref) < 1e-12 * ref
    assert np.min(rho) >= 0.0


def test_one_basis_function_gives_flat_density():
    d = _micro()
    zb = ZBasis(d["breakpoints"], d["order"], d["nq"])
    m, _ = gset(d, 0)
    C = np.zeros((1, len(m), zb.nb), dtype=np.complex128)
    C[0, 3, 4] = 1.0
    rho = density.density_grid(d, 0, C, [1.0])
    A = cell_area(d["a1"], d["a2"])
    ref = (zb.B[:, 4] ** 2 / A)[:, None, None] * np.ones_like(rho)
    assert np.max(np.abs(rho - ref)) < 1e-15 * np.max(ref) * 10


def test_two_plane_waves_beat():
    # |e^{i G0.rho} + e^{i G1.rho}|^2 B^2 / A = 2 B^2 (1 + cos((G1 - G0).rho)) / A
    d = _micro()
    zb = ZBasis(d["breakpoints"], d["order"], d["nq"])
    m, _ = gset(d, 0)
    g0, g1, i = 1, 7, 5
    C = np.zeros((1, len(m), zb.nb), dtype=np.complex128)
    C[0, g0, i] = 1.0
    C[0, g1, i] = 1.0
    rho = density.density_grid(d, 0, C, [1.0])
    N1, N2 = d["grid"]
    A = cell_area(d["a1"], d["a2"])
    dm = m[g1] - m[g0]
    j1 = np.arange(N1)[:, None]
    j2 = np.arange(N2)[None, :]
    beat = 1.0 + np.cos(2 * math.pi * (dm[0] * j1 / N1 + dm[1] * j2 / N2))
    ref = 2.0 * (zb.B[:, i] ** 2 / A)[:, None, None] * beat[None]
    assert np.max(np.abs(rho - ref)) < 1e-14 * np.max(ref)


def _sheet_potential(z, z0, s, g):
    # (2 pi / g) int exp(-(z' - z0)^2 / s^2) exp(-g |z - z'|) dz', written with erfcx
    x = z - z0
    a = g * s / 2 - x / s
    b = g * s / 2 + x / s
    return (2 * math.pi / g) * (math.sqrt(math.pi) * s / 2) * np.exp(-x * x / (s * s)) * (
        scipy.special.erfcx(a) + scipy.special.erfcx(b))


@pytest.mark.parametrize("g", [0.4, 1.7])
def test_gaussian_sheet_against_closed_form(g):
    z0, s = 0.3, 1.2
    errs = []
    for nint in (60, 240):
        d = dict(_micro(), breakpoints=list(np.linspace(-15.0, 15.0, nint + 1)))
        zb = ZBasis(d["breakpoints"], d["order"], d["nq"])
        f = np.exp(-((zb.zq - z0) / s) ** 2)
        v = density.coulomb_zg(d, f[:, None].astype(np.complex128), np.array([g]))[:, 0]
        ref = _sheet_potential(zb.zq, z0, s, g)
        errs.append(np.max(np.abs(v - ref)) / np.max(np.abs(ref)))
    # the kink of e^{-g|z - z'|} at z' = z limits the Gauss sums to second order in the
    # knot spacing: a quarter of the spacing gives 1/16 of the error
    assert errs[1] < 1e-3
    assert 12 < errs[0] / errs[1] < 20


def test_neutral_layer_potential_jump_is_four_pi_dipole():
    # g = 0: V(z_last) - V(z_first) = 4 pi sum_q w_q z_q rho_q for a neutral rho
    # (Helmholtz), exact for the Gauss sums since |z - z'| is linear on each side
    d = dict(_micro(), breakpoints=list(np.linspace(-12.0, 12.0, 41)))
    zb = ZBasis(d["breakpoints"], d["order"], d["nq"])
    f1 = np.exp(-((zb.zq - 1.1) / 0.9) ** 2)
    f2 = np.exp(-((zb.zq + 0.7) / 1.4) ** 2)
    rho = f1 - f2 * np.sum(zb.wq * f1) / np.sum(zb.wq * f2)
    assert abs(np.sum(zb.wq * rho)) < 1e-14
    v = density.coulomb_zg(d, rho[:, None].astype(np.complex128), np.array([0.0]))[:, 0].real
    p = np.sum(zb.wq * zb.zq * rho)
    assert abs((v[-1] - v[0]) - 4 * math.pi * p) < 1e-12 * abs(4 * math.pi * p)


def test_hartree_reciprocity_and_realness():
    # <rho1, V[rho2]> = <rho2, V[rho1]> (symmetric kernel, weights on both sides), and a
    # real potential on a hexagonal cell whose Nyquist frequencies have unequal aliases
    d = dict(workloads.graphene(), grid=[12, 12], breakpoints=list(np.linspace(-8.0, 8.0, 13)))
    zb = ZBasis(d["breakpoints"], d["order"], d["nq"])
    N1, N2 = d["grid"]
    rng = np.random.default_rng(3)
    r1 = rng.uniform(0, 1, (len(zb.zq), N1, N2))
    r2 = rng.uniform(0, 1, (len(zb.zq), N1, N2))
    v1 = density.hartree_grid(d, r1)
    v2 = density.hartree_grid(d, r2)
    assert np.max(np.abs(v1.imag)) < 1e-13 * np.max(np.abs(v1.real))
    a = np.sum(zb.wq[:, None, None] * r1 * v2.real)
    b = np.sum(zb.wq[:, None, None] * r2 * v1.real)
    assert abs(a - b) < 1e-12 * abs(a)
    # the shortest alias is even in g: |g(m)| = |g(-m)|
    _, gn = density.grid_g(d)
    neg = gn[(-np.arange(N1)) % N1][:, (-np.arange(N2)) % N2]
    assert np.max(np.abs(gn - neg)) < 1e-12


def test_planted_kernel_mistake_breaks_a_pin():
    # the pins above catch a misplaced weight (outer instead of inner Gauss weight)
    d = dict(_micro(), breakpoints=list(np.linspace(-12.0, 12.0, 41)))
    zb = ZBasis(d["breakpoints"], d["order"], d["nq"])
    f1 = np.exp(-((zb.zq - 1.1) / 0.9) ** 2)
    f2 = np.exp(-((zb.zq + 0.7) / 1.4) ** 2)
    rho = f1 - f2 * np.sum(zb.wq * f1) / np.sum(zb.wq * f2)
    dz = np.abs(zb.zq[:, None] - zb.zq[None, :])
    wrong = zb.wq * ((-2 * math.pi * dz) @ rho)
    p = np.sum(zb.wq * zb.zq * rho)
    assert abs((wrong[-1] - wrong[0]) - 4 * math.pi * p) > 1e-3 * abs(4 * math.pi * p)
