"""Pins of the oracle's B-spline layer (Sec. II.A, eqs. 1-3) against a library
routine, closed forms and exactness properties."""
import math

import numpy as np
import pytest
import scipy.interpolate

from oracle import bspline
from paper_1406_4960_amd import workloads

ORDER = 4


def _knot_sets():
    rng = np.random.default_rng(3)
    yield np.array(workloads.uniform_breakpoints(-15.0, 15.0, 39))
    yield np.array(workloads.graded_breakpoints(-20.0, 20.0, 79))
    yield np.sort(rng.uniform(-3.0, 5.0, size=12))


@pytest.mark.parametrize("bp", list(_knot_sets()))
@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_cox_de_boor_matches_scipy(bp, order):
    tau = bspline.clamped_knots(bp, order)
    z = np.linspace(bp[0], bp[-1], 997)[:-1]
    ours = bspline.bspline_values(tau, order, z)
    ref = scipy.interpolate.BSpline.design_matrix(z, tau, order - 1).toarray()
    assert np.max(np.abs(ours - ref)) < 1e-13
    d_ours = bspline.bspline_derivs(tau, order, z)
    nf = len(tau) - order
    d_ref = np.zeros_like(d_ours)
    for i in range(nf):
        c = np.zeros(nf)
        c[i] = 1.0
        d_ref[:, i] = scipy.interpolate.BSpline(tau, c, order - 1).derivative()(z)
    assert np.max(np.abs(d_ours - d_ref)) < 1e-10 * max(1.0, np.max(np.abs(d_ref)))


@pytest.mark.parametrize("bp", list(_knot_sets()))
def test_partition_of_unity(bp):
    tau = bspline.clamped_knots(bp, ORDER)
    z = np.concatenate([np.linspace(bp[0], bp[-1], 501), bp])
    B = bspline.bspline_values(tau, ORDER, z)
    dB = bspline.bspline_derivs(tau, ORDER, z[:-1])
    assert np.max(np.abs(B.sum(axis=1) - 1.0)) < 1e-14
    assert np.max(np.abs(dB.sum(axis=1))) < 1e-11
    assert np.all(B >= -1e-15)


def test_uniform_cubic_values_at_knots():
    # textbook: a uniform cubic B-spline takes 1/6, 2/3, 1/6 at its inner knots
    bp = np.arange(0.0, 11.0)
    tau = bspline.clamped_knots(bp, ORDER)
    B = bspline.bspline_values(tau, ORDER, bp)
    i = 6  # an interior spline with support [tau_6, tau_10] = [3, 7]
    assert tau[i] == 3.0 and tau[i + 4] == 7.0
    assert B[4, i] == pytest.approx(1 / 6, abs=1e-15)
    assert B[5, i] == pytest.approx(2 / 3, abs=1e-15)
    assert B[6, i] == pytest.approx(1 / 6, abs=1e-15)
    assert B[3, i] == 0.0 and B[7, i] == 0.0


@pytest.mark.parametrize("nq", [1, 3, 5, 6])
def test_gauss_rule_exact_for_polynomials(nq):
    bp = np.array(workloads.graded_breakpoints(-4.0, 6.0, 9))
    zq, wq = bspline.gauss_rule(bp, nq)
    assert np.all(wq > 0)
    for deg in range(2 * nq):
        exact = (bp[-1] ** (deg + 1) - bp[0] ** (deg + 1)) / (deg + 1)
        assert np.sum(wq * zq ** deg) == pytest.approx(exact, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("bp", list(_knot_sets()))
def test_spline_integrals(bp):
    # int B_i dz = (tau_{i+k} - tau_i) / k for the full set; so full S_z row sums
    # equal it and full D_z row sums vanish
    tau = bspline.clamped_knots(bp, ORDER)
    zq, wq = bspline.gauss_rule(bp, 5)
    B = bspline.bspline_values(tau, ORDER, zq)
    dB = bspline.bspline_derivs(tau, ORDER, zq)
    ints = B.T @ wq
    nf = len(tau) - ORDER
    closed = np.array([(tau[i + ORDER] - tau[i]) / ORDER for i in range(nf)])
    assert np.max(np.abs(ints - closed)) < 1e-13
    S = (B * wq[:, None]).T @ B
    D = (dB * wq[:, None]).T @ dB
    assert np.max(np.abs(S.sum(axis=1) - closed)) < 1e-13
    assert np.max(np.abs(D.sum(axis=1))) < 1e-11 * np.max(np.abs(D))


def test_uniform_overlap_closed_form():
    # Gram matrix of uniform cubic B-splines = order-8 B-spline at the integers:
    # h * (2416, 1191, 120, 1) / 5040 on the diagonals 0..3
    h = 0.7
    bp = np.arange(0, 21) * h
    zb = bspline.ZBasis(bp, ORDER, 5)
    S = zb.overlap()
    i = 10
    ref = h * np.array([2416, 1191, 120, 1]) / 5040.0
    assert np.max(np.abs(S[i, i:i + 4] - ref)) < 1e-15
    assert np.all(S[i, i + 4:] == 0.0)


@pytest.mark.parametrize("bp", list(_knot_sets()))
def test_overlap_banded_spd(bp):
    zb = bspline.ZBasis(bp, ORDER, 5)
    S = zb.overlap()
    D = zb.deriv_overlap()
    assert zb.nb == len(bp) + ORDER - 2 - 2
    for M in (S, D):
        assert np.max(np.abs(M - M.T)) <= 1e-15 * np.max(np.abs(M))
        i, j = np.nonzero(M)
        assert np.max(np.abs(i - j)) <= ORDER - 1
    assert np.linalg.eigvalsh(S).min() > 0
    np.linalg.cholesky(S)
    # hard walls: every kept spline vanishes at both ends
    Bend = zb.values(np.array([bp[0], bp[-1]]))
    assert np.max(np.abs(Bend)) == 0.0


def test_bilinear_forms_on_polynomials():
    # f(z) = (z - z0)(z1 - z)(1 + z/7) lies in the hard-wall cubic spline space;
    # its L2 projection reproduces it, so c^T S c and c^T D c equal the exact
    # integrals of f^2 and f'^2.
    bp = np.array(workloads.graded_breakpoints(-5.0, 5.0, 17))
    zb = bspline.ZBasis(bp, ORDER, 5)
    z0, z1 = bp[0], bp[-1]
    P = np.polynomial.Polynomial([-z0, 1.0]) * np.polynomial.Polynomial([z1, -1.0]) \
        * np.polynomial.Polynomial([1.0, 1.0 / 7.0])
    b = zb.weighted(P(zb.zq))
    S = zb.overlap()
    c = np.linalg.solve(S, b)
    zt = np.linspace(z0, z1, 301)
    assert np.max(np.abs(zb.values(zt) @ c - P(zt))) < 1e-12
    I2 = (P * P).integ()
    Id = (P.deriv() * P.deriv()).integ()
    assert c @ S @ c == pytest.approx(I2(z1) - I2(z0), rel=1e-12)
    assert c @ zb.deriv_overlap() @ c == pytest.approx(Id(z1) - Id(z0), rel=1e-12)


def test_graded_breakpoints_denser_in_centre():
    bp = np.array(workloads.graded_breakpoints(-20.0, 20.0, 79))
    h = np.diff(bp)
    assert h[39] == pytest.approx(20.0 * 2.0 / math.sinh(2.0) * (2.0 / 79), rel=0.02)
    assert h[0] / h[39] == pytest.approx(math.cosh(2.0), rel=0.05)
