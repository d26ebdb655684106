"""GPU parity beyond random-vector products:

* s_solve against the oracle's overlap, element by element (S = I_G (x) S_z,
  generalized form of Sec. II.B.2);
* lanczos_lowest with the plain S^{-1} H Krylov operator (sigma <= 0, the
  repeated-H sequence of Sec. II.C for the generalized problem) against the
  oracle's eigenvalues;
* exactly solvable potentials pushed through the library's grid path with
  mb_problem_set_potential: a plane-constant harmonic well (eps = 1/2|k+G|^2 +
  omega (n + 1/2)) and a separable V1(rho) + V2(z) (eps = in-plane eigenvalue +
  z eigenvalue), against their closed forms built without the library.
"""
import numpy as np
import pytest
import scipy.linalg
import torch

from oracle import lattice, operators, solve
from oracle.bspline import ZBasis
from paper_1406_4960_amd import mbks, workloads
from tests.helpers import gperm, lib_to_oracle, oracle_to_lib, random_lib_block, rel_err

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _lib_perm(p, d, ik=0):
    m, _ = p.gvectors(ik)
    return gperm(m, lattice.gset(d, ik)[0])


@pytest.mark.parametrize("cfg,prec", [("micro", "fp64"), ("micro", "fp32"), ("graphene", "fp64"),
                                      ("graphene", "fp32")])
def test_s_solve_matches_oracle_overlap(cfg, prec):
    # x = S^{-1} r with S the oracle's overlap: dense S on the small cell; on the
    # graphene-like slab (n = 39,000) the oracle's S_z per G, since S = I_G (x) S_z
    if cfg == "micro":
        d = workloads.micro(seed=3, natoms=2, mmax=2, nint=11, grid=8)
    else:
        d = workloads.graphene()
    print(f"[case] s_solve vs oracle {cfg} {prec}", flush=True)
    p = mbks.Problem(d, device=0)
    ik = 0
    dm = p.dims(ik)
    perm = _lib_perm(p, d, ik)
    r = random_lib_block(51, 3, dm["nb"], dm["ng"], dm["ld"])
    ct = torch.complex128 if prec == "fp64" else torch.complex64
    rt = torch.from_numpy(r).to(DEV).to(ct)
    xt = torch.full_like(rt, complex(3.0, 3.0))
    p.s_solve(ik, rt, xt, prec)
    torch.cuda.synchronize()
    x = xt.to(torch.complex128).cpu().numpy()
    p.close()
    r_used = r.astype(np.complex64).astype(np.complex128) if prec == "fp32" else r
    if cfg == "micro":
        S = operators.Problem(d, ik).overlap()
        ro = lib_to_oracle(r_used, dm["ng"], perm)
        ref = oracle_to_lib(scipy.linalg.solve(S, ro.T).T, dm["nb"], dm["ng"], dm["ld"], perm)
    else:
        Sz = ZBasis(d["breakpoints"], d["order"], d["nq"]).overlap()
        ref = np.zeros_like(r)
        for b in range(r.shape[0]):
            ref[b, :, :dm["ng"]] = scipy.linalg.solve(Sz, r_used[b, :, :dm["ng"]])
    # condition number of S_z times the working precision
    cond = np.linalg.cond(ZBasis(d["breakpoints"], d["order"], d["nq"]).overlap())
    tol = (1e-14 if prec == "fp64" else 1e-6) * cond
    print(f"cond(S_z) {cond:.1f}, rel err {rel_err(x, ref):.2e}, bar {tol:.1e}", flush=True)
    assert rel_err(x, ref) < tol
    assert np.all(x[:, :, dm["ng"]:] == 0)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("fp32", 1e-6)])
def test_lanczos_plain_inverse_overlap_operator(prec, tol):
    # sigma <= 0: Krylov vectors grown with K = S^{-1} (the generalized problem's
    # repeated application of S^{-1} H) instead of the kinetic preconditioner
    d = workloads.micro(seed=3, natoms=2, mmax=2, nint=11, grid=8, kfrac=(0.23, -0.31))
    print(f"[case] lanczos sigma=0 {prec}", flush=True)
    nev = 6
    ref = solve.solve_problem(d, 0, nev=nev)[3]
    p = mbks.Problem(d, device=0)
    o = p.default_opts()
    o.sigma = 0.0
    o.max_iter = 400
    eig, x, info, st = p.lanczos_lowest(0, nev, prec, opts=o)
    print(info, flush=True)
    assert st == 0
    assert np.max(np.abs(eig - ref)) < tol
    h = torch.empty_like(x)
    s = torch.empty_like(x)
    p.hpsi(0, x, h)
    p.spsi(0, x, s)
    res = torch.linalg.vector_norm((h - torch.from_numpy(eig).to(DEV).reshape(-1, 1, 1) * s).reshape(nev, -1), dim=1)
    assert float(res.max()) < 1e-6
    p.close()


def _grid_rho(d):
    N1, N2 = d["grid"]
    a1, a2 = np.array(d["a1"]), np.array(d["a2"])
    f1 = np.arange(N1)[:, None] / N1
    f2 = np.arange(N2)[None, :] / N2
    return f1 * a1[0] + f2 * a2[0], f1 * a1[1] + f2 * a2[1]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-7), ("fp32", 1e-6)])
def test_harmonic_well_through_library_grid(prec, tol):
    # V = 1/2 omega^2 z^2 on every grid point of every Gauss plane (box +-15 bohr,
    # 150 intervals: box and discretisation errors < 1e-7); the library's scatter,
    # inverse FFT, multiply, forward FFT and gather must return the plane-constant
    # operator, so eps = 1/2 |k+G|^2 + omega (n + 1/2)
    omega = 1.0
    d = workloads.micro(seed=0, nonlocal_=False, mmax=1, nint=150)
    d = dict(d, atoms=[], species=[], breakpoints=workloads.uniform_breakpoints(-15, 15, 150),
             kpts=[[0.0, 0.0]])
    print(f"[case] harmonic well {prec}", flush=True)
    zq = ZBasis(d["breakpoints"], d["order"], d["nq"]).zq
    N1, N2 = d["grid"]
    v = np.broadcast_to((0.5 * omega ** 2 * zq * zq)[:, None, None], (len(zq), N1, N2))
    p = mbks.Problem(d, device=0)
    p.set_potential(v)
    nev = 6
    eig, x, info, st = p.lanczos_lowest(0, nev, prec)
    p.close()
    assert st == 0
    _, kg = lattice.gset(d, 0)
    kin = np.sort(0.5 * np.sum(kg * kg, axis=1))
    ref = np.sort((kin[:, None] + omega * (np.arange(nev) + 0.5)[None, :]).ravel())[:nev]
    print(eig, ref, flush=True)
    assert np.max(np.abs(eig - ref)) < tol


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-6)])
def test_separable_potential_through_library_grid(prec, tol):
    # V = V1(rho) + V2(z) with V1 three complex Fourier components (no inversion
    # symmetry, k != 0) sampled on the grid: eigenvalues are all sums of the
    # in-plane plane-wave problem (from V1's known coefficients) and the 1D
    # B-spline problem with V2
    d = workloads.micro(seed=6, nonlocal_=False, mmax=2, nint=13, kfrac=(0.13, 0.29), grid=16)
    d = dict(d, atoms=[], species=[])
    print(f"[case] separable V1(rho)+V2(z) {prec}", flush=True)
    b1, b2 = lattice.reciprocal(d["a1"], d["a2"])
    comps = {(1, 0): 0.31 + 0.17j, (0, 1): -0.22 + 0.05j, (1, 1): 0.08 - 0.27j}
    X, Y = _grid_rho(d)
    v1 = np.zeros(X.shape)
    for (m1, m2), c in comps.items():
        g = m1 * b1 + m2 * b2
        v1 += 2.0 * np.real(c * np.exp(1j * (g[0] * X + g[1] * Y)))
    omega = 0.8
    zb = ZBasis(d["breakpoints"], d["order"], d["nq"])
    v = v1[None, :, :] + (0.5 * omega ** 2 * zb.zq ** 2)[:, None, None]
    p = mbks.Problem(d, device=0)
    p.set_potential(v)
    nev = 10
    eig, x, info, st = p.lanczos_lowest(0, nev, prec)
    p.close()
    assert st == 0
    coef = dict(comps)
    for (m1, m2), c in comps.items():
        coef[(-m1, -m2)] = np.conj(c)
    m, kg = lattice.gset(d, 0)
    Hin = np.diag(0.5 * np.sum(kg * kg, axis=1)).astype(complex)
    for a in range(len(m)):
        for b in range(len(m)):
            Hin[a, b] += coef.get((int(m[a, 0] - m[b, 0]), int(m[a, 1] - m[b, 1])), 0.0)
    ein = np.linalg.eigvalsh(Hin)
    A = 0.5 * zb.deriv_overlap() + zb.local(0.5 * omega ** 2 * zb.zq ** 2)
    ez = scipy.linalg.eigh(A, zb.overlap(), eigvals_only=True)[:nev]
    ref = np.sort((ein[:, None] + ez[None, :]).ravel())[:nev]
    print(eig - ref, flush=True)
    assert np.max(np.abs(eig - ref)) < tol
