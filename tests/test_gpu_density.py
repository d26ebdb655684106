"""GPU parity of the electron density and the Hartree potential (Sec. II.B.1: charge
density and the Coulomb potential in the (z, g) form) against the oracle:

* density_accumulate against the oracle's explicit sums on a small cell (every plane,
  FP64 and FP32 vectors, accumulation over two calls), on the graphene-like slab and the
  128x64 surface slab at sampled Gauss planes, and the total charge against
  sum_b w_b c_b^H S c_b with the library's own S; on the 128x64 grid the lane-split
  kernel against the LDS-transform kernel on every plane;
* hartree_potential against the oracle's direct double sums over Gauss points (every
  plane and grid frequency on a small cell and on the graphene-like slab's 36x36 grid);
  on the 128x64 grid V(z, g) at sampled frequencies against the oracle's z sums, and the
  potential against the inverse transform of V(z, g); in place (vh = rho) equals out of
  place.
"""
import numpy as np
import pytest
import torch

from oracle import density, lattice
from oracle.bspline import ZBasis
from paper_1406_4960_amd import mbks, workloads
from tests.helpers import gperm, random_lib_block, rel_err

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _oracle_vectors(x_lib, perm, ng_o):
    nv, nb, _ = x_lib.shape
    out = np.zeros((nv, ng_o, nb), dtype=np.complex128)
    out[:, perm, :] = np.transpose(x_lib[:, :, :len(perm)], (0, 2, 1))
    return out


def _setup(d, seed, nv, ik=0):
    p = mbks.Problem(d, device=0)
    dm = p.dims(ik)
    m, _ = p.gvectors(ik)
    mo = lattice.gset(d, ik)[0]
    perm = gperm(m, mo)
    x = random_lib_block(seed, nv, dm["nb"], dm["ng"], dm["ld"])
    return p, dm, perm, len(mo), x


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_density_matches_oracle_small_cell(prec):
    d = workloads.micro(seed=5, natoms=2, mmax=2, nint=11, grid=8, kfrac=(0.23, -0.31))
    print(f"[case] density micro {prec}", flush=True)
    p, dm, perm, ngo, x = _setup(d, 81, 3)
    w = np.array([2.0, 1.0, 0.5])
    ct = torch.complex128 if prec == "fp64" else torch.complex64
    xt = torch.from_numpy(x).to(DEV).to(ct)
    N1, N2 = d["grid"]
    rho = torch.zeros((dm["nzq"], N1, N2), dtype=torch.float64, device=DEV)
    wt = torch.from_numpy(w).to(DEV)
    p.density(0, xt, wt, rho, prec)
    r1 = rho.cpu().numpy().copy()
    p.density(0, xt, wt, rho, prec)
    r2 = rho.cpu().numpy()
    p.close()
    x_used = x.astype(np.complex64).astype(np.complex128) if prec == "fp32" else x
    ref = density.density_grid(d, 0, _oracle_vectors(x_used, perm, ngo), w)
    err = rel_err(r1, ref)
    print(f"rel err {err:.2e}", flush=True)
    assert err < 1e-12
    assert rel_err(r2, 2 * ref) < 1e-12


def test_density_graphene_slab_planes_and_total_charge():
    d = workloads.graphene()
    print("[case] density graphene sampled planes", flush=True)
    p, dm, perm, ngo, x = _setup(d, 82, 4, ik=1)
    w = np.array([2.0, 2.0, 1.0, 0.25])
    xt = torch.from_numpy(x).to(DEV)
    N1, N2 = d["grid"]
    rho = torch.zeros((dm["nzq"], N1, N2), dtype=torch.float64, device=DEV)
    p.density(1, xt, torch.from_numpy(w).to(DEV), rho)
    sx = torch.empty_like(xt)
    p.spsi(1, xt, sx)
    torch.cuda.synchronize()
    norms = torch.einsum("bij,bij->b", xt.conj(), sx).real.cpu().numpy()
    r = rho.cpu().numpy()
    p.close()
    planes = [0, 1, 100, 197, dm["nzq"] - 1]
    ref = density.density_grid(d, 1, _oracle_vectors(x, perm, ngo), w, planes=planes)
    assert rel_err(r[planes], ref) < 1e-12
    zb = ZBasis(d["breakpoints"], d["order"], d["nq"])
    area = lattice.cell_area(d["a1"], d["a2"])
    total = float(np.sum(zb.wq[:, None, None] * r) * area / (N1 * N2))
    assert abs(total - float(np.sum(w * norms))) < 1e-11 * total


def test_density_surface_slab_planes():
    d = workloads.surface()
    print("[case] density surface sampled planes", flush=True)
    p, dm, perm, ngo, x = _setup(d, 83, 2)
    w = np.array([1.0, 0.5])
    xt = torch.from_numpy(x).to(DEV).to(torch.complex64)
    N1, N2 = d["grid"]
    rho = torch.zeros((dm["nzq"], N1, N2), dtype=torch.float64, device=DEV)
    p.density(0, xt, torch.from_numpy(w).to(DEV), rho, "fp32")
    r = rho.cpu().numpy()
    p.close()
    planes = [0, 577, dm["nzq"] - 1]
    x_used = x.astype(np.complex64).astype(np.complex128)
    ref = density.density_grid(d, 0, _oracle_vectors(x_used, perm, ngo), w, planes=planes)
    assert rel_err(r[planes], ref) < 1e-12


@pytest.mark.parametrize("cfg", ["micro", "graphene"])
def test_hartree_matches_oracle(cfg):
    if cfg == "micro":
        d = workloads.micro(seed=5, natoms=2, mmax=2, nint=11, grid=8, kfrac=(0.23, -0.31))
    else:
        d = workloads.graphene()
    print(f"[case] hartree {cfg}", flush=True)
    p = mbks.Problem(d, device=0)
    nzq = p.dims(0)["nzq"]
    N1, N2 = d["grid"]
    rng = np.random.default_rng(91)
    rho = rng.uniform(0.0, 1.0, (nzq, N1, N2))
    rt = torch.from_numpy(rho).to(DEV)
    vh = torch.empty_like(rt)
    vzg = torch.empty((nzq, N1, N2), dtype=torch.complex128, device=DEV)
    p.hartree(rt, vh, vzg)
    torch.cuda.synchronize()
    v_gpu, vzg_gpu = vh.cpu().numpy(), vzg.cpu().numpy()
    # in place: the potential overwrites the density
    r2 = rt.clone()
    p.hartree(r2, r2)
    torch.cuda.synchronize()
    assert rel_err(r2.cpu().numpy(), v_gpu) < 1e-14
    p.close()
    v_ref, vzg_ref = density.hartree_grid(d, rho, return_zg=True)
    e1, e2 = rel_err(vzg_gpu, vzg_ref), rel_err(v_gpu, v_ref.real)
    print(f"rel err V(z,g) {e1:.2e}, V(rho,z) {e2:.2e}", flush=True)
    assert e1 < 1e-11 and e2 < 1e-11


def test_hartree_surface_grid_sampled_frequencies():
    d = workloads.surface()
    print("[case] hartree surface sampled", flush=True)
    p = mbks.Problem(d, device=0)
    nzq = p.dims(0)["nzq"]
    N1, N2 = d["grid"]
    rng = np.random.default_rng(92)
    rho = rng.uniform(0.0, 1.0, (nzq, N1, N2))
    rt = torch.from_numpy(rho).to(DEV)
    vh = torch.empty_like(rt)
    vzg = torch.empty((nzq, N1, N2), dtype=torch.complex128, device=DEV)
    p.hartree(rt, vh, vzg)
    torch.cuda.synchronize()
    vz = vzg.cpu().numpy()
    v = vh.cpu().numpy()
    p.close()
    _, gn = density.grid_g(d)
    picks = [(0, 0), (1, 0), (0, 1), (N1 // 2, N2 // 2), (N1 - 1, 3), (17, N2 - 5)]
    j1 = np.arange(N1)
    j2 = np.arange(N2)
    for a, b in picks:
        ph = np.exp(2j * np.pi * (a * j1[:, None] / N1 + b * j2[None, :] / N2))
        rg = np.einsum("qab,ab->q", rho, ph) / (N1 * N2)
        ref = density.coulomb_zg(d, rg[:, None], np.array([gn[a, b]]))[:, 0]
        assert rel_err(vz[:, a, b], ref) < 1e-11, (a, b)
    # the potential is the inverse transform of V(z, g) (real part)
    for q in (0, 600, nzq - 1):
        inv = np.fft.fft2(vz[q]).real  # sum_g V e^{-i g.rho}
        assert rel_err(v[q], inv) < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_density_plane_kernel_matches_generic_kernel(monkeypatch, prec):
    # the 128x64 grid's lane-split density kernel against the LDS-transform kernel on
    # every Gauss plane of the surface slab (6 bands), accumulating into a non-zero density
    d = workloads.surface()
    print(f"[case] density plane vs generic {prec}", flush=True)
    p = mbks.Problem(d, device=0)
    dm = p.dims(0)
    x = random_lib_block(84, 6, dm["nb"], dm["ng"], dm["ld"])
    ct = torch.complex128 if prec == "fp64" else torch.complex64
    xt = torch.from_numpy(x).to(DEV).to(ct)
    w = torch.tensor([2.0, 1.5, 1.0, 0.5, 0.25, 0.125], dtype=torch.float64, device=DEV)
    N1, N2 = d["grid"]
    base = torch.from_numpy(np.random.default_rng(85).uniform(0.0, 1.0, (dm["nzq"], N1, N2))).to(DEV)
    out = {}
    for kern in ("default", "generic"):
        if kern == "generic":
            monkeypatch.setenv("MBKS_DENSITY_KERNEL", "generic")
        rho = base.clone()
        p.density(0, xt, w, rho, prec)
        torch.cuda.synchronize()
        out[kern] = rho.cpu().numpy()
    p.close()
    assert rel_err(out["default"], out["generic"]) < 1e-13
