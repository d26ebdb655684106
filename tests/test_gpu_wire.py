"""GPU parity of the 1D-periodic form (B-splines along x and z, plane waves along y;
the extension at the end of Sec. II.B.2) against the oracle of oracle/wire.py:

* hpsi_apply / spsi_apply element by element against the dense H and S on small cells
  (several y-transform lengths and lane splits, several x rounds of the local kernel,
  projectors, k off zero), FP64 and FP32, padding outputs zero;
* s_solve against a dense solve with the oracle's S; in place;
* the 3-line ribbon: H against the oracle's matrix-free form, and lanczos_lowest
  (FP64 and mixed) against the stored LAPACK eigenvalues of the oracle's dense problem;
* the 19-line ribbon at full size: sampled outputs of H and S (first, last and
  projector-window rows, every G of a row) against the oracle's row form, and the
  lowest eigenpairs' residuals measured with the oracle's rows.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg
import torch

from oracle import wire
from paper_1406_4960_amd import mbks, workloads
from tests.helpers import rel_err

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _to_oracle(x_lib, nx, nz, ng):
    # [b][i][j][ld] -> [b][(g nx + i) nz + j]
    nv = x_lib.shape[0]
    return np.transpose(x_lib[..., :ng].reshape(nv, nx, nz, ng), (0, 3, 1, 2)).reshape(nv, -1)


def _from_oracle(x, nx, nz, ng, ld):
    nv = x.shape[0]
    out = np.zeros((nv, nx, nz, ld), dtype=np.complex128)
    out[..., :ng] = np.transpose(x.reshape(nv, ng, nx, nz), (0, 2, 3, 1))
    return out


def _setup(d, ik=0):
    p = mbks.Problem(d, device=0)
    dm, wd = p.dims(ik), p.wire_dims()
    m, _ = p.gvectors(ik)
    mo, _ = wire.gset(d, ik)
    assert np.array_equal(m[:, 0], mo)
    return p, dm, wd


def _block(seed, nv, nx, nz, ng, ld):
    rng = np.random.default_rng(seed)
    x = np.zeros((nv, nx, nz, ld), dtype=np.complex128)
    x[..., :ng] = rng.uniform(-1, 1, (nv, nx, nz, ng)) + 1j * rng.uniform(-1, 1, (nv, nx, nz, ng))
    # garbage in the padding must be ignored
    x[..., ng:] = 7.0 + 3.0j
    return x


def _apply(p, name, ik, x, prec):
    ct = torch.complex128 if prec == "fp64" else torch.complex64
    xt = torch.from_numpy(x.reshape(x.shape[0], -1, x.shape[-1])).to(DEV).to(ct)
    yt = torch.full_like(xt, 5.0)
    getattr(p, name)(ik, xt, yt, prec)
    torch.cuda.synchronize()
    return yt.cpu().numpy().astype(np.complex128).reshape(x.shape)


CASES = [
    # (seed, nint, ecut, ny, kfrac): ny 8 (2 lanes per line), 12 (4 lanes, radix 3),
    # 32 (8 lanes, several x rounds), 128 (16 lanes)
    (0, 6, 6.0, 8, 0.17),
    (1, 7, 9.0, 12, -0.29),
    (2, 16, 6.0, 32, 0.41),
    (3, 9, 6.0, 128, 0.0),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_wire_h_and_s_match_dense_oracle(case, prec):
    seed, nint, ecut, ny, kf = case
    d = workloads.wire_micro(seed=seed, nint=nint, ecut=ecut, ny=ny, kfrac=kf)
    print(f"[case] wire H/S seed {seed} ny {ny} {prec}", flush=True)
    p, dm, wd = _setup(d)
    ng, ld, nx, nz = dm["ng"], dm["ld"], wd["nbx"], wd["nbz"]
    x = _block(10 + seed, 3, nx, nz, ng, ld)
    y = _apply(p, "hpsi", 0, x, prec)
    sy = _apply(p, "spsi", 0, x, prec)
    p.close()
    pr = wire.WireProblem(d, 0)
    xo = _to_oracle(x if prec == "fp64" else x.astype(np.complex64).astype(np.complex128), nx, nz, ng)
    ref_h = (pr.hamiltonian() @ xo.T).T
    ref_s = (pr.overlap() @ xo.T).T
    tol = 1e-12 if prec == "fp64" else 1e-5
    eh, es = rel_err(_to_oracle(y, nx, nz, ng), ref_h), rel_err(_to_oracle(sy, nx, nz, ng), ref_s)
    print(f"rel err H {eh:.2e} S {es:.2e}", flush=True)
    assert eh < tol and es < tol
    assert np.all(y[..., ng:] == 0) and np.all(sy[..., ng:] == 0)


def test_wire_s_solve_matches_dense_solve():
    d = workloads.wire_micro(seed=4, nint=8, ecut=6.0, ny=16, kfrac=0.3)
    print("[case] wire s_solve", flush=True)
    p, dm, wd = _setup(d)
    ng, ld, nx, nz = dm["ng"], dm["ld"], wd["nbx"], wd["nbz"]
    r = _block(21, 2, nx, nz, ng, ld)
    x = _apply(p, "s_solve", 0, r, "fp64")
    rt = torch.from_numpy(r.reshape(2, -1, ld)).to(DEV)
    p.s_solve(0, rt, rt)  # in place
    torch.cuda.synchronize()
    x2 = rt.cpu().numpy().reshape(r.shape)
    p.close()
    S = wire.WireProblem(d, 0).overlap()
    ref = scipy.linalg.solve(S, _to_oracle(r, nx, nz, ng).T, assume_a="pos").T
    assert rel_err(_to_oracle(x, nx, nz, ng), ref) < 1e-12
    assert rel_err(x2[..., :ng], x[..., :ng]) < 1e-15


def test_wire_ribbon_narrow_h_against_matrix_free_oracle():
    d = workloads.ribbon_narrow()
    print("[case] wire narrow ribbon H", flush=True)
    for ik in range(len(d["kpts"])):
        p, dm, wd = _setup(d, ik)
        ng, ld, nx, nz = dm["ng"], dm["ld"], wd["nbx"], wd["nbz"]
        x = _block(30 + ik, 4, nx, nz, ng, ld)
        y = _apply(p, "hpsi", ik, x, "fp64")
        p.close()
        ref = wire.WireMatFree(d, ik).apply(_to_oracle(x, nx, nz, ng))
        assert rel_err(_to_oracle(y, nx, nz, ng), ref) < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_wire_ribbon_narrow_eigenvalues_match_stored_oracle(prec):
    d = workloads.ribbon_narrow()
    gold = json.load(open(os.path.join(GOLD, "ribbon_narrow_eigs.json")))
    print(f"[case] wire narrow ribbon eigen {prec}", flush=True)
    p = mbks.Problem(d, device=0)
    for ik in range(len(d["kpts"])):
        ref = np.array(gold["kpoints"][str(ik)]["eps"])
        eps, x, info, _ = p.lanczos_lowest(ik, len(ref), prec)
        err = np.max(np.abs(eps - ref))
        print(f"k{ik} iters {info['iters']} max err {err:.2e} resid {info['max_resid']:.1e}", flush=True)
        assert err < 1e-8
        assert info["max_resid"] < 1e-6
    p.close()


def _ribbon_rows(d, nx, nz, ng):
    rows = [(0, 0, 0), (ng - 1, nx - 1, nz - 1), (ng // 2, nx // 2, nz // 2), (3, 1, nz - 2), (ng - 2, nx - 2, 1)]
    xb, zb = wire.basis_x(d), wire.basis_z(d)
    F, X, Z, E = wire.projector_factors(d, 0, xb, zb)
    # edges of the windows of two projectors
    for q in (0, len(E) // 2 + 1):
        xs = np.nonzero(np.abs(X[q]) > 0)[0]
        zs = np.nonzero(np.abs(Z[q]) > 0)[0]
        rows += [(1, xs[0], zs[-1]), (ng - 3, xs[-1], zs[0])]
    return rows


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_wire_ribbon_full_size_sampled_rows(prec):
    d = workloads.ribbon()
    print(f"[case] wire ribbon sampled rows {prec}", flush=True)
    p, dm, wd = _setup(d)
    ng, ld, nx, nz = dm["ng"], dm["ld"], wd["nbx"], wd["nbz"]
    x = _block(40, 3, nx, nz, ng, ld)
    y = _apply(p, "hpsi", 0, x, prec)
    sy = _apply(p, "spsi", 0, x, prec)
    p.close()
    rr = wire.WireRows(d, 0)
    rows = _ribbon_rows(d, nx, nz, ng)
    xin = x if prec == "fp64" else x.astype(np.complex64).astype(np.complex128)
    tol = 1e-11 if prec == "fp64" else 2e-5
    for b in range(3):
        xo = np.transpose(xin[b, :, :, :ng], (2, 0, 1))
        hs, ss = rr.apply_rows(xo, rows)
        got_h = np.array([y[b, i, j, g] for g, i, j in rows])
        got_s = np.array([sy[b, i, j, g] for g, i, j in rows])
        scale = np.max(np.abs(hs))
        assert np.max(np.abs(got_h - hs)) < tol * scale, (b, np.max(np.abs(got_h - hs)) / scale)
        assert np.max(np.abs(got_s - ss)) < tol * np.max(np.abs(ss))


def test_wire_ribbon_full_size_eigenpairs_by_oracle_rows():
    d = workloads.ribbon()
    print("[case] wire ribbon eigenpairs", flush=True)
    p, dm, wd = _setup(d)
    ng, ld, nx, nz = dm["ng"], dm["ld"], wd["nbx"], wd["nbz"]
    nev = 24
    o = p.default_opts()
    o.max_iter = 80
    eps, x, info, _ = p.lanczos_lowest(0, nev, "fp32", opts=o)
    xs = x.cpu().numpy().reshape(nev, nx, nz, ld)
    p.close()
    print(f"iters {info['iters']} resid {info['max_resid']:.1e}", flush=True)
    assert info["max_resid"] < 1e-6
    assert np.all(np.diff(eps) >= -1e-12)
    rr = wire.WireRows(d, 0)
    rows = _ribbon_rows(d, nx, nz, ng)
    for b in (0, nev // 2, nev - 1):
        xo = np.transpose(xs[b, :, :, :ng], (2, 0, 1))
        hs, ss = rr.apply_rows(xo, rows)
        # residual of the returned pair with the oracle's operator, on the sampled rows
        assert np.max(np.abs(hs - eps[b] * ss)) < 1e-6


def test_wire_refuses_calls_of_the_slab_only():
    d = workloads.wire_micro()
    p = mbks.Problem(d, device=0)
    dm = p.dims(0)
    x = torch.zeros((1, dm["nb"], dm["ld"]), dtype=torch.complex128, device=DEV)
    rho = torch.zeros(8, dtype=torch.float64, device=DEV)
    w = torch.ones(1, dtype=torch.float64, device=DEV)
    for call in (lambda: p.density(0, x, w, rho), lambda: p.autotune(0, 1), lambda: p.hpsi_noalloc(0, x, x.clone()),
                 lambda: mbks.Batch([(p, 0)])):
        with pytest.raises(mbks.MbError) as e:
            call()
        assert e.value.status == -1
    p.close()


@pytest.mark.parametrize("cfg", ["micro", "narrow"])
def test_wire_kernel_variants_match(cfg, monkeypatch):
    # 256-thread local kernel (half the lines per round) and 8 z rows per combine thread
    # against the defaults (512 threads, 4 rows), FP64 and FP32
    d = workloads.wire_micro(seed=2, nint=16, ecut=6.0, ny=32, kfrac=0.41) if cfg == "micro" else workloads.ribbon_narrow()
    print(f"[case] wire kernel variants {cfg}", flush=True)
    p, dm, wd = _setup(d)
    ng, ld, nx, nz = dm["ng"], dm["ld"], wd["nbx"], wd["nbz"]
    x = _block(50, 3, nx, nz, ng, ld)
    for prec in ("fp64", "fp32"):
        ref = _apply(p, "hpsi", 0, x, prec)
        monkeypatch.setenv("MBKS_WIRE_LOCAL_THREADS", "256")
        monkeypatch.setenv("MBKS_WIRE_COMBINE_ROWS", "8")
        got = _apply(p, "hpsi", 0, x, prec)
        monkeypatch.delenv("MBKS_WIRE_LOCAL_THREADS")
        monkeypatch.delenv("MBKS_WIRE_COMBINE_ROWS")
        assert rel_err(got, ref) < (1e-13 if prec == "fp64" else 1e-6)
    p.close()
