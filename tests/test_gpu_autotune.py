"""mb_autotune: the kernel choices it stores leave the operator unchanged (up to the
summation-order differences of the kernels, the bars of the kernel cross-checks) and
the choice it reports is one of the kernels that support the grid; the choices saved to
the cache file and loaded into a fresh handle give the same choices and the same
operator, bit for bit."""
import pytest
import torch

from paper_1406_4960_amd import mbks, workloads
from tests.helpers import random_lib_block, rel_err

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("cfg,prec,kinds", [("graphene", "fp64", {0, 2, 3}), ("graphene", "fp32", {0, 2, 3}),
                                            ("graphene_2x2", "fp32", {1, 2}), ("graphene_2x2", "fp64", {1, 2}),
                                            ("surface", "fp32", {2, 3}), ("surface", "fp64", {1, 2, 3})])
def test_autotune_keeps_operator(cfg, prec, kinds):
    print(f"[case] autotune {cfg} {prec}", flush=True)
    d = workloads.CONFIGS[cfg]()
    p = mbks.Problem(d, device=0)
    dm = p.dims(0)
    ct = torch.complex128 if prec == "fp64" else torch.complex64
    x = torch.from_numpy(random_lib_block(90, 6, dm["nb"], dm["ng"], dm["ld"])).to(DEV).to(ct)
    y0 = torch.empty_like(x)
    p.hpsi(0, x, y0, prec)
    info = p.autotune(0, 16, prec)
    print(info, flush=True)
    assert info["local_kernel"] in kinds
    assert info["candidates"] >= 2 and info["local_ms"] > 0 and info["local_default_ms"] > 0
    if prec == "fp32":
        assert info["nl_matrix_cores"] in (0, 1)
    if info["local_kernel"] != 3:
        assert info["combine_bands"] in (1, 4)
    y1 = torch.empty_like(x)
    p.hpsi(0, x, y1, prec)
    torch.cuda.synchronize()
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert rel_err(y1.to(torch.complex128).cpu().numpy(), y0.to(torch.complex128).cpu().numpy()) < tol
    p.close()


def test_autotune_bad_args():
    p = mbks.Problem(workloads.tiny(), device=0)
    with pytest.raises(mbks.MbError):
        p.autotune(3, 8)
    with pytest.raises(mbks.MbError):
        p.autotune(0, 0)
    p.close()


@pytest.mark.parametrize("cfg,prec", [("graphene", "fp32"), ("surface", "fp32"), ("graphene_2x2", "fp64")])
def test_tune_cache_round_trip(tmp_path, cfg, prec):
    print(f"[case] tune cache {cfg} {prec}", flush=True)
    d = workloads.CONFIGS[cfg]()
    path = str(tmp_path / "tune.json")
    p = mbks.Problem(d, device=0)
    info = p.autotune(0, 16, prec)
    p.tune_save(path)
    q = mbks.Problem(d, device=0)
    assert q.tune_load(path) >= 1
    a, b = p.tune_get(0, prec), q.tune_get(0, prec)
    assert a == b and a["local_kernel"] == info["local_kernel"]
    dm = p.dims(0)
    ct = torch.complex128 if prec == "fp64" else torch.complex64
    x = torch.from_numpy(random_lib_block(93, 5, dm["nb"], dm["ng"], dm["ld"])).to(DEV).to(ct)
    y0, y1 = torch.empty_like(x), torch.empty_like(x)
    p.hpsi(0, x, y0, prec)
    q.hpsi(0, x, y1, prec)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    p.close()
    q.close()
