"""hpsi_apply_noalloc (work buffers in the library's fixed per-GPU array) against
hpsi_apply (work buffers allocated per k-point), through the C ABI: two calls in
a row, the second with a smaller input, and a call whose bands are split into
several groups; then a band too large for the array is refused."""
import numpy as np
import pytest
import torch

from paper_1406_4960_amd import mbks, workloads
from tests.helpers import random_lib_block, rel_err

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _both(p, ik, x, prec):
    ct = torch.complex128 if prec == "fp64" else torch.complex64
    xt = torch.from_numpy(x).to(DEV).to(ct)
    y_ref = torch.full_like(xt, complex(5.0, 5.0))
    y_na = torch.full_like(xt, complex(7.0, 7.0))
    p.hpsi(ik, xt, y_ref, prec)
    p.hpsi_noalloc(ik, xt, y_na, prec)
    torch.cuda.synchronize()
    return y_na.to(torch.complex128).cpu().numpy(), y_ref.to(torch.complex128).cpu().numpy()


def test_noalloc_matches_hpsi_two_calls_then_smaller():
    d = workloads.graphene()
    print("[case] noalloc graphene k0 32 bands fp64, then k1 6 bands fp32", flush=True)
    p = mbks.Problem(d, device=0)
    dm = p.dims(0)
    got, ref = _both(p, 0, random_lib_block(81, 32, dm["nb"], dm["ng"], dm["ld"]), "fp64")
    print("fp64 rel err", rel_err(got, ref), "bit-equal", np.array_equal(got, ref), flush=True)
    assert rel_err(got, ref) < 1e-12
    dm1 = p.dims(1)
    got, ref = _both(p, 1, random_lib_block(82, 6, dm1["nb"], dm1["ng"], dm1["ld"]), "fp32")
    print("fp32 rel err", rel_err(got, ref), flush=True)
    assert rel_err(got, ref) < 1e-6
    assert np.all(got[:, :, dm1["ng"]:] == 0)
    p.close()


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_noalloc_band_groups_on_the_surface_slab(prec):
    # one band of the 128x64 surface slab needs ~50 MiB of FP64 work space: 12 bands
    # run as several groups through the fixed array
    d = workloads.surface()
    print(f"[case] noalloc surface k2 12 bands {prec}", flush=True)
    p = mbks.Problem(d, device=0)
    dm = p.dims(2)
    got, ref = _both(p, 2, random_lib_block(83, 12, dm["nb"], dm["ng"], dm["ld"]), prec)
    print(prec, "rel err", rel_err(got, ref), flush=True)
    assert rel_err(got, ref) < (1e-12 if prec == "fp64" else 1e-6)
    p.close()


def test_noalloc_refuses_a_band_larger_than_the_array():
    # 128x64 grid with 1,200 knot intervals: one FP64 band needs > 256 MiB
    d = dict(workloads.surface(), breakpoints=workloads.graded_breakpoints(-30.0, 30.0, 1200), atoms=[],
             species=[], kpts=[[0.0, 0.0]])
    p = mbks.Problem(d, device=0)
    dm = p.dims(0)
    x = torch.zeros((1, dm["nb"], dm["ld"]), dtype=torch.complex128, device=DEV)
    with pytest.raises(mbks.MbError, match="MiB"):
        p.hpsi_noalloc(0, x, torch.empty_like(x))
    p.close()
