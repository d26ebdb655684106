"""hpsi_apply and spsi_apply inside a captured HIP graph (torch.cuda.CUDAGraph over
the library's stream argument): every replay, with eager work on the inputs in
between, must give exactly what an eager call gives on the same inputs (the same
kernels run in the same order)."""
import numpy as np
import pytest
import torch

from paper_1406_4960_amd import mbks, workloads
from tests.helpers import random_lib_block

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_hpsi_graph_replays_match_eager(prec):
    print(f"[case] graph hpsi {prec}", flush=True)
    d = workloads.graphene()
    p = mbks.Problem(d, device=0)
    ct = torch.complex128 if prec == "fp64" else torch.complex64
    xs, ys, ss = [], [], []
    for ik in (0, 1):
        dm = p.dims(ik)
        xs.append(torch.from_numpy(random_lib_block(70 + ik, 8, dm["nb"], dm["ng"], dm["ld"])).to(DEV).to(ct))
        ys.append(torch.empty_like(xs[-1]))
        ss.append(torch.empty_like(xs[-1]))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for ik in (0, 1):  # warm-up outside the capture: workspaces are allocated here
            p.hpsi(ik, xs[ik], ys[ik], prec)
            p.spsi(ik, xs[ik], ss[ik], prec)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for ik in (0, 1):
            p.hpsi(ik, xs[ik], ys[ik], prec)
            p.spsi(ik, xs[ik], ss[ik], prec)
    for rep in range(3):
        for ik in (0, 1):
            xs[ik].mul_(complex(0.5, 0.25 * (rep + 1)))  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        for ik in (0, 1):
            ye, se = torch.empty_like(xs[ik]), torch.empty_like(xs[ik])
            p.hpsi(ik, xs[ik], ye, prec)
            p.spsi(ik, xs[ik], se, prec)
            torch.cuda.synchronize()
            assert torch.equal(ys[ik], ye), (rep, ik)
            assert torch.equal(ss[ik], se), (rep, ik)
            assert float(torch.max(torch.abs(ye))) > 0
    del g
    p.close()
