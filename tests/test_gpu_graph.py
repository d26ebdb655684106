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


def test_reserved_locked_buffers_keep_a_captured_graph_valid():
    # a graph captured after mb_problem_reserve(lock) stays valid across a solve on the
    # same k-point (which would otherwise size the work buffers for its own blocks),
    # and a call that needs more than the reserved bands is refused instead of
    # reallocating them
    print("[case] graph with reserved, locked work buffers", flush=True)
    d = workloads.tiny()
    p = mbks.Problem(d, device=0)
    dm = p.dims(0)
    p.reserve(0, 24, lock=True)
    x = torch.from_numpy(random_lib_block(75, 4, dm["nb"], dm["ng"], dm["ld"])).to(DEV)
    y = torch.empty_like(x)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        p.hpsi(0, x, y)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        p.hpsi(0, x, y)
    o = p.default_opts()
    o.extra = 4
    eig, xv, info, st = p.lanczos_lowest(0, 8, "fp64", opts=o)  # H on up to 8 + 4 + 2 vectors
    assert st == 0
    big = torch.zeros((40, dm["nb"], dm["ld"]), dtype=torch.complex128, device=DEV)  # > 24 + 1/8 headroom
    with pytest.raises(mbks.MbError, match="locked"):
        p.hpsi(0, big, torch.empty_like(big))
    for rep in range(3):
        x.mul_(complex(0.5, 0.1 * (rep + 1)))
        g.replay()
        torch.cuda.synchronize()
        ye = torch.empty_like(x)
        p.hpsi(0, x, ye)
        torch.cuda.synchronize()
        assert torch.equal(y, ye), rep
    del g
    p.reserve(0, 0, lock=False)  # unlocked: larger calls grow the buffers again
    p.hpsi(0, big, torch.empty_like(big))
    torch.cuda.synchronize()
    p.close()


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_bound_batch_graph_replays_match_eager(prec):
    # hpsi_apply_batched_bound captured once: every replay (with eager work on the inputs
    # in between) equals an eager hpsi_apply_batched call on the same inputs; the list mixes
    # grids, k-points and projector counts (BF16x3 takes the matrix-core projections with
    # the bound partial buffers)
    print(f"[case] graph bound batch {prec}", flush=True)
    probs = [mbks.Problem(workloads.graphene(), device=0), mbks.Problem(workloads.tiny(), device=0),
             mbks.Problem(workloads.batched_member(12), device=0)]
    items = [(probs[0], 0), (probs[0], 1), (probs[1], 0), (probs[2], 0)]
    ct = torch.complex128 if prec == "fp64" else torch.complex64
    xs, ys = [], []
    for t, (pr, ik) in enumerate(items):
        dm = pr.dims(ik)
        xs.append(torch.from_numpy(random_lib_block(80 + t, 3 + t, dm["nb"], dm["ng"], dm["ld"])).to(DEV).to(ct))
        ys.append(torch.empty_like(xs[-1]))
    b = mbks.Batch(items)
    b.bind(xs, ys, prec)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.hpsi_bound()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.hpsi_bound()
    for rep in range(3):
        for x in xs:
            x.mul_(complex(0.5, 0.2 * (rep + 1)))
        g.replay()
        torch.cuda.synchronize()
        ye = [torch.empty_like(x) for x in xs]
        b.hpsi(xs, ye, prec)
        torch.cuda.synchronize()
        for t in range(len(items)):
            assert torch.equal(ys[t], ye[t]), (rep, t)
            assert float(torch.max(torch.abs(ye[t]))) > 0
    del g
    b.close()
    for pr in probs:
        pr.close()
