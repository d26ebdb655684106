#!/usr/bin/env python3
"""Benchmark of the mixed-basis eigen-search hot path on one MI355X.

Headline workload: the large surface slab (4x2 surface cell of 19.07 x 9.534 bohr,
128x64 in-plane grid, ~3,990 G per k-point, 192 graded cubic B-splines on
[-30, 30] with 6 Gauss points per interval, 64 atoms in 8 layers with 4
Kleinman-Bylander projectors each, 4x2 Monkhorst-Pack k-points, 320 bands;
n = 766,656 per k-point), synthetic and seeded.

One step = H applied to all 8 x 320 band-vectors (one hpsi_apply per k-point on
its 320 vectors, inputs resident in HBM) in the mixed form's reduced precision:
FP32 FFTs, potential multiply, projector contractions and spline projections,
FP64 banded kinetic and overlap sums.

Printed JSON line:
  value            band-vectors of H per second over the timed steps (8 x 320 per step)
  ms_per_step      time of one step
  surface          per-stage times of a step, the BF16x3 step, FP64 hpsi_apply on
                   k-point 0 (320 vectors), and the time to the 320 lowest eigenpairs of
                   k-point 0 mixed vs FP64 (with errors against the stored oracle values)
  graphene         the graphene-like slab (36x36 grid, 4 k-points x 32 bands): hpsi_apply
                   per precision and the time to all its eigenpairs mixed vs FP64
  batched_48       the 48-problem uneven batch: hpsi_apply_batched per precision and the
                   time to the eigenpairs of its first problems mixed vs FP64
  supercell_2x2    the 2x2 supercell (72x72 grid, 64 bands, 4 k-points): time to its
                   eigenpairs mixed vs FP64
  roofline         the local-potential plane kernel (largest share of a step), from HIP
                   events around its launches on the library's stream in the timed steps
                   (the projections run beside it there); roofline.standalone: the same
                   kernel in two more steps with the projections on the caller's stream
  cpu_baseline     the CPU FP64 oracle's matrix-free H (FFT local part) on a bounded
                   sample of the same workload
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def local_model(p, ik, csz_in, csz, planes=True):
    """Algorithmic flops and HBM bytes per band-vector of the local-potential kernel
    (B-spline evaluate, inverse 2D FFT, V multiply, forward 2D FFT, and either the
    per-plane output rows (plane kernel) or the kappa partial rows per interval)."""
    dm = p.dims(ik)
    N1, N2 = p.desc["grid"]
    N = N1 * N2
    nzq, ng, nb = dm["nzq"], dm["ng"], dm["nb"]
    nint = len(p.desc["breakpoints"]) - 1
    flops = nzq * (32 * ng + 10 * N * math.log2(N) + 2 * N)
    rows_out = nzq if planes else 4 * nint
    bytes_ = nb * ng * csz_in + rows_out * ng * csz
    vbytes = nzq * N * (csz // 2)
    return flops, bytes_, vbytes


def traffic_record(name):
    """HBM traffic per launch measured with rocprofv3 counters, if the kernel
    sources have not changed since (compared by hash)."""
    path = os.path.join(ROOT, "profiles", f"{name}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in rec.get("sources", []):
        h.update(open(os.path.join(ROOT, "paper_1406_4960_amd", "csrc", f), "rb").read())
    if rec.get("source_sha256") != h.hexdigest():
        return None
    return rec


def cpu_baseline(desc, nbands=8, budget_s=15.0):
    """Oracle matrix-free FP64 H application (local part through numpy FFTs) on the
    same workload, k-point 0, blocks of nbands band-vectors until ~budget_s seconds."""
    from oracle import matfree, operators
    from oracle.bspline import ZBasis
    from paper_1406_4960_amd import workloads
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    threads = max(threads, len(os.sched_getaffinity(0)))
    zb = ZBasis(desc["breakpoints"], desc["order"], desc["nq"])
    vg = operators.gaussian_potential_on_grid_separable(desc, zb.zq)
    mf = matfree.MatFree(desc, 0, local="fft", vgrid=vg)
    x = np.transpose(workloads.random_block(99, nbands, mf.nb, mf.ng), (0, 2, 1))
    mf.apply(x[:1])  # warm
    done, t0 = 0, time.perf_counter()
    while True:
        mf.apply(x)
        done += x.shape[0]
        el = time.perf_counter() - t0
        if el > budget_s:
            break
    return {"value": round(done / el, 3), "unit": "band-vectors/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{done} band-vectors of H on k-point 0 of {desc['name']} in blocks of {nbands} "
                      f"(FP64 matrix-free oracle, local part through numpy FFTs) in {el:.1f} s; "
                      f"potential grid and tables built before timing"}


def batched_leg(args, torch, mbks, workloads):
    """The 48-problem uneven batch: hpsi_apply_batched over every (problem, k-point)
    item with each problem's band count, in FP32 / BF16x3 / FP64, and the time to
    the eigenpairs of the first problems (all their k-points) mixed vs FP64."""
    descs = workloads.batched()
    probs = [mbks.Problem(d, device=0) for d in descs]
    items = [(pr, ik) for pr, d in zip(probs, descs) for ik in range(len(d["kpts"]))]
    nbt = [d["nbands"] for d in descs for _ in d["kpts"]]
    total = sum(nbt)
    res = {"problems": len(descs), "items": len(items), "band_vectors_per_call": total}
    b = mbks.Batch(items)
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(14064960)
    for prec, ct in (("fp32", torch.complex64), ("bf16x3", torch.complex64), ("fp64", torch.complex128)):
        xs, ys = [], []
        for (pr, ik), n in zip(items, nbt):
            dm = pr.dims(ik)
            x = torch.randn((n, dm["nb"], dm["ld"]), dtype=ct, device="cuda:0", generator=gen)
            x[:, :, dm["ng"]:] = 0
            xs.append(x)
            ys.append(torch.empty_like(x))
        b.hpsi(xs, ys, prec)
        torch.cuda.synchronize()
        reps = 5
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            b.hpsi(xs, ys, prec)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[f"hpsi_{prec}"] = {"band_vectors_per_s": round(total / (ms * 1e-3), 1), "ms_per_call": round(ms, 3)}
        log("batched hpsi", prec, res[f"hpsi_{prec}"])
        del xs, ys
        torch.cuda.empty_cache()
    b.close()
    npr = min(args.batched_solve_problems, len(descs))
    if npr > 0:
        sub = [(pr, ik) for pr, d in list(zip(probs, descs))[:npr] for ik in range(len(d["kpts"]))]
        nev = [d["nbands"] for d in descs[:npr] for _ in d["kpts"]]
        bs = mbks.Batch(sub)
        sol = {}
        for prec in ("fp32", "fp64"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            eigs, xs, infos, st = bs.lanczos_lowest(nev, prec, raise_not_converged=False)
            torch.cuda.synchronize()
            sol[prec] = {"ms": round(1e3 * (time.perf_counter() - t0), 1), "status": st,
                         "max_resid": max(i["max_resid"] for i in infos),
                         "h_applies": sum(i["h_applies"] for i in infos), "eigs": eigs}
            del xs
        diff = max(float(np.max(np.abs(a - c))) for a, c in zip(sol["fp32"]["eigs"], sol["fp64"]["eigs"]))
        for v in sol.values():
            del v["eigs"]
        res["solve"] = {"problems": npr, "items": len(sub), "eigenpairs": sum(nev), "mixed": sol["fp32"],
                        "fp64": sol["fp64"], "speedup_mixed_vs_fp64": round(sol["fp64"]["ms"] / sol["fp32"]["ms"], 3),
                        "max_eig_diff_mixed_vs_fp64": diff}
        log("batched solve", res["solve"])
        bs.close()
    for pr in probs:
        pr.close()
    return res


def c3_leg(torch, mbks, workloads):
    """The 2x2 supercell (72x72 grid, ~1,900 G, 96 splines, 8 atoms, 64 bands, 4
    k-points): time to the eigenpairs of all k-points (solved together) in the mixed
    form and in plain FP64, and the largest eigenvalue difference between the two."""
    d = workloads.graphene_2x2()
    p = mbks.Problem(d, device=0)
    nk, M = len(d["kpts"]), d["nbands"]
    b = mbks.Batch([(p, ik) for ik in range(nk)])
    o = p.default_opts()
    o.max_iter = 1
    b.lanczos_lowest([M] * nk, "fp64", opts=o, raise_not_converged=False)  # workspaces, factors
    res = {"workload": d["name"], "kpoints": nk, "bands": M}
    eigs = {}
    for prec in ("fp32", "fp64"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e, xs, infos, st = b.lanczos_lowest([M] * nk, prec, raise_not_converged=False)
        torch.cuda.synchronize()
        res[prec] = {"ms": round(1e3 * (time.perf_counter() - t0), 1), "status": st,
                     "iters": [i["iters"] for i in infos], "max_resid": max(i["max_resid"] for i in infos)}
        eigs[prec] = e
        del xs
    res["speedup_mixed_vs_fp64"] = round(res["fp64"]["ms"] / res["fp32"]["ms"], 3)
    res["max_eig_diff_mixed_vs_fp64"] = max(float(np.max(np.abs(a - c))) for a, c in zip(eigs["fp32"], eigs["fp64"]))
    log("c3", res)
    b.close()
    p.close()
    return res


def graphene_leg(torch, mbks, workloads, steps=2):
    """The graphene-like slab (36x36 grid, 4 k-points x 32 bands): hpsi_apply per
    precision (32 bands per call) and the time to all 4 x 32 eigenpairs solved
    together, mixed vs FP64, with errors against the stored oracle eigenvalues."""
    d = workloads.graphene()
    p = mbks.Problem(d, device=0)
    nk, M = len(d["kpts"]), d["nbands"]
    res = {"workload": d["name"], "kpoints": nk, "bands": M}
    for prec, ct in (("fp64", torch.complex128), ("fp32", torch.complex64)):
        xs, ys = [], []
        for ik in range(nk):
            dm = p.dims(ik)
            xt = torch.zeros((M, dm["nb"], dm["ld"]), dtype=ct, device="cuda:0")
            xt[:, :, :dm["ng"]] = torch.from_numpy(workloads.random_block(ik, M, dm["nb"], dm["ng"])).to("cuda:0").to(ct)
            xs.append(xt)
            ys.append(torch.empty_like(xt))
        for ik in range(nk):
            p.hpsi(ik, xs[ik], ys[ik], prec)
        torch.cuda.synchronize()
        reps = 10
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            for ik in range(nk):
                p.hpsi(ik, xs[ik], ys[ik], prec)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        res[f"hpsi_{prec}"] = {"band_vectors_per_s": round(reps * nk * M / (ms * 1e-3), 1),
                               "ms_per_call": round(ms / (reps * nk), 4)}
        del xs, ys
    golden = None
    gpath = os.path.join(ROOT, "tests", "golden", "graphene_eigs.json")
    if os.path.exists(gpath):
        golden = json.load(open(gpath))
    kb = mbks.Batch([(p, ik) for ik in range(nk)])
    kb.lanczos_lowest([M] * nk, "fp32")  # workspaces, factors
    for prec in ("fp32", "fp64"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            eigs, xs, infos, st = kb.lanczos_lowest([M] * nk, prec)
            del xs
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        err = None
        if golden:
            err = max(float(np.max(np.abs(eigs[ik] - np.array(golden["kpoints"][str(ik)]["eps"]))))
                      for ik in range(nk) if str(ik) in golden["kpoints"])
        res[prec] = {"ms_to_eigenpairs": round(ms, 2), "max_eig_err_vs_oracle": err,
                     "max_resid": max(i["max_resid"] for i in infos),
                     "h_applies": sum(i["h_applies"] for i in infos)}
    res["speedup_mixed_vs_fp64"] = round(res["fp64"]["ms_to_eigenpairs"] / res["fp32"]["ms_to_eigenpairs"], 3)
    log("graphene", res)
    kb.close()
    p.close()
    return res


def uspp_leg(torch, mbks, workloads, steps=2):
    """The graphene-like slab with augmentation charges (ultrasoft overlap): spsi_apply
    and s_solve per call of 32 bands (FP64; the norm-conserving banded S beside it),
    and the time to all 4 x 32 eigenpairs, mixed vs FP64, with errors against the
    stored oracle eigenvalues."""
    d = workloads.graphene_uspp()
    p = mbks.Problem(d, device=0)
    p_nc = mbks.Problem(workloads.graphene(), device=0)
    nk, M = len(d["kpts"]), d["nbands"]
    res = {"workload": d["name"], "kpoints": nk, "bands": M}
    dm = p.dims(0)
    xt = torch.zeros((M, dm["nb"], dm["ld"]), dtype=torch.complex128, device="cuda:0")
    xt[:, :, :dm["ng"]] = torch.from_numpy(workloads.random_block(7, M, dm["nb"], dm["ng"])).to("cuda:0")
    yt = torch.empty_like(xt)
    for name, fn in (("spsi_fp64", lambda: p.spsi(0, xt, yt)), ("s_solve_fp64", lambda: p.s_solve(0, xt, yt)),
                     ("spsi_fp64_norm_conserving", lambda: p_nc.spsi(0, xt, yt)),
                     ("s_solve_fp64_norm_conserving", lambda: p_nc.s_solve(0, xt, yt))):
        fn()
        torch.cuda.synchronize()
        reps = 20
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[name] = {"band_vectors_per_s": round(M / (ms * 1e-3), 1), "ms_per_call": round(ms, 4)}
    del xt, yt
    p_nc.close()
    golden = None
    gpath = os.path.join(ROOT, "tests", "golden", "graphene_uspp_eigs.json")
    if os.path.exists(gpath):
        golden = json.load(open(gpath))
    kb = mbks.Batch([(p, ik) for ik in range(nk)])
    kb.lanczos_lowest([M] * nk, "fp32")  # workspaces, factors
    for prec in ("fp32", "fp64"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            eigs, xs, infos, st = kb.lanczos_lowest([M] * nk, prec)
            del xs
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        err = None
        if golden:
            err = max(float(np.max(np.abs(eigs[ik] - np.array(golden["kpoints"][str(ik)]["eps"]))))
                      for ik in range(nk) if str(ik) in golden["kpoints"])
        res[prec] = {"ms_to_eigenpairs": round(ms, 2), "max_eig_err_vs_oracle": err,
                     "max_resid": max(i["max_resid"] for i in infos),
                     "h_applies": sum(i["h_applies"] for i in infos)}
    res["speedup_mixed_vs_fp64"] = round(res["fp64"]["ms_to_eigenpairs"] / res["fp32"]["ms_to_eigenpairs"], 3)
    log("uspp", res)
    kb.close()
    p.close()
    return res


def density_leg(torch, mbks, workloads, d, reps=3):
    """Electron density of 320 band-vectors (k-point 0 of the surface slab, FP64 vectors,
    weight 2/8 each) at all 1,146 Gauss planes, and the Hartree potential of that density
    in the (z, g) form."""
    p = mbks.Problem(d, device=0)
    dm = p.dims(0)
    M = d["nbands"]
    N1, N2 = d["grid"]
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(14064966)
    x = torch.randn((M, dm["nb"], dm["ld"]), dtype=torch.complex128, device="cuda:0", generator=gen)
    x[:, :, dm["ng"]:] = 0
    w = torch.full((M,), 2.0 / len(d["kpts"]), dtype=torch.float64, device="cuda:0")
    rho = torch.zeros((dm["nzq"], N1, N2), dtype=torch.float64, device="cuda:0")
    vh = torch.empty_like(rho)
    p.density(0, x, w, rho)
    p.hartree(rho, vh)
    torch.cuda.synchronize()
    res = {"workload": d["name"], "bands": M, "planes": dm["nzq"], "grid": [N1, N2]}
    for name, fn in (("density_fp64", lambda: p.density(0, x, w, rho)), ("hartree", lambda: p.hartree(rho, vh))):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        res[name] = {"ms_per_call": round(e0.elapsed_time(e1) / reps, 3)}
    res["density_fp64"]["band_vectors_per_s"] = round(M / (res["density_fp64"]["ms_per_call"] * 1e-3), 1)
    # flop model of the density kernel per band and plane: one inverse 2D FFT (5 N log2 N),
    # evaluate (8 N_G), |psi|^2 accumulate (3 N)
    n = N1 * N2
    fl = dm["nzq"] * (5 * n * np.log2(n) + 8 * dm["ng"] + 3 * n) * M
    res["density_fp64"]["tflops"] = round(float(fl) / (res["density_fp64"]["ms_per_call"] * 1e-3) / 1e12, 2)
    log("density", res)
    del x, rho, vh
    torch.cuda.empty_cache()
    p.close()
    return res


def ribbon_leg(torch, mbks, workloads, reps=5, full=True):
    """The 1D-periodic form on the 19-line armchair ribbon (B-splines along x and z,
    plane waves along y): hpsi_apply on k-point 0 with 96 band-vectors in FP64 and FP32,
    the local kernel against its flop model, and the time to the 96 lowest eigenpairs
    of k-point 0 (and of all 4 k-points one after another) mixed and FP64."""
    d = workloads.ribbon()
    p = mbks.Problem(d, device=0)
    dm, wd = p.dims(0), p.wire_dims()
    M = d["nbands"]
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(14064967)
    res = {"workload": d["name"], "kpoints": len(d["kpts"]), "bands": M, "n_per_k": dm["ng"] * dm["nb"],
           "plane_waves": dm["ng"], "splines_x": wd["nbx"], "splines_z": wd["nbz"], "ny": wd["ny"],
           "projectors": dm["np"]}
    # flop model of the local kernel per band: per (x_q, z_p) line two ny-point FFTs
    # (10 ny log2 ny), the potential multiply (2 ny), evaluate and project (32 N_G)
    ny = wd["ny"]
    lines = wd["nxq"] * wd["nzq"]
    fl_band = lines * (10 * ny * np.log2(ny) + 2 * ny + 32 * dm["ng"])
    res["local_gflop_per_band"] = round(float(fl_band) / 1e9, 4)
    for prec, ct in (("fp64", torch.complex128), ("fp32", torch.complex64)):
        x = torch.randn((M, dm["nb"], dm["ld"]), dtype=ct, device="cuda:0", generator=gen)
        x[:, :, dm["ng"]:] = 0
        y = torch.empty_like(x)
        p.hpsi(0, x, y, prec)
        torch.cuda.synchronize()
        mbks.timer_enable(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            p.hpsi(0, x, y, prec)
        e1.record()
        torch.cuda.synchronize()
        st = mbks.timer_read()
        mbks.timer_enable(False)
        ms = e0.elapsed_time(e1) / reps
        stage = {k: round(v[0] / reps, 3) for k, v in st.items() if v[1]}
        loc = stage.get("local" if prec == "fp64" else "local32")
        peak = 78.6 if prec == "fp64" else 157.3
        rec = {"band_vectors_per_s": round(M / (ms * 1e-3), 1), "ms_per_call": round(ms, 3),
               "stages_ms_per_call": stage}
        if loc:
            tf = fl_band * M / (loc * 1e-3) / 1e12
            rec["local_kernel_alu"] = {"achieved_tflops": round(float(tf), 2), "peak": peak,
                                       "frac": round(float(tf) / peak, 4)}
        res[f"hpsi_{prec}"] = rec
        del x, y
        torch.cuda.empty_cache()
        log("ribbon hpsi", prec, rec)
    nks = range(len(d["kpts"])) if full else [0]
    for prec in ("fp32", "fp64"):
        tot, iters, resid = 0.0, [], 0.0
        for ik in nks:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            eps, xs, info, stt = p.lanczos_lowest(ik, M, prec, raise_not_converged=False)
            torch.cuda.synchronize()
            dt = 1e3 * (time.perf_counter() - t0)
            if ik == 0:
                res[f"eig_k0_{prec}"] = {"ms": round(dt, 1), "status": stt, "iters": info["iters"],
                                         "iters_reduced_precision": info["iters_low"],
                                         "max_resid": info["max_resid"]}
            tot += dt
            iters.append(info["iters"])
            resid = max(resid, info["max_resid"])
            del xs
        res[f"eig_all_{prec}"] = {"ms": round(tot, 1), "eigenpairs": len(nks) * M, "iters_per_k": iters,
                                  "max_resid": resid}
        log("ribbon eigen", prec, res[f"eig_all_{prec}"])
    res["eig_all_speedup_mixed_vs_fp64"] = round(res["eig_all_fp64"]["ms"] / res["eig_all_fp32"]["ms"], 3)
    torch.cuda.empty_cache()
    p.close()
    return res


def gamma_leg(torch, mbks, workloads, reps=5):
    """Real wavefunctions at the Gamma point: the surface slab with k = 0, 320 seeded
    band-vectors made real in space (c(G) <- (c(G) + conj c(-G)) / 2), H in FP32 through
    hpsi_apply (band by band) and hpsi_apply_gamma (two bands per transform), and the
    largest difference between the two results relative to the largest entry."""
    d = workloads.at_gamma(workloads.surface())
    p = mbks.Problem(d, device=0)
    dm = p.dims(0)
    M, ng = d["nbands"], dm["ng"]
    m, _ = p.gvectors(0)
    at = {(int(a), int(b)): g for g, (a, b) in enumerate(m)}
    mir = torch.tensor([at[(-int(a), -int(b))] for a, b in m], device="cuda:0")
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(14064960)
    x = torch.randn((M, dm["nb"], dm["ld"]), dtype=torch.complex64, device="cuda:0", generator=gen)
    x[:, :, ng:] = 0
    x[:, :, :ng] = 0.5 * (x[:, :, :ng] + x[:, :, mir].conj())
    res = {"workload": d["name"], "bands": M, "precision": "fp32"}
    outs = {}
    for fn in ("hpsi", "hpsi_gamma"):
        y = torch.empty_like(x)
        f = getattr(p, fn)
        f(0, x, y, "fp32")
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            f(0, x, y, "fp32")
        e1.record()
        torch.cuda.synchronize()
        res[f"{fn}_ms"] = round(e0.elapsed_time(e1) / reps, 3)
        outs[fn] = y[:, :, :ng]
    diff = (outs["hpsi_gamma"] - outs["hpsi"]).abs().max() / outs["hpsi"].abs().max()
    res["rel_diff"] = float(diff)
    p.close()
    return res


def surface_fp64_and_eigen_leg(torch, mbks, workloads, d, full_eig=False):
    """FP64 hpsi_apply on k-point 0 (320 vectors), and the time to the 320 lowest
    eigenpairs of k-point 0 (the share of one GPU in a k-point split over 8) in the
    mixed form and in plain FP64, with the errors of the lowest ones against the
    stored oracle eigenvalues; optionally all 8 k-points (lanczos_lowest_batched)."""
    p = mbks.Problem(d, device=0)
    dm = p.dims(0)
    M = d["nbands"]
    res = {}
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(14064965)
    x = torch.randn((M, dm["nb"], dm["ld"]), dtype=torch.complex128, device="cuda:0", generator=gen)
    x[:, :, dm["ng"]:] = 0
    y = torch.empty_like(x)
    p.hpsi(0, x, y, "fp64")
    torch.cuda.synchronize()
    reps = 3
    mbks.timer_enable(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        p.hpsi(0, x, y, "fp64")
    e1.record()
    torch.cuda.synchronize()
    st = mbks.timer_read()
    mbks.timer_enable(False)
    ms = e0.elapsed_time(e1) / reps
    flops_b = local_model(p, 0, 16, 16)[0]
    lms, lcount, lunits = st["local"]
    ach = flops_b * lunits / (lms * 1e-3) / 1e12
    res["hpsi_fp64_k0"] = {"band_vectors_per_s": round(M / (ms * 1e-3), 1), "ms_per_call": round(ms, 3),
                           "stages_ms_per_call": {k: round(v[0] / reps, 3) for k, v in st.items() if v[1]},
                           "local_kernel_alu": {"achieved_tflops": round(ach, 3), "peak": PEAK_FP64_TFLOPS,
                                                "frac": round(ach / PEAK_FP64_TFLOPS, 4)}}
    log("surface fp64 hpsi", res["hpsi_fp64_k0"])
    del x, y
    torch.cuda.empty_cache()
    golden = None
    gpath = os.path.join(ROOT, "tests", "golden", "surface_eigs.json")
    if os.path.exists(gpath):
        golden = json.load(open(gpath))
    o = p.default_opts()
    o.max_iter = 1
    xs = p.lanczos_lowest(0, M, "fp64", opts=o, raise_not_converged=False)[1]  # workspaces, factors
    del xs
    eigs = {}
    for prec in ("fp32", "fp64"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e, xs, info, stt = p.lanczos_lowest(0, M, prec, raise_not_converged=False)
        torch.cuda.synchronize()
        rec = {"ms": round(1e3 * (time.perf_counter() - t0), 1), "status": stt, "iters": info["iters"],
               "iters_reduced_precision": info["iters_low"], "h_applies": info["h_applies"],
               "max_resid": info["max_resid"]}
        if golden and "0" in golden["kpoints"]:
            ref = np.array(golden["kpoints"]["0"]["eps"])
            err = np.abs(e[:len(ref)] - ref)
            rec["eig_err_vs_oracle_lowest"] = {"count": len(ref), "max": float(err.max()),
                                               "per_eigenvalue": [float(v) for v in err]}
        eigs[prec] = e
        res[f"eig_k0_{prec}"] = rec
        del xs
        torch.cuda.empty_cache()
        log("surface solve k0", prec, rec)
    res["eig_k0_speedup_mixed_vs_fp64"] = round(res["eig_k0_fp64"]["ms"] / res["eig_k0_fp32"]["ms"], 3)
    res["eig_k0_max_diff_mixed_vs_fp64"] = float(np.max(np.abs(eigs["fp32"] - eigs["fp64"])))
    if full_eig:
        # all 8 k-points x 320 eigenpairs in one lanczos_lowest_batched call per form (as
        # many k-points at a time as the free device memory holds)
        nk = len(d["kpts"])
        b = mbks.Batch([(p, ik) for ik in range(nk)])
        all_e = {}
        for prec in ("fp32", "fp64"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e, xs, infos, stt = b.lanczos_lowest([M] * nk, prec, raise_not_converged=False)
            torch.cuda.synchronize()
            rec = {"ms": round(1e3 * (time.perf_counter() - t0), 1), "status": stt,
                   "eigenpairs": nk * M, "iters_per_k": [i["iters"] for i in infos],
                   "max_resid": max(i["max_resid"] for i in infos)}
            if golden and "0" in golden["kpoints"]:
                ref = np.array(golden["kpoints"]["0"]["eps"])
                rec["k0_max_eig_err_vs_oracle"] = float(np.max(np.abs(e[0][:len(ref)] - ref)))
            res[f"eig_all_{prec}"] = rec
            all_e[prec] = e
            del xs
            torch.cuda.empty_cache()
            log("surface solve all k", prec, rec)
        res["eig_all_speedup_mixed_vs_fp64"] = round(res["eig_all_fp64"]["ms"] / res["eig_all_fp32"]["ms"], 3)
        res["eig_all_max_diff_mixed_vs_fp64"] = float(max(np.max(np.abs(all_e["fp32"][k] - all_e["fp64"][k]))
                                                       for k in range(nk)))
        b.close()
    p.close()
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "bf16x3", "fp64"],
                    help="precision of the headline H application (fp32: the mixed form's reduced precision)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-eigen", action="store_true", help="skip the surface FP64 / eigenpair leg")
    ap.add_argument("--no-full-eig", action="store_true",
                    help="skip the time to all 8 x 320 eigenpairs of the surface slab (mixed and FP64)")
    ap.add_argument("--full-eig", action="store_true", help="(default) kept for old command lines")
    ap.add_argument("--no-graphene", action="store_true", help="skip the graphene-like slab leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the 48-problem uneven batch leg")
    ap.add_argument("--no-c3", action="store_true", help="skip the 2x2-supercell mixed vs FP64 solve")
    ap.add_argument("--no-density", action="store_true", help="skip the density / Hartree leg")
    ap.add_argument("--no-ribbon", action="store_true", help="skip the 1D-periodic ribbon leg")
    ap.add_argument("--no-gamma", action="store_true", help="skip the Gamma-point real-band leg")
    ap.add_argument("--no-uspp", action="store_true",
                    help="skip the graphene-like slab with augmentation charges (ultrasoft overlap)")
    ap.add_argument("--batched-solve-problems", type=int, default=6,
                    help="problems of the uneven batch whose eigenpairs are timed (all their k-points)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run one device-to-device copy of BYTES (counter calibration) and exit")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported by this build", file=sys.stderr)
        return 2

    import torch
    from paper_1406_4960_amd import mbks, workloads

    if args.copy_calibration:
        n = args.copy_calibration // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n}))
        return 0

    d = workloads.surface()
    nk, M = len(d["kpts"]), d["nbands"]
    dev = "cuda:0"
    torch.cuda.set_device(0)
    head = args.prec
    ct = torch.complex128 if head == "fp64" else torch.complex64
    p = mbks.Problem(d, device=0)
    dims = [p.dims(ik) for ik in range(nk)]
    log("workload", d["name"], dims[0])
    tuned = None
    if not args.no_autotune:
        tuned = [p.autotune(ik, 64, head) for ik in range(nk)]
        log("autotune k0", tuned[0])
    gen = torch.Generator(device=dev)
    gen.manual_seed(14064964)
    xs, ys = [], []
    for ik in range(nk):
        x = torch.randn((M, dims[ik]["nb"], dims[ik]["ld"]), dtype=ct, device=dev, generator=gen)
        x[:, :, dims[ik]["ng"]:] = 0
        xs.append(x)
        ys.append(torch.empty_like(x))

    def step(prec):
        for ik in range(nk):
            p.hpsi(ik, xs[ik], ys[ik], prec)

    for _ in range(args.warmup):
        step(head)
    torch.cuda.synchronize()
    # timed steps; the stage timer brackets every kernel launch with HIP events on the
    # stream it is launched on (the library's stream argument = torch's current stream)
    mbks.timer_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(head)
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    stages = mbks.timer_read()
    mbks.timer_enable(False)
    ms_per_step = 1e3 * t_steps / args.steps
    value = args.steps * nk * M / t_steps
    log("headline", head, round(ms_per_step, 3), "ms/step", round(value, 1), "band-vectors/s")
    stage_ms = {k: round(v[0] / args.steps, 3) for k, v in stages.items() if v[1]}

    # BF16x3 projector contractions (same vectors)
    bf = None
    if head == "fp32":
        step("bf16x3")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(max(2, args.steps // 3)):
            step("bf16x3")
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t1) / max(2, args.steps // 3)
        bf = {"ms_per_step": round(1e3 * tb, 3), "band_vectors_per_s": round(nk * M / tb, 1)}

    # roofline of the dominant kernel: the local-potential plane kernel
    lname = "local" if head == "fp64" else "local32"
    lms, lcount, lunits = stages[lname]
    csz = 16 if head == "fp64" else 8
    flops_b, bytes_b, vbytes = local_model(p, 0, csz, csz)
    per_launch = lunits / lcount
    avg_ms = lms / lcount
    achieved = flops_b * per_launch / (avg_ms * 1e-3) / 1e12
    peak = PEAK_FP64_TFLOPS if head == "fp64" else PEAK_FP32_TFLOPS
    T = "double" if head == "fp64" else "float"
    var = (tuned[0]["plane_variant"] if tuned else (1 if head == "fp64" else 0))
    q1q2 = "8, 4" if var == 1 else "16, 8"
    tr = traffic_record(f"k_local_plane_surface_{'fp64' if head == 'fp64' else 'fp32'}_traffic")
    alg_bytes = bytes_b * per_launch + vbytes
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": tr["bytes_per_launch"] if tr else None,
                "kernel": f"k_local_plane<{T}, {T}, 128, 64, {q1q2}, 512, 1, false> (evaluate / 2D FFT / V / "
                          f"2D FFT / gather, one output row per Gauss plane)",
                "avg_launch_ms": round(avg_ms, 4), "launches": lcount, "bands_per_launch": per_launch,
                "flops_per_launch": flops_b * per_launch,
                "flop_model": "per Gauss plane 10 N log2 N (two 2D FFTs of N = N1 N2 points) + 2 N "
                              "(potential) + 32 N_G (evaluate, gather)",
                "algorithmic_bytes_per_launch": alg_bytes,
                "hbm_gbs_algorithmic": round(alg_bytes / (avg_ms * 1e-3) / 1e9, 1)}
    if tr:
        roofline["traffic_over_algorithmic"] = round(tr["bytes_per_launch"] / alg_bytes, 3)
    # In the timed steps the projections run beside the plane kernel on the k-point's own
    # stream, so the kernel's launch time above includes sharing the GPU with them.  Its
    # standalone rate, from two more steps with the projections on the caller's stream:
    prev = os.environ.get("MBKS_NL_OVERLAP")
    os.environ["MBKS_NL_OVERLAP"] = "0"
    mbks.timer_enable(True)
    for _ in range(2):
        step(head)
    torch.cuda.synchronize()
    solo = mbks.timer_read()
    mbks.timer_enable(False)
    if prev is None:
        del os.environ["MBKS_NL_OVERLAP"]
    else:
        os.environ["MBKS_NL_OVERLAP"] = prev
    sms, scount, _ = solo[lname]
    solo_ms = sms / scount
    solo_ach = flops_b * per_launch / (solo_ms * 1e-3) / 1e12
    roofline["standalone"] = {"avg_launch_ms": round(solo_ms, 4), "launches": scount,
                              "achieved": round(solo_ach, 3), "frac": round(solo_ach / peak, 4),
                              "note": "same kernel with the projections on the caller's stream "
                                      "(not beside it), two extra steps"}
    log("plane kernel standalone", round(solo_ms, 3), "ms", round(solo_ach, 2), "TFLOP/s")
    del xs, ys
    torch.cuda.empty_cache()
    p.close()

    surf = {"workload": d["name"], "stages_ms_per_step": stage_ms, "bf16x3": bf,
            "autotune_k0": tuned[0] if tuned else None}
    if not args.no_eigen:
        surf.update(surface_fp64_and_eigen_leg(torch, mbks, workloads, d, not args.no_full_eig))
    graphene = None if args.no_graphene else graphene_leg(torch, mbks, workloads)
    batched = None if args.no_batched else batched_leg(args, torch, mbks, workloads)
    c3 = None if args.no_c3 else c3_leg(torch, mbks, workloads)
    uspp = None if args.no_uspp else uspp_leg(torch, mbks, workloads)
    dens = None if args.no_density else density_leg(torch, mbks, workloads, d)
    ribbon = None if args.no_ribbon else ribbon_leg(torch, mbks, workloads)
    gamma = None if args.no_gamma else gamma_leg(torch, mbks, workloads)

    cpu = None
    if not args.no_cpu_baseline:
        try:
            cpu = cpu_baseline(d)
        except Exception as exc:  # report, do not fail the benchmark line
            cpu = {"value": None, "unit": "band-vectors/s", "cores": None, "kind": "oracle",
                   "sample": f"failed: {exc}"}

    out = {
        "metric": "Hψ band-vectors/s + time to N eigenpairs at 1e-6 Ha: mixed/batched vs FP64",
        "value": round(value, 1),
        "unit": "band-vectors/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": d["name"], "kpoints": nk, "bands": M, "band_vectors_per_step": nk * M,
                   "n_per_k": dims[0]["ng"] * dims[0]["nb"], "grid": d["grid"], "splines": dims[0]["nb"],
                   "gauss_planes": dims[0]["nzq"], "projectors": dims[0]["np"], "precision": head},
        "surface": surf,
        "graphene": graphene,
        "batched_48": batched,
        "supercell_2x2": c3,
        "ultrasoft_graphene": uspp,
        "density_hartree": dens,
        "ribbon_1d_periodic": ribbon,
        "gamma_real_bands": gamma,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
