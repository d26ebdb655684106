#!/usr/bin/env python3
"""Benchmark of the mixed-basis eigen-search hot path on one MI355X.

Workload: the graphene-like slab (hexagonal a = 4.65 bohr, 36x36 in-plane grid,
~483 G per k-point, 80 graded cubic B-splines on [-20, 20] with 5 Gauss points
per interval, 2 atoms with Gaussian local parts and 4 Kleinman-Bylander
projectors each, 2x2 Monkhorst-Pack k-points, 32 bands; n = 38,640 per k),
synthetic and seeded.

One step = the 32 lowest eigenpairs of every k-point from a seeded random start
(lanczos_lowest_batched over the 4 k-points, which runs them concurrently on
streams of their own), in the headline precision (mixed: FP32 local / nonlocal
parts of H until the residual reaches 1e-4, then FP64; FP64 orthonormalisation,
Krylov coefficients and projected problems throughout), to residual 1e-7.

Printed JSON line:
  value            H band-vectors applied per second over the timed steps
  ms_per_step      time to the 4 x 32 eigenpairs (all k-points)
  fp64             the same step in plain FP64 (time, eigenvalue errors)
  hpsi             pure hpsi_apply throughput (32 bands x 4 k per call) in FP64 / FP32,
                   eager and replayed from a captured HIP graph
  batched_48       the 48-problem uneven batch: hpsi_apply_batched throughput per
                   precision, and mixed vs FP64 time to the eigenpairs of its first
                   problems
  supercell_2x2    the 2x2 supercell (72x72 grid, 64 bands, 4 k-points): time to its
                   eigenpairs mixed vs FP64
  surface          the large surface slab (128x64 grid, 256 projectors, 320 bands),
                   k-point 0: hpsi_apply throughput per precision and time to its
                   320 eigenpairs mixed vs FP64
  roofline         the fused local-potential kernel (dominant kernel), from its
                   launches in the FP64 hpsi leg
  cpu_baseline     the CPU FP64 oracle's matrix-free H application, bounded sample
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


def local_model(p, ik, csz_in, csz):
    """Algorithmic flops and bytes per band-vector of the fused local kernel
    (B-spline evaluate, inverse FFT, V multiply, forward FFT, project)."""
    dm = p.dims(ik)
    N1, N2 = p.desc["grid"]
    N = N1 * N2
    nzq, ng, nb = dm["nzq"], dm["ng"], dm["nb"]
    nint = len(p.desc["breakpoints"]) - 1
    flops = nzq * (32 * ng + 10 * N * math.log2(N) + 2 * N)
    bytes_ = nb * ng * csz_in + 4 * nint * ng * csz
    vbytes = nzq * N * (csz // 2)
    return flops, bytes_, vbytes


def traffic_record(name):
    """HBM traffic per launch measured with rocprofv3 counters, if the kernel
    source has not changed since (compared by hash)."""
    path = os.path.join(ROOT, "profiles", f"{name}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    files = rec.get("sources", [rec.get("source", "k_local.hip")])
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_1406_4960_amd", "csrc", f), "rb").read())
    if rec.get("source_sha256") != h.hexdigest():
        return None
    return rec


def cpu_baseline(desc, budget_s=15.0):
    """Oracle matrix-free FP64 H application on the same workload (k-point 0),
    bounded sample: blocks of 8 band-vectors until ~budget_s seconds."""
    from oracle import matfree
    from paper_1406_4960_amd import workloads
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    mf = matfree.MatFree(desc, 0)
    x = workloads.random_block(99, 8, mf.ng, mf.nb)
    mf.apply(x[:1])  # warm
    done, t0 = 0, time.perf_counter()
    while True:
        mf.apply(x)
        done += x.shape[0]
        el = time.perf_counter() - t0
        if el > budget_s:
            break
    return {"value": done / el, "unit": "band-vectors/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{done} band-vectors of H (k-point 0, FP64 matrix-free oracle) in {el:.1f} s; "
                      f"potential tables built before timing"}


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


def surface_leg(torch, mbks, workloads):
    """The large surface slab (128x64 grid, ~3,990 G, 192 splines with 6 Gauss
    points, 64 atoms / 256 projectors, 320 bands) at k-point 0 of its 8: pure
    hpsi_apply throughput per precision on 320 band-vectors, and the time to its
    320 lowest eigenpairs in the mixed form and in plain FP64."""
    d = workloads.surface()
    p = mbks.Problem(d, device=0)
    dm = p.dims(0)
    M = d["nbands"]
    res = {"workload": d["name"], "kpoint": 0, "bands": M, "n_per_k": dm["ng"] * dm["nb"],
           "projectors": dm["np"], "gauss_planes": dm["nzq"]}
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(14064964)
    for prec, ct in (("fp64", torch.complex128), ("fp32", torch.complex64), ("bf16x3", torch.complex64)):
        x = torch.randn((M, dm["nb"], dm["ld"]), dtype=ct, device="cuda:0", generator=gen)
        x[:, :, dm["ng"]:] = 0
        y = torch.empty_like(x)
        p.hpsi(0, x, y, prec)
        torch.cuda.synchronize()
        reps = 3
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
        res[f"hpsi_{prec}"] = {"band_vectors_per_s": round(M / (ms * 1e-3), 1), "ms_per_call": round(ms, 3),
                               "stages_ms_per_call": {k: round(v[0] / reps, 3) for k, v in st.items() if v[1]}}
        # the fused local kernel against the vector ALU peak of its arithmetic type
        lname = "local" if prec == "fp64" else "local32"
        if st.get(lname, (0, 0, 0))[1]:
            lms, _, lunits = st[lname]
            flops_b = local_model(p, 0, 16, 16)[0]
            ach = flops_b * lunits / (lms * 1e-3) / 1e12
            peak = PEAK_FP64_TFLOPS if prec == "fp64" else PEAK_FP32_TFLOPS
            res[f"hpsi_{prec}"]["local_kernel_alu"] = {"achieved_tflops": round(ach, 3), "peak": peak,
                                                       "frac": round(ach / peak, 4)}
        log("surface hpsi", prec, res[f"hpsi_{prec}"])
        del x, y
        torch.cuda.empty_cache()
    o = p.default_opts()
    o.max_iter = 1
    xs = p.lanczos_lowest(0, M, "fp64", opts=o, raise_not_converged=False)[1]  # workspaces, factors
    del xs
    eigs = {}
    for prec in ("fp32", "fp64"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e, xs, info, st = p.lanczos_lowest(0, M, prec, raise_not_converged=False)
        torch.cuda.synchronize()
        res[prec] = {"ms": round(1e3 * (time.perf_counter() - t0), 1), "status": st, "iters": info["iters"],
                     "iters_reduced_precision": info["iters_low"], "h_applies": info["h_applies"],
                     "max_resid": info["max_resid"]}
        eigs[prec] = e
        del xs
        torch.cuda.empty_cache()
        log("surface solve", prec, res[prec])
    res["speedup_mixed_vs_fp64"] = round(res["fp64"]["ms"] / res["fp32"]["ms"], 3)
    res["max_eig_diff_mixed_vs_fp64"] = float(np.max(np.abs(eigs["fp32"] - eigs["fp64"])))
    p.close()
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="graphene")
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64"],
                    help="reduced precision of the headline step (fp32 = mixed FP32/FP64)")
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--hpsi-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 48-problem uneven batch leg")
    ap.add_argument("--no-c3", action="store_true", help="skip the 2x2-supercell mixed vs FP64 solve")
    ap.add_argument("--no-surface", action="store_true",
                    help="skip the surface-slab leg (320 bands: hpsi per precision, eigenpairs of one k-point)")
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

    desc = workloads.CONFIGS[args.workload]()
    nk = len(desc["kpts"])
    M = desc["nbands"]
    dev = "cuda:0"
    torch.cuda.set_device(0)
    p = mbks.Problem(desc, device=0)
    dims = [p.dims(ik) for ik in range(nk)]
    log("workload", desc["name"], dims[0])

    # ---- kernel choices measured per k-point (mb_autotune), kept for the run ----
    tuned = {}
    for prec in ("fp64", "fp32"):
        tuned[prec] = [p.autotune(ik, M, prec) for ik in range(nk)]
    log("autotune", tuned)

    # ---- pure H application throughput (inputs resident in HBM) ---------------
    hp = {}
    for prec, ct in (("fp64", torch.complex128), ("fp32", torch.complex64)):
        xs, ys = [], []
        for ik in range(nk):
            x = workloads.random_block(ik, M, dims[ik]["nb"], dims[ik]["ng"])
            xt = torch.zeros((M, dims[ik]["nb"], dims[ik]["ld"]), dtype=ct, device=dev)
            xt[:, :, :dims[ik]["ng"]] = torch.from_numpy(x).to(dev).to(ct)
            xs.append(xt)
            ys.append(torch.empty_like(xt))
        for _ in range(3):
            for ik in range(nk):
                p.hpsi(ik, xs[ik], ys[ik], prec)
        torch.cuda.synchronize()
        mbks.timer_enable(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.hpsi_reps):
            for ik in range(nk):
                p.hpsi(ik, xs[ik], ys[ik], prec)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        st = mbks.timer_read()
        mbks.timer_enable(False)
        # the same calls captured once in a HIP graph and replayed
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            for ik in range(nk):
                p.hpsi(ik, xs[ik], ys[ik], prec)
        gr.replay()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.hpsi_reps):
            gr.replay()
        e1.record()
        torch.cuda.synchronize()
        ms_graph = e0.elapsed_time(e1)
        del gr
        hp[prec] = {"band_vectors_per_s": args.hpsi_reps * nk * M / (ms * 1e-3),
                    "ms_per_call": ms / (args.hpsi_reps * nk),
                    "graph_band_vectors_per_s": args.hpsi_reps * nk * M / (ms_graph * 1e-3),
                    "stages_ms": {k: round(v[0], 4) for k, v in st.items() if v[1]},
                    "stage_raw": st}
        log("hpsi", prec, {k: v for k, v in hp[prec].items() if k != "stage_raw"})
        del xs, ys

    # ---- eigen-search steps --------------------------------------------------
    # all k-points of the step are solved together (lanczos_lowest_batched: one
    # stream per k-point, so their latency-bound small kernels overlap)
    kbatch = mbks.Batch([(p, ik) for ik in range(nk)])

    def solve_all(prec):
        eigs, xs, infos, stc = kbatch.lanczos_lowest([M] * nk, prec)
        del xs
        return eigs, infos

    golden = None
    gpath = os.path.join(ROOT, "tests", "golden", f"{args.workload}_eigs.json")
    if os.path.exists(gpath):
        golden = json.load(open(gpath))

    def errors(eigs):
        if golden is None:
            return None
        errs = [float(np.max(np.abs(eigs[ik] - np.array(golden["kpoints"][str(ik)]["eps"]))))
                for ik in range(nk) if str(ik) in golden["kpoints"]]
        return max(errs) if errs else None

    head = args.prec
    for _ in range(args.warmup):
        solve_all(head)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    applies = 0
    infos_all = []
    eigs = None
    for _ in range(args.steps):
        eigs, infos = solve_all(head)
        applies += sum(i["h_applies"] for i in infos)
        infos_all += infos
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    ms_per_step = 1e3 * t_steps / args.steps
    head_err = errors(eigs)
    head_res = max(i["max_resid"] for i in infos_all)
    log("step", head, ms_per_step, "ms; applies/step", applies / args.steps, "err", head_err)
    # one more, untimed step with the per-kernel stage timer (HIP events on the library's stream)
    mbks.timer_enable(True)
    solve_all(head)
    torch.cuda.synchronize()
    stages = mbks.timer_read()
    mbks.timer_enable(False)

    # plain FP64 form of the same step
    fp64 = None
    if head != "fp64" and args.fp64_steps > 0:
        solve_all("fp64")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        a64 = 0
        for _ in range(args.fp64_steps):
            e64, i64 = solve_all("fp64")
            a64 += sum(i["h_applies"] for i in i64)
        torch.cuda.synchronize()
        t64 = 1e3 * (time.perf_counter() - t1) / args.fp64_steps
        fp64 = {"ms_per_step": t64, "h_applies_per_step": a64 / args.fp64_steps,
                "max_eig_err_vs_oracle": errors(e64), "max_resid": max(i["max_resid"] for i in i64),
                "speedup_mixed_vs_fp64": t64 / ms_per_step}
        log("fp64 step", fp64)

    # ---- roofline of the dominant kernel ----------------------------------------
    # The fused local-potential kernel (k_local_lines, FP64 instantiation) takes the
    # largest share of the benchmark's kernel time.  Its launches in the pure hpsi_apply
    # leg all have one shape (32 bands, every knot interval), so the per-launch
    # figures are those of that leg: HIP events around each launch on the library's
    # stream (stage timer), algorithmic flops from the operation count model.
    def local_roofline(prec):
        name = "local" if prec == "fp64" else "local32"
        lms, lcount, lunits = hp[prec]["stage_raw"][name]
        csz = 16 if prec == "fp64" else 8
        flops_b, bytes_b, vbytes = local_model(p, 0, csz, csz)
        achieved = flops_b * lunits / (lms * 1e-3) / 1e12
        peak = PEAK_FP64_TFLOPS if prec == "fp64" else PEAK_FP32_TFLOPS
        per_launch = lunits / lcount
        return {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4),
                "avg_launch_ms": round(lms / lcount, 5), "launches": lcount, "bands_per_launch": per_launch,
                "flops_per_launch": flops_b * per_launch,
                "algorithmic_bytes_per_launch": bytes_b * per_launch + vbytes,
                "hbm_gbs_algorithmic": round((bytes_b * per_launch + vbytes) / (lms / lcount * 1e-3) / 1e9, 1)}

    roofline = local_roofline("fp64")
    tr = traffic_record(f"k_local_lines_{args.workload}_traffic")
    roofline["traffic"] = tr["bytes_per_launch"] if tr else None
    roofline["kernel"] = "k_local_lines<double, double, 36, 36, 256, 3> (fused evaluate / FFT / V / FFT / project)"
    roofline["fp32_instantiation"] = local_roofline("fp32")
    tot = {k: v for k, v in stages.items() if v[1]}
    roofline["step_stage_ms"] = {k: round(v[0], 3) for k, v in tot.items()}

    batched = None if args.no_batched else batched_leg(args, torch, mbks, workloads)
    c3 = None if args.no_c3 else c3_leg(torch, mbks, workloads)
    surf = None if args.no_surface else surface_leg(torch, mbks, workloads)

    cpu = None
    if not args.no_cpu_baseline:
        try:
            cpu = cpu_baseline(desc)
        except Exception as exc:  # report, do not fail the benchmark line
            cpu = {"value": None, "unit": "band-vectors/s", "cores": None, "kind": "oracle",
                   "sample": f"failed: {exc}"}

    value = applies / t_steps
    out = {
        "metric": "Hψ band-vectors/s + time to N eigenpairs at 1e-6 Ha: mixed/batched vs FP64",
        "value": round(value, 1),
        "unit": "band-vectors/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": desc["name"], "kpoints": nk, "bands": M, "n_per_k": dims[0]["ng"] * dims[0]["nb"],
                   "grid": desc["grid"], "splines": dims[0]["nb"], "projectors": dims[0]["np"],
                   "tol_resid": 1e-7},
        "time_to_eigenpairs_ms": round(ms_per_step, 2),
        "max_eig_err_vs_oracle": head_err,
        "max_resid": head_res,
        "h_applies_per_step": applies / args.steps,
        "fp64": fp64,
        "hpsi": {k: {kk: vv for kk, vv in v.items() if kk != "stage_raw"} for k, v in hp.items()},
        "autotune_k0": {k: v[0] for k, v in tuned.items()},
        "batched_48": batched,
        "supercell_2x2": c3,
        "surface": surf,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    kbatch.close()
    p.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
