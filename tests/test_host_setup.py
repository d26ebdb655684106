"""CPU checks of the library's host logic: it loads, exports every declared
symbol, and its set-up tables (built in C++) agree with the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import bspline, lattice, operators
from paper_1406_4960_amd import mbks, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    text = open(os.path.join(ROOT, "include", "mbks.h")).read()
    body = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:mb_status|void|const char\*)\s+(\w+)\s*\(", body, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = mbks.load()
    names = _header_symbols()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(mbks.EXPORTS) == names


@pytest.mark.parametrize("maker", [workloads.tiny, workloads.graphene, workloads.graphene_2x2,
                                   workloads.surface, lambda: workloads.micro(seed=3)])
def test_setup_tables_match_oracle(maker):
    d = maker()
    p = mbks.Problem(d, device=None)
    zb = bspline.ZBasis(d["breakpoints"], d["order"], d["nq"])
    for ik in range(min(2, len(d["kpts"]))):
        dm = p.dims(ik)
        m, kg2 = p.gvectors(ik)
        mo, kgo = lattice.gset(d, ik)
        assert dm["ng"] == len(mo) and dm["nb"] == zb.nb and dm["ld"] >= dm["ng"]
        assert {tuple(x) for x in m} == {tuple(x) for x in mo}
        perm = {(int(a), int(b)): n for n, (a, b) in enumerate(mo)}
        idx = np.array([perm[(int(a), int(b))] for a, b in m])
        assert np.max(np.abs(kg2 - np.sum(kgo[idx] ** 2, axis=1))) < 1e-11
        F, Z, E = p.projectors(ik)
        Fo, Zo, Eo = operators.projector_factors(d, ik, zb)
        assert F.shape == Fo[:, idx].shape
        if F.size:
            assert np.max(np.abs(F - Fo[:, idx])) < 1e-13 * np.max(np.abs(Fo))
            assert np.max(np.abs(Z - Zo)) < 1e-13 * np.max(np.abs(Zo))
            assert np.array_equal(E, Eo)
    zq, wq = p.zrule()
    assert np.max(np.abs(zq - zb.zq)) < 1e-13 and np.max(np.abs(wq - zb.wq)) < 1e-15
    s, dd = p.zbands()
    S, D = zb.overlap(), zb.deriv_overlap()
    for i in range(zb.nb):
        for k in range(4):
            ref_s = S[i, i + k] if i + k < zb.nb else 0.0
            ref_d = D[i, i + k] if i + k < zb.nb else 0.0
            assert abs(s[i, k] - ref_s) < 1e-14 * np.max(S)
            assert abs(dd[i, k] - ref_d) < 1e-13 * np.max(D)
    p.close()


def test_invalid_descriptions_rejected():
    d = workloads.tiny()
    bad = dict(d, breakpoints=[0.0, 1.0, 1.0, 2.0])
    with pytest.raises(mbks.MbError) as e:
        mbks.Problem(bad, device=None)
    assert e.value.status == -1
    with pytest.raises(mbks.MbError) as e:
        mbks.Problem(dict(d, grid=[6, 16]), device=None)  # 2*3+1 = 7 > 6: G would alias
    assert e.value.status == -1
    with pytest.raises(mbks.MbError) as e:
        mbks.Problem(dict(d, grid=[16, 14 * 7]), device=None)  # factor 7
    assert e.value.status == -1
    with pytest.raises(mbks.MbError):
        mbks.Problem(dict(d, nq=0), device=None)


def test_augmentation_charges_reach_the_library():
    # ultrasoft overlap (Sec. II.B.2): the charges of the seeded description, per
    # projector in the library's projector order, equal the oracle's; a description
    # without charges gives zeros; negative or non-finite charges are refused
    d = workloads.graphene_uspp()
    p = mbks.Problem(d, device=None)
    assert np.array_equal(p.augmentation(), operators.projector_augmentation(d))
    assert np.all(p.augmentation() > 0)
    p.close()
    p = mbks.Problem(workloads.graphene(), device=None)
    assert np.all(p.augmentation() == 0)
    p.close()
    for bad in (-0.1, float("nan")):
        sp = dict(d["species"][0], q_p=bad)
        with pytest.raises(mbks.MbError) as e:
            mbks.Problem(dict(d, species=[sp]), device=None)
        assert e.value.status == -1


def test_gpu_calls_on_host_only_handle_fail():
    p = mbks.Problem(workloads.tiny(), device=None)
    lib = mbks.load()
    st = lib.hpsi_apply(p.h, 0, ctypes.c_void_p(16), ctypes.c_void_p(4096), 1, p.dims(0)["ld"], 0, None)
    assert st == -7
    st = lib.s_solve(p.h, 0, ctypes.c_void_p(16), ctypes.c_void_p(16), 1, p.dims(0)["ld"], 0, None)
    assert st == -7
    assert b"host-only" in lib.mb_last_error()
    assert lib.mb_problem_reserve(p.h, 0, 8, 0, 1) == -7
    p.close()


def test_bench_runs_on_one_gpu_only():
    # the benchmark measures one GPU; asking for more exits with a message, before
    # any GPU work
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_tune_choices_persist_through_the_cache_file(tmp_path):
    # choices set on one handle are saved, merged with another problem's, and applied
    # to fresh handles of the same sizes only
    path = str(tmp_path / "tune.json")
    g = mbks.Problem(workloads.graphene(), device=None)
    for ik in range(4):
        g.tune_set(ik, "fp32", local_kernel=0, lds_budget_kb=66, nl_matrix_cores=0, combine_bands=4)
    g.tune_set(0, "fp64", local_kernel=2, combine_bands=1)
    g.tune_save(path)
    s = mbks.Problem(workloads.surface(), device=None)
    s.tune_set(0, "fp32", local_kernel=3, plane_variant=1, nl_matrix_cores=1)
    s.tune_save(path)
    text = open(path).read()
    assert '"format": "mbks-tune-1"' in text and text.count('"key"') >= 3
    g2 = mbks.Problem(workloads.graphene(), device=None)
    assert g2.tune_get(0, "fp32")["local_kernel"] == -1
    n = g2.tune_load(path)
    assert n >= 5  # four FP32 k-points (identical sizes share one entry) and the FP64 one
    for ik in range(4):
        t = g2.tune_get(ik, "fp32")
        assert (t["local_kernel"], t["lds_budget_kb"], t["nl_matrix_cores"], t["combine_bands"]) == (0, 66, 0, 4)
    assert g2.tune_get(0, "fp64")["local_kernel"] == 2 and g2.tune_get(0, "fp64")["combine_bands"] == 1
    s2 = mbks.Problem(workloads.surface(), device=None)
    assert s2.tune_load(path) >= 1
    t = s2.tune_get(0, "bf16x3")  # BF16x3 shares the FP32 class
    assert (t["local_kernel"], t["plane_variant"], t["nl_matrix_cores"]) == (3, 1, 1)
    # a problem of other sizes takes nothing; a missing file applies nothing
    t2 = mbks.Problem(workloads.graphene_2x2(), device=None)
    assert t2.tune_load(path) == 0
    assert t2.tune_load(str(tmp_path / "missing.json")) == 0
    # invalid choices and malformed files are refused
    for target, bad in ((g2, dict(local_kernel=7)), (g2, dict(local_kernel=0, lds_budget_kb=10)),
                        (t2, dict(local_kernel=3)), (g2, dict(local_kernel=0, combine_bands=3))):
        with pytest.raises(mbks.MbError) as e:
            target.tune_set(0, "fp32", **bad)  # kind 3: the 72x72 grid has no plane kernel
        assert e.value.status == -1
    open(str(tmp_path / "bad.json"), "w").write('{\n "format": "mbks-tune-1",\n "entries": [\n  {"key": 3}\n ]\n}\n')
    with pytest.raises(mbks.MbError):
        g2.tune_load(str(tmp_path / "bad.json"))
    # -1 restores the untuned rules
    g2.tune_set(1, "fp32", local_kernel=-1)
    assert g2.tune_get(1, "fp32")["local_kernel"] == -1
    for pr in (g, s, g2, s2, t2):
        pr.close()


def test_wire_handles_on_the_host():
    # 1D-periodic form: sizes and plane-wave sets against the oracle, calls of the slab
    # refused, inconsistent descriptions refused
    from oracle import wire
    for d in (workloads.wire_micro(), workloads.ribbon_narrow(), workloads.ribbon()):
        p = mbks.Problem(d, device=None)
        wd = p.wire_dims()
        xb, zb = wire.basis_x(d), wire.basis_z(d)
        assert (wd["nbx"], wd["nbz"], wd["nxq"], wd["nzq"], wd["ny"]) == (xb.nb, zb.nb, len(xb.zq), len(zb.zq), d["ny"])
        for ik in range(len(d["kpts"])):
            dm = p.dims(ik)
            m, kg2 = p.gvectors(ik)
            mo, q = wire.gset(d, ik)
            assert dm["nb"] == xb.nb * zb.nb and dm["ng"] == len(mo)
            assert np.array_equal(m[:, 0], mo) and np.all(m[:, 1] == 0)
            assert np.max(np.abs(kg2 - q * q)) < 1e-12 * np.max(q * q)
        for call in (p.zrule, p.zbands, p.projectors, p.augmentation, lambda: p.tune_get(0)):
            with pytest.raises(mbks.MbError) as e:
                call()
            assert e.value.status == -1
        p.close()
    slab = mbks.Problem(workloads.tiny(), device=None)
    with pytest.raises(mbks.MbError):
        slab.wire_dims()
    slab.close()
    base = workloads.wire_micro()
    bad = [dict(base, ny=10), dict(base, ny=8, ecut=40.0), dict(base, period=-1.0),
           dict(base, breakpoints_x=[0.0, 1.0, 1.0, 2.0]),
           dict(base, species=[dict(base["species"][0], q_s=0.2)] + base["species"][1:])]
    for d in bad:
        with pytest.raises(mbks.MbError) as e:
            mbks.Problem(d, device=None)
        assert e.value.status == -1
