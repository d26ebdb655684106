"""Write stored oracle eigenvalues for the full-size parity tests.

    python tests/golden/make_golden.py graphene       # -> tests/golden/graphene_eigs.json
    python tests/golden/make_golden.py graphene_uspp  # the same slab with augmentation charges
    python tests/golden/make_golden.py graphene_2x2   # 2x2 supercell, k-point 0, 64 lowest
    python tests/golden/make_golden.py surface        # 128x64 surface slab, k-point 0, 32 lowest
    python tests/golden/make_golden.py member12       # batch member 12 (60x60 grid), every k-point
    python tests/golden/make_golden.py member33       # batch member 33 (80x80 grid), every k-point
    python tests/golden/make_golden.py ribbon_narrow  # 1D-periodic 3-line ribbon, every k-point (dense)

Calls only the oracle: the matrix-free FP64 operator of oracle/matfree.py
(local part through the grid with numpy FFTs, or the dense per-plane sum for the
graphene-like slab) and scipy's LOBPCG to a residual of 1e-9 per eigenpair; for the
1D-periodic ribbon, the dense matrices of oracle/wire.py and LAPACK.  The
values are the lowest discrete eigenvalues of H c = eps S c (Sec. II.C) for the
stated k-points and band counts of each seeded workload.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import matfree, operators, wire  # noqa: E402
from oracle.bspline import ZBasis  # noqa: E402
from paper_1406_4960_amd import workloads  # noqa: E402

# name -> (description maker, k-points (None = all), eigenvalues per k-point (None = nbands), local mode)
SETS = {
    "graphene": (workloads.graphene, None, None, "dense"),
    "graphene_uspp": (workloads.graphene_uspp, None, None, "dense"),
    "graphene_2x2": (workloads.graphene_2x2, [0], 64, "fft"),
    "surface": (workloads.surface, [0], 32, "fft"),
    "member12": (lambda: workloads.batched_member(12), None, None, "fft"),
    "member33": (lambda: workloads.batched_member(33), None, None, "fft"),
    "ribbon_narrow": (workloads.ribbon_narrow, None, None, "wire-dense"),
}


def main(name: str, kpoints=None):
    make, ks_default, nev_set, local = SETS[name]
    desc = make()
    nev = nev_set or desc["nbands"]
    out = {"config": name, "desc_name": desc["name"], "nev": nev,
           "method": f"oracle.matfree (local={local}) + scipy lobpcg, tol 1e-9", "kpoints": {}}
    path = os.path.join(HERE, f"{name}_eigs.json")
    if os.path.exists(path):
        out = json.load(open(path))
    ks = kpoints if kpoints is not None else (ks_default if ks_default is not None else range(len(desc["kpts"])))
    vgrid = None
    if local == "fft" and desc["atoms"]:
        zb = ZBasis(desc["breakpoints"], desc["order"], desc["nq"])
        vgrid = operators.gaussian_potential_on_grid_separable(desc, zb.zq)
    if local == "wire-dense":
        out["method"] = "oracle.wire dense H, S + scipy eigh (LAPACK)"
    for ik in ks:
        if str(ik) in out["kpoints"]:
            continue
        t = time.time()
        if local == "wire-dense":
            eps, C = wire.lowest(desc, ik, nev)
            pr = wire.WireProblem(desc, ik)
            r = [float(v) for v in np.linalg.norm(pr.hamiltonian() @ C - (pr.overlap() @ C) * eps, axis=0)]
            out["kpoints"][str(ik)] = {"eps": [float(v) for v in eps], "resid": r, "seconds": time.time() - t}
            print(f"{name} k{ik}: max resid {max(r):.2e}, {time.time() - t:.0f} s", flush=True)
            json.dump(out, open(path, "w"), indent=1)
            continue
        mf = matfree.MatFree(desc, ik, local=local, vgrid=vgrid)
        eps, _, r = mf.lowest(nev, extra=8, tol=1e-9, maxiter=3000, seed=ik)
        out["kpoints"][str(ik)] = {"eps": [float(v) for v in eps], "resid": [float(v) for v in r],
                                   "seconds": time.time() - t}
        print(f"{name} k{ik}: max resid {max(r):.2e}, {time.time() - t:.0f} s", flush=True)
        json.dump(out, open(path, "w"), indent=1)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "graphene",
         [int(v) for v in sys.argv[2:]] if len(sys.argv) > 2 else None)
