"""Write stored oracle eigenvalues for the full-size parity tests.

    python tests/golden/make_golden.py graphene      # -> tests/golden/graphene_eigs.json

Calls only the oracle (matrix-free FP64 operator + scipy LOBPCG, residual
<= 1e-9 per eigenpair); the values are the discrete eigenvalues of the
graphene-like slab (hexagonal a = 4.65 bohr, 36x36 grid, 80 graded cubic
B-splines, 2 atoms with 4 Kleinman-Bylander projectors each, 2x2 MP k-points),
32 lowest per k-point.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import matfree  # noqa: E402
from paper_1406_4960_amd import workloads  # noqa: E402


def main(name: str, kpoints=None):
    desc = workloads.CONFIGS[name]()
    nev = desc["nbands"]
    out = {"config": name, "desc_name": desc["name"], "nev": nev, "method": "oracle.matfree + scipy lobpcg",
           "kpoints": {}}
    path = os.path.join(HERE, f"{name}_eigs.json")
    if os.path.exists(path):
        out = json.load(open(path))
    ks = kpoints if kpoints is not None else range(len(desc["kpts"]))
    for ik in ks:
        if str(ik) in out["kpoints"]:
            continue
        t = time.time()
        mf = matfree.MatFree(desc, ik)
        eps, _, r = mf.lowest(nev, extra=8, tol=1e-9, maxiter=3000, seed=ik)
        out["kpoints"][str(ik)] = {"eps": [float(v) for v in eps], "resid": [float(v) for v in r],
                                   "seconds": time.time() - t}
        print(f"k{ik}: max resid {max(r):.2e}, {time.time() - t:.0f} s", flush=True)
        json.dump(out, open(path, "w"), indent=1)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "graphene",
         [int(v) for v in sys.argv[2:]] if len(sys.argv) > 2 else None)
