"""Write oracle reference posteriors for workloads too large to re-run in a test.

Calls only the CPU oracle (oracle/) and the seeded input generator; the GPU
library is never imported. Output: tests/golden/oracle_<workload>.json with
the posterior matrix, log P(D) and the oracle's invariant residuals.

    python tests/golden/make_oracle_refs.py n25_binary_m2000_d4
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1408_1664_amd import datagen  # noqa: E402


def main(names):
    for name in names:
        ds, p = datagen.workload(name)
        t0 = time.time()
        r = O.edge_posteriors(ds.data, ds.arity, p["d"], ess=p["ess"])
        out = dict(workload=name, n=ds.n, m=ds.m, d=p["d"], ess=p["ess"],
                   generator="paper_1408_1664_amd.datagen.workload", oracle="oracle/bn_oracle.c",
                   log_LV=r["log_LV"], r_LR=r["r_LR"], r_layers=r["r_layers"],
                   r_gamma=r["r_gamma"], seconds=time.time() - t0,
                   threads=O.num_threads(), post=r["post"].tolist())
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"oracle_{name}.json")
        with open(path, "w") as f:
            json.dump(out, f)
        print(f"{name}: log L(V) {r['log_LV']:.6f}, {out['seconds']:.1f} s -> {path}")


if __name__ == "__main__":
    main(sys.argv[1:] or ["n25_binary_m2000_d4"])
