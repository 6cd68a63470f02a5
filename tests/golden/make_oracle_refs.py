"""Write oracle reference posteriors for workloads too large to re-run in a test.

Calls only the CPU oracle (oracle/) and the seeded input generator; the GPU
library is never imported. Output: tests/golden/oracle_<workload>.json with
the posterior matrix, log P(D) and the oracle's invariant residuals.

    python tests/golden/make_oracle_refs.py n25_binary_m2000_d4
    python tests/golden/make_oracle_refs.py n30_binary_m500_d3:27

A suffix ":k" keeps the first k variables of the workload's dataset (its
first k data rows and arities; the same samples, d and score), so that a
lattice too large for the oracle's host memory is pinned on its largest
prefix that fits (n = 27 needs about 40 GB).
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
    for spec in names:
        name, _, first = spec.partition(":")
        ds, p = datagen.workload(name)
        k = int(first) if first else ds.n
        data, arity = ds.data[:k], ds.arity[:k]
        t0 = time.time()
        r = O.edge_posteriors(data, arity, p["d"], ess=p["ess"])
        tag = name if k == ds.n else f"{name}_first{k}"
        out = dict(workload=name, first_vars=k, n=k, m=ds.m, d=p["d"], ess=p["ess"],
                   generator="paper_1408_1664_amd.datagen.workload", oracle="oracle/bn_oracle.c",
                   log_LV=r["log_LV"], r_LR=r["r_LR"], r_layers=r["r_layers"],
                   r_gamma=r["r_gamma"], seconds=time.time() - t0,
                   threads=O.num_threads(), post=r["post"].tolist())
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"oracle_{tag}.json")
        with open(path, "w") as f:
            json.dump(out, f)
        print(f"{tag}: log L(V) {r['log_LV']:.6f}, {out['seconds']:.1f} s -> {path}")


if __name__ == "__main__":
    main(sys.argv[1:] or ["n25_binary_m2000_d4"])
