"""Seeded synthetic inputs for the edge-posterior engine.

This module only draws data. It holds none of the method's arithmetic (no
scores, no transforms, no dynamic programme), so both the oracle tests and
the GPU path can take their inputs from it.

The paper evaluates on synthetic datasets of discrete random variables with
500 samples each (Sec. 4.1) but does not describe the generator. The recipe
used here:

* ``rng = numpy.random.default_rng(seed)`` (PCG64);
* a random topological order ``perm = rng.permutation(n)``;
* for the t-th node of ``perm``: ``k = rng.integers(0, min(maxdeg, t) + 1)``
  parents drawn with ``rng.choice(perm[:t], k, replace=False)``, then one
  conditional-probability row per parent configuration (mixed radix, first
  drawn parent most significant) from ``rng.dirichlet([a] * r)``;
* after the structure and every table are drawn, ``m`` samples by ancestral
  sampling in ``perm`` order, each value by inverse CDF on ``rng.random(m)``.

Data are returned column-major as ``uint8[n, m]`` (row i holds variable i).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Dataset:
    data: np.ndarray          # uint8 [n, m], row i = variable i
    arity: np.ndarray         # uint8 [n]
    parents: list             # true DAG: parents[i] = list of parent indices
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.data.shape[0])

    @property
    def m(self) -> int:
        return int(self.data.shape[1])


def random_dag_dataset(n: int, m: int, arity, maxdeg: int, dirichlet_a: float,
                       seed: int) -> Dataset:
    """Draw a random DAG with in-degree <= maxdeg, Dirichlet(a) tables and m samples."""
    if n < 1:
        raise ValueError("n must be >= 1")
    if m < 0:
        raise ValueError("m must be >= 0")
    rng = np.random.default_rng(seed)
    ar = np.broadcast_to(np.asarray(arity, dtype=np.int64), (n,)).copy()
    if np.any(ar < 2) or np.any(ar > 255):
        raise ValueError("arity must be in 2..255")
    perm = rng.permutation(n)
    parents: list = [[] for _ in range(n)]
    cpts: list = [None] * n
    for t, node in enumerate(perm):
        k = int(rng.integers(0, min(maxdeg, t) + 1))
        ps = [int(p) for p in rng.choice(perm[:t], k, replace=False)] if k > 0 else []
        parents[node] = ps
        q = int(np.prod([ar[p] for p in ps])) if ps else 1
        cpts[node] = rng.dirichlet([dirichlet_a] * int(ar[node]), size=q)
    data = np.zeros((n, m), dtype=np.uint8)
    for node in perm:
        ps = parents[node]
        cfg = np.zeros(m, dtype=np.int64)
        for p in ps:                       # first parent most significant
            cfg = cfg * ar[p] + data[p].astype(np.int64)
        cdf = np.cumsum(cpts[node][cfg], axis=1)
        u = rng.random(m)
        x = (u[:, None] >= cdf[:, :-1]).sum(axis=1)
        data[node] = np.minimum(x, ar[node] - 1).astype(np.uint8)
    return Dataset(data=data, arity=ar.astype(np.uint8), parents=parents, seed=seed,
                   meta=dict(n=n, m=m, maxdeg=maxdeg, dirichlet_a=dirichlet_a))


# Workloads. Each entry: data recipe + method parameters. The method parameters
# are d (in-degree bound) and ess (BDeu equivalent sample size); the prior is the
# library default (q == 1, rho_k = 1 / C(n-1, k)).
WORKLOADS = {
    # n=12 binary, m=200, DAG in-degree <= 3, Dirichlet(1); d=3
    "n12_binary_m200_d3": dict(n=12, m=200, arity=2, maxdeg=3, a=1.0, d=3, ess=1.0, seed=1),
    # n=20 ternary, m=1000, in-degree <= 4, Dirichlet(0.5); d=4
    "n20_ternary_m1000_d4": dict(n=20, m=1000, arity=3, maxdeg=4, a=0.5, d=4, ess=1.0, seed=2),
    # n=25 binary, m=2000, in-degree <= 4, Dirichlet(1); d=4
    "n25_binary_m2000_d4": dict(n=25, m=2000, arity=2, maxdeg=4, a=1.0, d=4, ess=1.0, seed=3),
    # n=30 binary, m=500, in-degree <= 3, Dirichlet(1); d=3
    "n30_binary_m500_d3": dict(n=30, m=500, arity=2, maxdeg=3, a=1.0, d=3, ess=1.0, seed=5),
}


def workload(name: str, **override) -> tuple[Dataset, dict]:
    """Return (dataset, method parameters) for a named workload."""
    w = dict(WORKLOADS[name])
    w.update(override)
    ds = random_dag_dataset(w["n"], w["m"], w["arity"], w["maxdeg"], w["a"], w["seed"])
    return ds, dict(d=w["d"], ess=w["ess"])


def serving_stream(num: int = 512, seed: int = 4, rate_hz: float | None = None):
    """Request stream for the serving workload.

    Request j: seed 4_000_000 + j, n ~ U{10..22}, m ~ U{100..2000}, one arity
    r ~ U{2,3} for all variables, DAG in-degree <= 3, Dirichlet(1); d = 3.
    Arrival gaps are exponential (Poisson arrivals) when ``rate_hz`` is given,
    else every request arrives at t = 0.
    """
    rng = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    for j in range(num):
        n = int(rng.integers(10, 23))
        m = int(rng.integers(100, 2001))
        r = int(rng.integers(2, 4))
        if rate_hz:
            t += float(rng.exponential(1.0 / rate_hz))
        reqs.append(dict(idx=j, seed=4_000_000 + j, n=n, m=m, arity=r, maxdeg=3,
                         a=1.0, d=3, ess=1.0, arrival_s=t))
    return reqs


def request_dataset(req: dict) -> Dataset:
    return random_dag_dataset(req["n"], req["m"], req["arity"], req["maxdeg"], req["a"],
                              req["seed"])


def subset_values(nbits: int, seed: int, dist: str = "uniform") -> np.ndarray:
    """2^nbits float64 values x[S] for the subset transforms.

    dist: "uniform" U[0, 1) (nonnegative, like the products the method sums);
    "signed" standard normal; "int" integers in [-1000, 1000] (every partial
    sum is exact in FP64 up to 2^43 terms); "wide" 2^u with u ~ U[-600, 0]
    (positive values spread over 180 decades, like probabilities);
    "ones" all 1. rng = numpy.random.default_rng(seed).
    """
    size = 1 << nbits
    rng = np.random.default_rng(seed)
    if dist == "uniform":
        return rng.random(size)
    if dist == "signed":
        return rng.standard_normal(size)
    if dist == "int":
        return rng.integers(-1000, 1001, size).astype(np.float64)
    if dist == "wide":
        return np.exp2(rng.uniform(-600.0, 0.0, size))
    if dist == "ones":
        return np.ones(size)
    raise ValueError(f"unknown distribution {dist!r}")
