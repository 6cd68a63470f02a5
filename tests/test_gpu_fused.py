"""GPU parity of the fused sweeps (FP32-scaled form, alpha never
materialised) against the CPU oracle.

The fused path is taken where materialised alpha would not fit (from n = 23);
BN_FUSED_ALPHA=1 takes it from n = 10, so that problems the oracle solves
in seconds exercise it:
* lattices whose 9-bit blocks have 1..11 high bits (n = 10..21), both seed
  kernels (per-seed below 8 high bits, grouped from 8), in-degree bounds
  0..6, mixed arities, K2 and a custom prior;
* BN_LINEAR_TILES=force, which runs every seed and every block in the number
  system itself (the path of blocks whose range exceeds one FP64 scale);
* near-copy data whose scores span about 2^2700, which sends real blocks and
  nodes down that path;
* the forward-only mode of the modular-feature entry point.
Tolerance 1e-5 absolute on every posterior (the FP32-scaled target), plus
the invariants of the number system.
"""
import numpy as np
import pytest

import paper_1408_1664_amd as bn
from oracle import oracle as O
from paper_1408_1664_amd import datagen

pytestmark = pytest.mark.gpu


def ranked_masks(N, d):
    """Compressed parent-set masks in the library's rank order (size, then colex)."""
    x = np.arange(1 << N, dtype=np.int64)
    pc = np.zeros_like(x)
    for b in range(N):
        pc += (x >> b) & 1
    return np.concatenate([x[pc == k] for k in range(min(d, N) + 1)])


def expand(c, i):
    return (c & ((1 << i) - 1)) | ((c >> i) << (i + 1))


def _check(post, rep, ref, tol=1e-5):
    err = np.abs(post - ref["post"]).max()
    print(f"  fused: max |dP| = {err:.3e}  log L(V) {rep['log_LV']:.6f} vs {ref['log_LV']:.6f}"
          f"  resid {rep['max_invariant_residual']:.2e} sat {rep['saturated']} "
          f"flush {rep['flushed']} slow blocks {rep['fallback_tiles']}", flush=True)
    assert err <= tol
    assert np.all(np.diag(post) == 0)
    assert abs(rep["log_LV"] - ref["log_LV"]) <= 1e-6 * max(1.0, abs(ref["log_LV"]))
    assert rep["max_invariant_residual"] < 1e-4
    assert rep["saturated"] == 0


CASES = [
    # (n, m, arity, maxdeg, d, seed)
    (10, 300, 2, 3, 3, 1), (11, 200, 3, 2, 2, 2), (12, 200, 2, 3, 3, 3), (13, 500, 2, 3, 0, 4),
    (14, 150, [2, 3] * 7, 2, 1, 5), (15, 400, 2, 4, 6, 6), (17, 800, 2, 3, 4, 7),
    (18, 300, 2, 3, 3, 8), (19, 1000, 3, 3, 2, 9), (21, 500, 2, 3, 3, 10),
]


@pytest.mark.parametrize("mode", ["1", "force"])
@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}d{c[4]}" for c in CASES])
def test_fused_matches_oracle(case, mode, monkeypatch):
    monkeypatch.setenv("BN_FUSED_ALPHA", "1")
    monkeypatch.setenv("BN_LINEAR_TILES", mode)
    n, m, ar, maxdeg, d, seed = case
    ds = datagen.random_dag_dataset(n, m, ar, maxdeg, 1.0, seed=seed)
    print(f"fused n={n} m={m} d={d} mode={mode}", flush=True)
    ref = O.edge_posteriors(ds.data, ds.arity, d)
    post, rep = bn.edge_posteriors(ds.data, ds.arity, d, precision="fp32")
    _check(post, rep, ref)
    if d == 0:
        assert np.all(post == 0)
    if mode == "force":
        assert rep["fallback_tiles"] > 0


@pytest.mark.parametrize("name", ["n12_binary_m200_d3", "n20_ternary_m1000_d4"])
def test_fused_workloads_and_parent_sets(name, monkeypatch):
    monkeypatch.setenv("BN_FUSED_ALPHA", "1")
    ds, p = datagen.workload(name)
    ref = O.edge_posteriors(ds.data, ds.arity, p["d"], ess=p["ess"])
    ps, post, rep = bn.parent_set_posteriors(ds.data, ds.arity, p["d"], precision="fp32",
                                             ess=p["ess"])
    _check(post, rep, ref)
    np.testing.assert_allclose(ps.sum(axis=1), 1.0, atol=1e-4)
    # the materialised form on the same inputs
    monkeypatch.setenv("BN_FUSED_ALPHA", "0")
    post0, _ = bn.edge_posteriors(ds.data, ds.arity, p["d"], precision="fp32", ess=p["ess"])
    assert np.abs(post - post0).max() <= 1e-5


def test_fused_custom_prior_and_k2(monkeypatch):
    monkeypatch.setenv("BN_FUSED_ALPHA", "1")
    ds = datagen.random_dag_dataset(14, 400, 3, 3, 1.0, seed=12)
    rng = np.random.default_rng(3)
    log_rho = rng.normal(size=4)
    log_q = rng.normal(size=14) * 3
    ref = O.edge_posteriors(ds.data, ds.arity, 3, kind=O.K2, log_rho=log_rho, log_q=log_q)
    post, rep = bn.edge_posteriors(ds.data, ds.arity, 3, precision="fp32", score="k2",
                                   log_rho=log_rho, log_q=log_q)
    _check(post, rep, ref)


def _near_copies(n, m, copies, flip, seed):
    rng = np.random.default_rng(seed)
    x = rng.integers(0, 2, size=(n, m)).astype(np.uint8)
    for j in range(1, copies + 1):
        x[j] = x[0] ^ (rng.random(m) < flip).astype(np.uint8)
    return x, np.full(n, 2, dtype=np.uint8)


@pytest.mark.parametrize("n", [14, 19])
def test_fused_wide_range_blocks(n, monkeypatch):
    """Near-deterministic copies make some scores about 2^2700 times the
    empty set's: those nodes' seeds and blocks run in the number system."""
    monkeypatch.setenv("BN_FUSED_ALPHA", "1")
    data, ar = _near_copies(n, 3000, 3, 0.01, seed=11)
    ref = O.edge_posteriors(data, ar, 3)
    post, rep = bn.edge_posteriors(data, ar, 3, precision="fp32")
    _check(post, rep, ref)
    assert rep["fallback_tiles"] > 0


@pytest.mark.parametrize("mode", ["1", "force"])
def test_fused_forward_only_feature(mode, monkeypatch):
    monkeypatch.setenv("BN_FUSED_ALPHA", "1")
    monkeypatch.setenv("BN_LINEAR_TILES", mode)
    ds = datagen.random_dag_dataset(15, 500, 2, 3, 1.0, seed=21)
    d = 3
    n = ds.n
    masks = ranked_masks(n - 1, d)
    rng = np.random.default_rng(5)
    log_f = np.log(rng.uniform(0.05, 2.0, size=(n, len(masks))))
    full = np.zeros((n, 1 << n))
    for v in range(n):
        full[v, expand(masks, v)] = log_f[v]
    logB = O.full_log_beta(ds.data, ds.arity, d)
    want = O.modular_feature_posterior(logB, d, full)
    got = bn.modular_feature_posterior(ds.data, ds.arity, d, log_f, precision="fp32")
    print(f"feature: {got['value']:.9e} vs {want['value']:.9e}", flush=True)
    assert abs(got["value"] - want["value"]) <= 1e-5 * abs(want["value"])
