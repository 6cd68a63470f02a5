"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (absolute, on posteriors):
* FP64 log-space form: 1e-10. Both sides evaluate the same sums in FP64
  logarithms; they differ only in summation order (tree versus sequential),
  i.e. by a few units of 2^-52 relative per value, far below 1e-10 even
  after the ~n layers of the lattice.
* FP32-scaled form: 1e-5, the target accuracy. FP32 rounding at each
  operation is ~6e-8 relative; over the zeta passes and the lattice layers
  the accumulated error stays around 1e-7..1e-6.
Local scores: relative 1e-12 (both are sums of FP64 log-gamma values).
"""
import os

import numpy as np
import pytest

import paper_1408_1664_amd as bn
from oracle import oracle as O
from paper_1408_1664_amd import datagen

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5}


def ranked_masks(N, d):
    """Compressed parent-set masks in the library's rank order (size, then colex)."""
    x = np.arange(1 << N, dtype=np.int64)
    pc = np.zeros_like(x)
    for b in range(N):
        pc += (x >> b) & 1
    return np.concatenate([x[pc == k] for k in range(min(d, N) + 1)])


def expand(c, i):
    low = c & ((1 << i) - 1)
    return low | ((c >> i) << (i + 1))


def _oracle(ds, d, ess=1.0, kind=O.BDEU, log_rho=None, log_q=None):
    return O.edge_posteriors(ds.data, ds.arity, d, kind=kind, ess=ess, log_rho=log_rho,
                             log_q=log_q)


def _check(post, rep, ref, prec):
    n = post.shape[0]
    err = np.abs(post - ref["post"]).max()
    print(f"  {prec}: max |dP| = {err:.3e}  log L(V) {rep['log_LV']:.6f} vs {ref['log_LV']:.6f}"
          f"  resid {rep['max_invariant_residual']:.2e} sat {rep['saturated']} "
          f"flush {rep['flushed']}", flush=True)
    assert err <= TOL[prec]
    assert np.all(np.diag(post) == 0)
    assert abs(rep["log_LV"] - ref["log_LV"]) <= (1e-9 if prec == "fp64" else 1e-6) * max(
        1.0, abs(ref["log_LV"]))
    assert rep["max_invariant_residual"] < (1e-9 if prec == "fp64" else 1e-4)
    assert rep["saturated"] == 0


# ------------------------------------------------------------- a1 scores

@pytest.mark.parametrize("name", ["n12_binary_m200_d3", "n20_ternary_m1000_d4"])
def test_local_scores_match_oracle(name):
    ds, p = datagen.workload(name)
    n, d = ds.n, p["d"]
    got = bn.local_scores(ds.data, ds.arity, d, ess=p["ess"])
    ref = O.local_scores(ds.data, ds.arity, d, O.BDEU, p["ess"])
    masks = ranked_masks(n - 1, d)
    assert got.shape == (n, len(masks))
    for i in range(n):
        want = ref[i, expand(masks, i)]
        np.testing.assert_allclose(got[i], want, rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("kind", ["bdeu", "k2"])
def test_local_scores_binary_bitplanes(kind):
    """All-binary data with d <= 4 is counted from bit planes; m not a
    multiple of 32 leaves a ragged last word."""
    ds = datagen.random_dag_dataset(11, 777, 2, 4, 1.0, seed=19)
    got = bn.local_scores(ds.data, ds.arity, 4, score=kind, ess=2.5)
    ref = O.local_scores(ds.data, ds.arity, 4, O.K2 if kind == "k2" else O.BDEU, 2.5)
    masks = ranked_masks(10, 4)
    for i in range(11):
        np.testing.assert_allclose(got[i], ref[i, expand(masks, i)], rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("kind", ["bdeu", "k2"])
@pytest.mark.parametrize("r,d,m", [(3, 3, 1001), (3, 4, 70), (4, 2, 257), (5, 4, 300)])
def test_local_scores_uniform_arity_tables(kind, r, d, m, monkeypatch):
    """Every variable of arity r, d <= 4: the log-gamma values come from
    tables (q = r^k for k parents). Against the oracle, and bitwise against
    the same kernel with lgamma evaluated per family (BN_SCORE_TABLES=0);
    m = 70 and 257 leave the four-sample steps ragged."""
    ds = datagen.random_dag_dataset(10, m, r, min(d, 3), 1.0, seed=31 + r + d)
    print(f"uniform arity scores r={r} d={d} m={m} kind={kind}", flush=True)
    got = bn.local_scores(ds.data, ds.arity, d, score=kind, ess=1.5)
    ref = O.local_scores(ds.data, ds.arity, d, O.K2 if kind == "k2" else O.BDEU, 1.5)
    masks = ranked_masks(9, d)
    for i in range(10):
        np.testing.assert_allclose(got[i], ref[i, expand(masks, i)], rtol=1e-12, atol=1e-10)
    monkeypatch.setenv("BN_SCORE_TABLES", "0")
    per_family = bn.local_scores(ds.data, ds.arity, d, score=kind, ess=1.5)
    assert np.array_equal(got, per_family)


def test_local_scores_k2_mixed_arity():
    ds = datagen.random_dag_dataset(9, 333, [2, 3, 4, 2, 5, 3, 2, 2, 3], 3, 0.7, seed=8)
    got = bn.local_scores(ds.data, ds.arity, 3, score="k2")
    ref = O.local_scores(ds.data, ds.arity, 3, O.K2)
    masks = ranked_masks(8, 3)
    for i in range(9):
        np.testing.assert_allclose(got[i], ref[i, expand(masks, i)], rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("kind", ["bdeu", "k2"])
def test_local_scores_large_histograms(kind):
    """Families with more than 2048 histogram bins (here up to 5 * 5*5*4*4*4
    = 8000 at d = 5) take the one-family-per-workgroup score kernel; smaller
    ones are counted four families per workgroup, one wave each (the tests
    above)."""
    ar = [5, 4, 5, 4, 3, 3, 2, 4, 5]
    ds = datagen.random_dag_dataset(9, 400, ar, 3, 0.8, seed=23)
    got = bn.local_scores(ds.data, ds.arity, 5, score=kind, ess=1.5)
    ref = O.local_scores(ds.data, ds.arity, 5, O.K2 if kind == "k2" else O.BDEU, 1.5)
    masks = ranked_masks(8, 5)
    for i in range(9):
        np.testing.assert_allclose(got[i], ref[i, expand(masks, i)], rtol=1e-12, atol=1e-10)


# ------------------------------------------------------- whole path, a1-a7

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["n12_binary_m200_d3", "n20_ternary_m1000_d4"])
def test_posteriors_match_oracle(name, prec):
    ds, p = datagen.workload(name)
    ref = _oracle(ds, p["d"], p["ess"])
    post, rep = bn.edge_posteriors(ds.data, ds.arity, p["d"], precision=prec, ess=p["ess"])
    _check(post, rep, ref, prec)


SMALL = [
    # (n, m, arity, maxdeg, d, seed)
    (2, 50, 2, 1, 1, 1), (3, 0, 2, 2, 2, 2), (4, 17, 3, 2, 1, 3), (5, 100, 2, 3, 0, 4),
    (6, 250, [2, 3, 4, 2, 3, 2], 2, 2, 5), (7, 400, 2, 3, 6, 6), (9, 1000, 2, 3, 3, 7),
    (11, 300, 3, 2, 2, 8), (13, 500, 2, 4, 4, 9), (14, 64, 2, 2, 3, 10),
    # large in-degree bounds on the 12-bit Gamma tile and the 13-bit alpha tile:
    # most lanes of the pattern layouts are live (every lane group for d >= 5)
    (15, 400, 2, 4, 6, 11), (16, 300, 2, 3, 8, 12),
    # alpha seeds by blocks of tiles (n >= 22) with a large in-degree bound
    (22, 200, 2, 3, 6, 13),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", SMALL, ids=[f"n{c[0]}m{c[1]}d{c[4]}" for c in SMALL])
def test_small_and_degenerate(case, prec):
    n, m, ar, maxdeg, d, seed = case
    ds = datagen.random_dag_dataset(n, m, ar, maxdeg, 1.0, seed=seed)
    ref = _oracle(ds, d)
    post, rep = bn.edge_posteriors(ds.data, ds.arity, d, precision=prec)
    _check(post, rep, ref, prec)
    if d == 0:
        assert np.all(post == 0)


TILES = ["1,1,1,1", "2,3,2,2", "3,4,3,3", "5,2,4,3", "4,6,2,5"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("tiles", TILES)
def test_every_tiling_path(tiles, prec, monkeypatch):
    """Small tiles force many sweep layers, multi-tile alpha and the two-level
    Gamma reduction on problems the oracle solves instantly."""
    monkeypatch.setenv("BN_TILE_BITS", tiles)
    ds = datagen.random_dag_dataset(12, 300, 2, 3, 1.0, seed=77)
    ref = _oracle(ds, 3)
    post, rep = bn.edge_posteriors(ds.data, ds.arity, 3, precision=prec)
    _check(post, rep, ref, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("mode", ["1", "force", "0"])
def test_linear_tiles_and_fallback(mode, prec, monkeypatch):
    """The alpha and Gamma in-tile zetas run on scaled doubles and hand the
    tiles whose range does not fit to the number-system kernels. 'force'
    sends every tile down that path, '0' turns the linear form off; all three
    must agree with the oracle. n = 20 uses 13-bit alpha tiles (64 per node)
    and 12-bit Gamma tiles (256)."""
    monkeypatch.setenv("BN_LINEAR_TILES", mode)
    ds, p = datagen.workload("n20_ternary_m1000_d4")
    ref = _oracle(ds, p["d"], p["ess"])
    post, rep = bn.edge_posteriors(ds.data, ds.arity, p["d"], precision=prec, ess=p["ess"])
    _check(post, rep, ref, prec)
    n = ds.n
    want = n * 2 ** (n - 1 - 13) + 2 ** (n - 12) if mode == "force" else 0
    assert rep["fallback_tiles"] == want


def _near_copies(n, m, copies, flip, seed):
    """Variable 0 uniform; variables 1..copies equal to it except for a
    fraction `flip` of samples; the rest independent uniform bits."""
    rng = np.random.default_rng(seed)
    x = rng.integers(0, 2, size=(n, m)).astype(np.uint8)
    for j in range(1, copies + 1):
        x[j] = x[0] ^ (rng.random(m) < flip).astype(np.uint8)
    return x, np.full(n, 2, dtype=np.uint8)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_wide_range_tiles_fall_back(prec):
    """Near-deterministic copies over 3000 samples make a parent set about
    2^2700 times likelier than the empty set, beyond what one FP64 scale per
    tile can hold: those tiles must take the fallback path and the result
    must still match the oracle."""
    data, ar = _near_copies(14, 3000, 3, 0.01, seed=11)
    ref = O.edge_posteriors(data, ar, 3)
    post, rep = bn.edge_posteriors(data, ar, 3, precision=prec)
    _check(post, rep, ref, prec)
    assert rep["fallback_tiles"] > 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["n12_binary_m200_d3", "n20_ternary_m1000_d4"])
def test_parent_set_posteriors_match_oracle(name, prec):
    """P(G_v = G | D) for every ranked parent set against the oracle; rows
    sum to 1; the edge posteriors returned alongside equal the edge entry."""
    ds, p = datagen.workload(name)
    n, d = ds.n, p["d"]
    logB = O.full_log_beta(ds.data, ds.arity, d, ess=p["ess"])
    ref = O.parent_set_posteriors(logB, d)
    ps, post, rep = bn.parent_set_posteriors(ds.data, ds.arity, d, precision=prec, ess=p["ess"])
    masks = ranked_masks(n - 1, d)
    want = np.stack([ref["ps"][v, expand(masks, v)] for v in range(n)])
    err = np.abs(ps - want).max()
    print(f"  {prec}: max |dP(G_v = G)| = {err:.3e}", flush=True)
    assert err <= TOL[prec]
    np.testing.assert_allclose(ps.sum(axis=1), 1.0, atol=TOL[prec] * 10)
    alone, _ = bn.edge_posteriors(ds.data, ds.arity, d, precision=prec, ess=p["ess"])
    assert np.array_equal(post, alone)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_custom_prior_and_k2(prec):
    ds = datagen.random_dag_dataset(10, 400, 3, 3, 1.0, seed=12)
    rng = np.random.default_rng(3)
    log_rho = rng.normal(size=4)
    log_q = rng.normal(size=10) * 3
    ref = _oracle(ds, 3, kind=O.K2, log_rho=log_rho, log_q=log_q)
    post, rep = bn.edge_posteriors(ds.data, ds.arity, 3, precision=prec, score="k2",
                                   log_rho=log_rho, log_q=log_q)
    _check(post, rep, ref, prec)


def test_deterministic_bitwise():
    ds, p = datagen.workload("n12_binary_m200_d3")
    for prec in ("fp64", "fp32"):
        a, _ = bn.edge_posteriors(ds.data, ds.arity, p["d"], precision=prec)
        b, _ = bn.edge_posteriors(ds.data, ds.arity, p["d"], precision=prec)
        assert np.array_equal(a, b)


def test_device_entry_matches_host_entry():
    import torch
    ds, p = datagen.workload("n20_ternary_m1000_d4")
    n, m = ds.n, ds.m
    for prec in ("fp64", "fp32"):
        host, rep = bn.edge_posteriors(ds.data, ds.arity, p["d"], precision=prec)
        ws = torch.empty(bn.workspace_bytes(n, p["d"], m, prec), dtype=torch.uint8,
                         device="cuda")
        data = torch.from_numpy(ds.data).cuda()
        post = torch.empty((n, n), dtype=torch.float64, device="cuda")
        diag = torch.zeros(8, dtype=torch.float64, device="cuda")
        bn.edge_posteriors_dev(data, ds.arity, p["d"], prec, ws, post, diag)
        torch.cuda.synchronize()
        assert np.array_equal(post.cpu().numpy(), host)
        assert diag[0].item() == pytest.approx(rep["log_LV"], abs=1e-12)


_FEATURE_REF = {}


def _ranked_feature(n, d, rng, kind):
    """log f as [n, K] in rank order and as the [n, 2^n] full-mask array of
    the oracle. kind: 'weights' (f in (0, 2]), 'mask' (random zeros, f(empty)
    = 1), 'noedges' (f_v(G) = [u not in G] for a few pairs)."""
    masks = ranked_masks(n - 1, d)
    K = len(masks)
    full = np.zeros((n, 1 << n))
    if kind == "weights":
        lf = np.log(rng.uniform(0.05, 2.0, size=(n, K)))
    elif kind == "mask":
        lf = np.where(rng.random((n, K)) < 0.3, -np.inf, 0.0)
        lf[:, 0] = 0.0
    else:
        lf = np.zeros((n, K))
        for _ in range(3):
            u, v = rng.choice(n, 2, replace=False)
            pu = u if u < v else u - 1          # u's bit in v's compressed masks
            lf[v] = np.where((masks >> pu) & 1, -np.inf, lf[v])
    for v in range(n):
        full[v, expand(masks, v)] = lf[v]
    return lf, full


@pytest.mark.parametrize("name", ["n12_binary_m200_d3", "n20_ternary_m1000_d4"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", ["weights", "mask", "noedges"])
def test_modular_feature_matches_oracle(name, prec, kind):
    """E[f | D] of modular features against the oracle (forward sums with and
    without f); relative tolerance of the number system on the ratio."""
    ds, p = datagen.workload(name)
    n, d = ds.n, p["d"]
    rng = np.random.default_rng(sum(map(ord, name + kind)))
    lf, full = _ranked_feature(n, d, rng, kind)
    key = (name, kind)
    if key not in _FEATURE_REF:     # the oracle once per workload and feature
        logB = O.full_log_beta(ds.data, ds.arity, d, ess=p["ess"])
        _FEATURE_REF[key] = O.modular_feature_posterior(logB, d, full)
    ref = _FEATURE_REF[key]
    got = bn.modular_feature_posterior(ds.data, ds.arity, d, lf, precision=prec, ess=p["ess"])
    print(f"  {name} {prec} {kind}: {got['value']:.12g} vs {ref['value']:.12g}", flush=True)
    assert got["value"] == pytest.approx(ref["value"], rel=TOL[prec], abs=1e-300)
    assert got["log_PD"] - got["log_PfD"] == pytest.approx(ref["log_LV"] - ref["log_LfV"],
                                                           abs=TOL[prec])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_modular_feature_edges_and_sets_agree_with_solve(prec):
    """f_v(G) = [u in G] gives the edge posterior of the full solve, f_v(G) =
    [G = G0] its parent-set posterior, f = 1 gives 1 (n = 25, GPU against
    GPU, both through the C ABI)."""
    ds, p = datagen.workload("n25_binary_m2000_d4")
    n, d = ds.n, p["d"]
    ps, post, _ = bn.parent_set_posteriors(ds.data, ds.arity, d, precision=prec, ess=p["ess"])
    masks = ranked_masks(n - 1, d)
    K = len(masks)
    one = bn.modular_feature_posterior(ds.data, ds.arity, d, np.zeros((n, K)), precision=prec,
                                       ess=p["ess"])
    assert one["value"] == pytest.approx(1.0, abs=TOL[prec])
    order = np.argsort(-post, axis=None)[:3]
    for flat in order:
        u, v = divmod(int(flat), n)
        pu = u if u < v else u - 1
        lf = np.zeros((n, K))
        lf[v] = np.where((masks >> pu) & 1, 0.0, -np.inf)
        r = bn.modular_feature_posterior(ds.data, ds.arity, d, lf, precision=prec, ess=p["ess"])
        print(f"  edge {u}->{v}: {r['value']:.9f} vs {post[u, v]:.9f}", flush=True)
        assert r["value"] == pytest.approx(post[u, v], abs=TOL[prec] * 10)
    v, r0 = divmod(int(np.argmax(ps)), K)
    lf = np.zeros((n, K))
    lf[v] = -np.inf
    lf[v, r0] = 0.0
    r = bn.modular_feature_posterior(ds.data, ds.arity, d, lf, precision=prec, ess=p["ess"])
    assert r["value"] == pytest.approx(ps[v, r0], abs=TOL[prec] * 10)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_modular_feature_custom_prior_and_k2(prec):
    """A modular feature under a custom order-modular prior (log rho, log q)
    and the K2 score, against the oracle."""
    ds = datagen.random_dag_dataset(10, 400, 3, 3, 1.0, seed=12)
    n, d = 10, 3
    rng = np.random.default_rng(5)
    log_rho = rng.normal(size=d + 1)
    log_q = rng.normal(size=n) * 3
    lf, full = _ranked_feature(n, d, rng, "weights")
    logB = O.full_log_beta(ds.data, ds.arity, d, kind=O.K2, log_rho=log_rho)
    ref = O.modular_feature_posterior(logB, d, full, log_q=log_q)
    got = bn.modular_feature_posterior(ds.data, ds.arity, d, lf, precision=prec, score="k2",
                                       log_rho=log_rho, log_q=log_q)
    assert got["value"] == pytest.approx(ref["value"], rel=TOL[prec])
