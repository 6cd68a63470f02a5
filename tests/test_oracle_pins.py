"""Pins for the CPU oracle: values the mathematics fixes, independent of the oracle's code.

Each test would fail on a plausible mistake in the oracle (a dropped term, a
wrong index, a transposed operand, an off-by-one in a layer, a wrong
hyperparameter):

* local scores: exact rational BDeu/K2 values, the 5/128 hand value,
  score equivalence, no-data scores;
* transforms: brute-force subset / superset sums (Eqs. 7 and 12);
* lattice: F(V) = R(V) read from the other end, per-layer sums, brute force
  over all orders (Eq. 8);
* posteriors: brute force over orders, over DAGs, the per-edge forward re-run,
  the no-data closed form, acyclicity and in-degree bounds, relabelling.
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_1408_1664_amd import datagen
from tests.ref import brute as B

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- scores ----

def test_bdeu_hand_value():
    g = _gold("bdeu_hand.json")
    data = np.array(g["data"], dtype=np.uint8)
    s = O.local_scores(data, g["arity"], 0, O.BDEU, g["ess"])
    assert s[0, 0] == pytest.approx(math.log(g["p_num"] / g["p_den"]), abs=1e-13)
    assert s[0, 0] == pytest.approx(g["log_p"], abs=1e-13)


def _count_table(data, arity, i, parents):
    q = int(np.prod([arity[p] for p in parents])) if parents else 1
    tab = [[0] * int(arity[i]) for _ in range(q)]
    for s in range(data.shape[1]):
        j = 0
        for p in parents:
            j = j * int(arity[p]) + int(data[p, s])
        tab[j][int(data[i, s])] += 1
    return tab


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("kind", [O.BDEU, O.K2])
def test_scores_exact_rational(seed, kind):
    rng = np.random.default_rng(100 + seed)
    n, m = 4, 9
    arity = rng.integers(2, 4, size=n).astype(np.uint8)
    data = np.stack([rng.integers(0, arity[i], size=m) for i in range(n)]).astype(np.uint8)
    ess = 1.0 + seed  # 1, 2, 3
    s = O.local_scores(data, arity, 2, kind, ess)
    for i in range(n):
        others = [j for j in range(n) if j != i]
        for k in range(3):
            for ps in itertools.combinations(others, k):
                G = sum(1 << p for p in ps)
                tab = _count_table(data, arity, i, list(ps))
                exact = (B.bdeu_rational(tab, Fraction(int(ess))) if kind == O.BDEU
                         else B.k2_rational(tab))
                assert s[i, G] == pytest.approx(math.log(exact), rel=1e-12, abs=1e-11)
        # families that must be absent: G containing i, |G| > d
        assert np.isneginf(s[i, 1 << i])


def test_scores_no_data_are_zero():
    data = np.zeros((5, 0), dtype=np.uint8)
    s = O.local_scores(data, 3, 2)
    assert np.all(s[np.isfinite(s)] == 0.0)
    assert np.isfinite(s).sum() == 5 * (1 + 4 + 6)


def test_bdeu_score_equivalence():
    """BDeu gives Markov-equivalent DAGs the same score: for a pair,
    i <- j and j <- i; for a chain a -> b -> c versus c -> b -> a."""
    ds = datagen.random_dag_dataset(5, 300, 3, 2, 1.0, seed=7)
    s = O.local_scores(ds.data, ds.arity, 2, O.BDEU, 1.0)
    for i, j in itertools.permutations(range(5), 2):
        lhs = s[i, 1 << j] + s[j, 0]
        rhs = s[j, 1 << i] + s[i, 0]
        assert lhs == pytest.approx(rhs, abs=1e-9)
    a, b, c = 0, 1, 2
    chain1 = s[a, 0] + s[b, 1 << a] + s[c, 1 << b]
    chain2 = s[c, 0] + s[b, 1 << c] + s[a, 1 << b]
    assert chain1 == pytest.approx(chain2, abs=1e-9)
    # K2 is not score-equivalent: the pin must be able to fail
    k = O.local_scores(ds.data, ds.arity, 2, O.K2)
    assert abs((k[0, 2] + k[1, 0]) - (k[1, 1] + k[0, 0])) > 1e-6


# ------------------------------------------------------------ transforms ----

def test_alpha_and_gamma_brute_force():
    """The oracle's A_i (Eq. 7) and Gamma_v (Eq. 12) against direct subset and
    superset sums written out per mask."""
    n, d = 7, 2
    rng = np.random.default_rng(5)
    logB = B.random_logB(n, d, rng)
    lq = rng.normal(size=n)
    r = O.posteriors_from_scores(logB, d, log_q=lq, dumps=True)
    A, F, Rp, Gm = r["alpha"], r["L"], r["Rp"], r["gamma"]
    N = 1 << n
    pc = [bin(x).count("1") for x in range(N)]
    for i in range(n):
        for S in range(N):
            if S >> i & 1:
                assert np.isneginf(A[i, S])
                continue
            terms = [logB[i, G] for G in range(N) if (G & ~S) == 0 and pc[G] <= d]
            assert A[i, S] == pytest.approx(lq[pc[S]] + B._lse(terms), abs=1e-11)
    for v in range(n):
        bv = 1 << v
        for G in range(N):
            if G & bv or pc[G] > d:
                assert np.isneginf(Gm[v, G])
                continue
            terms = [lq[pc[S]] + F[S] + Rp[S | bv] for S in range(N)
                     if not S & bv and (G & ~S) == 0]
            assert Gm[v, G] == pytest.approx(B._lse(terms), abs=1e-10)


def test_forward_backward_direct():
    """F (Eq. 9) and the backward function (Eq. 10, prefix-indexed:
    Rp(S) = R(V - S)) against their recursions written per mask."""
    n, d = 6, 3
    rng = np.random.default_rng(9)
    logB = B.random_logB(n, d, rng)
    r = O.posteriors_from_scores(logB, d, dumps=True)
    A, F, Rp = r["alpha"], r["L"], r["Rp"]
    full = (1 << n) - 1
    # R in the paper's own indexing: R(T) = sum_{i in T} A_i(V - T) R(T - i), R(empty) = 1
    R = {0: 0.0}
    for T in sorted(range(1, 1 << n), key=lambda x: bin(x).count("1")):
        R[T] = B._lse([A[i, full & ~T] + R[T & ~(1 << i)] for i in range(n) if T >> i & 1])
    for S in range(1 << n):
        assert Rp[S] == pytest.approx(R[full & ~S], abs=1e-11)
    assert F[0] == 0.0 and Rp[full] == 0.0
    assert F[full] == pytest.approx(Rp[0], abs=1e-11)


# ------------------------------------------------------------- posteriors ----

@pytest.mark.parametrize("n,d,seed", [(4, 2, 0), (5, 2, 1), (5, 4, 2), (6, 3, 3)])
def test_orders_brute_force_random_scores(n, d, seed):
    rng = np.random.default_rng(seed)
    logB = B.random_logB(n, d, rng, scale=3.0)
    lq = rng.normal(size=n)
    r = O.posteriors_from_scores(logB, d, log_q=lq, gamma_free=True)
    post, total = B.orders_posteriors(B.full_to_dict(logB, n), d, log_q=lq)
    assert r["log_LV"] == pytest.approx(total, abs=1e-10)
    np.testing.assert_allclose(r["post"], post, atol=1e-11)
    assert r["r_gamma_free"] < 1e-10


@pytest.mark.parametrize("wl_seed", [11, 12])
def test_orders_brute_force_data_scores(wl_seed):
    ds = datagen.random_dag_dataset(6, 400, 2, 3, 1.0, seed=wl_seed)
    logB = O.full_log_beta(ds.data, ds.arity, 3)
    r = O.edge_posteriors(ds.data, ds.arity, 3)
    post, total = B.orders_posteriors(B.full_to_dict(logB, 6), 3)
    assert r["log_LV"] == pytest.approx(total, abs=1e-9)
    np.testing.assert_allclose(r["post"], post, atol=1e-11)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_dag_enumeration(d):
    """Eq. 2 with the order-modular prior (q == 1): sum over DAGs weighted by
    their linear-extension counts."""
    ds = datagen.random_dag_dataset(4, 60, 3, 2, 1.0, seed=21 + d)
    logB = O.full_log_beta(ds.data, ds.arity, d)
    r = O.edge_posteriors(ds.data, ds.arity, d)
    post, total = B.dag_posteriors(B.full_to_dict(logB, 4), d)
    assert r["log_LV"] == pytest.approx(total, abs=1e-10)
    np.testing.assert_allclose(r["post"], post, atol=1e-12)


def _ps_dict_to_full(ps, n):
    out = np.zeros((n, 1 << n))
    for (v, G), x in ps.items():
        out[v, sum(1 << j for j in G)] = x
    return out


@pytest.mark.parametrize("n,d,seed", [(4, 2, 3), (5, 3, 4), (6, 2, 5)])
def test_parent_set_posteriors_orders_brute_force(n, d, seed):
    """P(G_v = G | D) against the sum over all orders with the parent-set
    feature; rows sum to 1 and the edge posteriors are their marginals."""
    rng = np.random.default_rng(seed)
    logB = B.random_logB(n, d, rng, scale=3.0)
    lq = rng.normal(size=n)
    r = O.parent_set_posteriors(logB, d, log_q=lq)
    want = _ps_dict_to_full(B.orders_parent_posteriors(B.full_to_dict(logB, n), d, log_q=lq), n)
    np.testing.assert_allclose(r["ps"], want, atol=1e-12)
    np.testing.assert_allclose(r["ps"].sum(axis=1), 1.0, atol=1e-12)
    for u in range(n):
        has_u = np.array([(G >> u) & 1 for G in range(1 << n)], dtype=bool)
        np.testing.assert_allclose(r["ps"][:, has_u].sum(axis=1), r["post"][u, :], atol=1e-12)


def test_parent_set_posteriors_dag_enumeration():
    ds = datagen.random_dag_dataset(4, 80, 2, 2, 1.0, seed=41)
    logB = O.full_log_beta(ds.data, ds.arity, 2)
    r = O.parent_set_posteriors(logB, 2)
    want = _ps_dict_to_full(B.dag_parent_posteriors(B.full_to_dict(logB, 4), 2), 4)
    np.testing.assert_allclose(r["ps"], want, atol=1e-12)


def test_per_edge_forward_rerun():
    n, d = 6, 2
    rng = np.random.default_rng(31)
    logB = B.random_logB(n, d, rng)
    lq = rng.normal(size=n)
    r = O.posteriors_from_scores(logB, d, log_q=lq)
    post, base = B.per_edge_forward(B.full_to_dict(logB, n), d, log_q=lq)
    assert r["log_LV"] == pytest.approx(base, abs=1e-10)
    np.testing.assert_allclose(r["post"], post, atol=1e-11)


def test_no_data_closed_form():
    g = _gold("m0_closed_form.json")
    for c in g["cases"]:
        n, d = c["n"], c["d"]
        data = np.zeros((n, 0), dtype=np.uint8)
        lr = (O.default_log_rho(n, d) if c["rho"] == "1/C(n-1,k)" else np.zeros(d + 1))
        r = O.edge_posteriors(data, 2, d, log_rho=lr)
        want = c["num"] / c["den"]
        # the closed form itself, recomputed exactly, must agree with the fixture
        rho = ([Fraction(1, math.comb(n - 1, k)) for k in range(d + 1)]
               if c["rho"] == "1/C(n-1,k)" else [Fraction(1)] * (d + 1))
        assert B.m0_closed_form(n, d, rho) == Fraction(c["num"], c["den"])
        off = r["post"][~np.eye(n, dtype=bool)]
        np.testing.assert_allclose(off, want, atol=1e-13)


def test_invariants_and_bounds_n12():
    ds, p = datagen.workload("n12_binary_m200_d3")
    logB = O.full_log_beta(ds.data, ds.arity, p["d"])
    r = O.posteriors_from_scores(logB, p["d"], gamma_free=True)
    P = r["post"]
    assert abs(r["r_LR"]) < 1e-11
    assert r["r_layers"] < 1e-10
    assert r["r_gamma"] < 1e-10
    assert r["r_gamma_free"] < 1e-10
    assert P.min() >= 0 and P.max() <= 1 + 1e-12
    assert np.all(P + P.T <= 1 + 1e-12)                  # acyclicity
    assert np.all(P.sum(axis=0) <= p["d"] + 1e-12)      # in-degree bound
    assert np.all(np.diag(P) == 0)


def test_relabelling_permutes_posteriors():
    ds = datagen.random_dag_dataset(9, 300, 2, 3, 1.0, seed=41)
    perm = np.random.default_rng(0).permutation(9)
    r1 = O.edge_posteriors(ds.data, ds.arity, 3)
    r2 = O.edge_posteriors(ds.data[perm], ds.arity[perm], 3)
    np.testing.assert_allclose(r2["post"], r1["post"][np.ix_(perm, perm)], atol=1e-12)
    assert r1["log_LV"] == pytest.approx(r2["log_LV"], abs=1e-9)


def test_degenerate_d0_and_full_d():
    ds = datagen.random_dag_dataset(6, 100, 2, 2, 1.0, seed=51)
    r0 = O.edge_posteriors(ds.data, ds.arity, 0)
    assert np.all(r0["post"] == 0.0)
    # d >= n-1 is clamped to n-1
    ra = O.edge_posteriors(ds.data, ds.arity, 5)
    rb = O.edge_posteriors(ds.data, ds.arity, 9)
    np.testing.assert_array_equal(ra["post"], rb["post"])


def _feature_dict(lf, logB_dict):
    """log f as logf[i][G] on the keys of logB (-inf entries kept)."""
    n = len(logB_dict)
    return [{G: float(lf[i, sum(1 << j for j in G)]) for G in logB_dict[i]} for i in range(n)]


def _random_feature(n, rng, kind):
    """log f_i(G) as [n, 2^n]: 'weights' (random f in (0, 2]), 'mask' (random
    0/1 per (i, G), keeping f_i(empty) = 1), 'edges' (u->v required for a few
    pairs, i.e. f_v(G) = [u in G])."""
    lf = np.zeros((n, 1 << n))
    if kind == "weights":
        lf = np.log(rng.uniform(0.05, 2.0, size=(n, 1 << n)))
    elif kind == "mask":
        lf = np.where(rng.random((n, 1 << n)) < 0.3, -np.inf, 0.0)
        lf[:, 0] = 0.0
    else:
        for _ in range(2):
            u, v = rng.choice(n, 2, replace=False)
            has = np.array([(G >> u) & 1 for G in range(1 << n)], dtype=bool)
            lf[v] = np.where(has, lf[v], -np.inf)
    return lf


@pytest.mark.parametrize("n,d,seed,kind", [(4, 2, 7, "weights"), (5, 3, 8, "mask"),
                                           (5, 2, 9, "edges"), (6, 2, 10, "weights")])
def test_modular_feature_orders_brute_force(n, d, seed, kind):
    """E[f | D] from the forward sum on f_i B_i against Eq. 5 with f summed
    over all orders (random q)."""
    rng = np.random.default_rng(seed)
    logB = B.random_logB(n, d, rng, scale=3.0)
    lq = rng.normal(size=n)
    lf = _random_feature(n, rng, kind)
    r = O.modular_feature_posterior(logB, d, lf, log_q=lq)
    Bd = B.full_to_dict(logB, n)
    want = B.orders_feature_posterior(Bd, d, _feature_dict(lf, Bd), log_q=lq)
    assert r["value"] == pytest.approx(want, rel=1e-11, abs=1e-14)


def test_modular_feature_dag_enumeration():
    ds = datagen.random_dag_dataset(4, 80, 2, 2, 1.0, seed=43)
    logB = O.full_log_beta(ds.data, ds.arity, 2)
    rng = np.random.default_rng(44)
    for kind in ["weights", "mask", "edges"]:
        lf = _random_feature(4, rng, kind)
        r = O.modular_feature_posterior(logB, 2, lf)
        Bd = B.full_to_dict(logB, 4)
        want = B.dag_feature_posterior(Bd, 2, _feature_dict(lf, Bd))
        assert r["value"] == pytest.approx(want, rel=1e-11, abs=1e-14)


def test_modular_feature_special_cases():
    """f == 1 gives 1; f_v(G) = [u in G] gives the edge posterior; f_v(G) =
    [G = G0] gives the parent-set posterior; f_v == 0 gives 0."""
    n, d = 6, 3
    rng = np.random.default_rng(45)
    logB = B.random_logB(n, d, rng, scale=3.0)
    r0 = O.parent_set_posteriors(logB, d)
    assert O.modular_feature_posterior(logB, d, np.zeros((n, 1 << n)))["value"] == pytest.approx(1.0, abs=1e-13)
    for u, v in [(0, 1), (4, 2), (5, 0)]:
        lf = np.zeros((n, 1 << n))
        lf[v] = np.where([(G >> u) & 1 for G in range(1 << n)], 0.0, -np.inf)
        assert O.modular_feature_posterior(logB, d, lf)["value"] == pytest.approx(r0["post"][u, v], abs=1e-12)
    for v, G0 in [(1, 0b000101), (3, 0)]:
        lf = np.zeros((n, 1 << n))
        lf[v] = -np.inf
        lf[v, G0] = 0.0
        assert O.modular_feature_posterior(logB, d, lf)["value"] == pytest.approx(r0["ps"][v, G0], abs=1e-12)
    lf = np.zeros((n, 1 << n))
    lf[2] = -np.inf
    assert O.modular_feature_posterior(logB, d, lf)["value"] == 0.0
