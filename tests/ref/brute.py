"""Independent brute-force and closed-form references that pin the oracle.

None of these share code with the oracle (oracle/bn_oracle.c) or with the GPU
library. They evaluate the defining sums directly, in ways a reader can check
against the paper by eye:

* ``orders_posteriors``: Eqs. 5 and 8 summed over all n! orders;
* ``dag_posteriors``: Eqs. 2-4 summed over every DAG with in-degree <= d,
  each weighted by its number of linear extensions (q == 1);
* ``per_edge_forward``: the forward recursion of Eq. 9 re-run once per edge
  with f_v(G) = [u in G] (the O(n^3 2^n) route of Sec. 2.2);
* ``orders_feature_posterior`` / ``dag_feature_posterior``: E[f | D] of a
  modular feature f(G) = prod_i f_i(G_i), over all orders (Eq. 5 with f) or
  over all DAGs;
* ``bdeu_rational``: the BDeu marginal likelihood as an exact rational number
  from rising factorials (Gamma(a+N)/Gamma(a) = a(a+1)...(a+N-1));
* ``m0_closed_form``: the exact posterior when every family score equals 1.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import numpy as np


def _lse(xs):
    xs = [x for x in xs if x != -math.inf]
    if not xs:
        return -math.inf
    m = max(xs)
    return m + math.log(sum(math.exp(x - m) for x in xs))


def _subsets_upto(items, d):
    for k in range(0, min(d, len(items)) + 1):
        for c in itertools.combinations(items, k):
            yield c


def orders_posteriors(logB, d, log_q=None):
    """P(u->v|D) and log P(D) by summing Eq. 5 over all orders.

    logB: dict-like, logB[i][G] with G a frozenset, for |G| <= d, i not in G.
    log_q: sequence, log q(k) by predecessor-set size (None: q == 1).
    """
    n = len(logB)
    lq = (lambda k: 0.0) if log_q is None else (lambda k: float(log_q[k]))
    joint = np.full((n, n), -math.inf)
    total = -math.inf
    for order in itertools.permutations(range(n)):
        pos = {v: t for t, v in enumerate(order)}
        # log A_i(L_i) for every i, and per-edge variants for v
        logA = []
        for i in range(n):
            L = [j for j in range(n) if pos[j] < pos[i]]
            logA.append(lq(len(L)) + _lse([logB[i][frozenset(G)] for G in _subsets_upto(L, d)]))
        lw = sum(logA)
        total = _lse([total, lw])
        for v in range(n):
            L = [j for j in range(n) if pos[j] < pos[v]]
            rest = lw - logA[v]
            for u in L:
                s = _lse([logB[v][frozenset(G)] for G in _subsets_upto(L, d) if u in G])
                joint[u, v] = _lse([joint[u, v], rest + lq(len(L)) + s])
    post = np.where(np.isfinite(joint), np.exp(joint - total), 0.0)
    np.fill_diagonal(post, 0.0)
    return post, total


def orders_feature_posterior(logB, d, logf, log_q=None):
    """E[f | D] for f(G) = prod_i f_i(G_i): Eq. 5 summed over all orders with
    and without f. logf[i][G] = log f_i(G) (same keys as logB)."""
    n = len(logB)
    lq = (lambda k: 0.0) if log_q is None else (lambda k: float(log_q[k]))
    num = den = -math.inf
    for order in itertools.permutations(range(n)):
        pos = {v: t for t, v in enumerate(order)}
        w = wf = 0.0
        for i in range(n):
            L = [j for j in range(n) if pos[j] < pos[i]]
            sets = [frozenset(G) for G in _subsets_upto(L, d)]
            w += lq(len(L)) + _lse([logB[i][G] for G in sets])
            wf += lq(len(L)) + _lse([logB[i][G] + logf[i][G] for G in sets])
        den = _lse([den, w])
        num = _lse([num, wf])
    return math.exp(num - den) if num > -math.inf else 0.0


def dag_feature_posterior(logB, d, logf):
    """E[f | D] for f(G) = prod_i f_i(G_i) over all DAGs with in-degree <= d
    (q == 1: each DAG weighted by its number of linear extensions)."""
    n = len(logB)
    choices = [list(_subsets_upto([j for j in range(n) if j != i], d)) for i in range(n)]
    num = den = -math.inf
    for pa in itertools.product(*choices):
        if not _is_acyclic(pa):
            continue
        lw = math.log(_linear_extensions(pa)) + sum(logB[i][frozenset(pa[i])] for i in range(n))
        den = _lse([den, lw])
        num = _lse([num, lw + sum(logf[i][frozenset(pa[i])] for i in range(n))])
    return math.exp(num - den) if num > -math.inf else 0.0


def _is_acyclic(parents):
    n = len(parents)
    state = [0] * n

    def visit(v):
        if state[v] == 1:
            return False
        if state[v] == 2:
            return True
        state[v] = 1
        for p in parents[v]:
            if not visit(p):
                return False
        state[v] = 2
        return True

    return all(visit(v) for v in range(n))


def _linear_extensions(parents):
    n = len(parents)
    cnt = 0
    for order in itertools.permutations(range(n)):
        pos = {v: t for t, v in enumerate(order)}
        if all(pos[p] < pos[v] for v in range(n) for p in parents[v]):
            cnt += 1
    return cnt


def dag_posteriors(logB, d):
    """P(u->v|D) by enumerating DAGs (Eqs. 2-4 with q == 1): each DAG G has
    weight (number of orders consistent with G) * prod_i B_i(G_i)."""
    n = len(logB)
    choices = [list(_subsets_upto([j for j in range(n) if j != i], d)) for i in range(n)]
    joint = np.full((n, n), -math.inf)
    total = -math.inf
    for pa in itertools.product(*choices):
        if not _is_acyclic(pa):
            continue
        lw = math.log(_linear_extensions(pa)) + sum(logB[i][frozenset(pa[i])] for i in range(n))
        total = _lse([total, lw])
        for v in range(n):
            for u in pa[v]:
                joint[u, v] = _lse([joint[u, v], lw])
    post = np.where(np.isfinite(joint), np.exp(joint - total), 0.0)
    return post, total


def dag_parent_posteriors(logB, d):
    """P(G_v = G | D) by enumerating DAGs (Eqs. 2-4 with q == 1):
    dict (v, frozenset G) -> probability."""
    n = len(logB)
    choices = [list(_subsets_upto([j for j in range(n) if j != i], d)) for i in range(n)]
    joint = {}
    total = -math.inf
    for pa in itertools.product(*choices):
        if not _is_acyclic(pa):
            continue
        lw = math.log(_linear_extensions(pa)) + sum(logB[i][frozenset(pa[i])] for i in range(n))
        total = _lse([total, lw])
        for v in range(n):
            key = (v, frozenset(pa[v]))
            joint[key] = _lse([joint.get(key, -math.inf), lw])
    return {k: math.exp(x - total) for k, x in joint.items()}


def orders_parent_posteriors(logB, d, log_q=None):
    """P(G_v = G | D) by summing Eq. 5 over all orders with the feature
    f = [G_v = G]: dict (v, frozenset G) -> probability."""
    n = len(logB)
    lq = (lambda k: 0.0) if log_q is None else (lambda k: float(log_q[k]))
    joint = {}
    total = -math.inf
    for order in itertools.permutations(range(n)):
        pos = {v: t for t, v in enumerate(order)}
        logA = []
        for i in range(n):
            L = [j for j in range(n) if pos[j] < pos[i]]
            logA.append(lq(len(L)) + _lse([logB[i][frozenset(G)] for G in _subsets_upto(L, d)]))
        lw = sum(logA)
        total = _lse([total, lw])
        for v in range(n):
            L = [j for j in range(n) if pos[j] < pos[v]]
            rest = lw - logA[v] + lq(len(L))
            for G in _subsets_upto(L, d):
                key = (v, frozenset(G))
                joint[key] = _lse([joint.get(key, -math.inf), rest + logB[v][frozenset(G)]])
    return {k: math.exp(x - total) for k, x in joint.items()}


def per_edge_forward(logB, d, log_q=None):
    """Eq. 9 re-run for each edge with B_v masked by [u in G]; divide by F(V)."""
    n = len(logB)
    lq = (lambda k: 0.0) if log_q is None else (lambda k: float(log_q[k]))
    full = (1 << n) - 1

    def forward(mask_fn):
        A = {}
        for i in range(n):
            for S in range(1 << n):
                if S >> i & 1:
                    continue
                members = [j for j in range(n) if S >> j & 1]
                A[i, S] = lq(len(members)) + _lse(
                    [logB[i][frozenset(G)] for G in _subsets_upto(members, d) if mask_fn(i, G)])
        F = {0: 0.0}
        for S in sorted(range(1, 1 << n), key=lambda x: bin(x).count("1")):
            F[S] = _lse([A[i, S & ~(1 << i)] + F[S & ~(1 << i)]
                         for i in range(n) if S >> i & 1])
        return F[full]

    base = forward(lambda i, G: True)
    post = np.zeros((n, n))
    for v in range(n):
        for u in range(n):
            if u == v:
                continue
            lj = forward(lambda i, G, u=u, v=v: (i != v) or (u in G))
            post[u, v] = math.exp(lj - base) if lj != -math.inf else 0.0
    return post, base


def rising(a: Fraction, N: int) -> Fraction:
    r = Fraction(1)
    for t in range(N):
        r *= a + t
    return r


def bdeu_rational(counts, ess=Fraction(1)) -> Fraction:
    """Exact BDeu marginal likelihood from a count table counts[j][k]
    (j = observed parent configuration, k = child value), with q the number
    of parent configurations (rows) and r the child arity (columns)."""
    q = len(counts)
    r = len(counts[0])
    a_j = Fraction(ess) / q
    a_jk = Fraction(ess) / (q * r)
    p = Fraction(1)
    for row in counts:
        Nj = sum(row)
        p /= rising(a_j, Nj)
        for c in row:
            p *= rising(a_jk, c)
    return p


def k2_rational(counts) -> Fraction:
    """Exact K2 marginal likelihood (all Dirichlet hyperparameters 1)."""
    r = len(counts[0])
    p = Fraction(1)
    for row in counts:
        p /= rising(Fraction(r), sum(row))
        for c in row:
            p *= rising(Fraction(1), c)
    return p


def m0_closed_form(n: int, d: int, rho) -> Fraction:
    """Exact P(u->v|D) with no data (every p(x_i|x_G) = 1) and q == 1.

    Every order then has the same weight, so v's predecessor count p is
    uniform on 0..n-1, u precedes v with probability p/(n-1), and given that,
    the fraction of v's parent-set mass containing u is
    sum_{k>=1} C(p-1,k-1) rho_k / sum_k C(p,k) rho_k.
    """
    rho = [Fraction(x) for x in rho]
    tot = Fraction(0)
    for p in range(n):
        num = sum((math.comb(p - 1, k - 1) * rho[k] for k in range(1, min(d, p) + 1)),
                  Fraction(0))
        den = sum((math.comb(p, k) * rho[k] for k in range(0, min(d, p) + 1)), Fraction(0))
        tot += Fraction(p, n - 1) * num / den
    return tot / n


def full_to_dict(logB_full, n):
    """[n, 2^n] full-mask log B array -> logB[i][frozenset(G)]."""
    out = []
    for i in range(n):
        dct = {}
        for G in range(1 << n):
            x = logB_full[i][G]
            if np.isfinite(x):
                dct[frozenset(j for j in range(n) if G >> j & 1)] = float(x)
        out.append(dct)
    return out


def random_logB(n, d, rng, scale=5.0):
    """Random log B_i(G) as [n, 2^n] (finite for |G| <= d, i not in G)."""
    out = np.full((n, 1 << n), -np.inf)
    for i in range(n):
        for G in range(1 << n):
            if G >> i & 1 or bin(G).count("1") > d:
                continue
            out[i, G] = rng.normal() * scale
    return out
