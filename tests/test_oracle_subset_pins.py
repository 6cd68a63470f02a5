"""Pins of the oracle's generic subset sums (oracle.subset_sums[_at]).

Each check ties the oracle to something other than itself:
* pure-Python brute force over explicit Python sets (no bit tricks) on tiny
  inputs, exact on integer values;
* the transform matrices as Kronecker powers: [S subset T] is the n-fold
  Kronecker power of [[1, 0], [1, 1]] and its inverse that of [[1, 0], [-1, 1]]
  (the zeta and Moebius functions of the Boolean lattice, Def. 1 and Def. 2);
* closed forms on all-ones input: sum_{k<=d} C(|T|, k) below T, 2^(n-|T|)
  above T, and the indicator of the bottom / top element for the inverses;
* inversion: the Moebius sums undo the zeta sums exactly on integer input.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1408_1664_amd import datagen

KINDS = ["zeta_up", "zeta_down", "mobius_up", "mobius_down"]


def _as_set(mask, nbits):
    return frozenset(j for j in range(nbits) if (mask >> j) & 1)


def _brute(x, kind, d, nbits):
    sets = [_as_set(S, nbits) for S in range(1 << nbits)]
    out = []
    for T in sets:
        acc = 0.0
        for S, xs in zip(sets, x):
            if kind in ("zeta_up", "mobius_up"):
                if not S <= T:
                    continue
                if kind == "zeta_up" and d >= 0 and len(S) > d:
                    continue
                sign = (-1) ** len(T - S) if kind == "mobius_up" else 1
            else:
                if not T <= S:
                    continue
                sign = (-1) ** len(S - T) if kind == "mobius_down" else 1
            acc += sign * xs
        out.append(acc)
    return np.array(out)


@pytest.mark.parametrize("nbits", [0, 1, 3, 5])
@pytest.mark.parametrize("kind", KINDS)
def test_brute_force_sets(nbits, kind):
    x = datagen.subset_values(nbits, 11 + nbits, "int")
    for d in ([-1, 0, 1, 2, nbits] if kind == "zeta_up" else [-1]):
        np.testing.assert_array_equal(O.subset_sums(x, kind, d), _brute(x, kind, d, nbits))


def _kron_power(m2, nbits):
    M = np.ones((1, 1))
    for _ in range(nbits):
        M = np.kron(m2, M)
    return M


@pytest.mark.parametrize("nbits", [4, 8])
def test_kronecker_matrices(nbits):
    Z = _kron_power(np.array([[1.0, 0.0], [1.0, 1.0]]), nbits)    # Z[T, S] = [S subset T]
    Mi = _kron_power(np.array([[1.0, 0.0], [-1.0, 1.0]]), nbits)
    np.testing.assert_array_equal(Z @ Mi, np.eye(1 << nbits))
    x = datagen.subset_values(nbits, 3, "int")
    np.testing.assert_array_equal(O.subset_sums(x, "zeta_up"), Z @ x)
    np.testing.assert_array_equal(O.subset_sums(x, "zeta_down"), Z.T @ x)
    np.testing.assert_array_equal(O.subset_sums(x, "mobius_up"), Mi @ x)
    np.testing.assert_array_equal(O.subset_sums(x, "mobius_down"), Mi.T @ x)
    pc = np.array([bin(S).count("1") for S in range(1 << nbits)])
    for d in range(nbits + 1):
        np.testing.assert_array_equal(O.subset_sums(x, "zeta_up", d), Z @ np.where(pc <= d, x, 0))
    y = datagen.subset_values(nbits, 4, "uniform")
    np.testing.assert_allclose(O.subset_sums(y, "zeta_up", 2), Z @ np.where(pc <= 2, y, 0),
                               rtol=1e-15, atol=0)


def test_closed_forms_on_ones():
    nbits = 10
    x = datagen.subset_values(nbits, 0, "ones")
    pc = np.array([bin(S).count("1") for S in range(1 << nbits)])
    for d in [-1, 0, 1, 3, 9, 10]:
        want = np.array([sum(math.comb(k, j) for j in range(k + 1 if d < 0 else min(d, k) + 1))
                         for k in pc], dtype=float)
        np.testing.assert_array_equal(O.subset_sums(x, "zeta_up", d), want)
    np.testing.assert_array_equal(O.subset_sums(x, "zeta_down"), 2.0 ** (nbits - pc))
    e0 = np.zeros(1 << nbits); e0[0] = 1
    eV = np.zeros(1 << nbits); eV[-1] = 1
    np.testing.assert_array_equal(O.subset_sums(x, "mobius_up"), e0)
    np.testing.assert_array_equal(O.subset_sums(x, "mobius_down"), eV)


def test_single_set_indicator():
    nbits = 9
    for S0 in [0, 5, 0b101100001, (1 << nbits) - 1]:
        x = np.zeros(1 << nbits); x[S0] = 2.5
        T = np.arange(1 << nbits)
        np.testing.assert_array_equal(O.subset_sums(x, "zeta_up"), np.where(T & S0 == S0, 2.5, 0))
        np.testing.assert_array_equal(O.subset_sums(x, "zeta_down"), np.where(T | S0 == S0, 2.5, 0))
        k = bin(S0).count("1")
        if k > 0:   # a bound below |S0| drops the only term
            np.testing.assert_array_equal(O.subset_sums(x, "zeta_up", k - 1),
                                          np.zeros(1 << nbits))


@pytest.mark.parametrize("pair", [("zeta_up", "mobius_up"), ("zeta_down", "mobius_down")])
def test_inversion_exact(pair):
    x = datagen.subset_values(12, 5, "int")
    z = O.subset_sums(x, pair[0])
    np.testing.assert_array_equal(O.subset_sums(z, pair[1]), x)
    np.testing.assert_array_equal(O.subset_sums(O.subset_sums(x, pair[1]), pair[0]), x)


def test_selected_outputs_and_absval():
    nbits = 11
    x = datagen.subset_values(nbits, 9, "signed")
    Ts = np.array([0, 1, 77, 1023, 2047, 1500], dtype=np.uint64)
    for kind in KINDS:
        for d in ([-1, 2] if kind == "zeta_up" else [-1]):
            full = O.subset_sums(x, kind, d)
            np.testing.assert_array_equal(O.subset_sums_at(x, kind, Ts, d), full[Ts.astype(int)])
            np.testing.assert_array_equal(O.subset_sums(x, kind, d, absval=True),
                                          O.subset_sums(np.abs(x), "zeta_down" if "down" in kind
                                                        else "zeta_up", d if kind == "zeta_up"
                                                        else -1))


def test_compensated_sum_is_exact_where_plain_sum_is_not():
    # 1 + 2^-53 added 2^10 times: plain sequential FP64 summation loses every
    # small term, the oracle's compensated sum keeps them.
    nbits = 10
    x = np.full(1 << nbits, 2.0 ** -53)
    x[0] = 1.0
    t = O.subset_sums_at(x, "zeta_up", np.array([(1 << nbits) - 1], np.uint64))[0]
    assert t == 1.0 + (2 ** nbits - 1) * 2.0 ** -53
