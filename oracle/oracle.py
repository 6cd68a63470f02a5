"""Python access to the CPU oracle (oracle/bn_oracle.c).

Test infrastructure only: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product path never does.

Everything is FP64 log-space with full n-bit masks (variable i <-> bit i).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bn_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")
_lib = None

BDEU = 0
K2 = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", "-o", tmp,
                        _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def build_sanitized() -> str:
    """The oracle under gcc's AddressSanitizer and UndefinedBehaviorSanitizer
    (liboracle_san.so; loaded with libasan preloaded and ORACLE_LIBRARY
    pointing at it)."""
    tmp = _LIB_SAN + ".tmp"
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-std=c11", "-fopenmp", "-shared", "-fPIC",
                    "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, _LIB_SAN)
    return _LIB_SAN


def _load():
    global _lib
    if _lib is None:
        # ORACLE_LIBRARY selects another build of the oracle (build_sanitized())
        path = os.environ.get("ORACLE_LIBRARY")
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.or_local_scores.argtypes = [ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_double, P, ctypes.c_int]
        lib.or_local_scores.restype = ctypes.c_int
        lib.or_posteriors_from_scores.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P, P,
                                                  P, P, ctypes.c_int, ctypes.c_int]
        lib.or_posteriors_from_scores.restype = ctypes.c_int
        lib.or_edge_posteriors.argtypes = [ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_double, P, P, P, P,
                                           ctypes.c_int]
        lib.or_edge_posteriors.restype = ctypes.c_int
        lib.or_subset_sums.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P,
                                       ctypes.c_int, ctypes.c_int]
        lib.or_subset_sums.restype = ctypes.c_int
        lib.or_subset_sums_at.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P,
                                          ctypes.c_int64, P, ctypes.c_int, ctypes.c_int]
        lib.or_subset_sums_at.restype = ctypes.c_int
        lib.or_num_threads.argtypes = []
        lib.or_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    """OpenMP threads the oracle uses (OMP_NUM_THREADS or all cores)."""
    return int(_load().or_num_threads())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def default_log_rho(n: int, d: int) -> np.ndarray:
    """log rho(k) = -log C(n-1, k), k = 0..d."""
    return np.array([-(math.lgamma(n) - math.lgamma(k + 1) - math.lgamma(n - k))
                     for k in range(d + 1)], dtype=np.float64)


def local_scores(data: np.ndarray, arity, d: int, kind: int = BDEU, ess: float = 1.0,
                 nthreads: int = 0) -> np.ndarray:
    """log p(x_i | x_G) as [n, 2^n] (full masks; -inf where G contains i or |G| > d)."""
    data = np.ascontiguousarray(data, dtype=np.uint8)
    n, m = data.shape
    ar = np.ascontiguousarray(np.broadcast_to(np.asarray(arity, np.uint8), (n,)))
    out = np.empty((n, 1 << n), dtype=np.float64)
    rc = _load().or_local_scores(n, m, _ptr(data), _ptr(ar), min(d, n - 1), kind, ess,
                                 _ptr(out), nthreads)
    if rc:
        raise RuntimeError(f"or_local_scores failed ({rc})")
    return out


def posteriors_from_scores(logB: np.ndarray, d: int, log_q=None, dumps: bool = False,
                           gamma_free: bool = False, nthreads: int = 0) -> dict:
    """Steps 2-7 of the method from log B_i(G) given as [n, 2^n] full-mask arrays."""
    logB = np.ascontiguousarray(logB, dtype=np.float64)
    n = logB.shape[0]
    assert logB.shape == (n, 1 << n)
    lq = None if log_q is None else np.ascontiguousarray(log_q, dtype=np.float64)
    post = np.zeros((n, n), dtype=np.float64)
    diag = np.zeros(5, dtype=np.float64)
    A = F = Rp = Gm = None
    if dumps:
        A = np.empty((n, 1 << n)); F = np.empty(1 << n); Rp = np.empty(1 << n)
        Gm = np.empty((n, 1 << n))
    rc = _load().or_posteriors_from_scores(n, min(d, n - 1), _ptr(logB), _ptr(lq), _ptr(post),
                                           _ptr(diag), _ptr(A), _ptr(F), _ptr(Rp), _ptr(Gm),
                                           1 if gamma_free else 0, nthreads)
    if rc:
        raise RuntimeError(f"or_posteriors_from_scores failed ({rc})")
    res = dict(post=post, log_LV=diag[0], r_LR=diag[1], r_layers=diag[2], r_gamma=diag[3],
               r_gamma_free=diag[4])
    if dumps:
        res.update(alpha=A, L=F, Rp=Rp, gamma=Gm)
    return res


def parent_set_posteriors(logB: np.ndarray, d: int, log_q=None, nthreads: int = 0) -> dict:
    """P(G_v = G | D) for every node v and parent set G (the parent-set
    feature of Sec. 2.1 put into Eq. 5): the Gamma_v of Eq. 12 weights each
    B_v(G), P(G_v = G | D) = B_v(G) Gamma_v(G) / F(V). Returns [n, 2^n]
    full-mask probabilities (0 where G is not a parent set of v), the edge
    posteriors and log F(V)."""
    r = posteriors_from_scores(logB, d, log_q=log_q, dumps=True, nthreads=nthreads)
    w = np.asarray(logB, dtype=np.float64) + r["gamma"]
    ps = np.where(np.isfinite(w), np.exp(w - r["log_LV"]), 0.0)
    return dict(ps=ps, post=r["post"], log_LV=r["log_LV"])


def edge_posteriors(data: np.ndarray, arity, d: int, kind: int = BDEU, ess: float = 1.0,
                    log_rho=None, log_q=None, nthreads: int = 0) -> dict:
    """Whole method from data. Returns posteriors [u, v], log L(V), residuals, seconds."""
    data = np.ascontiguousarray(data, dtype=np.uint8)
    n, m = data.shape
    ar = np.ascontiguousarray(np.broadcast_to(np.asarray(arity, np.uint8), (n,)))
    lr = None if log_rho is None else np.ascontiguousarray(log_rho, dtype=np.float64)
    lq = None if log_q is None else np.ascontiguousarray(log_q, dtype=np.float64)
    post = np.zeros((n, n), dtype=np.float64)
    diag = np.zeros(5, dtype=np.float64)
    t0 = time.perf_counter()
    rc = _load().or_edge_posteriors(n, m, _ptr(data), _ptr(ar), min(d, n - 1), kind, ess,
                                    _ptr(lr), _ptr(lq), _ptr(post), _ptr(diag), nthreads)
    dt = time.perf_counter() - t0
    if rc:
        raise RuntimeError(f"or_edge_posteriors failed ({rc})")
    return dict(post=post, log_LV=diag[0], r_LR=diag[1], r_layers=diag[2], r_gamma=diag[3],
                seconds=dt)


def full_log_beta(data: np.ndarray, arity, d: int, kind: int = BDEU, ess: float = 1.0,
                  log_rho=None, nthreads: int = 0) -> np.ndarray:
    """log B_i(G) = log rho(|G|) + log p(x_i|x_G) as [n, 2^n] full-mask arrays."""
    n = data.shape[0]
    d = min(d, n - 1)
    s = local_scores(data, arity, d, kind, ess, nthreads)
    lr = default_log_rho(n, d) if log_rho is None else np.asarray(log_rho, np.float64)
    pc = np.array([bin(x).count("1") for x in range(1 << n)])
    ok = np.isfinite(s)
    s[ok] += lr[np.broadcast_to(pc, s.shape)[ok]]
    return s


SUBSET_KINDS = {"zeta_up": 0, "zeta_down": 1, "mobius_up": 2, "mobius_down": 3}


def subset_sums(x: np.ndarray, kind: str, d: int = -1, absval: bool = False,
                nthreads: int = 0) -> np.ndarray:
    """Every output of a subset transform of x[0 .. 2^nbits), by its definition.

    zeta_up: t(T) = sum_{S subset T, |S| <= d} x(S) (Def. 1; d < 0: no bound);
    zeta_down: t(T) = sum_{S superset T} x(S) (Def. 2); mobius_up / mobius_down:
    the alternating sums that invert the untruncated forms. absval sums |x|.
    Cost 3^nbits.
    """
    x = np.ascontiguousarray(x, dtype=np.float64)
    nbits = int(x.size).bit_length() - 1
    assert x.size == 1 << nbits
    out = np.empty_like(x)
    rc = _load().or_subset_sums(nbits, SUBSET_KINDS[kind], int(d), _ptr(x), _ptr(out),
                                int(absval), int(nthreads))
    if rc:
        raise RuntimeError(f"or_subset_sums failed ({rc})")
    return out


def subset_sums_at(x: np.ndarray, kind: str, Ts, d: int = -1, absval: bool = False,
                   nthreads: int = 0) -> np.ndarray:
    """The outputs t(T) for the subsets in Ts only (same definitions)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    nbits = int(x.size).bit_length() - 1
    assert x.size == 1 << nbits
    Ts = np.ascontiguousarray(Ts, dtype=np.uint64)
    assert Ts.size == 0 or int(Ts.max()) < x.size
    out = np.empty(Ts.size, dtype=np.float64)
    rc = _load().or_subset_sums_at(nbits, SUBSET_KINDS[kind], int(d), _ptr(x), _ptr(Ts),
                                   Ts.size, _ptr(out), int(absval), int(nthreads))
    if rc:
        raise RuntimeError(f"or_subset_sums_at failed ({rc})")
    return out


def modular_feature_posterior(logB: np.ndarray, d: int, log_f: np.ndarray, log_q=None,
                              nthreads: int = 0) -> dict:
    """Posterior expectation E[f | D] of a modular feature f(G) = prod_i f_i(G_i)
    (Sec. 2.1; a 0/1 feature gives its posterior probability). With f put into
    Eq. 5, P(f, D) is the forward sum F(V) of Eq. 9 run on f_i(G) B_i(G) in
    place of B_i(G); P(D) is the plain F(V).
    logB, log_f: [n, 2^n] full-mask arrays (log_f -inf where f_i(G) = 0)."""
    logB = np.asarray(logB, dtype=np.float64)
    lf = logB + np.asarray(log_f, dtype=np.float64)
    base = posteriors_from_scores(logB, d, log_q=log_q, nthreads=nthreads)["log_LV"]
    feat = posteriors_from_scores(lf, d, log_q=log_q, nthreads=nthreads)["log_LV"]
    value = math.exp(feat - base) if feat > -math.inf else 0.0
    return dict(value=value, log_LV=base, log_LfV=feat)
