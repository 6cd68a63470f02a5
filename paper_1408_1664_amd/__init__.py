"""Exact Bayesian-network edge posteriors on an MI355X (gfx950).

Thin ctypes binding over ``libbnpost.so`` (C ABI in ``include/bn.h``): every
step of the computation runs in the library's HIP kernels; this module only
marshals arguments. Importing it does not load the library; the first call
does, and raises if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# BN_LIBRARY selects another build of the same library (the sanitizer build
# of the host code, libbnpost_san.so, for the CPU tests under ASan/UBSan).
LIB_PATH = os.environ.get("BN_LIBRARY") or os.path.join(_HERE, "libbnpost.so")

BN_OK, BN_EINVAL, BN_ENOMEM, BN_EDEVICE, BN_EAGAIN, BN_ECANCELED, BN_EINTERNAL = (
    0, -1, -2, -3, -4, -5, -6)
FP64_LOG = 0
FP32_SCALED = 1
SCORE_BDEU = 0
SCORE_K2 = 1

_PREC = {"fp64": FP64_LOG, "fp64_log": FP64_LOG, FP64_LOG: FP64_LOG,
         "fp32": FP32_SCALED, "fp32_scaled": FP32_SCALED, FP32_SCALED: FP32_SCALED}
_SCORE = {"bdeu": SCORE_BDEU, "k2": SCORE_K2, SCORE_BDEU: SCORE_BDEU, SCORE_K2: SCORE_K2}

EXPORTED = ["bn_num_parent_sets", "bn_local_scores", "bn_workspace_bytes",
            "bn_edge_posteriors", "bn_parent_set_posteriors", "bn_edge_posteriors_dev",
            "bn_timer_create",
            "bn_timer_destroy", "bn_timer_read", "bn_server_create", "bn_serve_submit",
            "bn_serve_poll", "bn_server_destroy", "bn_subset_transform",
            "bn_modular_feature_posterior", "bn_status_string", "bn_edge_posteriors_noalloc",
            "bn_zeta4_probe", "bn_subset_transform_x32"]

# Largest workspace the allocation-free entry point takes (BN_NOALLOC_MAX_BYTES).
NOALLOC_MAX_BYTES = 256 << 20


class BnError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


class Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("data", ctypes.c_void_p), ("arity", ctypes.c_void_p),
                ("d", ctypes.c_int32), ("score", ctypes.c_int32), ("ess", ctypes.c_double),
                ("log_rho", ctypes.c_void_p), ("log_q", ctypes.c_void_p)]


class Report(ctypes.Structure):
    _fields_ = [("log_LV", ctypes.c_double), ("max_invariant_residual", ctypes.c_double),
                ("saturated", ctypes.c_uint64), ("flushed", ctypes.c_uint64),
                ("ms_scores", ctypes.c_double), ("ms_alpha", ctypes.c_double),
                ("ms_fwd", ctypes.c_double), ("ms_bwd", ctypes.c_double),
                ("ms_gamma", ctypes.c_double), ("ms_edges", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("ms_queue", ctypes.c_double),
                ("ms_latency", ctypes.c_double), ("fallback_tiles", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libbnpost.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                              "python paper_1408_1664_amd/build.py")
        # torch ships its own copy of the HIP runtime under the same soname.
        # Loading torch first makes the library bind to that copy, so one
        # process never holds two HIP runtimes (which would hide the GPU from
        # one of them).
        try:
            import torch  # noqa: F401
        except Exception:  # torch absent: the library uses the system runtime
            pass
        L = ctypes.CDLL(LIB_PATH)
        P, I32, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64
        L.bn_num_parent_sets.argtypes = [I32, I32]
        L.bn_num_parent_sets.restype = ctypes.c_size_t
        L.bn_local_scores.argtypes = [P, P]
        L.bn_local_scores.restype = ctypes.c_int
        L.bn_workspace_bytes.argtypes = [I32, I32, I32, ctypes.c_int, P]
        L.bn_workspace_bytes.restype = ctypes.c_int
        L.bn_edge_posteriors.argtypes = [P, ctypes.c_int, P, P]
        L.bn_edge_posteriors.restype = ctypes.c_int
        L.bn_parent_set_posteriors.argtypes = [P, ctypes.c_int, P, P, P]
        L.bn_parent_set_posteriors.restype = ctypes.c_int
        L.bn_edge_posteriors_dev.argtypes = [P, ctypes.c_int, P, ctypes.c_size_t, P, P, P, P]
        L.bn_edge_posteriors_noalloc.argtypes = [P, ctypes.c_int, P, P, P]
        L.bn_edge_posteriors_noalloc.restype = ctypes.c_int
        L.bn_timer_create.argtypes = [P]
        L.bn_timer_create.restype = ctypes.c_int
        L.bn_timer_destroy.argtypes = [P]
        L.bn_timer_destroy.restype = ctypes.c_int
        L.bn_timer_read.argtypes = [P, P]
        L.bn_timer_read.restype = ctypes.c_int
        L.bn_edge_posteriors_dev.restype = ctypes.c_int
        L.bn_server_create.argtypes = [ctypes.c_size_t, I32, P]
        L.bn_server_create.restype = ctypes.c_int
        L.bn_serve_submit.argtypes = [P, P, ctypes.c_int, P]
        L.bn_serve_submit.restype = ctypes.c_int
        L.bn_serve_poll.argtypes = [P, U64, P, P, I32]
        L.bn_serve_poll.restype = ctypes.c_int
        L.bn_server_destroy.argtypes = [P]
        L.bn_server_destroy.restype = ctypes.c_int
        L.bn_modular_feature_posterior.argtypes = [P, ctypes.c_int, P, P, P]
        L.bn_modular_feature_posterior.restype = ctypes.c_int
        L.bn_subset_transform.argtypes = [P, I32, ctypes.c_int, I32, P]
        L.bn_subset_transform.restype = ctypes.c_int
        L.bn_subset_transform_x32.argtypes = [P, P, I32, ctypes.c_int, I32, P, P]
        L.bn_subset_transform_x32.restype = ctypes.c_int
        L.bn_zeta4_probe.argtypes = [P, P, U64, I32, I32, P, P]
        L.bn_zeta4_probe.restype = ctypes.c_int
        L.bn_status_string.argtypes = [ctypes.c_int]
        L.bn_status_string.restype = ctypes.c_char_p
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().bn_status_string(int(s)).decode()


def _check(status: int, where: str):
    if status != BN_OK:
        raise BnError(status, where)


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


class _ProblemHold:
    """A bn_problem plus the host arrays it points to (kept alive)."""

    def __init__(self, data, arity, d, score="bdeu", ess=1.0, log_rho=None, log_q=None,
                 data_ptr=None, device=False):
        """data: host array [n, m]; or, with device=True, the shape (n, m) of
        device data at data_ptr (None when m = 0)."""
        if not device and data_ptr is None:
            self.data = np.ascontiguousarray(data, dtype=np.uint8)
            n, m = self.data.shape
            dp = self.data.ctypes.data if m > 0 else None
        else:
            n, m = data
            dp = data_ptr
        self.arity = np.ascontiguousarray(np.broadcast_to(np.asarray(arity, np.uint8), (n,)))
        self.log_rho = None if log_rho is None else np.ascontiguousarray(log_rho, np.float64)
        self.log_q = None if log_q is None else np.ascontiguousarray(log_q, np.float64)
        self.p = Problem(n=n, m=m, data=dp, arity=self.arity.ctypes.data, d=int(d),
                         score=_SCORE[score], ess=float(ess),
                         log_rho=None if self.log_rho is None else self.log_rho.ctypes.data,
                         log_q=None if self.log_q is None else self.log_q.ctypes.data)
        self.n, self.m = n, m

    def ref(self):
        return ctypes.byref(self.p)


def num_parent_sets(n: int, d: int) -> int:
    return int(lib().bn_num_parent_sets(n, d))


def local_scores(data, arity, d, score="bdeu", ess=1.0) -> np.ndarray:
    """log p(x_i | x_G) for every node and ranked parent set: array [n, K(n-1,d)]."""
    h = _ProblemHold(data, arity, d, score, ess)
    K = num_parent_sets(h.n, d)
    out = np.empty((h.n, K), dtype=np.float64)
    _check(lib().bn_local_scores(h.ref(), _ptr(out)), "bn_local_scores")
    return out


def workspace_bytes(n: int, d: int, m: int, precision="fp32") -> int:
    b = ctypes.c_size_t(0)
    _check(lib().bn_workspace_bytes(n, d, m, _PREC[precision], ctypes.byref(b)),
           "bn_workspace_bytes")
    return int(b.value)


def edge_posteriors(data, arity, d, precision="fp64", score="bdeu", ess=1.0, log_rho=None,
                    log_q=None):
    """All edge posteriors from host data. Returns (post[u, v], report dict)."""
    h = _ProblemHold(data, arity, d, score, ess, log_rho, log_q)
    post = np.empty((h.n, h.n), dtype=np.float64)
    rep = Report()
    _check(lib().bn_edge_posteriors(h.ref(), _PREC[precision], _ptr(post), ctypes.byref(rep)),
           "bn_edge_posteriors")
    return post, rep.as_dict()


def parent_set_posteriors(data, arity, d, precision="fp64", score="bdeu", ess=1.0,
                          log_rho=None, log_q=None):
    """P(G_v = G | D) for every node v and parent set G, |G| <= d, as an
    [n, K(n-1, d)] array in the ranking of local_scores (each row sums to 1),
    with the edge posteriors and the report: (ps, post, report dict)."""
    h = _ProblemHold(data, arity, d, score, ess, log_rho, log_q)
    K = num_parent_sets(h.n, d)
    ps = np.empty((h.n, K), dtype=np.float64)
    post = np.empty((h.n, h.n), dtype=np.float64)
    rep = Report()
    _check(lib().bn_parent_set_posteriors(h.ref(), _PREC[precision], _ptr(ps), _ptr(post),
                                          ctypes.byref(rep)), "bn_parent_set_posteriors")
    return ps, post, rep.as_dict()


PHASES = ["scores", "alpha", "forward", "backward", "gamma", "edges", "total", "gamma_tile",
          "alpha_tile"]


class Timer:
    """Per-phase HIP events recorded by edge_posteriors_dev (bn_timer_*)."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(lib().bn_timer_create(ctypes.byref(h)), "bn_timer_create")
        self._h = h

    def read(self) -> dict:
        ms = np.zeros(9, dtype=np.float64)
        _check(lib().bn_timer_read(self._h, _ptr(ms)), "bn_timer_read")
        return dict(zip(PHASES, ms.tolist()))

    def close(self):
        if self._h:
            lib().bn_timer_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def edge_posteriors_dev(data_dev, arity, d, precision, ws, post_dev, diag_dev=None,
                        stream=None, score="bdeu", ess=1.0, log_rho=None, log_q=None,
                        timer: "Timer | None" = None):
    """Enqueue a solve on device-resident inputs (torch tensors on the GPU).

    data_dev: uint8 [n, m] device tensor; ws: device tensor of at least
    workspace_bytes() bytes; post_dev: float64 [n, n] device tensor;
    diag_dev: float64 [8] device tensor or None; stream: torch.cuda.Stream or
    None (current stream). Returns without synchronising.
    """
    import torch

    n, m = int(data_dev.shape[0]), int(data_dev.shape[1])
    assert data_dev.dtype == torch.uint8 and data_dev.is_contiguous() and data_dev.is_cuda
    assert post_dev.dtype == torch.float64 and post_dev.numel() >= n * n and post_dev.is_cuda
    h = _ProblemHold((n, m), arity, d, score, ess, log_rho, log_q,
                     data_ptr=data_dev.data_ptr() if m > 0 else None, device=True)
    st = (stream if stream is not None else torch.cuda.current_stream()).cuda_stream
    _check(lib().bn_edge_posteriors_dev(h.ref(), _PREC[precision], ctypes.c_void_p(ws.data_ptr()),
                                        ws.numel() * ws.element_size(), ctypes.c_void_p(st),
                                        ctypes.c_void_p(post_dev.data_ptr()),
                                        None if diag_dev is None
                                        else ctypes.c_void_p(diag_dev.data_ptr()),
                                        None if timer is None else timer._h),
           "bn_edge_posteriors_dev")


def edge_posteriors_noalloc(data_dev, arity, d, precision, post_dev, diag_dev=None,
                            stream=None, score="bdeu", ess=1.0, log_rho=None, log_q=None):
    """Enqueue a solve that allocates nothing (bn_edge_posteriors_noalloc):
    the library's static device array is the workspace, so it takes
    problems whose workspace_bytes() is at most NOALLOC_MAX_BYTES. Arguments
    as for edge_posteriors_dev without ws and timer. Calls whose work
    overlaps on one GPU share that array and race."""
    import torch

    n, m = int(data_dev.shape[0]), int(data_dev.shape[1])
    assert data_dev.dtype == torch.uint8 and data_dev.is_contiguous() and data_dev.is_cuda
    assert post_dev.dtype == torch.float64 and post_dev.numel() >= n * n and post_dev.is_cuda
    h = _ProblemHold((n, m), arity, d, score, ess, log_rho, log_q,
                     data_ptr=data_dev.data_ptr() if m > 0 else None, device=True)
    st = (stream if stream is not None else torch.cuda.current_stream()).cuda_stream
    _check(lib().bn_edge_posteriors_noalloc(h.ref(), _PREC[precision], ctypes.c_void_p(st),
                                            ctypes.c_void_p(post_dev.data_ptr()),
                                            None if diag_dev is None
                                            else ctypes.c_void_p(diag_dev.data_ptr())),
           "bn_edge_posteriors_noalloc")


def modular_feature_posterior(data, arity, d, log_f, precision="fp64", score="bdeu", ess=1.0,
                              log_rho=None, log_q=None) -> dict:
    """E[f | D] for f(G) = prod_i f_i(G_i) (bn_modular_feature_posterior).

    log_f: [n, K] array, log f_i(G) in the rank order of local_scores (-inf
    for a zero factor). Returns dict(value, log_PD, log_PfD)."""
    data = np.ascontiguousarray(data, dtype=np.uint8)
    n = data.shape[0]
    K = num_parent_sets(n, d)
    lf = np.ascontiguousarray(log_f, dtype=np.float64)
    if lf.shape != (n, K):
        raise ValueError(f"log_f must have shape ({n}, {K})")
    h = _ProblemHold(data, arity, d, score, ess, log_rho, log_q)
    out = np.zeros(1)
    pair = np.zeros(2)
    _check(lib().bn_modular_feature_posterior(h.ref(), _PREC[precision], _ptr(lf), _ptr(out),
                                              _ptr(pair)),
           "bn_modular_feature_posterior")
    return dict(value=float(out[0]), log_PD=float(pair[0]), log_PfD=float(pair[1]))


SUBSET_KINDS = {"zeta_up": 0, "zeta_down": 1, "mobius_up": 2, "mobius_down": 3}


def subset_transform(x_dev, kind: str, d: int = -1, stream=None):
    """In-place subset transform of a float64 device tensor of 2^nbits values
    (bn_subset_transform): "zeta_up" (Def. 1, truncated to |S| <= d when
    0 <= d < nbits), "zeta_down" (Def. 2), "mobius_up" / "mobius_down" (their
    untruncated inverses). Enqueued on `stream` (torch.cuda.Stream, default the
    current stream); returns without synchronising."""
    import torch

    assert x_dev.dtype == torch.float64 and x_dev.is_cuda and x_dev.is_contiguous()
    size = x_dev.numel()
    nbits = size.bit_length() - 1
    if size < 2 or size != 1 << nbits:
        raise ValueError("the array must hold 2^nbits values, nbits >= 1")
    st = (stream if stream is not None else torch.cuda.current_stream()).cuda_stream
    _check(lib().bn_subset_transform(ctypes.c_void_p(x_dev.data_ptr()), nbits,
                                     SUBSET_KINDS[kind], int(d), ctypes.c_void_p(st)),
           "bn_subset_transform")


def subset_transform_x32(f_dev, b_dev, kind: str, d: int = -1, counts_dev=None, stream=None):
    """In-place zeta transform ("zeta_up", truncated to |S| <= d when
    0 <= d < nbits, or "zeta_down") of 2^nbits non-negative values in the
    FP32-scaled storage: value = f * 2^(64 (b - 200)), b = 0 meaning 0
    (bn_subset_transform_x32). f_dev: float32 device tensor, b_dev: uint8
    device tensor of the same length; counts_dev: optional int64 device
    tensor of 2 entries that receives += (saturated, flushed). Enqueued on
    `stream` (default the current stream); returns without synchronising."""
    import torch

    assert f_dev.dtype == torch.float32 and f_dev.is_cuda and f_dev.is_contiguous()
    assert b_dev.dtype == torch.uint8 and b_dev.is_cuda and b_dev.is_contiguous()
    size = f_dev.numel()
    nbits = size.bit_length() - 1
    if size < 2 or size != 1 << nbits or b_dev.numel() != size:
        raise ValueError("both planes must hold 2^nbits values, nbits >= 1")
    cnt = None
    if counts_dev is not None:
        assert counts_dev.dtype == torch.int64 and counts_dev.is_cuda and counts_dev.numel() == 2
        cnt = ctypes.c_void_p(counts_dev.data_ptr())
    st = (stream if stream is not None else torch.cuda.current_stream()).cuda_stream
    _check(lib().bn_subset_transform_x32(ctypes.c_void_p(f_dev.data_ptr()),
                                         ctypes.c_void_p(b_dev.data_ptr()), nbits,
                                         SUBSET_KINDS[kind], int(d), cnt, ctypes.c_void_p(st)),
           "bn_subset_transform_x32")


def zeta4_probe(x_dev, y_dev, method: str, reps: int = 1, stream=None) -> float:
    """bn_zeta4_probe: the 4-bit upward zeta of every 16-entry group of the
    float64 device tensor x_dev into y_dev, by "valu" (register add steps) or
    "mfma" (the group matrix times the subset-inclusion matrix on the FP64
    matrix cores); reps > 1 repeats the arithmetic in registers. Waits for
    the kernel and returns its time in ms."""
    import torch

    for t in (x_dev, y_dev):
        assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
    assert x_dev.numel() == y_dev.numel() and x_dev.numel() % 16 == 0
    st = (stream if stream is not None else torch.cuda.current_stream()).cuda_stream
    ms = ctypes.c_float(0.0)
    _check(lib().bn_zeta4_probe(ctypes.c_void_p(x_dev.data_ptr()), ctypes.c_void_p(y_dev.data_ptr()),
                                x_dev.numel() // 16, {"valu": 0, "mfma": 1}[method], int(reps),
                                ctypes.c_void_p(st), ctypes.byref(ms)), "bn_zeta4_probe")
    return float(ms.value)


class Server:
    """Continuous-batching server (bn_server_* calls)."""

    def __init__(self, mem_budget_bytes: int = 0, max_active: int = 16):
        h = ctypes.c_void_p()
        _check(lib().bn_server_create(mem_budget_bytes, max_active, ctypes.byref(h)),
               "bn_server_create")
        self._h = h
        self._n = {}

    def submit(self, data, arity, d, precision="fp32", score="bdeu", ess=1.0, log_rho=None,
               log_q=None) -> int:
        h = _ProblemHold(data, arity, d, score, ess, log_rho, log_q)
        t = ctypes.c_uint64()
        _check(lib().bn_serve_submit(self._h, h.ref(), _PREC[precision], ctypes.byref(t)),
               "bn_serve_submit")
        self._n[t.value] = h.n
        return int(t.value)

    def poll(self, ticket: int, timeout_us: int = 0):
        """Returns (status, post or None, report dict or None)."""
        n = self._n.get(ticket, 1)
        post = np.empty((n, n), dtype=np.float64)
        rep = Report()
        s = lib().bn_serve_poll(self._h, ticket, _ptr(post), ctypes.byref(rep), timeout_us)
        if s == BN_OK:
            self._n.pop(ticket, None)
            return s, post, rep.as_dict()
        if s == BN_ECANCELED:
            self._n.pop(ticket, None)
        return s, None, None

    def close(self):
        if self._h:
            _check(lib().bn_server_destroy(self._h), "bn_server_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
