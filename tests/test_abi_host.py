"""Host-side checks of the C ABI (no GPU needed).

The library must load, export every function declared in include/bn.h, and
reject invalid problems before any device work.
"""
import os
import re

import numpy as np
import pytest

import paper_1408_1664_amd as bn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def built_library():
    if not os.path.exists(bn.LIB_PATH):
        from paper_1408_1664_amd import build
        build.build()
    return bn.lib()


def _declared():
    src = open(os.path.join(ROOT, "include", "bn.h")).read()
    return sorted(set(re.findall(r"\b(bn_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ["bn_local_scores", "bn_edge_posteriors", "bn_edge_posteriors_dev",
                 "bn_serve_submit", "bn_serve_poll", "bn_server_create", "bn_server_destroy",
                 "bn_workspace_bytes", "bn_num_parent_sets", "bn_status_string"]:
        assert want in names


def test_library_exports_every_declared_symbol():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", bn.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if " T " in l)
    for name in _declared():
        assert name in exported, name
        assert hasattr(bn.lib(), name)


def test_num_parent_sets():
    from math import comb
    for n in range(1, 32):
        for d in range(0, 6):
            want = sum(comb(n - 1, k) for k in range(min(d, n - 1) + 1))
            assert bn.num_parent_sets(n, d) == want
    assert bn.num_parent_sets(0, 2) == 0
    assert bn.num_parent_sets(5, -1) == 0


def test_workspace_grows_with_n_and_precision(monkeypatch):
    a = bn.workspace_bytes(20, 3, 500, "fp32")
    b = bn.workspace_bytes(21, 3, 500, "fp32")
    c = bn.workspace_bytes(20, 3, 500, "fp64")
    assert b > 1.9 * a
    assert c > a
    # dominant terms with alpha materialised: alpha n 2^(n-1) and the two 2^n sweeps
    n = 25
    w64 = bn.workspace_bytes(n, 4, 2000, "fp64")
    assert w64 >= 8 * n * 2 ** (n - 1) + 2 * 8 * 2 ** n
    w32m = bn.workspace_bytes(n, 4, 2000, "fp32")    # the default below 240 GiB
    assert w32m >= 5 * n * 2 ** (n - 1) + 2 * 5 * 2 ** n
    monkeypatch.setenv("BN_FUSED_ALPHA", "0")
    assert bn.workspace_bytes(n, 4, 2000, "fp32") == w32m
    # alpha never materialised: the two sweeps plus the 9-bit block seeds,
    # K(9, d - 1) of 8 bytes per block
    monkeypatch.setenv("BN_FUSED_ALPHA", "1")
    w32 = bn.workspace_bytes(n, 4, 2000, "fp32")
    seeds = 8 * n * 2 ** (n - 10) * (1 + 9 + 36 + 84)
    assert 2 * 5 * 2 ** n + seeds <= w32 < w32m - 5 * n * 2 ** (n - 1) + seeds + (64 << 20)
    # n = 31 fits one 288 GB device in both FP32-scaled forms, n = 32 does not exist
    monkeypatch.delenv("BN_FUSED_ALPHA")
    assert bn.workspace_bytes(31, 3, 500, "fp32") < 240 * 2 ** 30
    monkeypatch.setenv("BN_FUSED_ALPHA", "1")
    assert bn.workspace_bytes(31, 3, 500, "fp32") < 100e9
    monkeypatch.delenv("BN_FUSED_ALPHA")
    # the plan fuses by itself only where materialised alpha passes 240 GiB
    # and the fused plan is smaller: n = 31, d = 4 (253.6 -> 161.5 GiB); at
    # n = 30, d = 6 the 9-bit block seeds outgrow alpha, so alpha stays
    monkeypatch.setenv("BN_FUSED_ALPHA", "0")
    m31, m30 = bn.workspace_bytes(31, 4, 500, "fp32"), bn.workspace_bytes(30, 6, 500, "fp32")
    monkeypatch.setenv("BN_FUSED_ALPHA", "1")
    f31, f30 = bn.workspace_bytes(31, 4, 500, "fp32"), bn.workspace_bytes(30, 6, 500, "fp32")
    monkeypatch.delenv("BN_FUSED_ALPHA")
    assert m31 > 240 * 2 ** 30 > f31 and bn.workspace_bytes(31, 4, 500, "fp32") == f31
    assert f30 > m30 and bn.workspace_bytes(30, 6, 500, "fp32") == m30
    with pytest.raises(bn.BnError):
        bn.workspace_bytes(1, 2, 10, "fp32")
    with pytest.raises(bn.BnError):
        bn.workspace_bytes(32, 2, 10, "fp32")


@pytest.mark.parametrize("case", ["n_small", "n_big", "arity1", "value_ge_arity", "ess0",
                                  "neg_d", "bins"])
def test_invalid_problems_rejected_before_device_work(case):
    rng = np.random.default_rng(0)
    data = rng.integers(0, 2, size=(6, 40)).astype(np.uint8)
    arity = np.full(6, 2, np.uint8)
    kw = dict(d=2, ess=1.0)
    if case == "n_small":
        data, arity = data[:1], arity[:1]
    elif case == "n_big":
        data = np.zeros((32, 4), np.uint8)
        arity = np.full(32, 2, np.uint8)
    elif case == "arity1":
        arity = arity.copy(); arity[3] = 1
    elif case == "value_ge_arity":
        data = data.copy(); data[2, 7] = 2
    elif case == "ess0":
        kw["ess"] = 0.0
    elif case == "neg_d":
        kw["d"] = -1
    elif case == "bins":
        arity = np.full(6, 20, np.uint8)
        data = (data * 19).astype(np.uint8)
        kw["d"] = 3   # 20^4 bins > the histogram limit
    for fn in (lambda: bn.local_scores(data, arity, kw["d"], ess=kw["ess"]),
               lambda: bn.edge_posteriors(data, arity, kw["d"], "fp32", ess=kw["ess"]),
               lambda: bn.parent_set_posteriors(data, arity, kw["d"], "fp32", ess=kw["ess"])):
        with pytest.raises(bn.BnError) as ei:
            fn()
        assert ei.value.status == bn.BN_EINVAL


def test_status_strings():
    assert bn.status_string(0) == "ok"
    assert "invalid" in bn.status_string(-1)


def test_parent_set_posteriors_needs_an_output():
    import ctypes
    data = np.zeros((4, 10), np.uint8)
    arity = np.full(4, 2, np.uint8)
    h = bn._ProblemHold(data, arity, 2, "bdeu", 1.0, None, None)
    st = bn.lib().bn_parent_set_posteriors(h.ref(), 1, None, None, None)
    assert st == bn.BN_EINVAL


def test_subset_transform_rejects_bad_arguments():
    import ctypes
    L = bn.lib()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every case fails the checks
    assert L.bn_subset_transform(None, 10, 0, -1, None) == bn.BN_EINVAL
    assert L.bn_subset_transform(fake, 0, 0, -1, None) == bn.BN_EINVAL
    assert L.bn_subset_transform(fake, 33, 0, -1, None) == bn.BN_EINVAL
    assert L.bn_subset_transform(fake, 10, 4, -1, None) == bn.BN_EINVAL
    assert L.bn_subset_transform(fake, 10, 2, 3, None) == bn.BN_EINVAL   # truncated inverse
    assert L.bn_subset_transform(fake, 10, 3, 0, None) == bn.BN_EINVAL


def test_subset_transform_x32_rejects_bad_arguments():
    import ctypes
    L = bn.lib()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every case fails the checks
    assert L.bn_subset_transform_x32(None, fake, 10, 0, -1, None, None) == bn.BN_EINVAL
    assert L.bn_subset_transform_x32(fake, None, 10, 0, -1, None, None) == bn.BN_EINVAL
    assert L.bn_subset_transform_x32(fake, fake, 0, 0, -1, None, None) == bn.BN_EINVAL
    assert L.bn_subset_transform_x32(fake, fake, 33, 1, -1, None, None) == bn.BN_EINVAL
    assert L.bn_subset_transform_x32(fake, fake, 10, 2, -1, None, None) == bn.BN_EINVAL  # Moebius
    assert L.bn_subset_transform_x32(fake, fake, 10, 3, -1, None, None) == bn.BN_EINVAL
    assert L.bn_subset_transform_x32(fake, fake, 10, 4, -1, None, None) == bn.BN_EINVAL


def test_zeta4_probe_rejects_bad_arguments():
    import ctypes
    L = bn.lib()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every case fails the checks
    ms = ctypes.c_float()
    assert L.bn_zeta4_probe(None, fake, 16, 0, 1, None, ctypes.byref(ms)) == bn.BN_EINVAL
    assert L.bn_zeta4_probe(fake, fake, 16, 0, 1, None, None) == bn.BN_EINVAL
    assert L.bn_zeta4_probe(fake, fake, 8, 0, 1, None, ctypes.byref(ms)) == bn.BN_EINVAL
    assert L.bn_zeta4_probe(fake, fake, 40, 1, 1, None, ctypes.byref(ms)) == bn.BN_EINVAL
    assert L.bn_zeta4_probe(fake, fake, (1 << 32) + 16, 0, 1, None,
                            ctypes.byref(ms)) == bn.BN_EINVAL
    assert L.bn_zeta4_probe(fake, fake, 16, 2, 1, None, ctypes.byref(ms)) == bn.BN_EINVAL
    assert L.bn_zeta4_probe(fake, fake, 16, 0, 0, None, ctypes.byref(ms)) == bn.BN_EINVAL
    assert L.bn_zeta4_probe(fake, fake, 16, 1, 4097, None, ctypes.byref(ms)) == bn.BN_EINVAL


def test_modular_feature_rejects_bad_arguments():
    import ctypes
    data = np.zeros((4, 10), np.uint8)
    arity = np.full(4, 2, np.uint8)
    h = bn._ProblemHold(data, arity, 2, "bdeu", 1.0, None, None)
    K = bn.num_parent_sets(4, 2)
    out = np.zeros(1)
    lf = np.zeros((4, K))
    L = bn.lib()
    assert L.bn_modular_feature_posterior(h.ref(), 1, None, bn._ptr(out), None) == bn.BN_EINVAL
    assert L.bn_modular_feature_posterior(h.ref(), 1, bn._ptr(lf), None, None) == bn.BN_EINVAL
    for bad in [np.nan, np.inf]:
        lf2 = lf.copy()
        lf2[2, 3] = bad
        assert L.bn_modular_feature_posterior(h.ref(), 1, bn._ptr(lf2), bn._ptr(out), None) == bn.BN_EINVAL
    with pytest.raises(ValueError):
        bn.modular_feature_posterior(data, arity, 2, np.zeros((4, K + 1)))


def test_noalloc_rejects_problems_beyond_its_array():
    # checked against bn_workspace_bytes before any device call: a problem
    # whose workspace exceeds the static array gets BN_ENOMEM, and an
    # invalid one BN_EINVAL, without touching the (fake) device pointers
    import ctypes
    L = bn.lib()
    fake = ctypes.c_void_p(0x1000)
    for n, prec in [(22, 0), (22, 1), (25, 1)]:
        assert bn.workspace_bytes(n, 3, 100, prec) > bn.NOALLOC_MAX_BYTES
        h = bn._ProblemHold((n, 100), np.full(n, 2, np.uint8), 3, data_ptr=0x1000)
        assert L.bn_edge_posteriors_noalloc(h.ref(), prec, None, fake, None) == bn.BN_ENOMEM
    for n, prec in [(21, 1), (21, 0)]:
        assert bn.workspace_bytes(n, 3, 2000, prec) <= bn.NOALLOC_MAX_BYTES
    h = bn._ProblemHold((12, 100), np.full(12, 2, np.uint8), 3, data_ptr=0x1000)
    assert L.bn_edge_posteriors_noalloc(h.ref(), 1, None, None, None) == bn.BN_EINVAL
    assert L.bn_edge_posteriors_noalloc(h.ref(), 7, None, fake, None) == bn.BN_EINVAL
    assert L.bn_edge_posteriors_noalloc(None, 1, None, fake, None) == bn.BN_EINVAL
