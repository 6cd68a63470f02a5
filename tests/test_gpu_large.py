"""GPU checks of the largest lattices (n = 27..31) against references that do
not come from the GPU.

* n = 27: the first 27 variables of the n = 30 benchmark dataset (binary,
  m = 500, d = 3), both number systems and the FP32-scaled form without
  linear tiles, element by element against the oracle's posteriors stored in
  tests/golden/ (written by make_oracle_refs.py, which calls only the
  oracle). This is the largest lattice the oracle holds in host memory; the
  n = 28..30 regime rests on it plus the checks below.
* n = 28..31 with no data (m = 0): every local score is 1, so every order has
  the same weight and every edge posterior equals a closed form in n, d and
  the prior (tests/ref/brute.py m0_closed_form, pinned to exact rationals on
  the CPU). These runs cross 2^31 lattice entries per array (alpha from
  n = 28, L and Rp from n = 31), so every index path of the large sizes is
  exercised against a value fixed by the mathematics.
* n = 31 with data (binary, m = 500, d = 3; FP32-scaled only: FP64 does not
  fit in 288 GB): the invariants and the posterior bounds.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import paper_1408_1664_amd as bn
from paper_1408_1664_amd import datagen
from tests.ref.brute import m0_closed_form

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _fits(n, d, m, prec):
    import torch
    free, _ = torch.cuda.mem_get_info()
    return bn.workspace_bytes(n, d, m, prec) + (2 << 30) < free


def _solve_dev(data, arity, d, prec, ess=1.0):
    import torch
    n, m = data.shape
    ws = torch.empty(bn.workspace_bytes(n, d, m, prec), dtype=torch.uint8, device="cuda")
    dd = torch.from_numpy(np.ascontiguousarray(data)).cuda()
    post = torch.empty((n, n), dtype=torch.float64, device="cuda")
    diag = torch.zeros(8, dtype=torch.float64, device="cuda")
    bn.edge_posteriors_dev(dd, arity, d, prec, ws, post, diag, ess=ess)
    torch.cuda.synchronize()
    out = post.cpu().numpy(), diag.cpu().numpy()
    del ws, dd, post, diag
    torch.cuda.empty_cache()
    return out


def _bounds(P, d, tol):
    assert np.all(np.diag(P) == 0)
    assert P.min() >= 0.0 and P.max() <= 1.0 + tol
    assert np.all(P + P.T <= 1.0 + tol)
    assert np.all(P.sum(axis=0) <= d + d * tol)


@pytest.mark.parametrize("prec,tol,lin,fused", [("fp64", 1e-10, None, "0"),
                                                ("fp64", 1e-10, "force", "0"),
                                                ("fp64", 1e-10, "0", "0"),
                                                ("fp32", 1e-5, None, "0"),
                                                ("fp32", 1e-5, "0", "0"),
                                                ("fp32", 1e-5, "force", "0"),
                                                ("fp32", 1e-5, None, "1")])
def test_n27_prefix_of_n30_against_oracle(prec, tol, lin, fused, monkeypatch):
    ref = json.load(open(os.path.join(GOLD, "oracle_n30_binary_m500_d3_first27.json")))
    ds, p = datagen.workload("n30_binary_m500_d3")
    k = ref["first_vars"]
    assert k == 27 and ref["m"] == ds.m and ref["d"] == p["d"]
    if lin is not None:
        monkeypatch.setenv("BN_LINEAR_TILES", lin)
    monkeypatch.setenv("BN_FUSED_ALPHA", fused)   # 1: alpha never materialised
    print(f"n27 {prec} linear tiles {lin or 'on'} fused {fused}", flush=True)
    P, diag = _solve_dev(ds.data[:k], ds.arity[:k], p["d"], prec, p["ess"])
    err = np.abs(P - np.array(ref["post"])).max()
    print(f"n27 {prec}: max |dP| = {err:.3e}, log L(V) {diag[0]:.6f} vs {ref['log_LV']:.6f}, "
          f"residual {diag[1]:.2e}, fallback {diag[7]:.0f}", flush=True)
    assert err <= tol
    assert abs(diag[0] - ref["log_LV"]) <= 1e-9 * abs(ref["log_LV"])
    assert diag[2] == 0
    _bounds(P, p["d"], tol)


@pytest.mark.parametrize("n,prec,fused", [(28, "fp64", "0"), (28, "fp32", "0"), (29, "fp32", "0"),
                                          (30, "fp64", "0"), (30, "fp32", "0"), (31, "fp32", "0"),
                                          (30, "fp32", "1"), (31, "fp32", "1")])
def test_no_data_closed_form_at_large_n(n, prec, fused, monkeypatch):
    d = 3
    monkeypatch.setenv("BN_FUSED_ALPHA", fused)   # 1: alpha never materialised
    if not _fits(n, d, 0, prec):
        pytest.skip(f"n={n} {prec} workspace does not fit in free device memory")
    rho = [Fraction(1, math.comb(n - 1, k)) for k in range(d + 1)]
    want = float(m0_closed_form(n, d, rho))
    data = np.zeros((n, 0), np.uint8)
    print(f"m=0 n={n} {prec} fused {fused}", flush=True)
    P, diag = _solve_dev(data, np.full(n, 2, np.uint8), d, prec)
    tol = 1e-10 if prec == "fp64" else 1e-5
    off = P[~np.eye(n, dtype=bool)]
    err = np.abs(off - want).max()
    print(f"m=0 n={n} {prec}: closed form {want:.12f}, max |dP| = {err:.3e}, "
          f"residual {diag[1]:.2e}", flush=True)
    assert err <= tol
    assert np.all(np.diag(P) == 0)
    assert diag[1] < (1e-9 if prec == "fp64" else 1e-4)


def test_n31_d4_plan_fuses_by_itself(monkeypatch):
    """n = 31, d = 4: materialised alpha would take 253.6 GiB, so the plan
    takes the fused sweeps (161.5 GiB) without being asked; m = 0 has the
    closed form."""
    n, d = 31, 4
    monkeypatch.setenv("BN_FUSED_ALPHA", "1")
    fused_bytes = bn.workspace_bytes(n, d, 0, "fp32")
    monkeypatch.delenv("BN_FUSED_ALPHA")
    assert bn.workspace_bytes(n, d, 0, "fp32") == fused_bytes
    if not _fits(n, d, 0, "fp32"):
        pytest.skip("the n=31, d=4 workspace does not fit in free device memory")
    rho = [Fraction(1, math.comb(n - 1, k)) for k in range(d + 1)]
    want = float(m0_closed_form(n, d, rho))
    print("m=0 n=31 d=4 fp32, plan's own choice (fused)", flush=True)
    P, diag = _solve_dev(np.zeros((n, 0), np.uint8), np.full(n, 2, np.uint8), d, "fp32")
    off = P[~np.eye(n, dtype=bool)]
    err = np.abs(off - want).max()
    print(f"m=0 n=31 d=4: closed form {want:.12f}, max |dP| = {err:.3e}, "
          f"residual {diag[1]:.2e}", flush=True)
    assert err <= 1e-5
    assert diag[1] < 1e-4


@pytest.mark.parametrize("fused", ["0", "1"])
def test_n31_fp32_properties(fused, monkeypatch):
    n, m, d = 31, 500, 3
    monkeypatch.setenv("BN_FUSED_ALPHA", fused)   # 1: alpha never materialised
    if not _fits(n, d, m, "fp32"):
        pytest.skip("n=31 FP32-scaled workspace does not fit in free device memory")
    ds = datagen.random_dag_dataset(n, m, 2, 3, 1.0, seed=31)
    print(f"n31 fp32 m=500 fused {fused}", flush=True)
    P, diag = _solve_dev(ds.data, ds.arity, d, "fp32")
    print(f"n31 fp32: log L(V) {diag[0]:.6f}, residual {diag[1]:.2e}, saturated {diag[2]:.0f}, "
          f"flushed {diag[3]:.0f}, fallback {diag[7]:.0f}", flush=True)
    assert np.isfinite(diag[0])
    assert diag[1] < 1e-4
    assert diag[2] == 0
    _bounds(P, d, 1e-5)
