"""The literal block-only FP32 form, measured once against the oracle.

The FP32-scaled form keeps an exponent byte per value. Its literal reading
(exponent identically 0: every value a plain float, with only the per-node
and per-layer gauges applied in FP64 to the log scores) is built as
libbnpost_literal.so (BN_X32_LITERAL) and run here with the linear tiles and
the fused sweeps off, so that every zeta and sweep step is FP32 arithmetic.
Its posteriors on n12_binary_m200_d3 and n20_ternary_m1000_d4 are compared
with the oracle's; the measured errors are printed, and the test checks the
finding the library's design rests on: the literal form misses the 1e-5
target, while the form with the exponent byte meets it on the same inputs.
Measured on MI355X: n = 12 stays within the float range after the gauges
(max |dP| 4.0e-8, the same as with the exponent byte); at n = 20 (m = 1000,
three states) L(V) underflows to zero, log L(V) is -inf and the posteriors
are lost (max |dP| 1.0), where the exponent-byte form gives 1.7e-7.
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import paper_1408_1664_amd as bn
from oracle import oracle as O
from paper_1408_1664_amd import build as B
from paper_1408_1664_amd import datagen

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WORKLOADS = ["n12_binary_m200_d3", "n20_ternary_m1000_d4"]

_CHILD = r"""
import json, sys
import paper_1408_1664_amd as bn
from paper_1408_1664_amd import datagen
out = {}
for name in sys.argv[1:]:
    ds, p = datagen.workload(name)
    post, rep = bn.edge_posteriors(ds.data, ds.arity, p["d"], precision="fp32", ess=p["ess"])
    out[name] = dict(post=post.tolist(), log_LV=rep["log_LV"], saturated=rep["saturated"],
                     flushed=rep["flushed"])
print("RESULT " + json.dumps(out), flush=True)
"""


def _literal_run():
    env = dict(os.environ, BN_LIBRARY=B.LIB_LITERAL, BN_LINEAR_TILES="0", BN_FUSED_ALPHA="0",
               PYTHONPATH=ROOT)
    print("literal FP32 build: " + ", ".join(WORKLOADS), flush=True)
    r = subprocess.run([sys.executable, "-c", _CHILD, *WORKLOADS], env=env, cwd=ROOT,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    line = [x for x in r.stdout.splitlines() if x.startswith("RESULT ")][-1]
    return json.loads(line[len("RESULT "):])


@pytest.mark.skipif(not os.path.exists(B.LIB_LITERAL), reason="libbnpost_literal.so not built")
def test_literal_fp32_against_oracle(monkeypatch):
    lit = _literal_run()
    monkeypatch.setenv("BN_LINEAR_TILES", "0")
    monkeypatch.setenv("BN_FUSED_ALPHA", "0")
    worst_lit = 0.0
    for name in WORKLOADS:
        ds, p = datagen.workload(name)
        ref = O.edge_posteriors(ds.data, ds.arity, p["d"], ess=p["ess"])
        P = np.array(lit[name]["post"])
        assert P.shape == ref["post"].shape
        bad = ~np.isfinite(P)
        err_lit = float(np.abs(np.where(bad, 0.0, P) - ref["post"]).max())
        worst_lit = max(worst_lit, np.inf if bad.any() else err_lit)
        # the exponent-byte form on the same inputs, in this process (libbnpost.so)
        post, rep = bn.edge_posteriors(ds.data, ds.arity, p["d"], precision="fp32",
                                       ess=p["ess"])
        err_x32 = float(np.abs(post - ref["post"]).max())
        print(f"{name}: literal FP32 max |dP| = {err_lit:.3e} over finite entries, "
              f"{int(bad.sum())} non-finite, log L(V) {lit[name]['log_LV']:.6f} "
              f"(oracle {ref['log_LV']:.6f}); with the exponent byte {err_x32:.3e}", flush=True)
        assert err_x32 <= 1e-5
    assert worst_lit > 1e-5
