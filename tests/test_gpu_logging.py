"""BN_LOG_LEVEL: the plan of each solve (level 1) and its report (level 2)
on stderr. The level is read once per process, so the solve runs in a child
process."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_CHILD = r"""
import paper_1408_1664_amd as bn
from paper_1408_1664_amd import datagen
ds, p = datagen.workload("n12_binary_m200_d3")
post, rep = bn.edge_posteriors(ds.data, ds.arity, p["d"], precision="fp32", ess=p["ess"])
print("LOGV %.9f" % rep["log_LV"], flush=True)
"""


@pytest.mark.parametrize("level", ["0", "1", "2"])
def test_log_level(level):
    env = dict(os.environ, BN_LOG_LEVEL=level, PYTHONPATH=ROOT)
    print(f"BN_LOG_LEVEL={level}", flush=True)
    r = subprocess.run([sys.executable, "-c", _CHILD], env=env, cwd=ROOT, capture_output=True,
                       text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [x for x in r.stderr.splitlines() if x.startswith("[bn] ")]
    plan = [x for x in lines if x.startswith("[bn] solve ")]
    report = [x for x in lines if x.startswith("[bn] report ")]
    if level == "0":
        assert not lines
    else:
        assert len(plan) == 1 and "n=12 m=200 d=3 fp32_scaled alpha=materialised" in plan[0]
        assert len(report) == (1 if level == "2" else 0)
    if level == "2":
        logv = float([x for x in r.stdout.splitlines() if x.startswith("LOGV ")][0].split()[1])
        assert f"log_L(V)={logv:.9f}" in report[0]
