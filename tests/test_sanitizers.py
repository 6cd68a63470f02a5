"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

__graft_entry__.build() also builds libbnpost_san.so (the library's host
code -- validation, plans, workspace offsets, the server -- compiled with
-fsanitize=address,undefined; device code as usual) and the oracle as
liboracle_san.so. These tests rerun the host-side tests in a subprocess
against those builds, with the sanitizer runtimes preloaded, halting on the
first report. The GPU is never touched.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB_SAN = os.path.join(ROOT, "paper_1408_1664_amd", "libbnpost_san.so")
ORACLE_SAN = os.path.join(ROOT, "oracle", "liboracle_san.so")


def _run(tests, env_extra, tmp_path):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = f"detect_leaks=0:protect_shadow_gap=0:log_path={tmp_path}/asan"
    env["UBSAN_OPTIONS"] = f"print_stacktrace=1:halt_on_error=1:log_path={tmp_path}/ubsan"
    env.setdefault("OMP_NUM_THREADS", "4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider", *tests], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=900)
    reports = ""
    for f in sorted(glob.glob(os.path.join(str(tmp_path), "*san.*"))):
        reports += open(f).read()
    assert r.returncode == 0 and not reports, (r.stdout[-3000:], r.stderr[-3000:], reports[:6000])


def test_host_library_under_asan_ubsan(tmp_path):
    if not os.path.exists(LIB_SAN):
        pytest.skip("libbnpost_san.so not built (paper_1408_1664_amd/build.py --sanitize)")
    rt = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rt:
        pytest.skip("clang ASan runtime not found")
    _run(["tests/test_abi_host.py", "tests/test_serve.py"],
         {"BN_LIBRARY": LIB_SAN, "LD_PRELOAD": rt[0]}, tmp_path)


def test_oracle_under_asan_ubsan(tmp_path):
    if not os.path.exists(ORACLE_SAN):
        pytest.skip("liboracle_san.so not built (oracle.build_sanitized())")
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    _run(["tests/test_oracle_pins.py", "tests/test_oracle_subset_pins.py"],
         {"ORACLE_LIBRARY": ORACLE_SAN, "LD_PRELOAD": asan}, tmp_path)
