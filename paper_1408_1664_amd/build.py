"""Build libbnpost.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbnpost.so")
SOURCES = ["bn_kernels.hip", "bn_fused.hip", "bn_solver.hip", "bn_serve.hip", "bn_subset.hip",
           "bn_probe.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # no packed FP32 instructions anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer (device code is
# built as usual): each option applies to the host compilation only.
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
LIB_SAN = os.path.join(HERE, "libbnpost_san.so")
# Measurement build of the literal block-only FP32 form (every value a plain
# float under the per-node and per-layer gauges, no per-value exponent);
# selected with BN_LIBRARY.
LIB_LITERAL = os.path.join(HERE, "libbnpost_literal.so")


def build(verbose: bool = False, sanitize: bool = False, literal: bool = False) -> str:
    """Compile every source for gfx950 and link libbnpost.so; with sanitize,
    libbnpost_san.so with the host code under ASan and UBSan (loaded with
    the sanitizer runtime preloaded, BN_LIBRARY pointing at it); with
    literal, libbnpost_literal.so (BN_X32_LITERAL)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    flags = FLAGS + (SAN_FLAGS if sanitize else []) + (["-DBN_X32_LITERAL"] if literal else [])
    out_lib = LIB_SAN if sanitize else (LIB_LITERAL if literal else LIB)
    with tempfile.TemporaryDirectory() as td:
        objs = []
        procs = []
        for s in SOURCES:
            obj = os.path.join(td, s + ".o")
            cmd = [hipcc, *flags, "-c", os.path.join(CSRC, s), "-o", obj]
            procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                              stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        for s, p in procs:
            out, _ = p.communicate()
            if p.returncode != 0:
                sys.stderr.write(out)
                raise RuntimeError(f"hipcc failed on {s}")
            if verbose and out.strip():
                sys.stderr.write(out)
        tmp = out_lib + ".tmp"
        link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread",
                "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
        if sanitize:
            link += ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                     "-Xarch_host", "-shared-libsan"]
        subprocess.run(link, check=True)
        os.replace(tmp, out_lib)
    return out_lib


if __name__ == "__main__":
    print(build(verbose=True, sanitize="--sanitize" in sys.argv, literal="--literal" in sys.argv))
