"""Build the HIP library ``libhntt.so`` in-tree for gfx950 with hipcc.

Every call compiles from scratch (object files go to ``_build/`` next to this
file).  Usage: ``python -m paper_1205_2926_amd.build`` or ``build()``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhntt.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", f"-I{INCLUDE}", f"-I{CSRC}",
    "-Wall", "-Wno-unused-function",
    # packed fp32 instructions are kept out of all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]

SOURCES = ["ntt_kernels.hip", "hntt_api.cpp", "polymul.cpp", "polymul.hip", "static_scratch.hip",
           ("ntt_pass.hip", "u32_fwd", ["-DHNTT_WORD=32", "-DHNTT_INVERSE=0"]),
           ("ntt_pass.hip", "u32_inv", ["-DHNTT_WORD=32", "-DHNTT_INVERSE=1"]),
           ("ntt_pass.hip", "u64_fwd", ["-DHNTT_WORD=64", "-DHNTT_INVERSE=0"]),
           ("ntt_pass.hip", "u64_inv", ["-DHNTT_WORD=64", "-DHNTT_INVERSE=1"])]


def _compile(spec) -> str:
    """spec: a source file name, or (source, object tag, extra flags)."""
    src, tag, extra = (spec, None, []) if isinstance(spec, str) else spec
    stem = os.path.basename(src) + (f".{tag}" if tag else "")
    obj = os.path.join(OBJDIR, stem + ".o")
    cmd = [HIPCC, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {stem}")
    return obj


PROBE_SRC = os.path.join(HERE, "probe", "valu_rates.hip")
PROBE_BIN = os.path.join(HERE, "probe", "valu_rates")
LDS_PROBE_SRC = os.path.join(HERE, "probe", "lds_banks.hip")
LDS_PROBE_BIN = os.path.join(HERE, "probe", "lds_banks")


def build_probe() -> str:
    """The standalone measurement programs: instruction rates, shader clock and copy
    bandwidth (valu_rates), and the LDS lane grouping and bank mapping (lds_banks)."""
    for src, out in ((PROBE_SRC, PROBE_BIN), (LDS_PROBE_SRC, LDS_PROBE_BIN)):
        tmp = out + ".tmp"
        cmd = [HIPCC, "-O3", "-std=c++17", f"--offload-arch={ARCH}",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", src, "-o", tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"hipcc failed on {os.path.basename(src)}")
        os.replace(tmp, out)
    return PROBE_BIN


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    sources = list(SOURCES)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(sources))) as ex:
        objs = list(ex.map(_compile, sources))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libhntt.so failed")
    os.replace(tmp, LIB)
    build_probe()
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
