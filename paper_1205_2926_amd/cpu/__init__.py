"""Same-host CPU counterpart of the paper's Table 1 (Section 5): Algorithm 2 and
Algorithm 3 transforms of length 2^11 over a 62-bit prime on one core, compiled
with gcc -O2 as in the paper.  A measurement program for the host CPU, separate
from the GPU library."""
from __future__ import annotations

import ctypes
import os
import platform
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "table1.c")
LIB = os.path.join(_HERE, "libtable1.so")
_lib = None


def build() -> str:
    subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", SRC, "-o", LIB], check=True)
    return LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        u64, p64 = ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)
        lib.t1_plan_create.restype = ctypes.c_void_p
        lib.t1_plan_create.argtypes = [u64, u64, ctypes.c_int]
        lib.t1_plan_destroy.argtypes = [ctypes.c_void_p]
        lib.t1_forward.argtypes = [ctypes.c_void_p, ctypes.c_int, p64]
        lib.t1_time.argtypes = [ctypes.c_void_p, ctypes.c_int, p64, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double)]
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def forward(x, p: int, omega: int, alg: int) -> np.ndarray:
    """One transform of x (length 2^l) with Algorithm `alg` (2 or 3), reduced to [0, p)."""
    lib = load()
    a = np.ascontiguousarray(x, dtype=np.uint64).copy()
    l = a.size.bit_length() - 1
    pl = lib.t1_plan_create(p, omega, l)
    lib.t1_forward(pl, alg, _p(a))
    lib.t1_plan_destroy(pl)
    return np.where(a >= p, a - p, a)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def run(x, p: int, omega: int, reps: int = 20000) -> dict:
    """ns and time-stamp-counter ticks per butterfly for both algorithms (one core)."""
    lib = load()
    a = np.ascontiguousarray(x, dtype=np.uint64).copy()
    l = a.size.bit_length() - 1
    pl = lib.t1_plan_create(p, omega, l)
    out = {}
    for alg in (2, 3):
        ns, ticks = ctypes.c_double(), ctypes.c_double()
        b = a.copy()
        lib.t1_time(pl, alg, _p(b), reps, ctypes.byref(ns), ctypes.byref(ticks))
        out[f"alg{alg}"] = {"ns_per_butterfly": ns.value, "tsc_ticks_per_butterfly": ticks.value}
    lib.t1_plan_destroy(pl)
    gcc = subprocess.run(["gcc", "--version"], capture_output=True, text=True).stdout.splitlines()[0]
    out.update({"alg2_over_alg3": out["alg2"]["ns_per_butterfly"] / out["alg3"]["ns_per_butterfly"],
                "cpu": cpu_model(), "compiler": gcc + " -O2", "log2_len": l, "p": p, "reps": reps})
    return out
