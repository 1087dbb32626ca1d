"""The C oracle and the library's host code built with AddressSanitizer and
UndefinedBehaviorSanitizer, and the CPU tests run against those builds (host code
only: device code is never instrumented).  Each run is a subprocess with the
matching sanitizer runtime preloaded; any report fails the test."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _gcc_runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


def _run(files, preload, extra_env):
    env = dict(os.environ, LD_PRELOAD=preload, **SAN_ENV, **extra_env)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider", *files],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, out
    assert " passed" in r.stdout, out


def test_oracle_under_asan_and_ubsan(tmp_path):
    asan, ubsan = _gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc sanitizer runtimes not found")
    import oracle
    lib = oracle.build(("-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=all"), out=str(tmp_path / "libntt_oracle_san.so"))
    _run(["tests/test_oracle_pins.py", "tests/test_cpu_table1.py"], f"{asan}:{ubsan}", {"ORACLE_LIB": lib})


def test_host_runtime_under_asan_and_ubsan(tmp_path):
    rts = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rts:
        pytest.skip("clang sanitizer runtime not found")
    from paper_1205_2926_amd import build as B
    # host translation units with sanitizers (flags only on the host side), device code as built
    host_srcs = ["hntt_api.cpp", "polymul.cpp", "static_scratch.hip"]
    objs = []
    for src in host_srcs:
        obj = str(tmp_path / (src + ".o"))
        cmd = [B.HIPCC, *B.COMMON, "-g", "-fno-omit-frame-pointer",
               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-fno-sanitize-recover=all", "-c", os.path.join(B.CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(obj)
    for spec in B.SOURCES:
        src, tag = (spec, None) if isinstance(spec, str) else spec[:2]
        if src in host_srcs:
            continue
        obj = os.path.join(B.OBJDIR, os.path.basename(src) + (f".{tag}" if tag else "") + ".o")
        if not os.path.exists(obj):
            pytest.skip("library objects not built")
        objs.append(obj)
    lib = str(tmp_path / "libhntt_san.so")
    r = subprocess.run([B.HIPCC, "-shared", f"--offload-arch={B.ARCH}", "-fPIC", "-Xarch_host", "-fsanitize=address",
                        "-Xarch_host", "-fsanitize=undefined", *objs, "-o", lib], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    _run(["tests/test_abi_host.py"], rts[-1], {"HNTT_LIB": lib})
