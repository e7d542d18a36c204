"""The host code built with AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The FP64 oracle, the GF(2) encoder of the input generators and the library's
Tanner-graph builder (csrc/graph.cpp, host-only graphs) are compiled with
-fsanitize=address,undefined and driven by tests/sanitize_driver.py in a child
process that preloads the sanitizer runtime: every call must finish with no
sanitizer report (out-of-bounds access, use after free, signed overflow,
misaligned access, ...) and with the results numpy expects.
The server's admission bookkeeping runs only beside a device engine and is
covered by the GPU tests instead.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all", "-g", "-O1", "-fPIC",
       "-shared"]


def _runtime():
    out = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


def test_host_code_under_asan_and_ubsan(tmp_path):
    asan = _runtime()
    if asan is None:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    d = str(tmp_path)
    subprocess.check_call(["gcc", *SAN, "-std=c11", "-fopenmp", "-DORACLE_REAL=double",
                           "-o", os.path.join(d, "liboracle_san.so"), os.path.join(ROOT, "oracle", "ldpc_oracle.c"),
                           "-lm"])
    subprocess.check_call(["gcc", *SAN, "-std=c11", "-fopenmp", "-o", os.path.join(d, "libgf2enc_san.so"),
                           os.path.join(ROOT, "ldpc_inputs", "gf2enc.c")])
    subprocess.check_call(["g++", *SAN, "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                           "-I" + os.path.join(ROOT, "include"), "-o", os.path.join(d, "libgraph_san.so"),
                           os.path.join(ROOT, "paper_1609_01567_amd", "csrc", "graph.cpp"),
                           "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64"])
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0:exitcode=86"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=87"
    env["OMP_NUM_THREADS"] = "2"
    res = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitize_driver.py"), d], env=env,
                         capture_output=True, text=True, timeout=600)
    report = res.stdout[-3000:] + res.stderr[-6000:]
    assert res.returncode == 0, report
    assert "AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr, report
    assert "sanitized host code ok" in res.stdout, report
