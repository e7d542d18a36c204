"""FP64 CPU oracle for sum-product LDPC decoding -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may call
this package.  It shares no code with the GPU library: the C source here builds
its own adjacency lists from the COO input and decodes each frame with the
flooding schedule of the paper's Algorithms 1-4 and 7, in double precision
(see ldpc_oracle.c for the passage each step follows).

Parity status: every function here is pinned by the CPU tests
(tests/test_oracle_pins.py): brute-force bitwise MAP on cycle-free graphs,
the probability-domain form of Algorithm 1, closed forms on single-parity-check
and path codes, noiseless and all-zero inputs, the degree-1 clamp, sign
symmetry, and the paper's Tables I and II for the adjacency lists.  The
Min-Sum rules are pinned by brute-force max-log MAP on single parity checks,
brute-force max-marginals on cycle-free graphs, and the path-code closed form.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ldpc_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
# the same source built with FP32 arithmetic: a diagnostic of how two
# precisions of the algorithm drift apart (see decode(fp32_build=True))
_SO_F32 = os.path.join(_HERE, "liboracle_f32.so")
LMAX = 64.0
# check rules: name -> (code, default parameter); "ms" is the normalized rule with alpha = 1
RULES = {"sp": (0, 0.0), "nms": (1, 0.75), "oms": (2, 0.25), "ms": (1, 1.0)}
_libs = {}


def build() -> str:
    """Compile the oracle with gcc (OpenMP over frames, strict IEEE arithmetic),
    plus its FP32 build (the same steps in float; a diagnostic only)."""
    for so, real in ((_SO, "double"), (_SO_F32, "float")):
        tmp = so + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-Wextra", f"-DORACLE_REAL={real}", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, so)
    return _SO


def _load(fp32_build: bool = False):
    so = _SO_F32 if fp32_build else _SO
    if so not in _libs:
        if not os.path.exists(so):
            build()
        lib = ctypes.CDLL(so)
        P = ctypes.c_void_p
        lib.ldpc_oracle_decode.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_long, P, P, P,
                                           ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_double, P, P, P, P, P, P, ctypes.c_int]
        lib.ldpc_oracle_decode.restype = ctypes.c_int
        lib.ldpc_oracle_decode_rule.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_long, P, P, P,
                                                ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                                ctypes.c_double, ctypes.c_int, ctypes.c_double, P, P, P, P, P, P,
                                                ctypes.c_int]
        lib.ldpc_oracle_decode_rule.restype = ctypes.c_int
        lib.ldpc_oracle_adjacency.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_long, P, P, P, P, P, P]
        lib.ldpc_oracle_adjacency.restype = ctypes.c_int
        _libs[so] = lib
    return _libs[so]


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def decode(code, llr, max_iter: int, early_stop: bool = True, lmax: float = LMAX,
           threads: int = 0, want_lpost: bool = True, tie_margin: float = 1e-3, rule: str = "sp",
           param: float | None = None, fp32_build: bool = False) -> dict:
    """Decode every row of `llr` ([F][n] float32) on the CPU in FP64.

    rule: "sp" (sum-product, the paper's decoder), "ms" (Min-Sum), "nms"
    (normalized Min-Sum, param = alpha) or "oms" (offset Min-Sum, param = beta).

    Returns a dict with bits [F][n] u8, ok [F] u8, iters [F] i32,
    min_abs [F] f64 (smallest |Lpost| over all iterations run), tie_risk [F]
    u8 (1 if flipping the sign of bits with |Lpost| < tie_margin could change
    bits, ok or iters) and, if asked, lpost [F][n] f64.

    fp32_build: run the same algorithm compiled with FP32 arithmetic instead
    (a diagnostic of precision drift, never a reference).
    """
    lib = _load(fp32_build)
    rows = np.ascontiguousarray(code.rows, dtype=np.int32)
    cols = np.ascontiguousarray(code.cols, dtype=np.int32)
    llr = np.ascontiguousarray(np.atleast_2d(llr), dtype=np.float32)
    F, n = llr.shape
    if n != code.n:
        raise ValueError("llr width does not match the code length")
    bits = np.zeros((F, n), np.uint8)
    ok = np.zeros(F, np.uint8)
    iters = np.zeros(F, np.int32)
    min_abs = np.zeros(F, np.float64)
    tie_risk = np.zeros(F, np.uint8)
    lpost = np.zeros((F, n), np.float64) if want_lpost else None
    kind, default = RULES[rule]
    p = default if param is None or rule == "ms" else float(param)
    st = lib.ldpc_oracle_decode_rule(code.m, code.n, rows.size, _ptr(rows), _ptr(cols), _ptr(llr), F,
                                     int(max_iter), int(bool(early_stop)), float(lmax), float(tie_margin),
                                     kind, p, _ptr(lpost) if want_lpost else None, _ptr(bits), _ptr(ok),
                                     _ptr(iters), _ptr(min_abs), _ptr(tie_risk), int(threads))
    if st != 0:
        raise ValueError(f"oracle rejected the input (status {st})")
    out = dict(bits=bits, ok=ok, iters=iters, min_abs=min_abs, tie_risk=tie_risk)
    if want_lpost:
        out["lpost"] = lpost
    return out


def adjacency(code):
    """The oracle's own N_i / M_j lists: (bit_start, bit_edge, chk_start, chk_edge)."""
    lib = _load()
    rows = np.ascontiguousarray(code.rows, dtype=np.int32)
    cols = np.ascontiguousarray(code.cols, dtype=np.int32)
    bs = np.zeros(code.n + 1, np.int32)
    be = np.zeros(rows.size, np.int32)
    cs = np.zeros(code.m + 1, np.int32)
    ce = np.zeros(rows.size, np.int32)
    st = lib.ldpc_oracle_adjacency(code.m, code.n, rows.size, _ptr(rows), _ptr(cols),
                                   _ptr(bs), _ptr(be), _ptr(cs), _ptr(ce))
    if st != 0:
        raise ValueError(f"oracle rejected the graph (status {st})")
    return bs, be, cs, ce
