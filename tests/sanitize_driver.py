"""Runs the host code under AddressSanitizer / UndefinedBehaviorSanitizer.

Started by tests/test_host_sanitizers.py in a child process whose LD_PRELOAD
holds the sanitizer runtime; argv[1] is the folder with the sanitized builds:
  liboracle_san.so  the FP64 oracle (oracle/ldpc_oracle.c)
  libgf2enc_san.so  the systematic GF(2) encoder (ldpc_inputs/gf2enc.c)
  libgraph_san.so   the Tanner-graph builder of the library (csrc/graph.cpp)
Every call below must finish without a sanitizer report, and its results are
checked against numpy.  This process imports neither torch nor the HIP
library; graphs are built host-only.
"""
import ctypes
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import ldpc_inputs as li  # noqa: E402

P = ctypes.c_void_p


def ptr(a):
    return a.ctypes.data_as(P)


def load(folder):
    ora = ctypes.CDLL(os.path.join(folder, "liboracle_san.so"))
    ora.ldpc_oracle_decode_rule.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_long, P, P, P, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_int, ctypes.c_double, P, P, P, P, P, P, ctypes.c_int]
    ora.ldpc_oracle_adjacency.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_long, P, P, P, P, P, P]
    enc = ctypes.CDLL(os.path.join(folder, "libgf2enc_san.so"))
    enc.gf2enc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_long, P, P, ctypes.POINTER(P),
                                  ctypes.POINTER(ctypes.c_int)]
    enc.gf2enc_encode.argtypes = [P, ctypes.c_int, P, P]
    enc.gf2enc_info_columns.argtypes = [P, P]
    enc.gf2enc_free.argtypes = [P]
    gr = ctypes.CDLL(os.path.join(folder, "libgraph_san.so"))
    gr.ldpc_graph_create.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, P, P, ctypes.c_uint32,
                                     ctypes.POINTER(P)]
    gr.ldpc_graph_info.argtypes = [P, P, P, P, P, P, P]
    gr.ldpc_graph_arrays.argtypes = [P, P, P, P, P, P]
    gr.ldpc_graph_destroy.argtypes = [P]
    gr.ldpc_last_error.restype = ctypes.c_char_p
    return ora, enc, gr


def degenerate_code():
    # check 0 = {0}; check 1 = {0,1,2}; check 2 empty; check 3 = {2,3}; bit 4 unconnected
    return li.Code(m=4, n=5, rows=np.array([0, 1, 1, 1, 3, 3], np.int32), cols=np.array([0, 0, 1, 2, 2, 3], np.int32))


def hub_code():
    rng = np.random.default_rng(11)
    cdeg = np.concatenate([[300, 140, 64, 40, 33], rng.integers(3, 33, size=45)])
    E = int(cdeg.sum())
    bdeg = np.full(400, E // 400)
    bdeg[: E - bdeg.sum()] += 1
    return li.socket_code(bdeg, cdeg, seed=12)


def codes():
    return [li.code_14_7(), li.tiny_code(), li.random_small_code(300, 150, 3, seed=31), degenerate_code(),
            hub_code(), li.tree_code(4, seed=3), li.spc_code(9), li.path_code(7)]


def check_oracle(ora):
    for code in codes():
        rows, cols = np.ascontiguousarray(code.rows, np.int32), np.ascontiguousarray(code.cols, np.int32)
        bs = np.zeros(code.n + 1, np.int32)
        be = np.zeros(max(code.nnz, 1), np.int32)
        cs = np.zeros(code.m + 1, np.int32)
        ce = np.zeros(max(code.nnz, 1), np.int32)
        assert ora.ldpc_oracle_adjacency(code.m, code.n, code.nnz, ptr(rows), ptr(cols), ptr(bs), ptr(be), ptr(cs),
                                         ptr(ce)) == 0
        assert (be[:code.nnz] == np.argsort(cols, kind="stable")).all()
        assert (ce[:code.nnz] == np.argsort(rows, kind="stable")).all()
        F = 5
        llr = li.awgn_llr(code.n, F, 0.9, seed=code.n)
        for rule, param in ((0, 0.0), (1, 0.75), (2, 0.25)):
            for es in (0, 1):
                lp = np.zeros((F, code.n))
                bits = np.zeros((F, code.n), np.uint8)
                ok = np.zeros(F, np.uint8)
                it = np.zeros(F, np.int32)
                mn = np.zeros(F)
                tr = np.zeros(F, np.uint8)
                st = ora.ldpc_oracle_decode_rule(code.m, code.n, code.nnz, ptr(rows), ptr(cols), ptr(llr), F, 12, es,
                                                 64.0, 1e-3, rule, param, ptr(lp), ptr(bits), ptr(ok), ptr(it),
                                                 ptr(mn), ptr(tr), 2)
                assert st == 0
                assert (bits == (lp < 0)).all()
                assert (ok == ~code.syndrome(bits).any(axis=1)).all()
    # rejected input: an index out of range, and max_iter 0
    code = li.code_14_7()
    rows = np.ascontiguousarray(code.rows, np.int32).copy()
    rows[3] = 7
    cols = np.ascontiguousarray(code.cols, np.int32)
    llr = np.zeros((1, 14), np.float32)
    out = [np.zeros((1, 14)), np.zeros((1, 14), np.uint8), np.zeros(1, np.uint8), np.zeros(1, np.int32),
           np.zeros(1), np.zeros(1, np.uint8)]
    assert ora.ldpc_oracle_decode_rule(7, 14, code.nnz, ptr(rows), ptr(cols), ptr(llr), 1, 5, 1, 64.0, 1e-3, 0, 0.0,
                                       *[ptr(o) for o in out], 1) != 0
    print("oracle ok", flush=True)


def check_encoder(enc):
    for code in [li.code_14_7(), li.tiny_code(), li.random_small_code(300, 150, 3, seed=31), li.large_code()]:
        rows, cols = np.ascontiguousarray(code.rows, np.int32), np.ascontiguousarray(code.cols, np.int32)
        h = P()
        k = ctypes.c_int()
        assert enc.gf2enc_create(code.m, code.n, code.nnz, ptr(rows), ptr(cols), ctypes.byref(h), ctypes.byref(k)) == 0
        ic = np.zeros(k.value, np.int32)
        assert enc.gf2enc_info_columns(h, ptr(ic)) == k.value
        info = np.random.default_rng(1).integers(0, 2, size=(3, k.value), dtype=np.uint8)
        cw = np.zeros((3, code.n), np.uint8)
        assert enc.gf2enc_encode(h, 3, ptr(info), ptr(cw)) == 0
        assert not code.syndrome(cw).any()
        assert (cw[:, ic] == info).all()
        enc.gf2enc_free(h)
    print("encoder ok", flush=True)


def check_graph(gr):
    HOST_ONLY = 1
    for code in codes() + [li.large_code()]:
        rows, cols = np.ascontiguousarray(code.rows, np.int32), np.ascontiguousarray(code.cols, np.int32)
        g = P()
        st = gr.ldpc_graph_create(code.m, code.n, code.nnz, ptr(rows), ptr(cols), HOST_ONLY, ctypes.byref(g))
        assert st == 0, gr.ldpc_last_error()
        E = code.nnz
        row_ptr = np.zeros(code.m + 1, np.int32)
        col_idx = np.zeros(max(E, 1), np.int32)
        col_ptr = np.zeros(code.n + 1, np.int32)
        row_idx = np.zeros(max(E, 1), np.int32)
        c2c = np.zeros(max(E, 1), np.int32)
        assert gr.ldpc_graph_arrays(g, ptr(row_ptr), ptr(col_idx), ptr(col_ptr), ptr(row_idx), ptr(c2c)) == 0
        by_row = np.argsort(rows, kind="stable")
        by_col = np.argsort(cols, kind="stable")
        assert (row_ptr == np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=code.m))])).all()
        assert (col_idx[:E] == cols[by_row]).all()
        assert (col_ptr == np.concatenate([[0], np.cumsum(np.bincount(cols, minlength=code.n))])).all()
        assert (row_idx[:E] == rows[by_col]).all()
        vals = [ctypes.c_int64() for _ in range(3)] + [ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()]
        assert gr.ldpc_graph_info(g, *[ctypes.byref(v) for v in vals]) == 0
        assert vals[2].value == E
        assert gr.ldpc_graph_destroy(g) == 0
    # rejected graphs: duplicate edge, index out of range, bad sizes, unknown flags
    code = li.code_14_7()
    rows, cols = np.ascontiguousarray(code.rows, np.int32), np.ascontiguousarray(code.cols, np.int32)
    dup_r, dup_c = np.append(rows, rows[0]).astype(np.int32), np.append(cols, cols[0]).astype(np.int32)
    bad_r = rows.copy()
    bad_r[0] = 99
    for m, n, r, c, fl, want in ((7, 14, dup_r, dup_c, HOST_ONLY, 3), (7, 14, bad_r, cols, HOST_ONLY, 2),
                                 (0, 14, rows, cols, HOST_ONLY, 1), (7, 14, rows, cols, 1 << 5, 1)):
        g = P()
        assert gr.ldpc_graph_create(m, n, r.size, ptr(r), ptr(c), fl, ctypes.byref(g)) == want
    print("graph ok", flush=True)


if __name__ == "__main__":
    ora, enc, gr = load(sys.argv[1])
    check_oracle(ora)
    check_encoder(enc)
    check_graph(gr)
    print("sanitized host code ok", flush=True)
