"""Host-side checks of the C-ABI library: it loads, exports what include/ldpc.h
declares, builds the paper's address arrays, and rejects bad input.
No GPU is needed: graphs are built with LDPC_GRAPH_HOST_ONLY and every decode
call here is one that fails argument checks before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import ldpc_inputs as li
from paper_1609_01567_amd import ldpc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "ldpc.h")).read()
    return sorted(set(re.findall(r"LDPC_API\s+[\w\s\*]*?\b(ldpc_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ldpc.load_library()
    declared = _declared_symbols()
    assert len(declared) >= 8
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(ldpc.EXPORTED) == declared


def test_status_strings():
    lib = ldpc.load_library()
    assert lib.ldpc_status_str(0) == b"LDPC_OK"
    assert lib.ldpc_status_str(3) == b"LDPC_E_DUP_EDGE"
    assert lib.ldpc_status_str(99) == b"LDPC_E_UNKNOWN"


def test_address_arrays_match_paper_tables(tables):
    code = li.code_14_7()
    g = ldpc.Graph.from_code(code, host_only=True)
    a = g.arrays()
    E = code.nnz
    # Table I (bit-sorted positions)
    cp = a["col_ptr"]
    v = np.repeat(np.arange(code.n), np.diff(cp))
    assert v.tolist() == tables["v"]
    assert a["row_idx"].tolist() == tables["c"]
    assert [int(cp[x + 1] - cp[x]) for x in v] == tables["t"]
    assert [int(cp[x]) for x in v] == tables["s"]
    assert [k - int(cp[v[k]]) for k in range(E)] == tables["u"]
    # Table II (check-sorted positions)
    rp = a["row_ptr"]
    c = np.repeat(np.arange(code.m), np.diff(rp))
    assert a["csr_to_csc"].tolist() == tables["ebar"]
    assert a["col_idx"].tolist() == tables["vbar"]
    assert c.tolist() == tables["cbar"]
    assert [int(rp[x + 1] - rp[x]) for x in c] == tables["tbar"]
    assert [int(rp[x]) for x in c] == tables["sbar"]
    assert [k - int(rp[c[k]]) for k in range(E)] == tables["ubar"]
    info = g.info()
    assert (info["m"], info["n"], info["nnz"], info["max_check_deg"], info["max_bit_deg"]) == (7, 14, 31, 5, 4)
    assert info["device_bytes"] == 0


@pytest.mark.parametrize("maker", [li.tiny_code, li.extreme_code])
def test_address_arrays_consistent_on_random_codes(maker):
    code = maker()
    g = ldpc.Graph.from_code(code, host_only=True)
    a = g.arrays()
    rp, ci, cp, ri, m2c = a["row_ptr"], a["col_idx"], a["col_ptr"], a["row_idx"], a["csr_to_csc"]
    rows_csr = np.repeat(np.arange(code.m), np.diff(rp))
    cols_csc = np.repeat(np.arange(code.n), np.diff(cp))
    # same edge seen from both sides
    assert (ri[m2c] == rows_csr).all()
    assert (cols_csc[m2c] == ci).all()
    assert sorted(m2c.tolist()) == list(range(code.nnz))
    # stable order: within each check, input order is kept
    order = np.argsort(code.rows, kind="stable")
    assert (ci == code.cols[order]).all()
    info = g.info()
    assert info["max_check_deg"] == code.check_degrees().max()
    assert info["max_bit_deg"] == code.bit_degrees().max()


@pytest.mark.parametrize("m,n,rows,cols,status", [
    (0, 4, [0], [0], ldpc.E_INVAL),
    (2, 0, [0], [0], ldpc.E_INVAL),
    (2, 4, [2], [0], ldpc.E_RANGE),
    (2, 4, [0], [4], ldpc.E_RANGE),
    (2, 4, [-1], [0], ldpc.E_RANGE),
    (2, 4, [0, 1, 0], [1, 1, 1], ldpc.E_DUP_EDGE),
])
def test_graph_create_rejects_bad_input(m, n, rows, cols, status):
    with pytest.raises(ldpc.LdpcError) as ei:
        ldpc.Graph(m, n, np.array(rows), np.array(cols), host_only=True)
    assert ei.value.status == status


def _lifted_by_definition(Z, shifts):
    """COO of the lifted H straight from the definition of a circulant block:
    row i*Z + t of block (i, j) has its one in column j*Z + ((t + s_ij) mod Z)."""
    H = np.zeros((shifts.shape[0] * Z, shifts.shape[1] * Z), np.uint8)
    eye = np.eye(Z, dtype=np.uint8)
    for i, j in zip(*np.nonzero(shifts >= 0)):
        H[i * Z:(i + 1) * Z, j * Z:(j + 1) * Z] = np.roll(eye, shifts[i, j], axis=1)
    return H


@pytest.mark.parametrize("Z,mb,nb,seed", [(1, 3, 5, 1), (7, 4, 9, 2), (360, 90, 180, 3)])
def test_qc_graph_equals_lifted_matrix(Z, mb, nb, seed):
    rng = np.random.default_rng(seed)
    shifts = np.where(rng.random((mb, nb)) < 0.35, rng.integers(0, Z, (mb, nb)), -1).astype(np.int32)
    shifts[np.arange(mb), rng.integers(0, nb, mb)] = rng.integers(0, Z, mb)   # no empty base row
    g = ldpc.Graph.from_qc(Z, shifts, host_only=True)
    a = g.arrays()
    assert g.info()["nnz"] == int((shifts >= 0).sum()) * Z == a["col_idx"].size
    if Z * nb <= 2000:   # the dense definition for the small cases
        H = _lifted_by_definition(Z, shifts)
        rows_csr = np.repeat(np.arange(mb * Z), np.diff(a["row_ptr"]))
        D = np.zeros_like(H)
        D[rows_csr, a["col_idx"]] = 1
        assert (D == H).all() and H.sum() == a["col_idx"].size
    # the same tables as the COO graph of the lifted code, edges in base-column order within each check
    rows, cols = [], []
    for i in range(mb):
        js = np.nonzero(shifts[i] >= 0)[0]
        for t in range(Z):
            rows.extend([i * Z + t] * len(js))
            cols.extend((js * Z + (t + shifts[i, js]) % Z).tolist())
    ref = ldpc.Graph(mb * Z, nb * Z, np.array(rows), np.array(cols), host_only=True).arrays()
    for k in ref:
        assert (a[k] == ref[k]).all(), k


def test_qc_graph_of_the_structured_stand_in_equals_its_coo_graph():
    code = li.large_qc_code()
    Z, shifts = code.qc
    a = ldpc.Graph.from_qc(Z, shifts, host_only=True).arrays()
    b = ldpc.Graph.from_code(code, host_only=True).arrays()
    for k in a:
        assert (a[k] == b[k]).all(), k


@pytest.mark.parametrize("mb,nb,Z,shift,status", [
    (0, 2, 4, 0, ldpc.E_INVAL),
    (2, 2, 0, 0, ldpc.E_INVAL),
    (2, 2, 4, 4, ldpc.E_RANGE),
    (2, 2, 4, -2, ldpc.E_RANGE),
    (2, 1 << 20, 1 << 12, -1, ldpc.E_INVAL),    # n = nb * Z beyond 2^31
])
def test_qc_graph_rejects_bad_input(mb, nb, Z, shift, status):
    shifts = np.full((max(mb, 1), min(nb, 4)), -1, np.int32)
    shifts[0, 0] = shift
    lib = ldpc.load_library()
    h = ctypes.c_void_p()
    st = lib.ldpc_graph_create_qc(mb, nb, Z, shifts.ctypes.data, 1, ctypes.byref(h))
    assert st == status
    assert not h
    assert lib.ldpc_graph_create_qc(2, 2, 4, None, 1, ctypes.byref(h)) == ldpc.E_INVAL


def test_empty_rows_and_columns_are_accepted():
    g = ldpc.Graph(4, 6, np.array([0, 0, 2], np.int32), np.array([1, 3, 3], np.int32), host_only=True)
    a = g.arrays()
    assert a["row_ptr"].tolist() == [0, 2, 2, 3, 3]
    assert a["col_ptr"].tolist() == [0, 0, 1, 1, 3, 3, 3]
    g0 = ldpc.Graph(3, 3, np.zeros(0, np.int32), np.zeros(0, np.int32), host_only=True)
    assert g0.info()["nnz"] == 0


def test_workspace_size_rules():
    code = li.tiny_code()
    g = ldpc.Graph.from_code(code, host_only=True)
    assert ldpc.workspace_size(g, 0) == 0
    w32 = ldpc.workspace_size(g, 32)
    w16 = ldpc.workspace_size(g, 32, ldpc.MSG_FP16)
    w8 = ldpc.workspace_size(g, 32, ldpc.MSG_Q8)
    assert w32 > w16 > w8 > 0
    assert w16 - w8 >= code.nnz * 64 - 256          # one byte less per stored message
    # fp32: Lch + Lpost (n*S*4 each) + R (E*S*4) with S = 64 slots, plus small state
    assert w32 >= (2 * code.n + code.nnz) * 64 * 4
    assert ldpc.workspace_size(g, 1000) > ldpc.workspace_size(g, 100) > w32
    for bad in (ldpc.MSG_FP16 | ldpc.MSG_BF16, ldpc.MSG_FP16 | ldpc.MSG_Q8, ldpc.MSG_BF16 | ldpc.MSG_Q8):
        with pytest.raises(ldpc.LdpcError):
            ldpc.workspace_size(g, 8, bad)
    with pytest.raises(ldpc.LdpcError):
        ldpc.workspace_size(g, -1)
    with pytest.raises(ldpc.LdpcError):
        ldpc.workspace_size(g, 8, 1 << 8)               # no such flag


def test_compact_tail_workspace():
    """Tail compaction adds copies of the state for a half and a quarter of the
    slots, from 256 slots up, and nothing without early stopping."""
    code = li.tiny_code()
    g = ldpc.Graph.from_code(code, host_only=True)
    for msg, mb in ((0, 4), (ldpc.MSG_FP16, 2), (ldpc.MSG_Q8, 1)):
        base = ldpc.workspace_size(g, 1000, msg)
        comp = ldpc.workspace_size(g, 1000, msg | ldpc.COMPACT_TAIL)
        # S = 1024 slots (4 per lane): copies of 512 and 256 slots
        # Lch, Lpost, messages; iters, fail, map; 16-bit formats add a 16-bit posterior copy
        per_slot = 2 * code.n * 4 + code.nnz * mb + 3 * 4 + (2 * code.n if mb == 2 else 0)
        assert comp - base >= per_slot * 768
        assert comp - base <= per_slot * 768 + 16 * 256
        assert ldpc.workspace_size(g, 1000, msg | ldpc.COMPACT_TAIL | ldpc.NO_EARLY_STOP) == \
            ldpc.workspace_size(g, 1000, msg | ldpc.NO_EARLY_STOP)
    assert ldpc.workspace_size(g, 100, ldpc.COMPACT_TAIL) == ldpc.workspace_size(g, 100)   # 128 slots


def test_decode_argument_checks_fail_before_device_work():
    lib = ldpc.load_library()
    code = li.code_14_7()
    g = ldpc.Graph.from_code(code, host_only=True)
    call = lambda *a: lib.ldpc_decode(g.handle, *a)
    P = ctypes.c_void_p
    # host-only graph
    assert call(P(8), 1, 5, 0, P(8), P(8), P(8), None, P(256), 1 << 20, None) == ldpc.E_INVAL
    assert b"host-only" in lib.ldpc_last_error()
    # null graph
    assert lib.ldpc_decode(None, P(8), 1, 5, 0, P(8), P(8), P(8), None, P(256), 1, None) == ldpc.E_INVAL
    # frames == 0 is a no-op even with null buffers
    assert lib.ldpc_decode(g.handle, None, 0, 5, 0, None, None, None, None, None, 0, None) in (ldpc.OK, ldpc.E_INVAL)


def test_decode_rule_argument_checks():
    lib = ldpc.load_library()
    g = ldpc.Graph.from_code(li.code_14_7(), host_only=True)
    P = ctypes.c_void_p
    bufs = (P(8), P(8), None, P(256), 1 << 20, None)   # ok, iters, llr_out, workspace, bytes, stream
    cases = [(ldpc.Rule(7, 0.0), b"kind"), (ldpc.Rule(ldpc.RULE_MIN_SUM_NORMALIZED, 0.0), b"alpha"),
             (ldpc.Rule(ldpc.RULE_MIN_SUM_NORMALIZED, 1.5), b"alpha"),
             (ldpc.Rule(ldpc.RULE_MIN_SUM_NORMALIZED, float("nan")), b"alpha"),
             (ldpc.Rule(ldpc.RULE_MIN_SUM_OFFSET, -0.5), b"beta"), (ldpc.Rule(ldpc.RULE_MIN_SUM_OFFSET, 64.0), b"beta"),
             (ldpc.Rule(ldpc.RULE_SUM_PRODUCT, 0.0, (ctypes.c_int32 * 2)(1, 0)), b"reserved")]
    for rule, word in cases:
        st = lib.ldpc_decode_rule(g.handle, P(8), 1, 5, 0, ctypes.byref(rule), P(8), *bufs)
        assert st == ldpc.E_INVAL and word in lib.ldpc_last_error()
        st = lib.ldpc_simulate_rule(g.handle, 1, 1.0, 1, 0, 5, 0, ctypes.byref(rule), P(8), None, P(256), 1 << 20,
                                    None)
        assert st == ldpc.E_INVAL and word in lib.ldpc_last_error()
    # a valid rule gets as far as the graph checks
    for rule in (None, ldpc.make_rule("ms"), ldpc.make_rule("nms", 0.8), ldpc.make_rule("oms", 0.3)):
        st = lib.ldpc_decode_rule(g.handle, P(8), 1, 5, 0, ctypes.byref(rule) if rule else None, P(8), *bufs)
        assert st == ldpc.E_INVAL and b"host-only" in lib.ldpc_last_error()


def test_engine_argument_checks_fail_before_device_work():
    lib = ldpc.load_library()
    P = ctypes.c_void_p
    out = P()
    one = (ctypes.c_int32 * 1)(64)
    graphs = (P * 1)(None)
    assert lib.ldpc_engine_create(None, 1, one, one, 10, 0, None, ctypes.byref(out)) == ldpc.E_INVAL
    assert lib.ldpc_engine_create(graphs, 0, one, one, 10, 0, None, ctypes.byref(out)) == ldpc.E_INVAL
    assert lib.ldpc_engine_create(graphs, 33, one, one, 10, 0, None, ctypes.byref(out)) == ldpc.E_INVAL
    assert lib.ldpc_engine_create(graphs, 1, one, one, 0, 0, None, ctypes.byref(out)) == ldpc.E_INVAL
    assert lib.ldpc_engine_create(graphs, 1, one, one, 10, ldpc.MSG_FP16 | ldpc.MSG_BF16, None,
                                  ctypes.byref(out)) == ldpc.E_INVAL
    bad = ldpc.EngineOpts(3, 0)
    assert lib.ldpc_engine_create(graphs, 1, one, one, 10, 0, ctypes.byref(bad), ctypes.byref(out)) == ldpc.E_INVAL
    for ips in (-1, 17):
        bad = ldpc.EngineOpts(0, 0, 0, ips)
        assert lib.ldpc_engine_create(graphs, 1, one, one, 10, 0, ctypes.byref(bad), ctypes.byref(out)) == ldpc.E_INVAL
    for kind, p in ((9, 0.0), (ldpc.RULE_MIN_SUM_NORMALIZED, 0.0), (ldpc.RULE_MIN_SUM_OFFSET, 64.0)):
        bad = ldpc.EngineOpts(0, 0, 0, 0, kind, p)
        assert lib.ldpc_engine_create(graphs, 1, one, one, 10, 0, ctypes.byref(bad), ctypes.byref(out)) == ldpc.E_INVAL
    assert not out
    for f in ("ldpc_engine_step", "ldpc_engine_poll", "ldpc_engine_run", "ldpc_engine_info"):
        fn = getattr(lib, f)
        args = {"ldpc_engine_step": (None, 1), "ldpc_engine_poll": (None, None, None),
                "ldpc_engine_run": (None, 0, None), "ldpc_engine_info": (None, None, None)}[f]
        assert fn(*args) == ldpc.E_INVAL
    assert lib.ldpc_engine_destroy(None) == ldpc.OK
    assert ctypes.sizeof(ldpc.Frame) == 48
