"""GPU parity on the quasi-cyclic stand-in (the headline degree profile lifted by
Z = 360): sampled frames of a full 256-frame call against the oracle,
properties on every frame, and the graph built from the base matrix
(circulant indexing) against the graph built from the COO and the oracle."""
import numpy as np
import pytest

import ldpc_inputs as li
from parity import compare, gpu_decode

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")


def test_qc_code_full_batch_sampled_frames():
    code = li.large_qc_code()
    cw = li.Encoder(code).random_codewords(256, seed=3102)
    llr = li.awgn_llr(code.n, 256, li.ebn0_to_sigma2(1.2, code.rate), seed=2112, codewords=cw)
    print("[case] qc-64800 frames=256", flush=True)
    out = gpu_decode(code, llr, 50)
    assert ((out["lpost"] < 0) == out["bits"].astype(bool)).all()
    syn = code.syndrome(out["bits"]).any(axis=1)
    assert (syn == (out["ok"] == 0)).all()
    print(compare(code, llr, 50, frames=[0, 1, 128, 255], gpu=out))


def _same(a, b, what):
    for k in ("bits", "ok", "iters", "lpost"):
        assert (a[k] == b[k]).all(), f"{what}: {k} differs"


@pytest.mark.parametrize("msg,lane", [("fp32", 0), ("fp32", 1), ("fp16", 0), ("bf16", 2), ("fp32-compact", 0)])
def test_circulant_indexing_equals_column_table(msg, lane):
    """The check pass of a graph built from the base matrix (ldpc_graph_create_qc,
    bits computed from the shifts) against the same code built from its COO
    (bits read from the column table): identical results for every message
    format, lane width and the compacted schedule."""
    from paper_1609_01567_amd import ldpc
    code = li.large_qc_code()
    Z, shifts = code.qc
    flags = {"fp32": 0, "fp16": ldpc.MSG_FP16, "bf16": ldpc.MSG_BF16, "fp32-compact": ldpc.COMPACT_TAIL}[msg]
    flags |= {0: 0, 1: ldpc.LANE_SLOTS_1, 2: ldpc.LANE_SLOTS_2}[lane]
    cw = li.Encoder(code).random_codewords(256, seed=3103)
    llr = li.awgn_llr(code.n, 256, li.ebn0_to_sigma2(1.1, code.rate), seed=2113, codewords=cw)
    print(f"[case] qc circulant indexing {msg} lane={lane}", flush=True)
    qc = gpu_decode(code, llr, 50, flags=flags, graph=ldpc.Graph.from_qc(Z, shifts))
    coo = gpu_decode(code, llr, 50, flags=flags, graph=ldpc.Graph.from_code(code))
    _same(qc, coo, f"qc vs coo ({msg}, lane {lane})")
    assert len(np.unique(qc["iters"])) >= 3


def test_circulant_indexing_small_lifting_against_oracle():
    """A small lifted code (Z = 13, rows of 5..12 edges in both register classes)
    through the base-matrix graph against the oracle, with fixed iterations on
    every frame and with early stop."""
    from paper_1609_01567_amd import ldpc
    rng = np.random.default_rng(41)
    mb, nb, Z = 12, 30, 13
    shifts = np.full((mb, nb), -1, np.int32)
    for i in range(mb):
        d = 5 if i < 6 else 12
        js = rng.choice(nb, size=d, replace=False)
        shifts[i, js] = rng.integers(0, Z, size=d)
    rows, cols = [], []
    for i in range(mb):
        js = np.nonzero(shifts[i] >= 0)[0]
        for t in range(Z):
            rows.extend([i * Z + t] * len(js))
            cols.extend((js * Z + (t + shifts[i, js]) % Z).tolist())
    code = li.Code(m=mb * Z, n=nb * Z, rows=np.array(rows, np.int32), cols=np.array(cols, np.int32),
                   qc=(Z, shifts))
    g = ldpc.Graph.from_qc(Z, shifts)
    llr = li.awgn_llr(code.n, 100, 0.8, seed=42)
    print("[case] qc small lifting vs oracle", flush=True)
    compare(code, llr, 6, early_stop=False, posterior_all=True, gpu=gpu_decode(code, llr, 6, flags=ldpc.NO_EARLY_STOP,
                                                                                   graph=g))
    print(compare(code, llr, 30, gpu=gpu_decode(code, llr, 30, graph=g)))
