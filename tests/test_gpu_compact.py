"""GPU tests of tail compaction (LDPC_COMPACT_TAIL): once few frames of a call
still run, they move into a smaller slot range (with fewer slots per lane)
and finish there.  Only the schedule changes, so every output must be bit-identical to the
same decode without the flag (which is itself held to the oracle)."""
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


def _same(a, b, what):
    for k in ("bits", "ok", "iters", "lpost"):
        assert (a[k] == b[k]).all(), f"{what}: {k} differs"


def _mixed_code():
    rng = np.random.default_rng(31)
    cdeg = np.concatenate([[300, 140, 64, 40, 33], rng.integers(3, 33, size=95)])
    E = int(cdeg.sum())
    bdeg = np.full(700, E // 700)
    bdeg[: E - bdeg.sum()] += 1
    return li.socket_code(bdeg, cdeg, seed=32)


@pytest.mark.parametrize("msg", ["fp32", "fp16", "q8"])
@pytest.mark.parametrize("lane", [0, 2])
def test_compact_tail_equals_plain(msg, lane):
    from paper_1609_01567_amd import ldpc
    flags = {"fp32": 0, "fp16": ldpc.MSG_FP16, "q8": ldpc.MSG_Q8}[msg]
    flags |= {0: 0, 2: ldpc.LANE_SLOTS_2}[lane]
    rule = "oms" if msg == "q8" else None
    param = 0.5 if msg == "q8" else None
    code = li.random_small_code(600, 300, 3, seed=8)
    llr = li.awgn_llr(code.n, 1000, li.ebn0_to_sigma2(1.8, code.rate), seed=33)
    print(f"[case] compact msg={msg} lane={lane} frames=1000", flush=True)
    a = gpu_decode(code, llr, 40, flags=flags, rule=rule, param=param)
    b = gpu_decode(code, llr, 40, flags=flags | ldpc.COMPACT_TAIL, rule=rule, param=param)
    its = a["iters"]
    assert (its > 24).sum() > 0 and (its < 12).sum() > 400     # a tail that compaction reaches
    _same(a, b, f"{msg} lane {lane}")


def test_compact_tail_one_slot_per_lane_ragged_pool():
    """One slot per lane and 300 frames: 320 slots, copies of 128 and 64."""
    from paper_1609_01567_amd import ldpc
    code = li.random_small_code(600, 300, 3, seed=8)
    llr = li.awgn_llr(code.n, 300, li.ebn0_to_sigma2(1.8, code.rate), seed=36)
    print("[case] compact lane=1 frames=300", flush=True)
    a = gpu_decode(code, llr, 40, flags=ldpc.LANE_SLOTS_1)
    b = gpu_decode(code, llr, 40, flags=ldpc.LANE_SLOTS_1 | ldpc.COMPACT_TAIL)
    assert (a["iters"] > 20).sum() > 0
    _same(a, b, "lane 1, 300 frames")


def test_compact_tail_every_check_class():
    """Rows of every class (registers, chunks, more than 128 edges)."""
    from paper_1609_01567_amd import ldpc
    code = _mixed_code()
    llr = li.awgn_llr(code.n, 600, 0.2, seed=34)
    print("[case] compact mixed classes frames=600", flush=True)
    a = gpu_decode(code, llr, 30)
    b = gpu_decode(code, llr, 30, flags=ldpc.COMPACT_TAIL)
    assert len(set(a["iters"].tolist())) > 5
    _same(a, b, "mixed classes")


def test_compact_tail_all_stop_early():
    """Every frame stops early: the later iterations find no running frame."""
    from paper_1609_01567_amd import ldpc
    code = li.random_small_code(600, 300, 3, seed=8)
    llr = li.awgn_llr(code.n, 512, li.ebn0_to_sigma2(4.0, code.rate), seed=35)
    print("[case] compact all-stop frames=512", flush=True)
    a = gpu_decode(code, llr, 50)
    b = gpu_decode(code, llr, 50, flags=ldpc.COMPACT_TAIL)
    assert a["iters"].max() <= 10
    _same(a, b, "all stop early")


def test_compact_tail_large_code_and_oracle():
    """The headline code at 256 frames (copy of 64 slots), then the oracle on
    sampled frames of the compacted decode."""
    from paper_1609_01567_amd import ldpc
    code = li.large_code()
    cw = li.Encoder(code).random_codewords(256, seed=3005)
    llr = li.awgn_llr(code.n, 256, li.ebn0_to_sigma2(1.4, code.rate), seed=2042, codewords=cw)
    print("[case] compact large n=64800 frames=256", flush=True)
    a = gpu_decode(code, llr, 50)
    b = gpu_decode(code, llr, 50, flags=ldpc.COMPACT_TAIL)
    _same(a, b, "large code")
    late = [int(f) for f in np.argsort(-b["iters"])[:3]]
    print(compare(code, llr, 50, frames=late + [0], gpu=b))


def test_compact_tail_profiled_entry_point():
    """The profiled entry point takes the flag too and times every pass."""
    import torch
    from paper_1609_01567_amd import ldpc
    code = li.random_small_code(600, 300, 3, seed=8)
    llr = li.awgn_llr(code.n, 1000, li.ebn0_to_sigma2(1.8, code.rate), seed=33)
    g = ldpc.Graph.from_code(code)
    x = torch.from_numpy(llr).cuda()
    ref = gpu_decode(code, llr, 40, graph=g)
    res, tm = ldpc.decode_profiled(g, x, 40, flags=ldpc.COMPACT_TAIL)
    torch.cuda.synchronize()
    assert (res.iters.cpu().numpy() == ref["iters"]).all()
    assert (res.bits.cpu().numpy() == ref["bits"]).all()
    assert len(tm["check_ms"]) == 40 and (np.asarray(tm["check_ms"]) >= 0).all()


@pytest.mark.parametrize("msg,high", [("fp32", 300), ("fp32", 420), ("fp16", 420)])
def test_compact_tail_segmented_and_wide_rows(msg, high):
    """Rows beyond 512 edges (segmented path) and of 129..512 (16-wavefront
    path) in compacted decodes: 512 frames, `high` of them at 8 dB (they stop
    within 3 iterations) and the rest at 4 dB (most run all 30), so that the
    count after iteration 8 moves the running frames into the half-size copy
    (300) or straight into the quarter-size one (420)."""
    from paper_1609_01567_amd import ldpc
    from test_gpu_engine import _long_rows_code
    flags = {"fp32": 0, "fp16": ldpc.MSG_FP16}[msg]
    code = _long_rows_code()
    assert code.check_degrees().max() == 1200
    s8, s4 = li.ebn0_to_sigma2(8.0, code.rate), li.ebn0_to_sigma2(4.0, code.rate)
    llr = np.concatenate([li.awgn_llr(code.n, high, s8, seed=81), li.awgn_llr(code.n, 512 - high, s4, seed=82)])
    print(f"[case] compact long rows msg={msg} high={high} frames=512", flush=True)
    a = gpu_decode(code, llr, 30, flags=flags)
    b = gpu_decode(code, llr, 30, flags=flags | ldpc.COMPACT_TAIL)
    its = a["iters"]
    # frames still running after iteration 8 fit the intended copy, and some run on
    assert (its > 8).sum() <= (128 if high == 420 else 256) and (its > 12).sum() > 0
    _same(a, b, f"long rows {msg} {high}")


@pytest.mark.parametrize("T", [1, 8, 9, 12])
def test_compact_tail_short_runs(T):
    """Runs that end before, at and just after the first count (after iteration
    8): no count at all, and a move with a single iteration left before the
    results are copied back.  Half of the 512 frames stop within 3 iterations,
    so that count moves the others; posteriors are compared too."""
    from paper_1609_01567_amd import ldpc
    from test_gpu_engine import _long_rows_code
    code = _long_rows_code()
    s8, s4 = li.ebn0_to_sigma2(8.0, code.rate), li.ebn0_to_sigma2(4.0, code.rate)
    llr = np.concatenate([li.awgn_llr(code.n, 300, s8, seed=83), li.awgn_llr(code.n, 212, s4, seed=84)])
    print(f"[case] compact short runs T={T} frames=512", flush=True)
    a = gpu_decode(code, llr, T)
    b = gpu_decode(code, llr, T, flags=ldpc.COMPACT_TAIL)
    if T >= 9:
        assert (a["iters"] > 8).sum() <= 256 and (a["iters"] == T).sum() > 0
    _same(a, b, f"T={T}")
