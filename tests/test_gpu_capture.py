"""ldpc_decode under HIP graph capture.

The decode enqueues its kernels and returns, so a caller may capture it into a
graph and replay it.  Every replay, with other work and synchronizations
between replays, must give exactly the eager result.  Tail compaction takes
its decisions on the device, so a compacted decode captures and replays too,
and equals the plain decode.
"""
import numpy as np
import pytest

import ldpc_inputs as li

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1609_01567_amd import ldpc
    code = li.random_small_code(600, 300, 3, seed=8)
    llr = torch.from_numpy(li.awgn_llr(code.n, 300, li.ebn0_to_sigma2(1.5, code.rate), seed=61)).cuda()
    g = ldpc.Graph.from_code(code)
    return torch, ldpc, code, llr, g


def _alloc(torch, ldpc, F, n):
    return ldpc.DecodeResult(bits=torch.empty((F, n), dtype=torch.uint8, device="cuda"),
                             ok=torch.empty(F, dtype=torch.uint8, device="cuda"),
                             iters=torch.empty(F, dtype=torch.int32, device="cuda"),
                             llr=torch.empty((F, n), dtype=torch.float32, device="cuda"))


def test_captured_decode_replays_equal_eager(setup):
    torch, ldpc, code, llr, g = setup
    F, n, T = llr.shape[0], code.n, 30
    print("[case] capture: plain decode, 3 replays", flush=True)
    eager = ldpc.decode(g, llr, T, want_llr=True)
    torch.cuda.synchronize()
    ref = {k: getattr(eager, k).cpu().numpy() for k in ("bits", "ok", "iters", "llr")}
    ws = ldpc.Workspace(ldpc.workspace_size(g, F, 0))
    out = _alloc(torch, ldpc, F, n)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ldpc.decode(g, llr, T, want_llr=True, workspace=ws, out=out, stream=side)   # warm-up outside capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=side):
        ldpc.decode(g, llr, T, want_llr=True, workspace=ws, out=out, stream=side)
    for rep in range(3):
        for k in ("bits", "ok", "iters", "llr"):
            getattr(out, k).zero_()                  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k in ("bits", "ok", "iters", "llr"):
            assert np.array_equal(getattr(out, k).cpu().numpy(), ref[k]), (rep, k)
    assert (ref["iters"] > 1).any()


@pytest.mark.parametrize("msg", ["fp32", "fp16"])
def test_captured_compact_tail_replays_equal_plain(setup, msg):
    """A decode with LDPC_COMPACT_TAIL (300 frames in 512 slots: copies of 256
    and 128 slots) captured into a graph: every replay equals the eager decode
    without compaction, posteriors included (with FP16 messages the fp32
    posterior output moves between the copies too)."""
    torch, ldpc, code, _, g = setup
    llr = torch.from_numpy(li.awgn_llr(code.n, 300, li.ebn0_to_sigma2(1.8, code.rate), seed=36)).cuda()
    F, n, T = llr.shape[0], code.n, 40
    flags = ldpc.MSG_FP16 if msg == "fp16" else 0
    print(f"[case] capture: LDPC_COMPACT_TAIL {msg}, 3 replays", flush=True)
    plain = ldpc.decode(g, llr, T, flags=flags, want_llr=True)
    torch.cuda.synchronize()
    ref = {k: getattr(plain, k).cpu().numpy() for k in ("bits", "ok", "iters", "llr")}
    # a tail that the counts after iterations 8, 12, ... reach: at most 256
    # running frames (the first copy) by iteration 16, some still running at 20
    assert (ref["iters"] <= 16).sum() >= 44 and (ref["iters"] > 20).any()
    cflags = flags | ldpc.COMPACT_TAIL
    ws = ldpc.Workspace(ldpc.workspace_size(g, F, cflags))
    out = _alloc(torch, ldpc, F, n)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ldpc.decode(g, llr, T, flags=cflags, want_llr=True, workspace=ws, out=out, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for k in ("bits", "ok", "iters", "llr"):
        assert np.array_equal(getattr(out, k).cpu().numpy(), ref[k]), ("eager", k)
    with torch.cuda.graph(graph, stream=side):
        ldpc.decode(g, llr, T, flags=cflags, want_llr=True, workspace=ws, out=out, stream=side)
    for rep in range(3):
        for k in ("bits", "ok", "iters", "llr"):
            getattr(out, k).zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k in ("bits", "ok", "iters", "llr"):
            assert np.array_equal(getattr(out, k).cpu().numpy(), ref[k]), (rep, k)
