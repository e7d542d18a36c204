"""ldpc_decode under HIP graph capture.

The decode enqueues its kernels and returns, so a caller may capture it into a
graph and replay it.  Every replay, with other work and synchronizations
between replays, must give exactly the eager result.  Tail compaction waits on
the host for its counts, so a call with LDPC_COMPACT_TAIL on a capturing
stream is refused with LDPC_E_INVAL before anything is enqueued.
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


def test_compact_tail_refused_on_capturing_stream(setup):
    torch, ldpc, code, llr, g = setup
    F, n = llr.shape[0], code.n
    print("[case] capture: LDPC_COMPACT_TAIL refused", flush=True)
    ws = ldpc.Workspace(ldpc.workspace_size(g, F, ldpc.COMPACT_TAIL))
    out = _alloc(torch, ldpc, F, n)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    err = None
    with torch.cuda.graph(graph, stream=side):
        try:
            ldpc.decode(g, llr, 30, flags=ldpc.COMPACT_TAIL, workspace=ws, out=out, stream=side)
        except ldpc.LdpcError as e:
            err = e
        # something to capture, so the graph is not empty
        out.ok.zero_()
    assert err is not None and err.status == ldpc.E_INVAL
    assert "capturing" in str(err)
    # the same call outside capture still runs
    res = ldpc.decode(g, llr, 30, flags=ldpc.COMPACT_TAIL, workspace=ws, out=out)
    torch.cuda.synchronize()
    assert (res.iters.cpu().numpy() >= 1).all()
