"""ldpc_decode_noalloc: the decode with its state in the library's static device array.

Its outputs must equal those of ldpc_decode (same kernels, same plan) exactly,
call after call: the array keeps the previous call's contents, and a smaller
second call must not see any of them, also with tail compaction (whose
control words and copies live in the array too).  Sizes beyond the array are
refused before anything is enqueued.
"""
import numpy as np
import pytest

import ldpc_inputs as li

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1609_01567_amd import ldpc
    return torch, ldpc


def _classes_code():
    """Checks of degree 3..300: every row class, the segmented one included."""
    rng = np.random.default_rng(11)
    cdeg = np.concatenate([[300, 140, 64, 40, 33], rng.integers(3, 33, size=95)])
    E = int(cdeg.sum())
    n = 700
    bdeg = np.full(n, E // n)
    bdeg[: E - bdeg.sum()] += 1
    return li.socket_code(bdeg, cdeg, seed=12)


def _host(res):
    return {k: getattr(res, k).cpu().numpy() for k in ("bits", "ok", "iters", "llr")}


def _assert_same(a, b, what):
    for k in ("bits", "ok", "iters", "llr"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=f"{what}: {k}")


@pytest.mark.parametrize("name,flags_name", [("tiny", 0), ("classes", 0), ("classes", "MSG_FP16"),
                                             ("tiny", "NO_EARLY_STOP"), ("classes", "COMPACT_TAIL")])
def test_noalloc_equals_decode_on_consecutive_calls(lib, name, flags_name):
    torch, ldpc = lib
    flags = 0 if not flags_name else getattr(ldpc, flags_name)
    code = li.tiny_code() if name == "tiny" else _classes_code()
    g = ldpc.Graph.from_code(code)
    T = 30
    # first call the larger one, then a smaller one on the same array
    for frames, seed in ((300, 501), (37, 502)):
        print(f"[case] noalloc {name} flags={flags} frames={frames}", flush=True)
        llr = torch.from_numpy(li.awgn_llr(code.n, frames, li.ebn0_to_sigma2(1.5, code.rate), seed=seed)).cuda()
        ref = ldpc.decode(g, llr, T, flags=flags, want_llr=True)
        got = ldpc.decode_noalloc(g, llr, T, flags=flags, want_llr=True)
        torch.cuda.synchronize()
        r, o = _host(ref), _host(got)
        assert ((o["iters"] >= 1) & (o["iters"] <= T)).all()
        _assert_same(o, r, f"{name} frames={frames}")


def test_noalloc_with_preallocated_outputs_and_no_llr(lib):
    torch, ldpc = lib
    code = li.random_small_code(600, 300, 3, seed=8)
    g = ldpc.Graph.from_code(code)
    F = 200
    llr = torch.from_numpy(li.awgn_llr(code.n, F, li.ebn0_to_sigma2(1.2, code.rate), seed=9)).cuda()
    print("[case] noalloc preallocated outputs", flush=True)
    out = ldpc.DecodeResult(bits=torch.empty((F, code.n), dtype=torch.uint8, device="cuda"),
                            ok=torch.empty(F, dtype=torch.uint8, device="cuda"),
                            iters=torch.empty(F, dtype=torch.int32, device="cuda"), llr=None)
    got = ldpc.decode_noalloc(g, llr, 25, out=out)
    ref = ldpc.decode(g, llr, 25)
    torch.cuda.synchronize()
    assert got is out
    for k in ("bits", "ok", "iters"):
        assert torch.equal(getattr(got, k), getattr(ref, k)), k


def test_noalloc_refusals(lib):
    torch, ldpc = lib
    code = li.large_code()
    g = ldpc.Graph.from_code(code)
    # the n=64800 code's state is about 1.2 MB per frame slot in fp32: 512 slots are far beyond the array
    F = 512
    assert ldpc.workspace_size(g, F, 0) > ldpc.NOALLOC_SCRATCH_BYTES
    assert ldpc.workspace_size(g, 64, 0) <= ldpc.NOALLOC_SCRATCH_BYTES
    llr = torch.zeros((F, code.n), dtype=torch.float32, device="cuda")
    print("[case] noalloc refusals", flush=True)
    with pytest.raises(ldpc.LdpcError) as ei:
        ldpc.decode_noalloc(g, llr, 10)
    assert ei.value.status == ldpc.E_RANGE
    assert "static scratch" in str(ei.value)
    # frames = 0 is a no-op
    empty = ldpc.decode_noalloc(g, llr[:0].contiguous(), 10)
    torch.cuda.synchronize()
    assert empty.bits.shape == (0, code.n)
    # the largest size that fits still decodes, identically to ldpc_decode (all-zero LLRs: one iteration)
    small = llr[:64].contiguous()
    got = ldpc.decode_noalloc(g, small, 10, want_llr=True)
    ref = ldpc.decode(g, small, 10, want_llr=True)
    torch.cuda.synchronize()
    for k in ("bits", "ok", "iters", "llr"):
        assert torch.equal(getattr(got, k), getattr(ref, k)), k
    assert (got.iters == 1).all() and (got.ok == 1).all()
