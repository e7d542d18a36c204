"""GPU parity on every frame of the throughput workload, decoded the way the
benchmark times it.

The workload is the rate-1/2 n = 64800 code with 256 random codewords at each
of 0.8 / 1.0 / 1.2 / 1.4 dB, at most 50 iterations with syndrome early stop,
FP32 messages.  The decode configuration (frames per call, flags, lane width,
one workspace shared by the calls) is the one `bench.py` times, taken from
`paper_1609_01567_amd.workloads`.  Every frame of every point is compared with
the FP64 oracle; at 1.0 dB every frame is also compared after 1, 2, 5 and 10
iterations with early stop off, posteriors included.
"""
import numpy as np
import pytest

import ldpc_inputs as li
from parity import compare

pytestmark = pytest.mark.gpu

T = 50


@pytest.fixture(scope="module")
def headline():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1609_01567_amd import ldpc, workloads
    code, cws, llrs = li.headline_workload()
    g = ldpc.Graph.from_code(code)
    print(f"[case] headline decode: {len(llrs)} points x {llrs[0].shape[0]} frames", flush=True)
    runs = workloads.headline_decode(g, [torch.from_numpy(x).cuda() for x in llrs], T, want_llr=True)
    torch.cuda.synchronize()
    results = [dict(bits=r.bits.cpu().numpy(), ok=r.ok.cpu().numpy(), iters=r.iters.cpu().numpy(),
                    lpost=r.llr.cpu().numpy()) for r in runs]
    return code, cws, llrs, g, results


@pytest.mark.parametrize("point", range(len(li.HEADLINE_POINTS_DB)))
def test_headline_every_frame_equals_oracle(headline, point):
    code, cws, llrs, _, results = headline
    eb = li.HEADLINE_POINTS_DB[point]
    gpu = results[point]
    print(f"[case] headline {eb} dB: oracle on all {llrs[point].shape[0]} frames", flush=True)
    # properties that need no oracle
    syn = code.syndrome(gpu["bits"]).any(axis=1)
    assert (syn == (gpu["ok"] == 0)).all()
    assert ((gpu["lpost"] < 0) == gpu["bits"].astype(bool)).all()
    assert ((gpu["iters"] >= 1) & (gpu["iters"] <= T)).all()
    st = compare(code, llrs[point], T, gpu=gpu)
    print(eb, st)
    # the comparison covers nearly every frame (tie-risk frames are counted, not hidden)
    assert st["clear"] >= 0.95 * st["frames"]


@pytest.mark.parametrize("fixed_t", [1, 2, 5, 10])
def test_headline_fixed_iterations_every_frame(headline, fixed_t):
    from paper_1609_01567_amd import workloads
    import torch
    code, _, llrs, g, _ = headline
    x = llrs[1]                                      # 1.0 dB
    print(f"[case] headline 1.0 dB fixed T={fixed_t}: all {x.shape[0]} frames", flush=True)
    gpu = workloads.headline_decode(g, [torch.from_numpy(x).cuda()], fixed_t, want_llr=True, early_stop=False)[0]
    torch.cuda.synchronize()
    gpu = dict(bits=gpu.bits.cpu().numpy(), ok=gpu.ok.cpu().numpy(), iters=gpu.iters.cpu().numpy(),
               lpost=gpu.llr.cpu().numpy())
    st = compare(code, x, fixed_t, early_stop=False, gpu=gpu, posterior_all=True)
    print(fixed_t, st)
    assert st["posterior_checked"] >= 0.95 * st["frames"]
