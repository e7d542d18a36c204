"""GPU parity at the large ends of the size range: a code of 2^20 bits
(3.1 M edges) and 65 499 frames of one code in a single call (a slot count
that is not a multiple of 64).  Index arithmetic past 2^31 bytes of messages
and many slot groups are exercised; the oracle checks sampled frames and
properties are checked on every frame."""
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


def _properties(code, out, T):
    assert ((out["iters"] >= 1) & (out["iters"] <= T)).all()
    assert ((out["lpost"] < 0) == out["bits"].astype(bool)).all()
    syn = code.syndrome(out["bits"]).any(axis=1)
    assert (syn == (out["ok"] == 0)).all()


def test_million_bit_code_sampled_frames():
    code = li.random_small_code(1 << 20, 1 << 19, 3, seed=5)
    llr = li.awgn_llr(code.n, 64, li.ebn0_to_sigma2(2.5, code.rate), seed=6)
    print(f"[case] n={code.n} E={code.nnz} frames=64", flush=True)
    out = gpu_decode(code, llr, 20)
    _properties(code, out, 20)
    assert (out["ok"] == 1).mean() > 0.9
    print(compare(code, llr, 20, frames=[0, 31, 63], gpu=out))


def test_many_frames_in_one_call():
    code = li.tiny_code()
    F = 65499
    llr = li.awgn_llr(code.n, F, li.ebn0_to_sigma2(2.0, code.rate), seed=7)
    print(f"[case] n={code.n} frames={F}", flush=True)
    out = gpu_decode(code, llr, 30)
    _properties(code, out, 30)
    # messages of this call: E x S x 4 bytes = 0.94 GB; every slot group up to the ragged last one
    print(compare(code, llr, 30, frames=[0, 1, 63, 64, 32767, 65471, 65472, F - 1], gpu=out))


def test_batched_mix_full_size_engine_equals_plain():
    """The batched workload at full size (eight codes, 4096 frames) through the
    engine in the shape the autotuner picks for it (4 slots per lane, 4 steps
    per replay, 2 iterations per step, the tuned pools), FP16 messages: every
    frame is bit-identical to a plain FP16 decode of its code.  The plain FP32
    decode of every code is held to the oracle on its first and last frames."""
    import torch
    from paper_1609_01567_amd import ldpc, workloads
    mix = workloads.batched_mix()
    T = 50
    print(f"[case] batched mix, {sum(F for _, F, *_ in mix)} frames", flush=True)
    graphs = [ldpc.Graph.from_code(c) for c, *_ in mix]
    eng = ldpc.Engine(graphs, [1507, 754, 502, 377, 302, 256, 256, 256], [F for _, F, *_ in mix], T,
                      flags=ldpc.MSG_FP16, lane_slots=4, graph_steps=4, iters_per_step=2)
    jobs = [(i, torch.from_numpy(np.ascontiguousarray(x)).cuda()) for i, (*_, x) in enumerate(mix)]
    res = ldpc.decode_batch(eng, jobs, want_llr=True, max_replays=200)
    torch.cuda.synchronize()
    eng.close()
    for (code, F, eb, cw, llr), g, r in zip(mix, graphs, res):
        plain = gpu_decode(code, llr, T, flags=ldpc.MSG_FP16, graph=g)
        for k, v in (("bits", r.bits), ("ok", r.ok), ("iters", r.iters), ("lpost", r.llr)):
            assert (v.cpu().numpy() == plain[k]).all(), f"{code.name}: engine {k} differs from plain"
        p32 = gpu_decode(code, llr, T, graph=g)
        _properties(code, p32, T)
        print(code.name, compare(code, llr, T, frames=[0, F - 1], gpu=p32), flush=True)
