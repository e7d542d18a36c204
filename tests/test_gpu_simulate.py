"""GPU tests of the Monte-Carlo runs (ldpc_simulate): channel noise drawn on the
device, decode, error counting.

* The device's channel LLRs equal the host's counter-based draw
  (ldpc_inputs.counter_noise, pinned by the generator's known-answer vectors)
  to float32 rounding of the transcendentals.
* The counts equal those of ldpc_decode run on the same LLRs (the decode is the
  same kernels; ldpc_decode itself is held to the FP64 oracle elsewhere), and
  the oracle agrees on tie-free frames.
* A run split over calls (first_frame) or repeated gives the same totals.
"""
import numpy as np
import pytest

import ldpc_inputs as li
import oracle
from ldpc_inputs.counter_noise import sim_channel_llr
from parity import gpu_decode

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")


def _run(code, frames, ebn0, seed, T, first_frame=0, flags=0, want_llr=True):
    import torch
    from paper_1609_01567_amd import ldpc
    g = ldpc.Graph.from_code(code)
    counts, llr = ldpc.simulate(g, frames, ebn0, seed, T, flags=flags, first_frame=first_frame, want_llr=want_llr)
    torch.cuda.synchronize()
    return ldpc.sim_counts(counts), (llr.cpu().numpy() if llr is not None else None)


def _counts_from(out, T):
    err = out["bits"].astype(np.int64).sum(axis=1)
    return dict(frames=int(err.size), frame_errors=int((err > 0).sum()), bit_errors=int(err.sum()),
                undetected=int(((err > 0) & (out["ok"] == 1)).sum()), iterations=int(out["iters"].sum()))


@pytest.mark.parametrize("which", ["tiny", "large"])
def test_device_channel_equals_host_draw(which):
    code = li.tiny_code() if which == "tiny" else li.large_code()
    frames = 40 if which == "tiny" else 6
    seed = 0x1234_5678_9ABC
    first = 2 ** 32 - 3          # the frame index crosses into the counter's high word
    print(f"[case] channel {which} frames={frames}", flush=True)
    _, llr = _run(code, frames, 1.0, seed, 2, first_frame=first)
    host = sim_channel_llr(code.n, code.m, frames, 1.0, seed, first_frame=first)
    # float32 log/sqrt/sincospi on the device against float64 on the host: a
    # few units in the last place of k1 z, i.e. ~1e-6 of the noise magnitude
    err = np.abs(llr.astype(np.float64) - host)
    assert (err <= 5e-6 * (1.0 + np.abs(host))).all(), f"max {err.max():.3e}"
    assert err.max() > 0 or frames * code.n < 100   # the device computed its own draw


def test_counts_equal_decode_of_the_same_llrs_and_oracle():
    code = li.tiny_code()
    T = 50
    print("[case] counts tiny 1.2 dB", flush=True)
    counts, llr = _run(code, 300, 1.2, seed=77, T=T)
    out = gpu_decode(code, llr, T)
    assert counts == _counts_from(out, T)
    assert counts["frame_errors"] > 0 and counts["frames"] == 300
    # the oracle on the same inputs: tie-free frames decide identically
    ora = oracle.decode(code, llr[:64], T)
    clear = ora["tie_risk"] == 0
    assert clear.sum() > 50
    assert (ora["bits"][clear] == out["bits"][:64][clear]).all()
    assert (ora["iters"][clear] == out["iters"][:64][clear]).all()


@pytest.mark.parametrize("flags_name", ["fp16", "no_early_stop", "compact_tail"])
def test_counts_equal_decode_under_flags(flags_name):
    from paper_1609_01567_amd import ldpc
    flags = {"fp16": ldpc.MSG_FP16, "no_early_stop": ldpc.NO_EARLY_STOP,
             "compact_tail": ldpc.COMPACT_TAIL}[flags_name]
    code = li.random_small_code(600, 300, 3, seed=8)
    print(f"[case] counts flags={flags_name}", flush=True)
    counts, llr = _run(code, 257, 1.4, seed=5, T=30, flags=flags)
    out = gpu_decode(code, llr, 30, flags=flags)
    assert counts == _counts_from(out, 30)


def test_split_and_repeated_runs_agree():
    import torch
    from paper_1609_01567_amd import ldpc
    code = li.random_small_code(600, 300, 3, seed=8)
    g = ldpc.Graph.from_code(code)
    print("[case] split runs", flush=True)
    whole, _ = ldpc.simulate(g, 500, 1.3, 99, 40)
    parts, _ = ldpc.simulate(g, 300, 1.3, 99, 40)
    ldpc.simulate(g, 200, 1.3, 99, 40, first_frame=300, counts=parts)
    again, _ = ldpc.simulate(g, 500, 1.3, 99, 40)
    torch.cuda.synchronize()
    a, b, c = ldpc.sim_counts(whole), ldpc.sim_counts(parts), ldpc.sim_counts(again)
    assert a == b == c
    other, _ = ldpc.simulate(g, 500, 1.3, 100, 40)
    assert ldpc.sim_counts(other) != a


def test_error_free_at_high_snr_and_argument_checks():
    import torch
    from paper_1609_01567_amd import ldpc
    code = li.tiny_code()
    print("[case] high snr", flush=True)
    counts, _ = _run(code, 128, 8.0, seed=1, T=20, want_llr=False)
    assert counts["frames"] == 128 and counts["frame_errors"] == 0 and counts["bit_errors"] == 0
    # a frame with no channel bit error stops after one iteration; a few still have one
    assert 128 <= counts["iterations"] < 128 * 3
    g = ldpc.Graph.from_code(code)
    with pytest.raises(ldpc.LdpcError):
        ldpc.simulate(g, 10, float("nan"), 1, 10)
    with pytest.raises(ldpc.LdpcError):
        ldpc.simulate(g, 10, 1.0, 1, 0)
    torch.cuda.synchronize()
