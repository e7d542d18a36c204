"""GPU tests of reduced-precision message storage (FP16 / BF16 storage, FP32 arithmetic).

Iteration 1 has a provable bound.  The check message R(c->v) combines the
clamped channel LLRs of the other bits of c, and the magnitude of the exact
check combination never exceeds the smallest magnitude among its inputs.  So
|R(c->v)| <= min(64, min over v' in N(c)\\{v} of |Lch(v')|).  Storing R rounds it once
to the nearest value of the storage format (relative error at most u = 2^-11
for FP16, 2^-8 for BF16).  With 16-bit messages the check pass also reads the
channel LLRs from their FP16 copy (relative error at most 2^-11 each), and the
check combination changes by at most the sum of its inputs' changes (each
two-input step a (+) b has |d(a (+) b)/da| <= 1).  The posterior sums the
stored messages in FP32.  Against the FP64 oracle, the posterior after one
iteration therefore stays within the FP32 parity bar plus, over the checks of
v, u times the smallest other input plus 2^-11 times the sum of the other
(clamped) inputs.
Later iterations have no such closed bound; the decodes must still be
self-consistent (flags agree with the syndrome of the returned bits) and
independent of the tile shape.
"""
import numpy as np
import pytest

import ldpc_inputs as li
import oracle
from parity import ATOL, RTOL, first_iteration_bound, first_iteration_input_bound, gpu_decode

pytestmark = pytest.mark.gpu

UNIT_ROUNDOFF = {"fp16": 2.0 ** -11, "bf16": 2.0 ** -8}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")


def _flag(name):
    from paper_1609_01567_amd import ldpc
    return {"fp16": ldpc.MSG_FP16, "bf16": ldpc.MSG_BF16}[name]


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("which", ["tiny", "classes"])
def test_first_iteration_within_rounding_bound(prec, which):
    from paper_1609_01567_amd import ldpc
    if which == "tiny":
        code = li.tiny_code()
        llr = li.awgn_llr(code.n, 70, li.ebn0_to_sigma2(2.0, code.rate), seed=71)
    else:
        rng = np.random.default_rng(11)
        cdeg = np.concatenate([[300, 140, 64, 40, 33], rng.integers(3, 33, size=95)])
        E = int(cdeg.sum())
        bdeg = np.full(700, E // 700)
        bdeg[: E - bdeg.sum()] += 1
        code = li.socket_code(bdeg, cdeg, seed=12)
        llr = li.awgn_llr(code.n, 70, 0.7, seed=72)
    print(f"[case] first-iteration bound {prec} {which} n={code.n}", flush=True)
    gpu = gpu_decode(code, llr, 1, flags=_flag(prec) | ldpc.NO_EARLY_STOP)
    ora = oracle.decode(code, llr, 1, early_stop=False)
    bound = (ATOL + RTOL * np.abs(ora["lpost"]) + UNIT_ROUNDOFF[prec] * first_iteration_bound(code, llr)
             + 2.0 ** -11 * first_iteration_input_bound(code, llr))
    err = np.abs(gpu["lpost"].astype(np.float64) - ora["lpost"])
    assert (err <= bound).all(), f"max excess {(err - bound).max():.3e}"
    # the messages really are stored rounded: FP32 storage stays below 1e-5 here
    assert err.max() > 1e-4


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_first_iteration_long_rows_against_rounded_inputs(prec):
    """Rows of 129..512 edges (LDS path) and of 513..1200 (segmented path).
    The check pass of iteration 1 reads the channel LLRs from their FP16 copy,
    so the FP64 oracle is given those rounded values: the message sums
    Lpost - Lch of both then differ only by the storage rounding of each
    message (at most u times the smallest other input of its check) and the
    FP32 bar.  (The input-change term of the general bound grows with the row
    length and would hide a wrong message scale on these rows.)"""
    from paper_1609_01567_amd import ldpc
    rng = np.random.default_rng(31)
    cdeg = np.concatenate([[1200, 700, 513, 512, 300, 129], rng.integers(3, 12, size=200)])
    E = int(cdeg.sum())
    bdeg = np.full(1500, E // 1500)
    bdeg[: E - bdeg.sum()] += 1
    code = li.socket_code(bdeg, cdeg, seed=32)
    llr = li.awgn_llr(code.n, 70, li.ebn0_to_sigma2(6.0, code.rate), seed=73)
    llr16 = llr.astype(np.float16).astype(np.float64)
    print(f"[case] long rows first iteration {prec}", flush=True)
    gpu = gpu_decode(code, llr, 1, flags=_flag(prec) | ldpc.NO_EARLY_STOP)
    ora = oracle.decode(code, llr16, 1, early_stop=False)
    sum_gpu = gpu["lpost"].astype(np.float64) - llr.astype(np.float64)
    sum_ora = ora["lpost"] - llr16
    bound = ATOL + RTOL * np.abs(ora["lpost"]) + UNIT_ROUNDOFF[prec] * first_iteration_bound(code, llr16)
    err = np.abs(sum_gpu - sum_ora)
    assert (err <= bound).all(), f"max excess {(err - bound).max():.3e}"
    assert err.max() > 1e-4


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_reduced_precision_decodes_are_consistent(prec):
    code = li.extreme_code()
    llr = li.awgn_llr(code.n, 200, li.ebn0_to_sigma2(5.0, code.rate), seed=2013)
    print(f"[case] consistency {prec} extreme 5.0 dB", flush=True)
    out = gpu_decode(code, llr, 100, flags=_flag(prec))
    syn = code.syndrome(out["bits"]).any(axis=1)
    assert (syn == (out["ok"] == 0)).all()
    assert ((out["lpost"] < 0) == out["bits"].astype(bool)).all()
    assert ((out["iters"] >= 1) & (out["iters"] <= 100)).all()
    assert (out["iters"][out["ok"] == 0] == 100).all()
    assert (out["ok"] == 1).mean() > 0.2        # the waterfall region of this code


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_reduced_precision_tile_shapes_identical(prec):
    from paper_1609_01567_amd import ldpc
    code = li.random_small_code(600, 300, 3, seed=8)
    llr = li.awgn_llr(code.n, 300, li.ebn0_to_sigma2(1.2, code.rate), seed=9)
    print(f"[case] tile shapes {prec}", flush=True)
    ref = gpu_decode(code, llr, 30, flags=_flag(prec) | ldpc.LANE_SLOTS_1)
    for fl in (ldpc.LANE_SLOTS_2, ldpc.LANE_SLOTS_4):
        out = gpu_decode(code, llr, 30, flags=_flag(prec) | fl)
        for k in ref:
            assert (out[k] == ref[k]).all(), (fl, k)
