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
