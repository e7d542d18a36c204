"""GPU parity on the quasi-cyclic stand-in (the headline degree profile lifted by
Z = 360): sampled frames of a full 256-frame call against the oracle, and
properties on every frame."""
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
