"""GPU parity: the HIP decoder (through the C ABI) against the FP64 oracle.

Cases span several tiles and ragged tails (frame counts not a multiple of the
64-lane slot groups, codes whose n is not a multiple of 64), every check-degree
class (register rows up to 8/16/32 edges and the segmented path for longer
rows), the degenerate cases (degree-1 checks, empty rows/columns, all-zero and
noiseless inputs) and the full-size rate-1/2 n=64800 code on sampled frames.
"""
import numpy as np
import pytest

import ldpc_inputs as li
import oracle
from parity import compare, gpu_decode

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1609_01567_amd import ldpc
    ldpc.load_library()


def _announce(name, **kw):
    print(f"[case] {name} {kw}", flush=True)


# ------------------------------------------------------------------ small

def test_noiseless_codewords_14_7_one_iteration():
    import itertools
    code = li.code_14_7()
    words = np.array(list(itertools.product([0, 1], repeat=14)), np.uint8)
    cw = words[code.syndrome(words).sum(1) == 0]
    llr = (2.0 * (1.0 - 2.0 * cw) / 0.5).astype(np.float32)
    _announce("noiseless-14-7", frames=len(cw))
    out = gpu_decode(code, llr, 50)
    assert (out["iters"] == 1).all() and (out["ok"] == 1).all()
    assert (out["bits"] == cw).all()
    compare(code, llr, 50)


def test_all_zero_llr():
    code = li.tiny_code()
    llr = np.zeros((5, code.n), np.float32)
    _announce("all-zero-llr", frames=5)
    out = gpu_decode(code, llr, 10)
    assert (out["lpost"] == 0).all() and out["bits"].sum() == 0
    assert (out["ok"] == 1).all() and (out["iters"] == 1).all()


def test_tiny_code_early_stop():
    code = li.tiny_code()
    llr = li.awgn_llr(code.n, 32, li.ebn0_to_sigma2(2.0, code.rate), seed=2001)
    _announce("tiny-2dB", frames=32)
    st = compare(code, llr, 50)
    print(st)


@pytest.mark.parametrize("T", [1, 2, 5, 10])
def test_tiny_code_fixed_iterations_every_frame(T):
    code = li.tiny_code()
    llr = li.awgn_llr(code.n, 32, li.ebn0_to_sigma2(2.0, code.rate), seed=2001)
    _announce("tiny-fixed", T=T)
    compare(code, llr, T, early_stop=False, require_all=(T <= 2), posterior_all=True)


@pytest.mark.parametrize("frames", [1, 63, 65, 130, 200, 257])
def test_ragged_frame_counts(frames):
    code = li.random_small_code(300, 150, 3, seed=31)
    llr = li.awgn_llr(code.n, frames, li.ebn0_to_sigma2(1.5, code.rate), seed=40 + frames)
    _announce("ragged", frames=frames, n=code.n)
    print(compare(code, llr, 30))


def test_low_snr_many_iterations():
    code = li.random_small_code(500, 250, 3, seed=5)
    llr = li.awgn_llr(code.n, 96, li.ebn0_to_sigma2(0.5, code.rate), seed=6)
    _announce("low-snr", frames=96)
    st = compare(code, llr, 40)
    print(st)


def test_degree_classes_and_segmented_rows():
    """Checks of degree 3..300 in one code: every kernel class is used."""
    rng = np.random.default_rng(11)
    cdeg = np.concatenate([[300, 140, 64, 40, 33], rng.integers(3, 33, size=95)])
    E = int(cdeg.sum())
    n = 700
    bdeg = np.full(n, E // n)
    bdeg[: E - bdeg.sum()] += 1
    code = li.socket_code(bdeg, cdeg, seed=12)
    assert code.check_degrees().max() == 300
    llr = li.awgn_llr(n, 70, 0.7, seed=13)
    _announce("classes", frames=70, max_deg=300)
    print(compare(code, llr, 25))
    compare(code, llr, 3, early_stop=False, posterior_all=True)


def test_long_rows_wide_and_segmented_paths():
    """Rows just inside and just beyond the LDS path's 512-edge limit, and far
    beyond it (segmented path), with iterations fixed and with early stop."""
    rng = np.random.default_rng(31)
    cdeg = np.concatenate([[1200, 700, 513, 512, 300, 129], rng.integers(3, 12, size=200)])
    E = int(cdeg.sum())
    n = 1500
    bdeg = np.full(n, E // n)
    bdeg[: E - bdeg.sum()] += 1
    code = li.socket_code(bdeg, cdeg, seed=32)
    assert sorted(code.check_degrees())[-4:] == [512, 513, 700, 1200]
    llr = li.awgn_llr(n, 70, li.ebn0_to_sigma2(6.0, code.rate), seed=33)
    _announce("long-rows", frames=70, max_deg=1200)
    compare(code, llr, 4, early_stop=False, posterior_all=True)
    print(compare(code, llr, 20))


def test_degree_classes_converging_frames():
    """Rows of every register and chunk class (degrees 3..64) on frames that
    converge at different iterations, so the syndrome fold of each class
    decides when a frame stops."""
    rng = np.random.default_rng(21)
    cdeg = np.concatenate([[64, 48, 33, 20, 17], rng.integers(3, 17, size=115)])
    E = int(cdeg.sum())
    n = 2 * len(cdeg) + 400
    bdeg = np.full(n, E // n)
    bdeg[: E - bdeg.sum()] += 1
    code = li.socket_code(bdeg, cdeg, seed=22)
    sigma2 = li.ebn0_to_sigma2(3.5, code.rate)
    llr = li.awgn_llr(n, 130, sigma2, seed=23)
    _announce("classes-converging", frames=130, max_deg=64)
    st = compare(code, llr, 30)
    print(st)
    ora = oracle.decode(code, llr, 30)
    assert (ora["ok"] == 1).sum() >= 20, "too few converging frames to exercise early stopping"
    assert len(np.unique(ora["iters"][ora["ok"] == 1])) >= 3


def test_degree_one_checks_and_empty_nodes():
    # check 0 = {0}; check 1 = {0,1,2}; check 2 empty; check 3 = {2,3}; bit 4 unconnected
    code = li.Code(m=4, n=5, rows=np.array([0, 1, 1, 1, 3, 3], np.int32),
                   cols=np.array([0, 0, 1, 2, 2, 3], np.int32))
    rng = np.random.default_rng(2)
    llr = rng.normal(0.5, 2.0, size=(20, 5)).astype(np.float32)
    _announce("degenerate", frames=20)
    out = gpu_decode(code, llr, 6)
    np.testing.assert_array_equal(out["lpost"][:, 4], llr[:, 4])
    compare(code, llr, 6)
    compare(code, llr, 4, early_stop=False, posterior_all=True)


def test_extreme_code_sampled():
    code = li.extreme_code()
    llr = li.awgn_llr(code.n, 128, li.ebn0_to_sigma2(1.5, code.rate), seed=2003)
    _announce("extreme", frames=128)
    gpu = gpu_decode(code, llr, 100)
    syn = code.syndrome(gpu["bits"]).any(axis=1)
    assert (syn == (gpu["ok"] == 0)).all()
    st = compare(code, llr, 100, frames=[0, 1, 63, 64, 127], gpu=gpu)
    print(st)


def test_determinism_and_sign_symmetry():
    import itertools
    code = li.code_14_7()
    words = np.array(list(itertools.product([0, 1], repeat=14)), np.uint8)
    cw = words[code.syndrome(words).sum(1) == 0]
    base = li.awgn_llr(14, 1, 0.8, seed=3)
    flip = (1.0 - 2.0 * cw).astype(np.float32)
    llr = base * flip
    _announce("symmetry", frames=len(cw))
    a = gpu_decode(code, llr, 20)
    b = gpu_decode(code, llr, 20)
    for k in a:
        assert (a[k] == b[k]).all()
    assert (a["iters"] == a["iters"][0]).all()
    assert (a["lpost"] == a["lpost"][0] * flip).all()
    assert (a["bits"] == (a["bits"][0] ^ cw)).all()


# ------------------------------------------------------------- full size

def test_large_code_full_batch_sampled_frames():
    code = li.large_code()
    frames = 256
    cw = li.Encoder(code).random_codewords(frames, seed=3002)
    llr = li.awgn_llr(code.n, frames, li.ebn0_to_sigma2(1.0, code.rate), seed=2012, codewords=cw)
    _announce("large-1.0dB", frames=frames)
    gpu = gpu_decode(code, llr, 50)
    # properties on every frame
    assert ((gpu["iters"] >= 1) & (gpu["iters"] <= 50)).all()
    syn = code.syndrome(gpu["bits"]).any(axis=1)
    assert (syn == (gpu["ok"] == 0)).all()
    assert ((gpu["lpost"] < 0) == gpu["bits"].astype(bool)).all()
    assert (gpu["bits"][gpu["ok"] == 1] == cw[gpu["ok"] == 1]).mean() > 0.999
    # oracle on sampled frames: first, last and across slot groups
    st = compare(code, llr, 50, frames=[0, 1, 127, 128, 200, 255], gpu=gpu)
    print(st)


def test_tile_shapes_give_identical_results():
    """The slots-per-lane tile shape changes the memory access width only."""
    from paper_1609_01567_amd import ldpc
    code = li.random_small_code(600, 300, 3, seed=8)
    llr = li.awgn_llr(code.n, 300, li.ebn0_to_sigma2(1.2, code.rate), seed=9)
    _announce("tile-shapes", frames=300)
    ref = gpu_decode(code, llr, 30, flags=ldpc.LANE_SLOTS_1)
    for fl in (ldpc.LANE_SLOTS_2, ldpc.LANE_SLOTS_4, 0):
        out = gpu_decode(code, llr, 30, flags=fl)
        for k in ref:
            assert (out[k] == ref[k]).all(), (fl, k)
    compare(code, llr, 30, gpu=ref)
