"""Host-side pins of the counter-based channel noise used by Monte-Carlo runs.

The generator is fixed by its published definition: its known-answer vectors
(tests/golden/philox4x32_10_kat.txt) pin every round of the host implementation;
the Box-Muller output and the channel LLRs are pinned by their distribution and
by the counter layout (a frame's noise depends only on its global index).
"""
import os

import numpy as np

import ldpc_inputs as li
from ldpc_inputs.counter_noise import frame_normals, philox4x32_10, sim_channel_llr, unit_open

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        ctr = [int(x, 16) for x in r[0:4]]
        key = [int(x, 16) for x in r[4:6]]
        want = [int(x, 16) for x in r[6:10]]
        assert philox4x32_10(ctr, key).tolist() == want


def test_philox_vectorised_equals_single_calls():
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 2 ** 32, size=(7, 4), dtype=np.uint64)
    key = rng.integers(0, 2 ** 32, size=2, dtype=np.uint64)
    batch = philox4x32_10(ctr, key)
    for i in range(7):
        assert (batch[i] == philox4x32_10(ctr[i], key)).all()


def test_uniforms_open_interval_and_exact_in_float32():
    x = np.array([0, 1, 511, 512, 2 ** 31, 2 ** 32 - 1], dtype=np.uint32)
    u = unit_open(x)
    assert (u > 0).all() and (u < 1).all()
    assert (u.astype(np.float32).astype(np.float64) == u).all()
    assert u[0] == 0.5 * 2.0 ** -23 and u[-1] == 1.0 - 0.5 * 2.0 ** -23


def test_normals_moments_and_independence_of_frames():
    z = frame_normals(4001, 64, seed=11)
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1.0) < 0.01
    assert abs(np.mean(z ** 3)) < 0.03 and abs(np.mean(z ** 4) - 3.0) < 0.05
    # a frame's noise depends only on its global index: shifted windows agree
    w = frame_normals(4001, 16, seed=11, first_frame=40)
    assert (w == z[40:56]).all()
    # distinct seeds and the high word of the frame index matter
    assert not np.allclose(frame_normals(64, 2, seed=12), frame_normals(64, 2, seed=11))
    assert not np.allclose(frame_normals(64, 2, seed=11, first_frame=2 ** 32),
                           frame_normals(64, 2, seed=11, first_frame=0))


def test_channel_llr_statistics_match_awgn():
    code = li.tiny_code()
    ebn0 = 2.0
    llr = sim_channel_llr(code.n, code.m, 512, ebn0, seed=3).astype(np.float64)
    sigma2 = li.ebn0_to_sigma2(ebn0, (code.n - code.m) / code.n)
    # L = 2/sigma^2 + (2/sigma) z: mean 2/sigma^2, variance 4/sigma^2 (the consistency of LLRs)
    assert abs(llr.mean() / (2 / sigma2) - 1) < 0.01
    assert abs(llr.var() / (4 / sigma2) - 1) < 0.02
