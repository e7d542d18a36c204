"""CPU checks of the seeded input generators (codes, encoder, channel)."""
import itertools

import numpy as np
import pytest

import ldpc_inputs as li


def test_code_profiles():
    c = li.tiny_code()
    assert (c.m, c.n, c.nnz) == (512, 1024, 3585)
    assert sorted(set(c.check_degrees().tolist())) == [7, 8]
    assert np.bincount(c.bit_degrees()).nonzero()[0].tolist() == [2, 3, 8]
    c = li.large_code()
    assert (c.m, c.n, c.nnz) == (32400, 64800, 226800)
    assert set(c.check_degrees().tolist()) == {7}
    bd = c.bit_degrees()
    assert ((bd == 8).sum(), (bd == 3).sum(), (bd == 2).sum()) == (12960, 19440, 32400)
    c = li.extreme_code()
    cd, bd = c.check_degrees(), c.bit_degrees()
    assert cd.min() >= 4 and cd.max() <= 512 and (cd > 256).sum() == 8
    assert bd.min() >= 2 and bd.max() <= 64
    for code, (n, m) in zip(li.batch_codes(), li.BATCH_SPECS):
        assert (code.n, code.m) == (n, m)
    assert li.batch_frame_split().tolist() == [1507, 754, 502, 377, 302, 251, 215, 188]


@pytest.mark.parametrize("maker", [li.tiny_code, li.extreme_code])
def test_no_repeated_edges(maker):
    c = maker()
    key = c.rows.astype(np.int64) * c.n + c.cols
    assert np.unique(key).size == key.size


def test_codes_are_reproducible():
    a, b = li.tiny_code(), li.tiny_code()
    assert (a.rows == b.rows).all() and (a.cols == b.cols).all()
    assert (li.awgn_llr(100, 3, 0.5, 7) == li.awgn_llr(100, 3, 0.5, 7)).all()


def test_encoder_spans_the_14_7_code():
    code = li.code_14_7()
    enc = li.Encoder(code)
    assert enc.k == 7
    info = np.array(list(itertools.product([0, 1], repeat=7)), np.uint8)
    cw = enc.encode(info)
    words = np.array(list(itertools.product([0, 1], repeat=14)), np.uint8)
    brute = words[code.syndrome(words).sum(1) == 0]
    assert sorted(map(bytes, cw)) == sorted(map(bytes, brute))
    assert (cw[:, enc.info_cols] == info).all()


@pytest.mark.parametrize("maker", [li.tiny_code, li.large_code, li.extreme_code])
def test_encoder_codewords_satisfy_h(maker):
    code = maker()
    enc = li.Encoder(code)
    assert enc.k == code.n - code.m        # these random codes have full-rank H
    cw = enc.random_codewords(8, seed=3002)
    assert code.syndrome(cw).sum() == 0
    assert 0.4 < cw.mean() < 0.6


def test_encoder_rank_deficient_matrix():
    # rows 0 and 1 equal rows 2 xor 3 in sum: rank 3 of 4 rows
    H = np.array([[1, 1, 0, 0, 1, 0], [0, 1, 1, 0, 0, 1], [1, 0, 1, 1, 0, 0], [0, 0, 0, 1, 1, 1]], np.uint8)
    r, c = np.nonzero(H)
    code = li.Code(m=4, n=6, rows=r.astype(np.int32), cols=c.astype(np.int32))
    enc = li.Encoder(code)
    assert enc.k == 3
    info = np.array(list(itertools.product([0, 1], repeat=3)), np.uint8)
    cw = enc.encode(info)
    assert code.syndrome(cw).sum() == 0 and len(set(map(bytes, cw))) == 8


def test_channel_llr_statistics():
    s2 = li.ebn0_to_sigma2(2.0, 0.5)
    assert s2 == pytest.approx(0.6309573, rel=1e-6)
    llr = li.awgn_llr(20000, 4, s2, seed=1)
    mu = 2.0 / s2
    assert llr.mean() == pytest.approx(mu, rel=0.01)
    assert llr.var() == pytest.approx(2 * mu, rel=0.02)
    cw = np.zeros((4, 20000), np.uint8)
    cw[:, ::2] = 1
    flipped = li.awgn_llr(20000, 4, s2, seed=1, codewords=cw)
    # same noise: a transmitted 1 moves y by -2, i.e. the LLR by -4/sigma^2
    np.testing.assert_allclose(llr[:, ::2] - flipped[:, ::2], 4.0 / s2, rtol=0, atol=2e-5)
    assert (flipped[:, 1::2] == llr[:, 1::2]).all()


def test_lifted_code_structure():
    """Each base edge expands to a Z x Z circulant: check i*Z + r meets bit
    j*Z + ((r + s) mod Z) for one shift s per base edge, degrees scale by Z."""
    base = li.random_small_code(12, 6, 3, seed=3)
    Z = 16
    code = li.lifted_code(base, Z, seed=4)
    assert (code.m, code.n, code.nnz) == (base.m * Z, base.n * Z, base.nnz * Z)
    np.testing.assert_array_equal(np.bincount(code.cols, minlength=code.n), np.repeat(base.bit_degrees(), Z))
    np.testing.assert_array_equal(code.check_degrees(), np.repeat(base.check_degrees(), Z))
    bi, bj = code.rows // Z, code.cols // Z
    for i, j in zip(base.rows.tolist(), base.cols.tolist()):
        sel = (bi == i) & (bj == j)
        r, c = code.rows[sel] % Z, code.cols[sel] % Z
        assert sel.sum() == Z and sorted(r.tolist()) == list(range(Z))
        shift = (c - r) % Z
        assert (shift == shift[0]).all()            # one circulant per base edge
    key = code.rows.astype(np.int64) * code.n + code.cols
    assert np.unique(key).size == key.size


def test_large_qc_code_profile_and_encoder():
    code = li.large_qc_code()
    assert (code.n, code.m, code.nnz) == (64800, 32400, 226800)
    assert set(code.check_degrees().tolist()) == {7}
    assert np.bincount(np.bincount(code.cols, minlength=code.n)).tolist() == [0, 0, 32400, 19440, 0, 0, 0, 0, 12960]
    cw = li.Encoder(code).random_codewords(3, seed=5)
    assert not code.syndrome(cw).any()
