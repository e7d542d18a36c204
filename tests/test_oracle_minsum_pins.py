"""Pins of the oracle's Min-Sum rules against facts that do not come from the oracle.

The Min-Sum family keeps the sum-product bit rule and replaces the check
magnitude by the smallest other |Q| (normalized by alpha, or reduced by an
offset beta and floored at 0), the derived decoders the paper's Section 3.1
names for the edge-level approach.  What fixes them independently:

* max-log MAP by enumeration: for a single parity check, the extrinsic
  max-log LLR of bit j (the best even-weight word with c_j = 0 minus the best
  with c_j = 1, counting the other bits only) is the Min-Sum message, so one
  iteration on a single-parity-check code gives Lpost_j = L_j + that value
  (times alpha, or with the offset applied);
* max-marginals by enumeration: on a cycle-free graph Min-Sum is exact
  max-product, so after enough iterations Lpost_j equals the best codeword
  metric with c_j = 0 minus the best with c_j = 1 (which catches a dropped
  term, a wrong sign or a non-extrinsic message in either rule);
* closed forms and special cases: degree-2 checks pass the other message
  through, so a path code sums its channel values like sum-product; a degree-1
  check sends +LMAX; sign symmetry is exact.
"""
import itertools

import numpy as np
import pytest

import ldpc_inputs as li
import oracle


def _even_words(d):
    w = np.array(list(itertools.product([0, 1], repeat=d)), dtype=np.uint8)
    return w[w.sum(axis=1) % 2 == 0]


def _maxlog_extrinsic_spc(L):
    """Extrinsic max-log LLR of every bit of one parity check, by enumeration."""
    L = np.asarray(L, np.float64)
    d = L.size
    words = _even_words(d).astype(np.float64)
    out = np.empty(d)
    for j in range(d):
        others = np.delete(np.arange(d), j)
        metric = ((1.0 - 2.0 * words[:, others]) * L[others] / 2.0).sum(axis=1)
        out[j] = metric[words[:, j] == 0].max() - metric[words[:, j] == 1].max()
    return out


def _max_marginals(code, L):
    words = np.array(list(itertools.product([0, 1], repeat=code.n)), dtype=np.uint8)
    cw = words[code.syndrome(words).sum(axis=1) == 0].astype(np.float64)
    metric = ((1.0 - 2.0 * cw) * np.asarray(L, np.float64)[None, :] / 2.0).sum(axis=1)
    return np.array([metric[cw[:, j] == 0].max() - metric[cw[:, j] == 1].max() for j in range(code.n)])


@pytest.mark.parametrize("d", [2, 3, 5, 8, 11])
def test_min_sum_single_parity_check_is_max_log_map(d):
    code = li.spc_code(d)
    rng = np.random.default_rng(40 + d)
    llr = rng.uniform(-4, 4, size=(3, d)).astype(np.float32)
    got = oracle.decode(code, llr, max_iter=1, early_stop=False, rule="ms")["lpost"]
    for f in range(3):
        want = llr[f].astype(np.float64) + _maxlog_extrinsic_spc(llr[f])
        np.testing.assert_allclose(got[f], want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("alpha", [0.5, 0.75, 1.0])
def test_normalized_min_sum_single_parity_check(alpha):
    code = li.spc_code(6)
    rng = np.random.default_rng(7)
    llr = rng.uniform(-3, 3, size=(4, 6)).astype(np.float32)
    got = oracle.decode(code, llr, max_iter=1, early_stop=False, rule="nms", param=alpha)["lpost"]
    for f in range(4):
        want = llr[f].astype(np.float64) + alpha * _maxlog_extrinsic_spc(llr[f])
        np.testing.assert_allclose(got[f], want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("beta", [0.0, 0.3, 1.0])
def test_offset_min_sum_single_parity_check(beta):
    code = li.spc_code(5)
    rng = np.random.default_rng(8)
    # magnitudes straddle the offset, so some messages are floored at 0
    llr = rng.uniform(-1.5, 1.5, size=(6, 5)).astype(np.float32)
    got = oracle.decode(code, llr, max_iter=1, early_stop=False, rule="oms", param=beta)["lpost"]
    floored = 0
    for f in range(6):
        ext = _maxlog_extrinsic_spc(llr[f])
        shrunk = np.sign(ext) * np.maximum(np.abs(ext) - beta, 0.0)
        floored += int(((np.abs(ext) <= beta) & (ext != 0)).sum())
        np.testing.assert_allclose(got[f], llr[f].astype(np.float64) + shrunk, rtol=0, atol=1e-12)
    if beta >= 0.3:
        assert floored > 0


@pytest.mark.parametrize("seed", range(10))
def test_min_sum_tree_decode_equals_max_marginals(seed):
    rng = np.random.default_rng(300 + seed)
    code = li.tree_code(int(rng.integers(2, 6)), seed=seed, max_check_deg=4)
    if code.n > 16:
        pytest.skip("tree too large for enumeration")
    llr = rng.uniform(-2.0, 2.0, size=(2, code.n)).astype(np.float32)
    got = oracle.decode(code, llr, max_iter=code.m + 1, early_stop=False, rule="ms")["lpost"]
    for f in range(2):
        np.testing.assert_allclose(got[f], _max_marginals(code, llr[f]), rtol=0, atol=1e-9)


@pytest.mark.parametrize("rule,param", [("ms", None), ("nms", 1.0), ("oms", 0.0)])
def test_min_sum_path_code_posterior_is_total_sum(rule, param):
    """Checks of degree 2 forward the other message unchanged under alpha = 1
    and beta = 0, so the path code sums its channel values."""
    n = 7
    code = li.path_code(n)
    rng = np.random.default_rng(n)
    llr = rng.uniform(-3, 3, size=(2, n)).astype(np.float32)
    got = oracle.decode(code, llr, max_iter=n - 1, early_stop=False, rule=rule, param=param)["lpost"]
    want = llr.astype(np.float64).sum(axis=1, keepdims=True) * np.ones((1, n))
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def test_normalized_min_sum_path_code_geometric_weights():
    """Under alpha, a message crossing k degree-2 checks is scaled by alpha^k:
    after n - 1 iterations Lpost_j = sum_i alpha^|i - j| L_i on a path."""
    n, alpha = 6, 0.75
    code = li.path_code(n)
    rng = np.random.default_rng(5)
    llr = rng.uniform(-3, 3, size=(1, n)).astype(np.float32)
    got = oracle.decode(code, llr, max_iter=n - 1, early_stop=False, rule="nms", param=alpha)["lpost"][0]
    L = llr[0].astype(np.float64)
    want = np.array([sum(alpha ** abs(i - j) * L[i] for i in range(n)) for j in range(n)])
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("rule,param", [("ms", None), ("nms", 0.75), ("oms", 0.5)])
def test_min_sum_degree_one_check_adds_lmax(rule, param):
    code = li.Code(m=2, n=2, rows=np.array([0, 1, 1], np.int32), cols=np.array([0, 0, 1], np.int32))
    llr = np.array([[-1.5, 2.5]], np.float32)
    got = oracle.decode(code, llr, max_iter=1, early_stop=False, rule=rule, param=param)["lpost"][0]
    through = {"ms": 2.5, "nms": 0.75 * 2.5, "oms": 2.5 - 0.5}[rule]
    assert got[0] == pytest.approx(-1.5 + 64.0 + through, abs=1e-12)


@pytest.mark.parametrize("rule,param", [("ms", None), ("nms", 0.75), ("oms", 0.25)])
def test_min_sum_sign_symmetry_is_exact(rule, param):
    code = li.code_14_7()
    words = np.array(list(itertools.product([0, 1], repeat=14)), dtype=np.uint8)
    cw = words[code.syndrome(words).sum(axis=1) == 0]
    rng = np.random.default_rng(2)
    base = rng.normal(1.5, 2.0, size=(1, 14)).astype(np.float32)
    ref = oracle.decode(code, base, max_iter=20, rule=rule, param=param)
    flip = (1 - 2 * cw.astype(np.int32)).astype(np.float32)
    got = oracle.decode(code, base * flip, max_iter=20, rule=rule, param=param)
    assert (got["iters"] == ref["iters"][0]).all()
    assert (got["lpost"] == ref["lpost"][0] * flip).all()
    assert (got["bits"] == (ref["bits"][0] ^ cw)).all()


def test_min_sum_rules_reject_bad_parameters():
    code = li.spc_code(3)
    llr = np.zeros((1, 3), np.float32)
    for rule, param in (("nms", 0.0), ("nms", 1.5), ("oms", -0.1), ("oms", 64.0)):
        with pytest.raises(ValueError):
            oracle.decode(code, llr, max_iter=1, rule=rule, param=param)
