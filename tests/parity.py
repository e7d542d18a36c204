"""Shared helpers for the GPU parity tests: run the HIP decoder through the C ABI
and compare it with the FP64 oracle on the same seeded inputs.

Parity bar (from the decoder's contract):
  * hard decisions, syndrome flags and iteration counts are bit-exact on every
    frame that is clear of decision ties.  The contract excludes frames whose
    trajectory has any |Lpost| < 1e-3; at n = 64800 and tens of iterations
    that excludes every frame, so the oracle instead flags a frame only when
    flipping the bits with |Lpost| < 1e-3 could change an output (zero a
    failing syndrome early, or touch the returned estimate).  Every frame the
    contract keeps is also kept here (the test is stricter); tie-risk frames
    are counted and their mismatches reported;
  * posterior LLRs agree to |L_gpu - L_oracle| <= 1e-3 + 1e-4 |L_oracle| on
    those frames when the oracle decodes them to a codeword, and on every
    frame in the fixed-iteration checks (posterior_all=True).
  * a frame that never converges keeps oscillating until max_iter, and any
    two precisions drift apart on it, more with every iteration: the oracle's
    own source built with FP32 arithmetic exceeds the bar on such frames by
    orders of magnitude at 80 iterations (a CPU pin in test_oracle_pins.py).
    On those frames the GPU posterior must stay within the bar plus
    DRIFT_FACTOR times the drift of that FP32 build from FP64 (frame maximum);
    bits, flag and iteration count are still held bit-exact.
"""
from __future__ import annotations

import numpy as np

import oracle

ATOL = 1e-3
RTOL = 1e-4
TIE_MARGIN = 1e-3
# GPU drift allowed on non-converging frames, as a multiple of the drift of an
# FP32 build of the oracle's own arithmetic: the GPU rounds the same algorithm
# in FP32 but through the hardware exp2/log2/reciprocal (about 1 ulp each) and
# a different exact form of the check rule, so its rounding noise per
# iteration is a small multiple of that build's; the iterations amplify both
# the same way.
DRIFT_FACTOR = 8.0


def gpu_decode(code, llr: np.ndarray, max_iter: int, flags: int = 0, graph=None, rule=None, param=None):
    import torch
    from paper_1609_01567_amd import ldpc
    g = graph if graph is not None else ldpc.Graph.from_code(code)
    x = torch.from_numpy(np.ascontiguousarray(llr, dtype=np.float32)).cuda()
    res = ldpc.decode(g, x, max_iter, flags=flags, want_llr=True, rule=rule, rule_param=param)
    torch.cuda.synchronize()
    return dict(bits=res.bits.cpu().numpy(), ok=res.ok.cpu().numpy(), iters=res.iters.cpu().numpy(),
                lpost=res.llr.cpu().numpy())


def compare(code, llr, max_iter: int, early_stop: bool = True, flags: int = 0, frames=None,
            gpu=None, atol: float = ATOL, rtol: float = RTOL, margin: float = TIE_MARGIN,
            require_all: bool = False, posterior_all: bool = False, rule=None, param=None):
    """Decode on both sides and assert the parity bar; returns a stats dict.

    `frames` restricts the oracle to a subset of rows of `llr` (full-size
    cases); `gpu` may carry a GPU result decoded earlier for all rows.
    `rule` / `param` select the check rule on both sides (None: sum-product).
    """
    from paper_1609_01567_amd import ldpc
    if not early_stop:
        flags |= ldpc.NO_EARLY_STOP
    if gpu is None:
        gpu = gpu_decode(code, llr, max_iter, flags, rule=rule, param=param)
    idx = np.arange(llr.shape[0]) if frames is None else np.asarray(frames)
    ora = oracle.decode(code, llr[idx], max_iter, early_stop=early_stop, tie_margin=margin,
                        rule=rule or "sp", param=param)
    g = {k: v[idx] for k, v in gpu.items()}
    clear = ora["tie_risk"] == 0
    if require_all:
        clear[:] = True
    same_bits = (g["bits"] == ora["bits"]).all(axis=1)
    same_iter = g["iters"] == ora["iters"]
    same_ok = g["ok"] == ora["ok"]
    err = np.abs(g["lpost"].astype(np.float64) - ora["lpost"])
    within = (err <= atol + rtol * np.abs(ora["lpost"])).all(axis=1)
    conv = ora["ok"] == 1
    post = clear & (conv | posterior_all)
    if not early_stop and posterior_all:
        # Without early stop no decision feeds back into the decode, so ties
        # cannot change the posterior: it is held on every frame, and every
        # hard decision is held except those of bits within the tie margin.
        post = np.ones_like(clear)
        sure = np.abs(ora["lpost"]) >= margin
        same_bits = ((g["bits"] == ora["bits"]) | ~sure).all(axis=1)
        same_ok = same_ok | ~clear
        clear = np.ones_like(clear)
    bad = (clear & ~(same_bits & same_iter & same_ok)) | (post & ~within)
    drift = clear & ~post
    drift_ratio = np.zeros(0)
    if drift.any():
        sel = np.flatnonzero(drift)
        o32 = oracle.decode(code, llr[idx][sel], max_iter, early_stop=early_stop, tie_margin=margin,
                            rule=rule or "sp", param=param, fp32_build=True)
        d32 = np.abs(o32["lpost"] - ora["lpost"][sel]).max(axis=1)
        excess = (err[sel] - (atol + rtol * np.abs(ora["lpost"][sel]))).max(axis=1)
        drift_ratio = np.where(excess > 0, excess / np.maximum(d32, 1e-30), 0.0)
        over = excess > DRIFT_FACTOR * d32
        bad[sel[over]] = True
    stats = dict(frames=int(idx.size), clear=int(clear.sum()), near_tie=int((~clear).sum()),
                 clear_by_min_abs=int((ora["min_abs"] >= margin).sum()),
                 mismatched_near_tie=int((~clear & ~(same_bits & same_iter & same_ok)).sum()),
                 posterior_checked=int(post.sum()),
                 max_err=float(err[post].max()) if post.any() else 0.0,
                 max_rel=float((err / (1.0 + np.abs(ora["lpost"])))[post].max()) if post.any() else 0.0,
                 nonconverged_clear=int(drift.sum()),
                 nonconverged_max_err=float(err[drift].max()) if drift.any() else 0.0,
                 nonconverged_max_excess_over_fp32_drift=float(drift_ratio.max()) if drift_ratio.size else 0.0)
    if bad.any():
        f = int(np.flatnonzero(bad)[0])
        raise AssertionError(
            f"parity failure on frame {int(idx[f])}: bits_equal={bool(same_bits[f])} "
            f"iters gpu/oracle={int(g['iters'][f])}/{int(ora['iters'][f])} ok gpu/oracle="
            f"{int(g['ok'][f])}/{int(ora['ok'][f])} max|dL|={float(err[f].max()):.3e} stats={stats}")
    return stats


def first_iteration_bound(code, llr, lmax: float = 64.0):
    """[F][n]: sum over the checks of v of min(lmax, min |Lch| over the check's other bits)."""
    F = llr.shape[0]
    a = np.minimum(np.abs(llr.astype(np.float64)), lmax)          # [F][n]
    rows, cols = code.rows.astype(np.int64), code.cols.astype(np.int64)
    mag = a[:, cols]                                               # [F][E]
    big = np.full((F, code.m), np.inf)
    first = big.copy()
    arg = np.full((F, code.m), -1, np.int64)
    for e in range(code.nnz):     # smallest per check, and which edge holds it
        c = rows[e]
        upd = mag[:, e] < first[:, c]
        first[upd, c] = mag[upd, e]
        arg[upd, c] = e
    second = big.copy()
    for e in range(code.nnz):
        c = rows[e]
        x = np.where(arg[:, c] == e, np.inf, mag[:, e])
        second[:, c] = np.minimum(second[:, c], x)
    excl = np.where(arg[:, rows] == np.arange(code.nnz)[None, :], second[:, rows], first[:, rows])
    excl = np.minimum(excl, lmax)                                  # degree-1 checks: clamp of the empty rule
    bound = np.zeros((F, code.n))
    np.add.at(bound.T, cols, excl.T)
    return bound


def first_iteration_input_bound(code, llr, lmax: float = 64.0):
    """[F][n]: sum over the checks of v of the sum of min(lmax, |Lch|) over the check's other bits."""
    a = np.minimum(np.abs(llr.astype(np.float64)), lmax)          # [F][n]
    rows, cols = code.rows.astype(np.int64), code.cols.astype(np.int64)
    row_sum = np.zeros((llr.shape[0], code.m))
    np.add.at(row_sum.T, rows, a[:, cols].T)                       # per check: sum over its bits
    other = row_sum[:, rows] - a[:, cols]                          # per edge: the other bits of its check
    bound = np.zeros((llr.shape[0], code.n))
    np.add.at(bound.T, cols, other.T)
    return bound
