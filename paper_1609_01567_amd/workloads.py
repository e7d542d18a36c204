"""Benchmark workloads built on the decoder: the batched uneven-code mix and its
operating points.

The batched mix is eight seeded random codes (ldpc_inputs.batch_codes) with a
Zipf split of 4096 frames.  Each code runs 0.5 dB above its waterfall, the
Eb/N0 where the FP32 decoder's frame-error rate at 50 iterations crosses 0.5.
`calibrate()` finds those points by bisection on a 0.05 dB grid (2000 random
codewords per point) and writes them to operating_points.json.  They are
workload parameters of the benchmark only.
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import ldpc_inputs as li  # noqa: E402

POINTS_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "operating_points.json")
GRID_DB = 0.05
MARGIN_DB = 0.5


def frame_error_rate(code, graph, encoder, ebn0, frames, T, seed):
    import torch
    from . import ldpc
    cw = encoder.random_codewords(frames, seed=seed)
    llr = li.awgn_llr(code.n, frames, li.ebn0_to_sigma2(ebn0, code.rate), seed=seed + 1, codewords=cw)
    res = ldpc.decode(graph, torch.from_numpy(llr).cuda(), T)
    bits = res.bits.cpu().numpy()
    return float((bits != cw).any(axis=1).mean())


def find_waterfall(code, frames=2000, T=50, lo_db=-1.0, hi_db=6.0, seed=9000):
    """Bisection on the 0.05 dB grid for the lowest Eb/N0 with FER <= 0.5."""
    from . import ldpc
    graph = ldpc.Graph.from_code(code)
    enc = li.Encoder(code)
    lo, hi = int(round(lo_db / GRID_DB)), int(round(hi_db / GRID_DB))
    fer = {}

    def f(i):
        if i not in fer:
            fer[i] = frame_error_rate(code, graph, enc, i * GRID_DB, frames, T, seed + i)
        return fer[i]

    if f(lo) <= 0.5 or f(hi) > 0.5:
        raise RuntimeError(f"{code.name}: FER does not cross 0.5 in [{lo_db}, {hi_db}] dB")
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if f(mid) > 0.5:
            lo = mid
        else:
            hi = mid
    return hi * GRID_DB, {round(i * GRID_DB, 2): v for i, v in sorted(fer.items())}


def calibrate(frames=2000, T=50):
    out = {"method": f"FER of the FP32 plain decoder at T={T} with {frames} random codewords per point; "
                     f"bisection on a {GRID_DB} dB grid for the first point with FER <= 0.5; "
                     f"operating point = waterfall + {MARGIN_DB} dB",
           "codes": []}
    for code in li.batch_codes():
        wf, trace = find_waterfall(code, frames=frames, T=T)
        out["codes"].append({"name": code.name, "n": code.n, "m": code.m, "waterfall_db": round(wf, 2),
                             "operating_db": round(wf + MARGIN_DB, 2), "fer_trace": trace})
        print(f"[calibrate] {code.name}: waterfall {wf:.2f} dB", flush=True)
    with open(POINTS_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def operating_points():
    with open(POINTS_FILE) as fh:
        return {c["name"]: c["operating_db"] for c in json.load(fh)["codes"]}


def batched_mix(frames_total=4096, seed_base=0):
    """[(code, frames, ebn0_db, codewords [F][n], llr [F][n])] for the eight batch codes."""
    pts = operating_points()
    split = li.batch_frame_split(frames_total)
    out = []
    for i, (code, F) in enumerate(zip(li.batch_codes(), split)):
        eb = pts[code.name]
        cw = li.Encoder(code).random_codewords(int(F), seed=3101 + i + seed_base)
        llr = li.awgn_llr(code.n, int(F), li.ebn0_to_sigma2(eb, code.rate), seed=2101 + i + seed_base, codewords=cw)
        out.append((code, int(F), eb, cw, llr))
    return out


# ---------------------------------------------------------------------------
# the rate-1/2 n = 64800 throughput workload, decoded as the benchmark times it
# ---------------------------------------------------------------------------

HEADLINE_FRAMES_PER_CALL = 256     # one ldpc_decode per Eb/N0 point


def headline_flags(early_stop: bool = True) -> int:
    from . import ldpc
    return ldpc.COMPACT_TAIL if early_stop else ldpc.NO_EARLY_STOP


def headline_decode(graph, d_llrs, max_iter: int, want_llr: bool = False, early_stop: bool = True,
                    workspace=None, outs=None, stream=None):
    """Enqueue the decode of each point's frames ([F][n] float32 device tensors
    in `d_llrs`) the way the benchmark times them: calls of
    HEADLINE_FRAMES_PER_CALL frames, headline_flags(), the default lane width,
    one workspace shared by the calls.  Returns one DecodeResult per point."""
    from . import ldpc
    flags = headline_flags(early_stop)
    if workspace is None:
        workspace = ldpc.Workspace(ldpc.workspace_size(graph, HEADLINE_FRAMES_PER_CALL, flags))
    res = []
    for i, x in enumerate(d_llrs):
        if x.shape[0] > HEADLINE_FRAMES_PER_CALL:
            raise ValueError("more frames than one headline call holds")
        res.append(ldpc.decode(graph, x, max_iter, flags=flags, want_llr=want_llr, workspace=workspace,
                               stream=stream, out=None if outs is None else outs[i]))
    return res


if __name__ == "__main__":
    calibrate()
