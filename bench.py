"""Throughput benchmark of the MI355X sum-product LDPC decoder.

Workload (one "step"): the n=64800, m=32400 rate-1/2 random irregular code
(bit degrees 8/3/2), 256 frames at each Eb/N0 in {0.8, 1.0, 1.2, 1.4} dB,
at most 50 iterations with syndrome early stop, fp32 messages.  Channel LLRs
are seeded and synthetic and already resident in HBM when timing starts.

Prints ONE JSON line: decoded information Gbit/s (k = n - m per frame), the
fraction of HBM peak of the whole step, a roofline entry for the dominant
kernel (the check-node pass) from HIP events recorded on the decode stream,
and the FP64 CPU oracle's rate on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak, GB/s
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "check_rows_kernel_n64800_f256_4pts.json")
DOMINANT = "void check_rows_kernel<0, 4, 8, 1, 0, false>"   # FP32, 4 slots per lane, rows <= 8, steady state, sum-product, column table


def kernel_source_sha():
    """Hash of the sources the plain decoder's kernels are built from."""
    import hashlib
    h = hashlib.sha256()
    for f in ("decode.hip", "device_common.h"):
        h.update(open(os.path.join(ROOT, "paper_1609_01567_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 PMC record.

    FETCH_SIZE and WRITE_SIZE per dispatch, scaled by what the same counters read
    for a plain 1 GiB copy.  None when the kernel source changed since the counters
    were taken.
    """
    try:
        rec = json.load(open(TRAFFIC_RECORD))
    except (OSError, ValueError):
        return None
    if kernel_source_sha() != rec.get("source_sha"):
        return None
    k = rec["kernels"].get(DOMINANT)
    if not k:
        return None
    return int(round(k["fetch_bytes_per_dispatch"] + k["write_bytes_per_dispatch"]))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--ebn0", type=str, default="0.8,1.0,1.2,1.4")
    ap.add_argument("--frames", type=int, default=256)
    ap.add_argument("--max-iter", type=int, default=50)
    ap.add_argument("--msg", choices=["fp32", "fp16", "bf16"], default="fp32")
    ap.add_argument("--lane-slots", type=int, choices=[0, 1, 2, 4], default=0,
                    help="frame slots per wavefront lane (0: library default)")
    ap.add_argument("--cpu-frames", type=int, default=64,
                    help="oracle sample on all host threads: frames per Eb/N0 point")
    ap.add_argument("--cpu-frames-1core", type=int, default=4,
                    help="oracle sample on one thread: frames per Eb/N0 point")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--engine-slots", type=str, default="256,512",
                    help="slot-pool sizes tried for the refill engine on the same workload")
    ap.add_argument("--no-engine", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--extreme-only", action="store_true",
                    help="only the throughput of the extreme code (1024 frames at 1.5 dB, every message format)")
    ap.add_argument("--no-simulate", action="store_true")
    ap.add_argument("--no-minsum", action="store_true")
    ap.add_argument("--no-structured", action="store_true")
    ap.add_argument("--served-requests", type=int, default=20000,
                    help="counted requests per load point (after a 2 s warm-up)")
    ap.add_argument("--served-iters-per-step", type=int, default=4,
                    help="decoder iterations per engine step in the server")
    ap.add_argument("--no-compact", action="store_true",
                    help="time the headline decode without tail compaction (LDPC_COMPACT_TAIL)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates rocprof byte counters) and exit")
    ap.add_argument("--engine-timeline", action="store_true",
                    help="only run the batched mix through the autotuned FP16 engine one replay at a time, "
                         "printing each replay's time and the frames still pending per code, and exit")
    ap.add_argument("--timeline-one-iteration", action="store_true",
                    help="with --engine-timeline: one step of one iteration per replay (per-iteration counts)")
    return ap.parse_args()


def engine_timeline(torch, ldpc, T=50, reps=2, gap_s=0.002, one_iteration=False):
    """The batched mix, one engine replay at a time (FP16 messages, autotuned).

    After every replay the host waits for the engine and records the replay's
    wall time and the frames still pending per code; a short sleep between
    replays separates them in a kernel trace.  The last of `reps` batches is
    reported, with the edge-frames each code still had running (the work an
    iteration at full activity would do for them).  one_iteration: the tuned
    pools and lane width, but one step of one iteration per replay.
    """
    from paper_1609_01567_amd import workloads
    mix = workloads.batched_mix()
    graphs = [ldpc.Graph.from_code(c) for c, *_ in mix]
    d_llr = [torch.from_numpy(x).cuda() for *_, x in mix]
    outs = [ldpc.DecodeResult(bits=torch.empty((F, c.n), dtype=torch.uint8, device="cuda"),
                              ok=torch.empty(F, dtype=torch.uint8, device="cuda"),
                              iters=torch.empty(F, dtype=torch.int32, device="cuda"), llr=None) for c, F, *_ in mix]
    frame_lists = [ldpc.frames_for(x, o.bits, o.ok, o.iters) for x, o in zip(d_llr, outs)]
    torch.cuda.synchronize()
    tune = ldpc.autotune(graphs, frame_lists, T, ldpc.MSG_FP16)
    if one_iteration:
        tune.update(graph_steps=1, iters_per_step=1)
    eng = ldpc.Engine(graphs, tune["slots"], [len(fl) for fl in frame_lists], T, flags=ldpc.MSG_FP16,
                      lane_slots=tune["lane_slots"], graph_steps=tune["graph_steps"],
                      iters_per_step=tune["iters_per_step"])
    edges = [c.nnz for c, *_ in mix]
    replays = []
    for _ in range(reps):
        for gi, fl in enumerate(frame_lists):
            eng.submit(gi, fl)
        torch.cuda.synchronize()
        replays = []
        while True:
            t0 = time.perf_counter()
            eng.step(1)
            _, pending = eng.poll()
            ms = (time.perf_counter() - t0) * 1e3
            replays.append({"ms": round(ms, 3), "pending": pending.tolist(),
                            "pending_edge_frames": int(sum(e * p for e, p in zip(edges, pending.tolist())))})
            time.sleep(gap_s)
            if not pending.any():
                break
            if len(replays) > 4 * T:
                raise RuntimeError("engine timeline: frames still pending after many replays")
    eng.close()
    iters = [o.iters.cpu().numpy() for o in outs]
    return {"metric": "engine_timeline", "tuning": tune,
            "iterations_per_replay": tune["graph_steps"] * tune["iters_per_step"],
            "codes": [{"code": c.name, "frames": F, "edges": c.nnz, "mean_iters": round(float(it.mean()), 2),
                       "frac_at_max_iter": round(float((it == T).mean()), 4)} for (c, F, *_), it in zip(mix, iters)],
            "replays": replays, "total_ms": round(sum(r["ms"] for r in replays), 3)}


def copy_ceiling(torch, nbytes=1 << 30, reps=5):
    """GB/s of a plain device-to-device copy of nbytes (read + write counted)."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


def algorithmic_bytes(iters: np.ndarray, T: int, E: int, n: int, msg_bytes: int):
    """Bytes the method must move, per pass, from each frame's iteration count.

    s is the message size and p the posterior size the check pass reads (2
    bytes with 16-bit messages, whose posterior is stored in FP16; else 4).
    Check pass t reads every message and the previous posterior and writes
    every message: 2 E s + p n per active frame (iteration 1 reads the channel
    LLRs and writes messages only: E s + p n).  It runs for frame f while
    t <= iters_f + 1 (the pass after the last estimate also evaluates its
    syndrome).  Bit pass t reads every message and the FP32 channel LLRs and
    writes the posterior: E s + (4 + p) n, for t <= iters_f.
    """
    p = 2 if msg_bytes == 2 else 4
    check = np.zeros(T)
    bit = np.zeros(T)
    for t in range(1, T + 1):
        a = int((iters >= t - 1).sum()) if t > 1 else iters.size
        b = int((iters >= t).sum())
        check[t - 1] = a * ((2 if t > 1 else 1) * E * msg_bytes + p * n)
        bit[t - 1] = b * (E * msg_bytes + (4 + p) * n)
    return check, bit


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(code, llrs, T, frames_per_point, frames_per_point_1core):
    """The FP64 oracle on the host cores, on a bounded sample of the same frames:
    every thread this process may use, and one thread (the paper's serial CPU
    program is the other point of its Table III comparison)."""
    import oracle
    threads = os.cpu_count() or 1
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    k = code.n - code.m
    oracle.decode(code, llrs[0][:1], 2, threads=threads, want_lpost=False)   # load/warm

    def run(fpp, nthreads):
        sample = [x[:fpp] for x in llrs]
        t0 = time.perf_counter()
        iters = [oracle.decode(code, x, T, threads=nthreads, want_lpost=False)["iters"] for x in sample]
        dt = time.perf_counter() - t0
        nf = sum(x.shape[0] for x in sample)
        return nf * k / dt / 1e9, nf, float(np.concatenate(iters).mean()), dt

    v, nf, mi, dt = run(frames_per_point, threads)
    v1, nf1, mi1, dt1 = run(frames_per_point_1core, 1)
    model = cpu_model()
    return {"value": v, "unit": "Gbit/s", "cores": threads, "kind": "oracle",
            "sample": f"{frames_per_point} frames at each of {len(llrs)} Eb/N0 points of the same workload "
                      f"({nf} frames, {mi:.1f} mean iterations), FP64 C oracle (gcc -O2, OpenMP over frames), "
                      f"{dt:.1f} s wall on {threads} threads",
            "cpu_model": model,
            "single_core": {"value": v1, "unit": "Gbit/s", "cores": 1,
                            "sample": f"{frames_per_point_1core} frames at each point ({nf1} frames, {mi1:.1f} mean "
                                      f"iterations), {dt1:.1f} s wall on one thread"}}


def engine_large(torch, ldpc, g, d_llr, T, flags, slots, steps, warmup, graph_steps=8):
    """The same frames through the refill engine (one graph, `slots` slots)."""
    F = sum(x.shape[0] for x in d_llr)
    n = g.n
    eng = ldpc.Engine([g], [slots], [F], T, flags=flags & (ldpc.MSG_FP16 | ldpc.MSG_BF16),
                      lane_slots=4, graph_steps=graph_steps)
    bits = torch.empty((F, n), dtype=torch.uint8, device="cuda")
    ok = torch.empty(F, dtype=torch.uint8, device="cuda")
    it = torch.empty(F, dtype=torch.int32, device="cuda")
    llr_all = torch.cat(d_llr, 0).contiguous()
    frames = ldpc.frames_for(llr_all, bits, ok, it)
    torch.cuda.synchronize()

    def one():
        eng.submit(0, frames)
        return eng.run()

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    replays = 0
    for _ in range(steps):
        replays += one()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    out = {"slots": eng.info()["slots"][0], "ms_per_step": round(ms, 3), "replays_per_step": replays / steps,
           "graph_steps": graph_steps, "iters": it.cpu().numpy(), "ok": ok.cpu().numpy()}
    eng.close()
    return out


def bench_batched(torch, ldpc, steps, warmup, T=50):
    """Eight uneven codes, 4096 frames (Zipf split), each 0.5 dB above its waterfall.

    (a) plain FP32: one ldpc_decode per code, back to back on one stream;
    (b) engine FP16: every code in one engine (autotuned), continuous refill;
    (c) engine FP32: the same engine with FP32 messages (separates the batching
        gain from the storage-precision gain).
    Frame errors are counted against the transmitted codewords; (a) and (b)
    see the same noise, so their difference is reported as paired counts.
    """
    from paper_1609_01567_amd import workloads
    mix = workloads.batched_mix()
    graphs = [ldpc.Graph.from_code(c) for c, *_ in mix]
    d_llr = [torch.from_numpy(x).cuda() for *_, x in mix]
    info_bits = sum(F * (c.n - c.m) for c, F, *_ in mix)
    stream = torch.cuda.current_stream()

    def plain_run(flags):
        wss = [ldpc.Workspace(ldpc.workspace_size(g, F, flags)) for g, (_, F, *_) in zip(graphs, mix)]
        outs = [ldpc.DecodeResult(bits=torch.empty((F, c.n), dtype=torch.uint8, device="cuda"),
                                  ok=torch.empty(F, dtype=torch.uint8, device="cuda"),
                                  iters=torch.empty(F, dtype=torch.int32, device="cuda"), llr=None)
                for c, F, *_ in mix]

        def plain_step():
            for g, x, w, o in zip(graphs, d_llr, wss, outs):
                ldpc.decode(g, x, T, flags=flags, workspace=w, stream=stream, out=o)

        for _ in range(warmup):
            plain_step()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record(stream)
        for _ in range(steps):
            plain_step()
        e.record(stream)
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / steps
        err = [(o.bits.cpu().numpy() != cw).any(axis=1) for o, (_, _, _, cw, _) in zip(outs, mix)]
        iters = [o.iters.cpu().numpy() for o in outs]
        del wss
        return ms, err, iters

    plain_ms, plain_err, plain_iters = plain_run(0)
    p16_ms, p16_err, _ = plain_run(ldpc.MSG_FP16)

    def alg_bytes(msg_bytes):
        tot = 0.0
        for (c, *_), it in zip(mix, plain_iters):
            cb, bb = algorithmic_bytes(it, T, c.nnz, c.n, msg_bytes)
            tot += cb.sum() + bb.sum()
        return tot

    b32, b16 = alg_bytes(4), alg_bytes(2)

    def engine_run(flags):
        eouts = [ldpc.DecodeResult(bits=torch.empty((F, c.n), dtype=torch.uint8, device="cuda"),
                                   ok=torch.empty(F, dtype=torch.uint8, device="cuda"),
                                   iters=torch.empty(F, dtype=torch.int32, device="cuda"), llr=None)
                 for c, F, *_ in mix]
        frame_lists = [ldpc.frames_for(x, o.bits, o.ok, o.iters) for x, o in zip(d_llr, eouts)]
        torch.cuda.synchronize()
        tune = ldpc.autotune(graphs, frame_lists, T, flags)
        eng = ldpc.Engine(graphs, tune["slots"], [len(fl) for fl in frame_lists], T, flags=flags,
                          lane_slots=tune["lane_slots"], graph_steps=tune["graph_steps"],
                          iters_per_step=tune["iters_per_step"])

        def one():
            for gi, fl in enumerate(frame_lists):
                eng.submit(gi, fl)
            eng.run()

        for _ in range(warmup):
            one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            one()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        info = eng.info()
        eng.close()
        err = [(o.bits.cpu().numpy() != cw).any(axis=1) for o, (_, _, _, cw, _) in zip(eouts, mix)]
        iters = [o.iters.cpu().numpy() for o in eouts]
        return ms, tune, info, err, iters

    f16_ms, f16_tune, f16_info, f16_err, f16_iters = engine_run(ldpc.MSG_FP16)
    f32_ms, f32_tune, _, f32_err, f32_iters = engine_run(0)
    same32 = all((a == b).all() for a, b in zip(f32_iters, plain_iters))
    per_code = []
    for (c, F, eb, *_), pe, he in zip(mix, plain_err, f16_err):
        per_code.append({"code": c.name, "frames": F, "ebn0_db": eb, "fer_plain_fp32": round(float(pe.mean()), 5),
                         "fer_engine_fp16": round(float(he.mean()), 5),
                         "fail_only_fp16": int((he & ~pe).sum()), "fail_only_fp32": int((pe & ~he).sum())})
    pe_all, he_all = np.concatenate(plain_err), np.concatenate(f16_err)
    gb = lambda ms: round(info_bits / (ms * 1e-3) / 1e9, 4)
    tbs = lambda b, ms: round(b / (ms * 1e-3) / 1e9, 1)
    return {
        "workload": "8 random irregular codes n in {576..64800}, rates 1/3..9/10, 4096 frames (Zipf split), "
                    "random codewords, Eb/N0 = waterfall + 0.5 dB per code, max 50 iterations",
        "info_bits_per_step": int(info_bits),
        "algorithmic_bytes_per_step": {"fp32": round(b32), "fp16": round(b16)},
        "plain_fp32_per_code": {"ms_per_step": round(plain_ms, 3), "gbits": gb(plain_ms),
                                "alg_gbs": tbs(b32, plain_ms)},
        "plain_fp16_per_code": {"ms_per_step": round(p16_ms, 3), "gbits": gb(p16_ms), "alg_gbs": tbs(b16, p16_ms),
                                "fer": round(float(np.concatenate(p16_err).mean()), 5)},
        "engine_fp16": {"ms_per_step": round(f16_ms, 3), "gbits": gb(f16_ms), "tuning": f16_tune,
                        "device_bytes": f16_info["device_bytes"], "alg_gbs": tbs(b16, f16_ms)},
        "engine_fp32": {"ms_per_step": round(f32_ms, 3), "gbits": gb(f32_ms), "tuning": f32_tune,
                        "iters_equal_plain": bool(same32), "alg_gbs": tbs(b32, f32_ms)},
        "speedup_engine_fp16_vs_plain_fp32": round(plain_ms / f16_ms, 3),
        "fer_plain_fp32": round(float(pe_all.mean()), 5), "fer_engine_fp16": round(float(he_all.mean()), 5),
        "paired": {"fail_only_fp16": int((he_all & ~pe_all).sum()), "fail_only_fp32": int((pe_all & ~he_all).sum()),
                   "frames": int(pe_all.size)},
        "per_code": per_code,
    }


def bench_simulate(torch, ldpc, code, points, frames=1024, calls=2, T=50, seed=2026, compact=True):
    """Monte-Carlo error-rate runs on the device (ldpc_simulate): all-zero
    codeword, counter-based channel noise drawn on the GPU, decode, error
    counts; frames/s and info Gbit/s include the noise generation."""
    g = ldpc.Graph.from_code(code)
    flags = ldpc.COMPACT_TAIL if compact else 0
    ws = ldpc.Workspace(ldpc.simulate_workspace_size(g, frames, flags))
    ldpc.simulate(g, frames, points[0], seed, T, flags=flags, workspace=ws)       # warm
    torch.cuda.synchronize()
    out = {"workload": f"n={code.n} m={code.m}, all-zero codeword, device noise (Philox4x32-10 + Box-Muller), "
                       f"{frames * calls} frames per Eb/N0 point, max {T} iterations, fp32 messages",
           "tail_compaction": compact, "points": []}
    k = code.n - code.m
    for i, eb in enumerate(points):
        counts = torch.zeros(len(ldpc.SIM_FIELDS), dtype=torch.int64, device="cuda")
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for c in range(calls):
            ldpc.simulate(g, frames, eb, seed + i, T, flags=flags, first_frame=c * frames, counts=counts,
                          workspace=ws)
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e)
        r = ldpc.sim_counts(counts)
        out["points"].append({"ebn0_db": eb, **r, "fer": r["frame_errors"] / r["frames"],
                              "ber": r["bit_errors"] / (r["frames"] * code.n),
                              "mean_iters": r["iterations"] / r["frames"],
                              "frames_per_s": round(r["frames"] / (ms * 1e-3), 1),
                              "gbits": round(r["frames"] * k / (ms * 1e-3) / 1e9, 4)})
    return out


def bench_minsum(torch, ldpc, g, d_llr, cws, points, T, steps, rules=(("oms", 0.25, "fp32"), ("oms", 0.25, "fp16"),
                                                                    ("oms", 0.25, "q8"), ("nms", 0.875, "fp32"),
                                                                    ("ms", None, "fp32"))):
    """Min-Sum family check rules (ldpc_decode_rule) on the headline workload:
    throughput and frame errors against sum-product on the same frames (paired).
    On this degree-2-heavy code a normalization below ~0.85 stalls decoding
    (messages along chains of degree-2 bits shrink by alpha per check), so the
    offset rule is the one listed first."""
    F, n = d_llr[0].shape
    k = g.n - g.m
    E = g.nnz

    def run(rule, param, msg):
        flags = {"fp32": 0, "fp16": ldpc.MSG_FP16, "q8": ldpc.MSG_Q8}[msg]
        ws = ldpc.Workspace(ldpc.workspace_size(g, F, flags))
        outs = [None] * len(points)

        def step():
            for i in range(len(points)):
                outs[i] = ldpc.decode(g, d_llr[i], T, flags=flags, workspace=ws, rule=rule, rule_param=param)

        step()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(steps):
            step()
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / steps
        fails = [(o.bits.cpu().numpy() != cw).any(axis=1) for o, cw in zip(outs, cws)]
        iters = np.concatenate([o.iters.cpu().numpy() for o in outs])
        return ms, fails, iters

    base_ms, base_fail, base_it = run(None, None, "fp32")
    frames = F * len(points)
    out = {"workload": "the headline frames (random codewords, every Eb/N0 point), same LLRs for every rule",
           "sum_product_fp32": {"ms_per_step": round(base_ms, 3),
                                "gbits": round(frames * k / (base_ms * 1e-3) / 1e9, 4),
                                "fer": [round(float(f.mean()), 5) for f in base_fail],
                                "mean_iters": round(float(base_it.mean()), 2)},
           "rules": []}
    for rule, param, msg in rules:
        ms, fail, it = run(rule, param, msg)
        b = sum(int((f & ~bf).sum()) for f, bf in zip(fail, base_fail))     # fails only under this rule
        c = sum(int((bf & ~f).sum()) for f, bf in zip(fail, base_fail))     # fails only under sum-product
        out["rules"].append({"rule": rule, "param": param, "msg": msg, "ms_per_step": round(ms, 3),
                             "gbits": round(frames * k / (ms * 1e-3) / 1e9, 4),
                             "speedup_vs_sum_product_fp32": round(base_ms / ms, 3),
                             "ns_per_edge_iteration": round(ms * 1e6 / (float(it.sum()) * E), 5),
                             "fer": [round(float(f.mean()), 5) for f in fail],
                             "mean_iters": round(float(it.mean()), 2),
                             "paired_vs_sum_product": {"fail_only_rule": b, "fail_only_sp": c,
                                                       "fer_diff_ci95": _mcnemar(b, c, frames)}})
    out["sum_product_fp32"]["ns_per_edge_iteration"] = round(base_ms * 1e6 / (float(base_it.sum()) * E), 5)
    return out


def bench_structured(torch, ldpc, li, points, F, T, steps, compact=True):
    """The headline workload on a quasi-cyclic stand-in: the same degree profile
    lifted by Z = 360 from a 90 x 180 base graph, decoded through two graphs of
    the same code: one built from the base matrix (ldpc_graph_create_qc: the
    check pass computes each edge's bit from its circulant shift) and one built
    from the COO (the check pass reads the column table).  Both give identical
    results; the figures say what the circulant indexing changes."""
    code = li.large_qc_code()
    Z, shifts = code.qc
    n, E, k = code.n, code.nnz, code.n - code.m
    enc = li.Encoder(code)
    cws = [enc.random_codewords(F, seed=3102 + i) for i in range(len(points))]
    llrs = [li.awgn_llr(n, F, li.ebn0_to_sigma2(eb, code.rate), seed=2102 + 10 * i, codewords=cws[i])
            for i, eb in enumerate(points)]
    d_llr = [torch.from_numpy(x).cuda() for x in llrs]
    timed_flags = ldpc.COMPACT_TAIL if compact else 0

    def run(g):
        ws = ldpc.Workspace(ldpc.workspace_size(g, F, timed_flags))
        outs = [None] * len(points)

        def step():
            for i in range(len(points)):
                outs[i] = ldpc.decode(g, d_llr[i], T, flags=timed_flags, workspace=ws)

        step()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(steps):
            step()
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / steps
        res = [(o.bits.cpu().numpy(), o.iters.cpu().numpy()) for o in outs]
        chk_ms, chk_bytes, launches = 0.0, 0.0, 0
        for i in range(len(points)):
            r, tm = ldpc.decode_profiled(g, d_llr[i], T, workspace=ws)
            cb, _ = algorithmic_bytes(r.iters.cpu().numpy(), T, E, n, 4)
            chk_ms += float(tm["check_ms"].sum())
            chk_bytes += float(cb.sum())
            launches += T
        achieved = chk_bytes / launches / (chk_ms / launches * 1e-3) / 1e9
        del ws
        return res, {"ms_per_step": round(ms, 3), "gbits": round(len(points) * F * k / (ms * 1e-3) / 1e9, 4),
                     "check_avg_launch_ms": round(chk_ms / launches, 5), "check_achieved_gbs": round(achieved, 1),
                     "check_frac": round(achieved / HBM_PEAK_GBS, 4)}

    res_qc, circ = run(ldpc.Graph.from_qc(Z, shifts))
    res_coo, table = run(ldpc.Graph.from_code(code))
    same = all((a[0] == b[0]).all() and (a[1] == b[1]).all() for a, b in zip(res_qc, res_coo))
    fer = [round(float((bits != cw).any(axis=1).mean()), 5) for (bits, _), cw in zip(res_qc, cws)]
    it = np.concatenate([iters for _, iters in res_qc])
    out = {"workload": f"n={n} m={code.m} E={E} quasi-cyclic (Z=360, base 90x180, the headline degree profile), "
                       f"{F} random codewords at each Eb/N0 in {points} dB, max {T} iterations, fp32 messages",
           "tail_compaction": compact, "fer": fer, "mean_iters": round(float(it.mean()), 2)}
    out.update(circ)   # the structured path: circulant indexing
    out["column_table"] = table
    out["results_identical"] = bool(same)
    return out


def _mcnemar(b, c, N):
    """Paired difference (b - c) / N of two decoders' frame-error rates with a 95% interval."""
    d = (b - c) / N
    half = 1.96 * np.sqrt(max(b + c - (b - c) ** 2 / N, 0.0)) / N
    return [round(d - half, 5), round(d + half, 5)]


def extreme_throughput(torch, ldpc, code, g, d, T, variants, reps=2):
    """Decode throughput of every message format on one batch of the extreme code
    (all check classes, hub rows included): info Gbit/s of whole decodes timed
    with events, and per pass the algorithmic bytes of the active frames per
    second from a profiled decode (HIP events around every pass)."""
    F, n, E = d.shape[0], code.n, code.nnz
    k = code.n - code.m
    stream = torch.cuda.current_stream()
    out = {}
    for name, fl in variants:
        ws = ldpc.Workspace(ldpc.workspace_size(g, F, fl))
        o = ldpc.DecodeResult(bits=torch.empty((F, n), dtype=torch.uint8, device="cuda"),
                              ok=torch.empty(F, dtype=torch.uint8, device="cuda"),
                              iters=torch.empty(F, dtype=torch.int32, device="cuda"), llr=None)
        ldpc.decode(g, d, T, flags=fl, workspace=ws, stream=stream, out=o)
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        s.record(stream)
        for _ in range(reps):
            ldpc.decode(g, d, T, flags=fl, workspace=ws, stream=stream, out=o)
        e.record(stream)
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / reps
        _, tm = ldpc.decode_profiled(g, d, T, flags=fl, workspace=ws, stream=stream, out=o)
        it = o.iters.cpu().numpy()
        cb, bb = algorithmic_bytes(it, T, E, n, 4 if fl == 0 else 2)
        out[name] = {"ms": round(ms, 3), "gbits": round(F * k / (ms * 1e-3) / 1e9, 4),
                     "mean_iters": round(float(it.mean()), 2),
                     "check_ms_per_iter": round(float(tm["check_ms"].mean()), 4),
                     "bit_ms_per_iter": round(float(tm["bit_ms"].mean()), 4),
                     "check_alg_gbs": round(float(cb.sum() / (tm["check_ms"].sum() * 1e-3) / 1e9), 1),
                     "bit_alg_gbs": round(float(bb.sum() / (tm["bit_ms"].sum() * 1e-3) / 1e9), 1)}
        del ws
    return out


def bench_precision(torch, ldpc, frames=1024, T=100, points=(1.5, 5.0), oracle_frames=32):
    """Extreme-irregularity code (n=16200, check degrees 4..509): FP32 vs FP16 vs
    BF16 message storage (FP32 arithmetic), all-zero codeword.

    On the GPU, all frames at each Eb/N0 with early stop: FER, BER, mean
    iterations, and paired discordance against FP32.  Against the FP64 oracle on
    the first `oracle_frames` frames: posterior error at fixed T in {1, 5}
    (every frame, no early stop) and, at max_iter with early stop, agreement of
    hard decisions / iteration counts / flags and the posterior error of frames
    the oracle decodes to a codeword.  1.5 dB lies below this code's threshold
    (no precision decodes there); 5.0 dB is in its waterfall.
    """
    import oracle
    import ldpc_inputs as li
    code = li.extreme_code()
    g = ldpc.Graph.from_code(code)
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    variants = (("fp32", 0), ("fp16", ldpc.MSG_FP16), ("bf16", ldpc.MSG_BF16))

    def run(x, Tm, fl):
        r = ldpc.decode(g, x, Tm, flags=fl, want_llr=True)
        torch.cuda.synchronize()
        return dict(bits=r.bits.cpu().numpy(), ok=r.ok.cpu().numpy(), iters=r.iters.cpu().numpy(),
                    lpost=r.llr.cpu().numpy().astype(np.float64))

    def err_stats(gl, ol):
        e = np.abs(gl - ol)
        rel = e / (1.0 + np.abs(ol))
        if e.size == 0:
            return None
        return {"max": float(e.max()), "p99": float(np.percentile(e, 99)), "mean": float(e.mean()),
                "max_rel": float(rel.max())}

    out = {"workload": f"n={code.n} m={code.m} E={code.nnz}, check degrees {int(code.check_degrees().min())}.."
                       f"{int(code.check_degrees().max())}, bit degrees 2..64 (power law), all-zero codeword, "
                       f"{frames} frames per point, max {T} iterations, early stop",
           "oracle_sample_frames": oracle_frames, "points": []}
    for i, eb in enumerate(points):
        llr = li.awgn_llr(code.n, frames, li.ebn0_to_sigma2(eb, code.rate), seed=2003 + 10 * i)
        d = torch.from_numpy(llr).cuda()
        res = {name: run(d, T, fl) for name, fl in variants}
        fe = {name: (r["bits"] != 0).any(axis=1) for name, r in res.items()}
        pt = {"ebn0_db": eb, "gpu": {}, "vs_oracle": {}}
        for name, r in res.items():
            b = int((fe[name] & ~fe["fp32"]).sum())
            c = int((fe["fp32"] & ~fe[name]).sum())
            pt["gpu"][name] = {"fer": float(fe[name].mean()), "ber": float((r["bits"] != 0).mean()),
                               "mean_iters": float(r["iters"].mean()),
                               "fail_only_this": b, "fail_only_fp32": c,
                               "fer_diff_ci95": _mcnemar(b, c, frames)}
        pt["throughput"] = extreme_throughput(torch, ldpc, code, g, d, T, variants)
        xs = llr[:oracle_frames]
        dx = d[:oracle_frames].contiguous()
        for Tf in (1, 5):
            ora = oracle.decode(code, xs, Tf, early_stop=False, threads=threads)
            for name, fl in variants:
                gr = run(dx, Tf, fl | ldpc.NO_EARLY_STOP)
                pt["vs_oracle"].setdefault(name, {})[f"fixed_T{Tf}"] = err_stats(gr["lpost"], ora["lpost"])
        ora = oracle.decode(code, xs, T, threads=threads)
        conv = ora["ok"] == 1
        for name, _ in variants:
            r = {k: v[:oracle_frames] for k, v in res[name].items()}
            same = (r["bits"] == ora["bits"]).all(axis=1) & (r["iters"] == ora["iters"]) & (r["ok"] == ora["ok"])
            both = conv & (r["ok"] == 1)
            pt["vs_oracle"][name]["early_stop"] = {
                "frames_identical": int(same.sum()), "oracle_converged": int(conv.sum()),
                "posterior_err_converged": err_stats(r["lpost"][both], ora["lpost"][both])}
        out["points"].append(pt)
        print(f"[bench] precision {eb} dB: " + ", ".join(f"{k} FER {v['fer']:.4f}" for k, v in pt["gpu"].items()),
              file=sys.stderr, flush=True)
    return out


def bench_served(torch, ldpc, capacity_fps, requests, loads=(0.25, 0.5, 0.75, 0.95), T=50, seed=4001,
                 warmup_s=2.0, client_threads=4, iters_per_step=4):
    """Poisson arrivals of requests (1..64 frames of one of the eight batch codes,
    code drawn Zipf(1) by ascending n) at fractions of the measured batch
    capacity; the server (continuous batching, FP16 messages) against plain
    per-request FP32 launches in arrival order on one stream."""
    from paper_1609_01567_amd import workloads
    import ldpc_inputs as li
    codes = li.batch_codes()
    pts = workloads.operating_points()
    pool_f = 128
    pools = []
    for i, c in enumerate(codes):
        cw = li.Encoder(c).random_codewords(pool_f, seed=5100 + i)
        pools.append(li.awgn_llr(c.n, pool_f, li.ebn0_to_sigma2(pts[c.name], c.rate), seed=5200 + i, codewords=cw))
    kinfo = np.array([c.n - c.m for c in codes], np.float64)
    zipf = 1.0 / np.arange(1, len(codes) + 1)
    zipf /= zipf.sum()
    mean_frames = 32.5
    graphs = [ldpc.Graph.from_code(c) for c in codes]
    import queue
    import threading
    out = {"capacity_frames_per_s": round(capacity_fps, 1), "requests_per_load": requests, "warmup_s": warmup_s,
           "client_threads": client_threads, "iters_per_step": iters_per_step,
           "workload": "Poisson arrivals; request = U{1..64} frames of one code (Zipf(1) over the 8 batch codes), "
                       "Eb/N0 = waterfall + 0.5 dB, max 50 iterations", "loads": []}
    # slot pools follow each code's share of the request stream (the batched mix's Zipf split)
    slots = [int(x) for x in li.batch_frame_split(4096, len(codes))]
    out["slots"] = slots
    srv = ldpc.Server(graphs, slots, T, flags=ldpc.MSG_FP16, hbm_budget=2 << 30,
                      host_budget=1 << 30, lane_slots=4, graph_steps=2, iters_per_step=iters_per_step)
    for rho in loads:
        rng = np.random.default_rng(seed + int(rho * 100))
        lam = rho * capacity_fps / mean_frames
        warm = int(round(warmup_s * lam))            # requests of the warm-up, not counted
        total = warm + requests
        gaps = rng.exponential(1.0 / lam, size=total)
        gis = rng.choice(len(codes), size=total, p=zipf)
        fs = rng.integers(1, 65, size=total)
        starts = rng.integers(0, pool_f - 64 + 1, size=total)
        lat, info = [], 0.0
        pending = {}
        unmatched = []
        lock = threading.Lock()
        work = queue.Queue()
        t_first = t_last = None

        # Client threads make the submit calls (each copies about 1 MB of LLRs on
        # average), so the arrival process is not limited by one thread's copy rate.
        # A request's latency runs from its arrival: the wait for a client thread
        # plus the server's own submit-to-completion time.
        def submitter():
            while True:
                item = work.get()
                if item is None:
                    return
                r, gi, F, st, t_arrival = item
                t_sub = time.perf_counter()
                rid = srv.submit(gi, pools[gi][st:st + F])
                with lock:
                    pending[rid] = (r, F * kinfo[gi], t_sub - t_arrival)

        def collect(rids):
            nonlocal info, t_last
            for rid in unmatched + rids:
                with lock:
                    entry = pending.pop(rid, None)
                if entry is None:                      # completed before its submitter recorded it
                    if rid not in unmatched:
                        unmatched.append(rid)
                    continue
                if rid in unmatched:
                    unmatched.remove(rid)
                _, _, _, l = srv.result(rid, want_bits=False)
                r, bits, wait = entry
                if r >= warm:
                    lat.append(l + wait)
                    info += bits
                    t_last = time.perf_counter()

        threads = [threading.Thread(target=submitter, daemon=True) for _ in range(client_threads)]
        for th in threads:
            th.start()
        t0 = time.perf_counter()
        t_arr = t0
        for r in range(total):
            t_arr += gaps[r]
            while time.perf_counter() < t_arr:
                collect(srv.poll(0))
            if r == warm:
                t_first = time.perf_counter()
            work.put((r, int(gis[r]), int(fs[r]), int(starts[r]), t_arr))
        for _ in threads:
            work.put(None)
        for th in threads:
            th.join()
        deadline = time.perf_counter() + 60
        while (pending or unmatched) and time.perf_counter() < deadline:
            collect(srv.poll(20))
        lat = np.array(lat)
        window = (t_last or time.perf_counter()) - (t_first or t0)
        out["loads"].append({"offered": rho, "offered_req_per_s": round(lam, 1), "warmup_requests": warm,
                             "completed": int(lat.size),
                             "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                             "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                             "gbits": round(info / window / 1e9, 4), "window_s": round(window, 2)})
        print(f"[bench] served load {rho}: p50 {out['loads'][-1]['p50_ms']} ms p99 {out['loads'][-1]['p99_ms']} ms "
              f"{out['loads'][-1]['gbits']} Gbit/s", file=sys.stderr, flush=True)
    out["server_stats"] = srv.stats()
    srv.close()

    # plain per-request FP32 launches, FIFO in arrival order, same request stream at the lowest load
    rho = loads[0]
    rng = np.random.default_rng(seed + int(rho * 100))
    lam = rho * capacity_fps / mean_frames
    n_plain = min(requests, 400)
    gaps = rng.exponential(1.0 / lam, size=requests)[:n_plain]
    gis = rng.choice(len(codes), size=requests, p=zipf)[:n_plain]
    fs = rng.integers(1, 65, size=requests)[:n_plain]
    starts = rng.integers(0, pool_f - 64 + 1, size=requests)[:n_plain]
    d_pools = [torch.from_numpy(x).cuda() for x in pools]
    lat, info = [], 0.0
    t0 = time.perf_counter()
    t_arr = t0
    for r in range(n_plain):
        t_arr += gaps[r]
        while time.perf_counter() < t_arr:
            pass
        gi, F, st = int(gis[r]), int(fs[r]), int(starts[r])
        x = d_pools[gi][st:st + F].contiguous()
        res = ldpc.decode(graphs[gi], x, T)
        res.bits.cpu()
        lat.append(time.perf_counter() - t_arr)
        info += F * kinfo[gi]
    wall = time.perf_counter() - t0
    lat = np.array(lat)
    # the same requests back to back (no arrival gaps): the most the per-request path sustains
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(n_plain):
        gi, F, st = int(gis[r]), int(fs[r]), int(starts[r])
        res = ldpc.decode(graphs[gi], d_pools[gi][st:st + F].contiguous(), T)
        res.bits.cpu()
    sat = info / (time.perf_counter() - t0) / 1e9
    out["plain_per_request_fp32"] = {"offered": rho, "requests": n_plain, "saturated_gbits": round(sat, 4),
                                     "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                                     "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                                     "gbits": round(info / wall / 1e9, 4),
                                     "note": "one ldpc_decode per request in arrival order; the stream falls behind "
                                             "when its service time exceeds the arrival gap, so latency grows"}
    best = max(x["gbits"] for x in out["loads"])
    out["served_fp16_vs_plain_per_request_fp32"] = round(best / sat, 3) if sat > 0 else None
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build decodes on one GPU only; --gpus {args.gpus} is not supported "
              "(frames shard across GPUs with no per-iteration exchange, see the design notes)", file=sys.stderr)
        sys.exit(2)
    import torch

    import ldpc_inputs as li
    from paper_1609_01567_amd import ldpc

    torch.cuda.set_device(0)
    if args.calib_copy:
        a = torch.ones((1 << 30) // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)          # one dispatch: reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes_read": 1 << 30, "calib_copy_bytes_written": 1 << 30}))
        return
    if args.engine_timeline:
        print(json.dumps(engine_timeline(torch, ldpc, one_iteration=args.timeline_one_iteration)))
        return
    if args.extreme_only:
        code = li.extreme_code()
        g = ldpc.Graph.from_code(code)
        d = torch.from_numpy(li.awgn_llr(code.n, 1024, li.ebn0_to_sigma2(1.5, code.rate), seed=2003)).cuda()
        variants = (("fp32", 0), ("fp16", ldpc.MSG_FP16), ("bf16", ldpc.MSG_BF16))
        print(json.dumps({"metric": "extreme_throughput", "workload": f"n={code.n} m={code.m} E={code.nnz}, "
                          "1024 frames at 1.5 dB, max 100 iterations",
                          "throughput": extreme_throughput(torch, ldpc, code, g, d, 100, variants)}))
        return
    flags = {"fp32": 0, "fp16": ldpc.MSG_FP16, "bf16": ldpc.MSG_BF16}[args.msg]
    flags |= {0: 0, 1: ldpc.LANE_SLOTS_1, 2: ldpc.LANE_SLOTS_2, 4: ldpc.LANE_SLOTS_4}[args.lane_slots]
    msg_bytes = 4 if args.msg == "fp32" else 2
    points = [float(x) for x in args.ebn0.split(",")]
    code, cws, llrs = li.headline_workload(args.frames, points)
    n, m, E, F, T = code.n, code.m, code.nnz, args.frames, args.max_iter
    k = n - m
    g = ldpc.Graph.from_code(code)
    d_llr = [torch.from_numpy(x).cuda() for x in llrs]
    # the timed decodes compact their tails; the profiled pass below times the
    # full-width kernels without it
    from paper_1609_01567_amd import workloads
    # the decode configuration of the timed step (and of the full-size parity
    # tests): one call of F frames per point with the headline flags
    timed_flags = flags | (0 if args.no_compact else workloads.headline_flags())
    if F > workloads.HEADLINE_FRAMES_PER_CALL:
        raise SystemExit(f"--frames above {workloads.HEADLINE_FRAMES_PER_CALL} per call is not the timed configuration")
    ws = ldpc.Workspace(ldpc.workspace_size(g, F, timed_flags))
    outs = [ldpc.DecodeResult(bits=torch.empty((F, n), dtype=torch.uint8, device="cuda"),
                              ok=torch.empty(F, dtype=torch.uint8, device="cuda"),
                              iters=torch.empty(F, dtype=torch.int32, device="cuda"), llr=None) for _ in points]
    stream = torch.cuda.current_stream()

    def step():
        for i in range(len(points)):
            ldpc.decode(g, d_llr[i], T, flags=timed_flags, workspace=ws, stream=stream, out=outs[i])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(args.steps):
        step()
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / args.steps
    frames_per_step = F * len(points)
    value = frames_per_step * k / (ms * 1e-3) / 1e9
    print(f"[bench] timed {args.steps} steps: {ms:.3f} ms/step", file=sys.stderr, flush=True)

    # each point's decode timed on its own (after the timed steps, same calls)
    point_ms = []
    for i in range(len(points)):
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        for _ in range(args.steps):
            ldpc.decode(g, d_llr[i], T, flags=timed_flags, workspace=ws, stream=stream, out=outs[i])
        s1.record(stream)
        torch.cuda.synchronize()
        point_ms.append(s0.elapsed_time(s1) / args.steps)
    k_rank = li.Encoder(code).k   # n - rank(H) over GF(2)

    per_point = []
    step_bytes = 0.0
    all_check = []
    for i, eb in enumerate(points):
        it = outs[i].iters.cpu().numpy()
        ok = outs[i].ok.cpu().numpy()
        bits = outs[i].bits.cpu().numpy()
        cb, bb = algorithmic_bytes(it, T, E, n, msg_bytes)
        step_bytes += cb.sum() + bb.sum() + F * (4 * n + 4 * n + n)   # + LLR in/transposes, bits out
        err = bits != cws[i]
        per_point.append({"ebn0_db": eb, "mean_iters": float(it.mean()), "max_iters": int(it.max()),
                          "fer": float(err.any(axis=1).mean()), "ber": float(err.mean()),
                          "syndrome_ok_frames": int(ok.sum()), "ms": round(point_ms[i], 3),
                          "gbits": round(F * k / (point_ms[i] * 1e-3) / 1e9, 4)})
        all_check.append((it, cb, bb))
    hbm_frac = step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS

    roofline = None
    phase = None
    if not args.no_profile:
        # Same workload again through the profiled entry point: the library
        # records HIP events on the decode stream around every pass.
        chk_ms = np.zeros(T)
        bit_ms = np.zeros(T)
        chk_bytes = np.zeros(T)
        bit_bytes = np.zeros(T)
        launches = 0
        for _ in range(args.steps):
            for i in range(len(points)):
                res, tm = ldpc.decode_profiled(g, d_llr[i], T, flags=flags, workspace=ws, stream=stream,
                                               out=outs[i])
                it = res.iters.cpu().numpy()
                cb, bb = algorithmic_bytes(it, T, E, n, msg_bytes)
                chk_ms += tm["check_ms"]
                bit_ms += tm["bit_ms"]
                chk_bytes += cb
                bit_bytes += bb
                launches += T
        avg_ms = chk_ms.sum() / launches
        achieved = chk_bytes.sum() / launches / (avg_ms * 1e-3) / 1e9
        traffic = measured_traffic() if flags == 0 else None
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "traffic_note": "HBM bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0, "
                                    "copy-calibrated) from " + os.path.relpath(TRAFFIC_RECORD, ROOT),
                    "kernel": "check_rows_kernel (check-node pass, rows of degree <= 8)",
                    "avg_launch_ms": round(avg_ms, 5), "launches": launches,
                    "bytes_per_launch": round(chk_bytes.sum() / launches),
                    "per_unit": f"{2 * msg_bytes} B per edge-frame (message read + write) + "
                                f"{2 if msg_bytes == 2 else 4} B per bit-frame "
                                f"(posterior gather); units = active frames x (E={E} edges, n={n} bits)"}
        phase = {"check_ms_per_step": round(chk_ms.sum() / args.steps, 3),
                 "bit_ms_per_step": round(bit_ms.sum() / args.steps, 3),
                 "bit_achieved_gbs": round(bit_bytes.sum() / (bit_ms.sum() * 1e-3) / 1e9, 1)}
        print(f"[bench] profiled pass done", file=sys.stderr, flush=True)

    engine = None
    if not args.no_engine:
        tries = []
        for sl in [int(x) for x in args.engine_slots.split(",") if x]:
            r = engine_large(torch, ldpc, g, d_llr, T, flags, sl, args.steps, args.warmup)
            ref_it = np.concatenate([o.iters.cpu().numpy() for o in outs])
            same = bool((r["iters"] == ref_it).all())
            tries.append({"slots": r["slots"], "ms_per_step": r["ms_per_step"],
                          "gbits": round(frames_per_step * k / (r["ms_per_step"] * 1e-3) / 1e9, 4),
                          "replays_per_step": r["replays_per_step"], "iters_equal_plain": same})
        engine = {"note": "same 1024 frames per step through the refill engine (ldpc_engine_*); wall clock "
                          "includes submission and host polling", "tries": tries}
        print(f"[bench] engine done", file=sys.stderr, flush=True)

    batched = None
    if not args.no_batched:
        batched = bench_batched(torch, ldpc, max(1, args.steps), args.warmup)
        print(f"[bench] batched done", file=sys.stderr, flush=True)
    served = None
    if not args.no_served:
        cap = 4096.0 / (batched["engine_fp16"]["ms_per_step"] * 1e-3) if batched else 150000.0
        served = bench_served(torch, ldpc, cap, args.served_requests, iters_per_step=args.served_iters_per_step)
        print(f"[bench] served done", file=sys.stderr, flush=True)

    simulate = None
    if not args.no_simulate:
        simulate = bench_simulate(torch, ldpc, code, points, compact=not args.no_compact)
        print(f"[bench] simulate done", file=sys.stderr, flush=True)

    structured = None
    if not args.no_structured:
        structured = bench_structured(torch, ldpc, li, points, F, T, max(1, args.steps), compact=not args.no_compact)
        print(f"[bench] structured done", file=sys.stderr, flush=True)

    minsum = None
    if not args.no_minsum:
        minsum = bench_minsum(torch, ldpc, g, d_llr, cws, points, T, max(1, args.steps))
        print(f"[bench] min-sum done", file=sys.stderr, flush=True)

    precision = None
    if not args.no_precision:
        precision = bench_precision(torch, ldpc)
        print(f"[bench] precision done", file=sys.stderr, flush=True)

    ceiling = copy_ceiling(torch)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(code, llrs, T, args.cpu_frames, args.cpu_frames_1core)
        print(f"[bench] cpu baseline done", file=sys.stderr, flush=True)

    line = {
        "metric": "decoded info Gbit/s (n=64800 r1/2, <=50 it) + %HBM peak; p50/p99 latency",
        "value": round(value, 4),
        "unit": "Gbit/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp16": "f32 math, f16 messages", "bf16": "f32 math, bf16 messages"}[args.msg],
        "data": "synthetic: seeded random irregular code, random codewords (systematic GF(2) encoder, info "
                "seed 3002+i) over BPSK/AWGN, FP32 LLRs",
        "config": {"workload": f"n={n} m={m} E={E} rate-1/2 random irregular LDPC (bit degrees 8/3/2, check "
                               f"degree 7), {F} frames at each Eb/N0 in {points} dB, max {T} iterations, "
                               f"syndrome early stop, {args.msg} messages",
                   "frames_per_step": frames_per_step, "info_bits_per_frame": k,
                   "info_bits_per_frame_n_minus_rank": k_rank},
        "tail_compaction": not args.no_compact,
        "hbm_frac_step": round(hbm_frac, 4),
        "copy_ceiling_gbs": round(ceiling, 1),
        "per_point": per_point,
        "roofline": roofline,
        "phases": phase,
        "engine_same_workload": engine,
        "batched": batched,
        "served": served,
        "precision": precision,
        "simulate": simulate,
        "minsum": minsum,
        "structured": structured,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
