"""GPU tests of the batched engine (continuous refill over several codes).

The engine runs each frame with the same per-frame arithmetic and order as
ldpc_decode, so its outputs must be bit-identical to decoding that frame with
ldpc_decode alone, whatever else shares the launch; the plain path is itself
held to the FP64 oracle (test_gpu_parity.py) and the engine is also checked
against the oracle directly here.
"""
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


def _announce(name, **kw):
    print(f"[case] {name} {kw}", flush=True)


def _engine_decode(codes, llrs, slots, T, flags=0, lane_slots=0, graph_steps=0, want_llr=True, cap=None,
                   repack=True, iters_per_step=0, rule=None, param=None):
    import torch
    from paper_1609_01567_amd import ldpc
    graphs = [ldpc.Graph.from_code(c) for c in codes]
    caps = cap or [max(1, x.shape[0]) for x in llrs]
    eng = ldpc.Engine(graphs, slots, caps, T, flags=flags, lane_slots=lane_slots, graph_steps=graph_steps,
                      repack=repack, iters_per_step=iters_per_step, rule=rule, rule_param=param)
    jobs = [(i, torch.from_numpy(np.ascontiguousarray(x)).cuda()) for i, x in enumerate(llrs)]
    # bound: every frame needs at most T+1 steps once admitted; admissions follow slot turnover
    steps = sum((x.shape[0] // max(1, sl) + 2) * (T + 2) for x, sl in zip(llrs, slots)) + 8
    res = ldpc.decode_batch(eng, jobs, want_llr=want_llr, max_replays=steps)
    torch.cuda.synchronize()
    out = [dict(bits=r.bits.cpu().numpy(), ok=r.ok.cpu().numpy(), iters=r.iters.cpu().numpy(),
                lpost=r.llr.cpu().numpy() if r.llr is not None else None) for r in res]
    eng.close()
    return out


def _assert_same(a, b, what):
    for k in ("bits", "ok", "iters", "lpost"):
        if a.get(k) is None or b.get(k) is None:
            continue
        assert (a[k] == b[k]).all(), f"{what}: {k} differs"


def test_engine_all_frames_at_once_equals_plain():
    code = li.tiny_code()
    llr = li.awgn_llr(code.n, 32, li.ebn0_to_sigma2(2.0, code.rate), seed=2001)
    _announce("engine-once", frames=32)
    eng = _engine_decode([code], [llr], [64], 50)[0]
    plain = gpu_decode(code, llr, 50)
    _assert_same(eng, plain, "engine vs plain")


@pytest.mark.parametrize("lane_slots", [1, 2, 4])
def test_engine_refill_equals_plain(lane_slots):
    code = li.random_small_code(600, 300, 3, seed=8)
    llr = li.awgn_llr(code.n, 700, li.ebn0_to_sigma2(1.2, code.rate), seed=9)
    _announce("engine-refill", frames=700, lane_slots=lane_slots)
    eng = _engine_decode([code], [llr], [64 * lane_slots], 30, lane_slots=lane_slots, graph_steps=5)[0]
    plain = gpu_decode(code, llr, 30)
    _assert_same(eng, plain, "engine refill vs plain")
    compare(code, llr[:96], 30, gpu={k: v[:96] for k, v in eng.items()})


def _mixed_codes():
    rng = np.random.default_rng(11)
    cdeg = np.concatenate([[300, 140, 64, 40, 33], rng.integers(3, 33, size=95)])
    E = int(cdeg.sum())
    bdeg = np.full(700, E // 700)
    bdeg[: E - bdeg.sum()] += 1
    hub = li.socket_code(bdeg, cdeg, seed=12)
    codes = [li.tiny_code(), hub, li.random_small_code(300, 150, 3, seed=31), li.code_14_7()]
    frames = [150, 70, 333, 40]
    snr = [2.0, None, 1.5, None]
    llrs = []
    for i, (c, f) in enumerate(zip(codes, frames)):
        s2 = li.ebn0_to_sigma2(snr[i], c.rate) if snr[i] else 0.7
        llrs.append(li.awgn_llr(c.n, f, s2, seed=50 + i))
    return codes, llrs


@pytest.mark.parametrize("iters_per_step", [2, 3, 4])
def test_engine_iterations_per_step_each_frame_as_alone(iters_per_step):
    """Several decoder iterations between turnovers: frames that stop inside a
    step sit out its remaining passes, and slots refill at step ends (pools
    smaller than the frame counts), over every check-degree class."""
    codes, llrs = _mixed_codes()
    _announce("engine-iters-per-step", iters_per_step=iters_per_step)
    out = _engine_decode(codes, llrs, [64, 64, 128, 64], 25, lane_slots=2, graph_steps=3,
                         iters_per_step=iters_per_step)
    for c, x, o in zip(codes, llrs, out):
        _assert_same(o, gpu_decode(c, x, 25), f"{iters_per_step} iterations per step: {c.name}")


@pytest.mark.parametrize("rule,param,ips", [("ms", None, 1), ("nms", 0.75, 2), ("oms", 0.25, 3)])
def test_engine_min_sum_rules_each_frame_as_alone(rule, param, ips):
    """Min-Sum family rules in the engine, over every check-degree class, with
    slot refill: each frame equals its plain ldpc_decode_rule decode."""
    from paper_1609_01567_amd import ldpc
    codes, llrs = _mixed_codes()
    _announce("engine-min-sum", rule=rule, iters_per_step=ips)
    for flags in (0, ldpc.MSG_FP16, ldpc.MSG_Q8):
        out = _engine_decode(codes, llrs, [64, 64, 128, 64], 25, flags=flags, lane_slots=2, graph_steps=3,
                             iters_per_step=ips, rule=rule, param=param)
        for c, x, o in zip(codes, llrs, out):
            _assert_same(o, gpu_decode(c, x, 25, flags=flags, rule=rule, param=param), f"{rule} {flags}: {c.name}")


def test_engine_iterations_per_step_repack_and_max_iter():
    """Repacking between multi-iteration steps, and max_iter not a multiple of
    the iterations per step (with and without early stop)."""
    from paper_1609_01567_amd import ldpc
    code = li.random_small_code(600, 300, 3, seed=8)
    llr = li.awgn_llr(code.n, 900, li.ebn0_to_sigma2(1.0, code.rate), seed=19)
    _announce("engine-iters-per-step-repack")
    on = _engine_decode([code], [llr], [1024], 40, flags=ldpc.MSG_FP16, graph_steps=2, iters_per_step=3)[0]
    _assert_same(on, gpu_decode(code, llr, 40, flags=ldpc.MSG_FP16), "3 iterations per step, repack")
    small = llr[:100]
    for T in (1, 7):
        eng = _engine_decode([code], [small], [64], T, flags=ldpc.NO_EARLY_STOP, iters_per_step=4)[0]
        assert (eng["iters"] == T).all()
        _assert_same(eng, gpu_decode(code, small, T, flags=ldpc.NO_EARLY_STOP), f"T={T}, 4 per step")


def test_engine_mixed_codes_each_frame_as_alone():
    """Uneven codes (all check-degree classes, rows up to 300 edges) in one engine."""
    rng = np.random.default_rng(11)
    cdeg = np.concatenate([[300, 140, 64, 40, 33], rng.integers(3, 33, size=95)])
    E = int(cdeg.sum())
    bdeg = np.full(700, E // 700)
    bdeg[: E - bdeg.sum()] += 1
    hub = li.socket_code(bdeg, cdeg, seed=12)
    codes = [li.tiny_code(), hub, li.random_small_code(300, 150, 3, seed=31), li.code_14_7()]
    frames = [150, 70, 333, 40]
    snr = [2.0, None, 1.5, None]
    llrs = []
    for i, (c, f) in enumerate(zip(codes, frames)):
        s2 = li.ebn0_to_sigma2(snr[i], c.rate) if snr[i] else 0.7
        llrs.append(li.awgn_llr(c.n, f, s2, seed=50 + i))
    _announce("engine-mixed", frames=frames)
    out = _engine_decode(codes, llrs, [64, 64, 128, 64], 25, graph_steps=3)
    for c, x, o in zip(codes, llrs, out):
        _assert_same(o, gpu_decode(c, x, 25), f"mixed {c.name}")
    compare(codes[1], llrs[1], 25, gpu=out[1])


@pytest.mark.parametrize("msg", ["fp16", "bf16"])
def test_engine_reduced_precision_equals_plain(msg):
    from paper_1609_01567_amd import ldpc
    flag = ldpc.MSG_FP16 if msg == "fp16" else ldpc.MSG_BF16
    code = li.random_small_code(500, 250, 3, seed=5)
    llr = li.awgn_llr(code.n, 300, li.ebn0_to_sigma2(1.5, code.rate), seed=6)
    _announce("engine-precision", msg=msg)
    eng = _engine_decode([code], [llr], [128], 40, flags=flag)[0]
    plain = gpu_decode(code, llr, 40, flags=flag)
    _assert_same(eng, plain, f"engine {msg} vs plain")


def test_engine_no_early_stop_and_max_iter_one():
    from paper_1609_01567_amd import ldpc
    code = li.tiny_code()
    llr = li.awgn_llr(code.n, 100, li.ebn0_to_sigma2(1.5, code.rate), seed=3)
    _announce("engine-no-early-stop")
    for T in (1, 7):
        eng = _engine_decode([code], [llr], [64], T, flags=ldpc.NO_EARLY_STOP)[0]
        assert (eng["iters"] == T).all()
        _assert_same(eng, gpu_decode(code, llr, T, flags=ldpc.NO_EARLY_STOP), f"no early stop T={T}")


def test_engine_queue_backpressure_and_incremental_submit():
    import torch
    from paper_1609_01567_amd import ldpc
    code = li.random_small_code(300, 150, 3, seed=31)
    llr = li.awgn_llr(code.n, 200, li.ebn0_to_sigma2(1.5, code.rate), seed=77)
    _announce("engine-backpressure")
    g = ldpc.Graph.from_code(code)
    eng = ldpc.Engine([g], [64], [50], 30, graph_steps=2)
    x = torch.from_numpy(llr).cuda()
    bits = torch.empty((200, code.n), dtype=torch.uint8, device="cuda")
    ok = torch.empty(200, dtype=torch.uint8, device="cuda")
    it = torch.empty(200, dtype=torch.int32, device="cuda")
    done = torch.zeros(1, dtype=torch.int32, device="cuda")
    fr = ldpc.frames_for(x, bits, ok, it, done=done)
    with pytest.raises(ldpc.LdpcError):
        eng.submit(0, fr[:51])                     # more than the queue holds
    sent = 0
    for _ in range(400):                          # bounded: the loop must not spin forever
        if sent >= 200:
            break
        free = eng.capacity(0)
        k = min(free, 200 - sent)
        if k > 0:
            eng.submit(0, fr[sent:sent + k])
            sent += k
        eng.step(1)
        eng.poll()
    assert sent == 200
    eng.run(max_replays=400)
    torch.cuda.synchronize()
    assert int(done.item()) == 200
    ref = gpu_decode(code, llr, 30)
    assert (bits.cpu().numpy() == ref["bits"]).all()
    assert (it.cpu().numpy() == ref["iters"]).all() and (ok.cpu().numpy() == ref["ok"]).all()
    r, p = eng.poll()
    assert r.tolist() == [200] and p.tolist() == [0]
    eng.close()


@pytest.mark.parametrize("lane_slots", [1, 2, 4])
@pytest.mark.parametrize("msg", ["fp32", "fp16"])
def test_engine_repack_equals_plain(lane_slots, msg):
    """All frames admitted at once into a large pool: as frames finish, the
    scattered survivors are repacked into the low slots again and again."""
    from paper_1609_01567_amd import ldpc
    flags = {"fp32": 0, "fp16": ldpc.MSG_FP16}[msg]
    code = li.random_small_code(600, 300, 3, seed=8)
    llr = li.awgn_llr(code.n, 900, li.ebn0_to_sigma2(1.0, code.rate), seed=19)
    _announce("engine-repack", frames=900, lane_slots=lane_slots, msg=msg)
    on = _engine_decode([code], [llr], [1024], 40, flags=flags, lane_slots=lane_slots, graph_steps=3)[0]
    off = _engine_decode([code], [llr], [1024], 40, flags=flags, lane_slots=lane_slots, graph_steps=3,
                         repack=False)[0]
    plain = gpu_decode(code, llr, 40, flags=flags)
    assert len(set(on["iters"].tolist())) > 10     # a spread of stopping iterations
    _assert_same(on, off, "repack vs no repack")
    _assert_same(on, plain, "repack vs plain")


@pytest.mark.parametrize("lane_slots", [2, 4])
@pytest.mark.parametrize("msg", ["fp32", "fp16"])
def test_engine_chunked_rows_drained_pools_equal_plain(lane_slots, msg):
    """Rows of 17..64 edges (the chunked class).  A pool whose extent is at most
    32 V slots runs them at one slot per lane: here one graph starts that way
    (40 frames), and one gets there by finishing and repacking (700 frames)."""
    from paper_1609_01567_amd import ldpc
    flags = {"fp32": 0, "fp16": ldpc.MSG_FP16}[msg]
    rng = np.random.default_rng(23)
    cdeg = rng.integers(17, 65, size=150)
    E = int(cdeg.sum())
    bdeg = np.full(1500, E // 1500)
    bdeg[: E - bdeg.sum()] += 1
    code = li.socket_code(bdeg, cdeg, seed=24)
    assert int(cdeg.min()) > 16
    small = li.awgn_llr(code.n, 40, li.ebn0_to_sigma2(4.0, code.rate), seed=25)
    big = li.awgn_llr(code.n, 700, li.ebn0_to_sigma2(4.0, code.rate), seed=26)
    _announce("engine-chunk-drained", lane_slots=lane_slots, msg=msg)
    out = _engine_decode([code, code], [small, big], [256, 768], 30, flags=flags, lane_slots=lane_slots,
                         graph_steps=2, iters_per_step=2)
    for x, o, what in ((small, out[0], "40 frames"), (big, out[1], "700 frames")):
        plain = gpu_decode(code, x, 30, flags=flags)
        _assert_same(o, plain, f"{what}: engine vs plain")
    assert len(set(out[1]["iters"].tolist())) > 5


def test_engine_repack_with_long_rows_and_many_graphs():
    """Repacking under rows of every class (the >128-edge path keeps per-slot
    scratch) and with 16 graphs in one engine (counters of every graph)."""
    rng = np.random.default_rng(11)
    cdeg = np.concatenate([[300, 140, 64, 40, 33], rng.integers(3, 33, size=95)])
    E = int(cdeg.sum())
    bdeg = np.full(700, E // 700)
    bdeg[: E - bdeg.sum()] += 1
    hub = li.socket_code(bdeg, cdeg, seed=12)
    codes = [hub] + [li.random_small_code(200 + 40 * i, 100 + 20 * i, 3, seed=60 + i) for i in range(15)]
    llrs = [li.awgn_llr(hub.n, 150, 0.7, seed=13)]
    llrs += [li.awgn_llr(c.n, 40 + 7 * i, li.ebn0_to_sigma2(1.0, c.rate), seed=80 + i)
             for i, c in enumerate(codes[1:])]
    _announce("engine-repack-16-graphs", frames=sum(x.shape[0] for x in llrs))
    slots = [256] * len(codes)
    on = _engine_decode(codes, llrs, slots, 25, lane_slots=2, graph_steps=4)
    off = _engine_decode(codes, llrs, slots, 25, lane_slots=2, graph_steps=4, repack=False)
    for i, (c, x) in enumerate(zip(codes, llrs)):
        plain = gpu_decode(c, x, 25)
        _assert_same(on[i], off[i], f"graph {i}: repack vs no repack")
        _assert_same(on[i], plain, f"graph {i}: engine vs plain")


def _long_rows_code():
    """Rows just inside and beyond the 512-edge limit of the LDS path, and far
    beyond it (segmented path), among short rows."""
    rng = np.random.default_rng(31)
    cdeg = np.concatenate([[1200, 700, 513, 512, 300, 129], rng.integers(3, 12, size=200)])
    E = int(cdeg.sum())
    n = 1500
    bdeg = np.full(n, E // n)
    bdeg[: E - bdeg.sum()] += 1
    return li.socket_code(bdeg, cdeg, seed=32)


@pytest.mark.parametrize("msg", ["fp32", "fp16", "bf16"])
def test_engine_segmented_and_wide_rows_equal_plain(msg):
    """The engine's long-row kernels (16-wavefront rows up to 512 edges and the
    segmented path beyond) against the plain decoder, with repacking and several
    iterations per step, in every floating-point message format."""
    from paper_1609_01567_amd import ldpc
    flags = {"fp32": 0, "fp16": ldpc.MSG_FP16, "bf16": ldpc.MSG_BF16}[msg]
    code = _long_rows_code()
    assert code.check_degrees().max() == 1200
    llr = li.awgn_llr(code.n, 200, li.ebn0_to_sigma2(6.0, code.rate), seed=33)
    _announce("engine-long-rows", msg=msg, frames=200)
    eng = _engine_decode([code], [llr], [128], 20, flags=flags, iters_per_step=2)[0]
    plain = gpu_decode(code, llr, 20, flags=flags)
    _assert_same(eng, plain, f"engine {msg} long rows vs plain")
    assert len(np.unique(plain["iters"])) >= 2     # frames leave and enter at different steps
