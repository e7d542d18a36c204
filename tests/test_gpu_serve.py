"""GPU tests of the serving loop (continuous batching over the engine).

Each request's result must be bit-identical to decoding its frames alone with
ldpc_decode, whatever else is in flight; admission must respect the device
memory budget.  Every wait is bounded so a lost request fails the test.
"""
import threading
import time

import numpy as np
import pytest

import ldpc_inputs as li
from parity import gpu_decode

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")


def _codes():
    return [li.tiny_code(), li.random_small_code(600, 300, 3, seed=8), li.code_14_7()]


def _requests(codes, count, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(count):
        gi = int(rng.integers(len(codes)))
        c = codes[gi]
        F = int(rng.integers(1, 65))
        llr = li.awgn_llr(c.n, F, li.ebn0_to_sigma2(1.6, c.rate) if c.n > 14 else 0.7, seed=seed * 1000 + r)
        reqs.append((gi, llr))
    return reqs


def _drain(srv, ids, deadline_s=60.0):
    out = {}
    t0 = time.time()
    while len(out) < len(ids):
        assert time.time() - t0 < deadline_s, f"only {len(out)}/{len(ids)} requests finished"
        for rid in srv.poll(wait_ms=50):
            out[rid] = srv.result(rid)
    return out


@pytest.mark.parametrize("iters_per_step", [1, 4])
def test_served_results_equal_alone(iters_per_step):
    from paper_1609_01567_amd import ldpc
    codes = _codes()
    graphs = [ldpc.Graph.from_code(c) for c in codes]
    srv = ldpc.Server(graphs, [128, 128, 64], 30, graph_steps=2, iters_per_step=iters_per_step)
    reqs = _requests(codes, 60, seed=1)
    print(f"[case] serve-mix requests={len(reqs)} iters_per_step={iters_per_step}", flush=True)
    ids = [srv.submit(gi, llr) for gi, llr in reqs]
    res = _drain(srv, ids)
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs) and st["waiting"] == 0 and st["in_flight"] == 0
    for rid, (gi, llr) in zip(ids, reqs):
        bits, ok, iters, lat = res[rid]
        ref = gpu_decode(codes[gi], llr, 30)
        assert (bits == ref["bits"]).all() and (ok == ref["ok"]).all() and (iters == ref["iters"]).all(), rid
        assert lat > 0


def test_served_min_sum_results_equal_alone():
    from paper_1609_01567_amd import ldpc
    codes = _codes()
    graphs = [ldpc.Graph.from_code(c) for c in codes]
    srv = ldpc.Server(graphs, [128, 128, 64], 30, flags=ldpc.MSG_FP16, graph_steps=2, rule="oms", rule_param=0.25)
    reqs = _requests(codes, 40, seed=3)
    print(f"[case] serve-min-sum requests={len(reqs)}", flush=True)
    ids = [srv.submit(gi, llr) for gi, llr in reqs]
    res = _drain(srv, ids)
    srv.close()
    for rid, (gi, llr) in zip(ids, reqs):
        bits, ok, iters, _ = res[rid]
        ref = gpu_decode(codes[gi], llr, 30, flags=ldpc.MSG_FP16, rule="oms", param=0.25)
        assert (bits == ref["bits"]).all() and (ok == ref["ok"]).all() and (iters == ref["iters"]).all(), rid


def test_admission_respects_device_budget():
    from paper_1609_01567_amd import ldpc
    code = li.random_small_code(600, 300, 3, seed=8)
    g = ldpc.Graph.from_code(code)
    per_frame = code.n * 5
    budget = 1 << 20                       # ~ 350 frames of this code at a time
    srv = ldpc.Server([g], [128], 30, hbm_budget=budget, host_budget=1 << 20, graph_steps=2)
    reqs = [(0, li.awgn_llr(code.n, 64, li.ebn0_to_sigma2(1.6, code.rate), seed=500 + r)) for r in range(24)]
    print(f"[case] serve-budget budget={budget} per_frame={per_frame}", flush=True)
    ids = [srv.submit(0, llr) for _, llr in reqs]
    res = _drain(srv, ids)
    st = srv.stats()
    srv.close()
    assert 0 < st["device_bytes_peak"] <= budget
    for rid, (_, llr) in zip(ids, reqs):
        ref = gpu_decode(code, llr, 30)
        assert (res[rid][0] == ref["bits"]).all()
    with pytest.raises(ldpc.LdpcError):
        srv2 = ldpc.Server([g], [128], 30, hbm_budget=budget, host_budget=1 << 20)
        try:
            srv2.submit(0, np.zeros((400, code.n), np.float32))   # can never fit the budget
        finally:
            srv2.close()


def test_concurrent_submitters():
    from paper_1609_01567_amd import ldpc
    codes = _codes()
    graphs = [ldpc.Graph.from_code(c) for c in codes]
    srv = ldpc.Server(graphs, [128, 128, 64], 30, graph_steps=2)
    lists = [_requests(codes, 25, seed=10 + t) for t in range(2)]
    ids = [[], []]
    print("[case] serve-threads", flush=True)

    def client(t):
        for gi, llr in lists[t]:
            ids[t].append(srv.submit(gi, llr))
            time.sleep(0.001)

    th = [threading.Thread(target=client, args=(t,)) for t in range(2)]
    for x in th:
        x.start()
    for x in th:
        x.join(timeout=30)
    res = _drain(srv, ids[0] + ids[1])
    srv.close()
    for t in range(2):
        for rid, (gi, llr) in zip(ids[t], lists[t]):
            ref = gpu_decode(codes[gi], llr, 30)
            assert (res[rid][0] == ref["bits"]).all() and (res[rid][2] == ref["iters"]).all()
