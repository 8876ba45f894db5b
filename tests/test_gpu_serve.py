"""GPU tests of the amplitude server (continuous admission by HBM footprint).

Requests are seeded random-circuit amplitudes of uneven size.  Each result
is checked against the oracle, and every request's amplitude must be the
same bits whether it ran alone or among others.
"""
import sys
import threading
import time

import numpy as np
import pytest

import oracle
from workloads import circuits, configs, paths, rng

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def mini_request(i, seed=8800):
    """Small stand-in of the serving workload: 9-20 sites, 4-9 cycles, sliced
    to max rank <= 12 (the oracle checks these quickly)."""
    r = rng.SplitMix64(seed + i)
    n = r.randint(9, 20)
    cycles = r.randint(4, 9)
    rows, cols = circuits.grid_shape(n)
    return configs.circuit_workload(rows, cols, cycles, seed * 7 + i, max_rank=12, n_sites=n,
                                    restarts=2)


@pytest.fixture(scope="module")
def requests_():
    return [mini_request(i) for i in range(12)]


@pytest.fixture(scope="module")
def oracle_amps(requests_):
    out = []
    for w in requests_:
        a, _ = oracle.contract_network(w.network.tensors, w.network.labels, w.path, w.sliced)
        out.append(complex(a))
    return out


def submit(srv, w, mode):
    return srv.submit(w.network.tensors, w.network.labels, w.path, w.sliced, mode)


@pytest.mark.parametrize("mode", ["fp64", "fp32_4m"])
def test_server_results_match_oracle(requests_, oracle_amps, mode):
    import paper_2201_06620_amd as rn
    tol = 1e-12 if mode == "fp64" else 1e-5
    srv = rn.Server(0, hbm_budget=1 << 30, max_active=4)
    tickets = [submit(srv, w, mode) for w in requests_]
    for w, t, ref in zip(requests_, tickets, oracle_amps):
        res = srv.wait(t)
        assert res["status"] == 0
        err = abs(res["amp"] - ref) / max(abs(ref), 2.0 ** (-w.circuit.n / 2))
        assert err < tol, (w.meta, err)
        assert res["latency_s"] >= res["run_s"] >= 0
    srv.close()


def overlapping_pairs(results):
    """Pairs of requests whose running intervals [start, done] overlap."""
    n = 0
    for i in range(len(results)):
        for j in range(i + 1, len(results)):
            a, b = results[i], results[j]
            if a["start_s"] < b["done_s"] and b["start_s"] < a["done_s"]:
                n += 1
    return n


def test_alone_equals_in_mix(requests_):
    import paper_2201_06620_amd as rn
    srv = rn.Server(0, hbm_budget=1 << 30, max_active=4)
    alone = []
    for w in requests_:
        alone.append(srv.wait(submit(srv, w, "fp32_4m"))["amp"])
    # A burst: every request queued at once, so up to four run at the same
    # time on their slots; the run intervals must overlap, and every
    # amplitude must be the same bits as alone.
    tk = [submit(srv, w, "fp32_4m") for w in requests_]
    burst = [srv.wait(t) for t in tk]
    pairs = overlapping_pairs(burst)
    log(f"  burst: {pairs} overlapping pairs of running requests")
    assert pairs > 0
    for i, r in enumerate(burst):
        assert r["status"] == 0 and r["amp"] == alone[i], i
    # The same requests again, arriving as a Poisson stream from another
    # thread while earlier ones are still on the GPU, in a shuffled order.
    order = rng.SplitMix64(5).permutation(len(requests_))
    tickets = {}
    gaps = np.random.default_rng(3).exponential(0.002, size=len(order))

    def client():
        for g, i in zip(gaps, order):
            time.sleep(g)
            tickets[i] = submit(srv, requests_[i], "fp32_4m")

    th = threading.Thread(target=client)
    th.start()
    th.join()
    for i in order:
        res = srv.wait(tickets[i])
        assert res["status"] == 0
        assert res["amp"] == alone[i], i
    srv.close()


@pytest.mark.parametrize("policy", ["fifo", "smallest", "aged"])
def test_admission_order(policy):
    # One slot: a large request runs first; a big and a small one arrive
    # while it runs.  Arrival order admits the big one next; smallest-first
    # admits the small one first; with max_overtakes = 0 every waiting
    # request counts as aged, which is arrival order again.
    import paper_2201_06620_amd as rn
    blocker = configs.config5_request(0, 16)              # ~1.4e13 flops
    big = configs.circuit_workload(5, 6, 10, 9191, max_rank=24, restarts=1)
    small = configs.circuit_workload(2, 3, 4, 9192, restarts=1)
    srv = rn.Server(0, hbm_budget=16 << 30, max_active=1)
    if policy == "fifo":
        srv.set_admission("fifo")
    elif policy == "aged":
        srv.set_admission("smallest", 0)
    t0 = submit(srv, blocker, "fp32_4m")
    t1 = submit(srv, big, "fp32_4m")
    t2 = submit(srv, small, "fp32_4m")
    r0, r1, r2 = srv.wait(t0), srv.wait(t1), srv.wait(t2)
    srv.close()
    assert r0["status"] == r1["status"] == r2["status"] == 0
    sub1, sub2 = r1["start_s"] - r1["queue_s"], r2["start_s"] - r2["queue_s"]
    log(f"  {policy}: blocker done {r0['done_s']:.4f}s, big submitted {sub1:.4f}s start "
        f"{r1['start_s']:.4f}s, small submitted {sub2:.4f}s start {r2['start_s']:.4f}s")
    assert max(sub1, sub2) < r0["done_s"], "both arrived while the blocker ran"
    if policy == "smallest":
        assert r2["start_s"] < r1["start_s"]
    else:
        assert r1["start_s"] < r2["start_s"]


def test_request_over_budget_is_rejected():
    import paper_2201_06620_amd as rn
    w = configs.circuit_workload(4, 4, 8, 123, max_rank=30, restarts=1)
    big = rn.Server(0, hbm_budget=1 << 30, max_active=1)
    fp = big.wait(submit(big, w, "fp64"))["footprint"]
    big.close()
    srv = rn.Server(0, hbm_budget=int(fp) // 2, max_active=2)
    res = srv.wait(submit(srv, w, "fp64"))
    assert res["status"] == 5  # RN_ERR_OOM: can never fit the budget
    small = configs.circuit_workload(2, 3, 4, 124, restarts=1)
    res2 = srv.wait(submit(srv, small, "fp64"))
    assert res2["status"] == 0
    srv.close()


def test_admission_respects_budget(requests_):
    # Budget for roughly two requests at a time: all still complete, and the
    # server never holds more than the budget.
    import paper_2201_06620_amd as rn
    srv = rn.Server(0, hbm_budget=64 << 20, max_active=4)
    tickets = [submit(srv, w, "fp64") for w in requests_]
    peak = 0
    done = 0
    t0 = time.time()
    while done < len(tickets) and time.time() - t0 < 60:
        st = srv.stats()
        peak = max(peak, st["bytes_in_use"])
        done = st["completed"]
        time.sleep(0.0005)
    for t in tickets:
        assert srv.wait(t)["status"] == 0
    assert peak <= 64 << 20
    srv.close()


def test_sliced_request_fitted_to_budget():
    # A sliced request whose all-batched footprint exceeds the budget runs
    # with fewer slices batched per pass instead of being refused.
    import paper_2201_06620_amd as rn
    w = configs.circuit_workload(3, 4, 10, 4242, n_slices=5, restarts=2)
    ref, _ = oracle.contract_network(w.network.tensors, w.network.labels, w.path, w.sliced)
    ref = complex(ref)
    big = rn.Server(0, hbm_budget=1 << 30, max_active=1)
    full = big.wait(submit(big, w, "fp64"))
    big.close()
    assert full["status"] == 0
    budget = int(full["footprint"]) * 3 // 4
    srv = rn.Server(0, hbm_budget=budget, max_active=2)
    res = srv.wait(submit(srv, w, "fp64"))
    srv.close()
    log(f"  footprint all-batched={full['footprint']:.0f} fitted={res['footprint']:.0f}")
    assert res["status"] == 0
    assert res["footprint"] <= budget
    assert abs(res["amp"] - ref) / max(abs(ref), 2.0 ** (-w.circuit.n / 2)) < 1e-12


def fullsize_requests(count=3, scan=32):
    """Serving-workload requests at their real size for the oracle check: the
    first `count` of the first `scan` requests with at least 40 sites, at
    least 2 sliced bonds and at most 6e9 flops per slice (so the oracle
    finishes a slice in seconds), each checked on its own slicing."""
    out = []
    for i in range(scan):
        w = configs.config5_request(0, i)
        if (w.meta["sites"] >= 40 and len(w.sliced) >= 2
                and w.meta["flops_per_slice"] <= 6e9):
            out.append((i, w))
            if len(out) == count:
                break
    assert len(out) == count
    return out


@pytest.fixture(scope="module")
def fullsize():
    return fullsize_requests()


@pytest.mark.parametrize("mode", ["fp32_4m", "fp64"])
def test_serving_requests_at_full_size_per_slice_vs_oracle(fullsize, mode):
    # Config-5 requests (40-50 sites, 8-10 cycles, 4-6 sliced bonds) through
    # rn_contract_network with per-slice values: the first and the last slice
    # of each are compared with the oracle's single-slice projection (slice-
    # subsampled: the other slices are checked only through the FP64 sum).
    # FP32-4M on all three requests, FP64 on the first.
    import torch
    import paper_2201_06620_amd as rn
    ctx = rn.Context(0)
    tol = 1e-12 if mode == "fp64" else 1e-5
    dt = torch.complex128 if mode == "fp64" else torch.complex64
    picks = fullsize[:1] if mode == "fp64" else fullsize
    for i, w in picks:
        net, S = w.network, len(w.sliced)
        log(f"request {i}: {w.meta['sites']} sites, {w.meta['cycles']} cycles, {S} sliced, "
            f"max rank {w.meta['max_rank']}, {w.meta['flops_per_slice']:.3g} flops/slice")
        ts = [torch.from_numpy(np.ascontiguousarray(t.reshape(-1))).to(dt).cuda()
              for t in net.tensors]
        sl = torch.zeros(2 << S, dtype=torch.float64, device="cuda")
        amp = ctx.contract_network(ts, net.labels, w.path, w.sliced, mode, slices=sl)
        torch.cuda.synchronize()
        got = sl.cpu().numpy().view(np.complex128)
        which = [0, (1 << S) - 1]
        ref = oracle.contract_network_slices(net.tensors, net.labels, w.path, w.sliced, which)
        # Amplitude scale 2^(-n/2), spread over 2^S slices of random phase.
        scale = 2.0 ** (-(w.meta["sites"] + S) / 2)
        for s, r in zip(which, ref):
            err = abs(got[s] - r) / max(abs(r), scale)
            log(f"  slice {s}: |a| = {abs(r):.3e}, e_amp = {err:.3e}")
            assert err < tol, (i, s, err)
        a = amp.cpu().numpy()
        assert abs(complex(a[0], a[1]) - np.sum(got)) <= 1e-14 * max(np.sum(np.abs(got)), 1e-300)
