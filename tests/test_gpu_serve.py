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


def test_alone_equals_in_mix(requests_):
    import paper_2201_06620_amd as rn
    srv = rn.Server(0, hbm_budget=1 << 30, max_active=4)
    alone = []
    for w in requests_:
        alone.append(srv.wait(submit(srv, w, "fp32_4m"))["amp"])
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
