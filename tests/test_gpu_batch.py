"""GPU parity of batched block tensordots, autotuned tiles and graph replay.

The uneven batch (256 problems, operand ranks 8-24, 2-10 contracted axes,
output rank <= 24, blocked on the first three axes) is checked on sampled
outputs of every problem against the oracle; a smaller batch is checked
whole.  Normal inputs: e_F and e_max within the mode's tolerance and every
compared entry within its rounding bound (tests/parity.py).  Graph replays
are compared bit for bit with the eager run.
"""
import sys

import numpy as np
import pytest

import oracle
import parity
from workloads import circuits, configs, paths, rng

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2201_06620_amd as rn
    assert torch.cuda.is_available()
    return rn.Context(0)


def to_dev(x, mode):
    import torch
    dt = torch.complex128 if mode == "fp64" else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(x)).to(dt).to("cuda")


def dense(op):
    return oracle.from_blocked(op.data, op.dims, op.grid)


def blocked_flat_index(dims, grid, flat_dense):
    # Position in C's block-major buffer of dense (row-major) index flat_dense.
    flat_dense = np.asarray(flat_dense, dtype=np.int64)
    if len(dims) == 0:
        return np.zeros_like(flat_dense)
    idx = np.array(np.unravel_index(flat_dense, dims)).T
    ext = np.array(dims) // np.array(grid)
    bcoord, icoord = idx // ext, idx % ext
    blin = np.ravel_multi_index(tuple(bcoord.T), grid)
    ilin = np.ravel_multi_index(tuple(icoord.T), tuple(ext))
    return blin * int(np.prod(ext)) + ilin


def small_batch(count=24, seed=5150, integer=False):
    r = rng.SplitMix64(seed)
    probs = []
    while len(probs) < count:
        ra, rb, k = r.randint(3, 12), r.randint(3, 12), r.randint(0, 6)
        if k > min(ra, rb) or ra + rb - 2 * k > 14:
            continue
        axa, axb = r.sample(ra, k), r.sample(rb, k)
        probs.append(configs.make_problem(ra, rb, axa, axb, configs.split_first(ra),
                                          configs.split_first(rb), seed + 31 * len(probs),
                                          integer))
    return probs


def run_batch(ctx, probs, mode, autotune=False, workspace=None, outs=None):
    import torch
    items = [(to_dev(p.a.data, mode), p.a.dims, p.a.grid, to_dev(p.b.data, mode), p.b.dims,
              p.b.grid, p.axes_a, p.axes_b) for p in probs]
    res, fl = ctx.block_tensordot_batch(items, mode, autotune=autotune, workspace=workspace,
                                        outs=outs)
    torch.cuda.synchronize()
    return items, res


@pytest.mark.parametrize("mode", ["fp64", "fp32_4m", "fp32_3m", "bf16x3"])
def test_small_batch_full(ctx, mode):
    probs = small_batch()
    _, res = run_batch(ctx, probs, mode)
    for i, (p, (c, cd, cg)) in enumerate(zip(probs, res)):
        ref, rd, rg = oracle.block_tensordot(p.a.data, p.a.dims, p.a.grid, p.b.data, p.b.dims,
                                             p.b.grid, p.axes_a, p.axes_b)
        assert cd == rd and cg == rg
        got = c.cpu().numpy().astype(np.complex128)
        parity.check(got, ref, parity.abs_product_blocked(p), 2 ** p.k, mode, f"problem {i}")


@pytest.mark.parametrize("mode", ["fp64", "fp32_4m", "bf16x3"])
def test_small_batch_integers_bitwise_and_autotune(ctx, mode, tmp_path):
    probs = small_batch(16, seed=6161, integer=True)
    _, res = run_batch(ctx, probs, mode, autotune=True)
    for p, (c, _, _) in zip(probs, res):
        ref, _, _ = oracle.block_tensordot(p.a.data, p.a.dims, p.a.grid, p.b.data, p.b.dims,
                                           p.b.grid, p.axes_a, p.axes_b)
        assert np.array_equal(c.cpu().numpy().astype(np.complex128), ref)
    f = str(tmp_path / "tune.txt")
    ctx.tune_save(f)
    text = open(f).read()
    assert text.startswith("rn_tune 1") and len(text.splitlines()) > 1
    ctx.tune_clear()
    ctx.tune_load(f)


def test_config4_sampled(ctx):
    import torch
    log("config4: generating 256 problems")
    probs = configs.config4()
    assert len(probs) == 256
    _, res = run_batch(ctx, probs, "fp32_4m", autotune=True)
    rs = np.random.default_rng(44)
    worst = 0.0
    for i, (p, (c, cd, cg)) in enumerate(zip(probs, res)):
        n = int(np.prod(cd)) if cd else 1
        idx = np.unique(rs.integers(0, n, size=min(n, 48)))
        da, db = dense(p.a), dense(p.b)
        ref = oracle.tensordot_entries(da, db, p.axes_a, p.axes_b, idx)
        absprod = parity.abs_product_entries(da, db, p.axes_a, p.axes_b, idx)
        pos = torch.from_numpy(blocked_flat_index(cd, cg, idx)).to("cuda")
        got = c[pos].cpu().numpy().astype(np.complex128)
        r = parity.check(got, ref, absprod, 2 ** p.k, "fp32_4m", f"problem {i}")
        worst = max(worst, r["e_F"])
    log(f"config4 worst sampled e_F = {worst:.3e}")


def test_batch_graph_replay_matches_eager(ctx):
    import torch
    probs = small_batch(20, seed=777)
    items = [(to_dev(p.a.data, "fp32_4m"), p.a.dims, p.a.grid, to_dev(p.b.data, "fp32_4m"),
              p.b.dims, p.b.grid, p.axes_a, p.axes_b) for p in probs]
    side = torch.cuda.Stream()
    ws = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    ctx.set_graphs(False)
    eager, _ = ctx.block_tensordot_batch(items, "fp32_4m", workspace=ws)
    torch.cuda.synchronize()
    eager = [c.clone() for c, _, _ in eager]
    ctx.set_graphs(True)
    outs = [torch.empty_like(c) for c in eager]
    for rep in range(4):      # direct, capture, then replays
        for o in outs:
            o.zero_()
        with torch.cuda.stream(side):
            ctx.block_tensordot_batch(items, "fp32_4m", workspace=ws, outs=outs)
        side.synchronize()
        scratch = torch.randn(1 << 20, device="cuda").sum()   # eager work in between
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            assert torch.equal(o, e), rep


def test_network_graph_replay_matches_eager(ctx):
    import torch
    circ = circuits.random_circuit(3, 4, 8, seed=91)
    net = circuits.circuit_network(circ, circuits.random_bitstring(12, 92))
    path = paths.greedy_path(net.labels, 93, restarts=2)
    sliced = paths.greedy_slices(net.labels, path, 94, n_slices=3)
    ts = [torch.from_numpy(np.ascontiguousarray(t.reshape(-1))).to("cuda")
          for t in net.tensors]
    ws_n, _, _ = ctx.contract_network_plan(ts, net.labels, path, sliced, "fp64")
    ws = torch.empty(max(ws_n, 1), dtype=torch.uint8, device="cuda")
    ctx.set_graphs(False)
    eager = ctx.contract_network(ts, net.labels, path, sliced, "fp64", workspace=ws).clone()
    torch.cuda.synchronize()
    ctx.set_graphs(True)
    side = torch.cuda.Stream()
    amp = torch.zeros(2, dtype=torch.float64, device="cuda")
    for rep in range(4):
        amp.zero_()
        with torch.cuda.stream(side):
            ctx.contract_network(ts, net.labels, path, sliced, "fp64", amp=amp, workspace=ws)
        side.synchronize()
        torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.equal(amp, eager), rep


def test_prepared_batch_replays_new_values(ctx):
    # A prepared batch on a side stream runs directly, is captured, then
    # replayed without planning; operands rewritten in place before every
    # call must show up in every result (Gaussian integers: bit-exact).
    import torch
    import paper_2201_06620_amd as rn
    probs = small_batch(12, seed=4242, integer=True)
    items = [(to_dev(p.a.data, "fp32_4m"), p.a.dims, p.a.grid, to_dev(p.b.data, "fp32_4m"),
              p.b.dims, p.b.grid, p.axes_a, p.axes_b) for p in probs]
    side = torch.cuda.Stream()
    ctx.set_graphs(True)
    pb = ctx.prepare_batch(items, "fp32_4m")
    for rep in range(4):
        log(f"prepared batch call {rep}")
        rs = np.random.default_rng(99 + rep)
        news = []
        for (a, _, _, b, _, _, _, _), p in zip(items, probs):
            na = rs.integers(-8, 9, a.numel()) + 1j * rs.integers(-8, 9, a.numel())
            nb = rs.integers(-8, 9, b.numel()) + 1j * rs.integers(-8, 9, b.numel())
            a.copy_(torch.from_numpy(na).to(torch.complex64))
            b.copy_(torch.from_numpy(nb).to(torch.complex64))
            news.append((na, nb))
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            outs = pb.run()
        side.synchronize()
        for p, (na, nb), o in zip(probs, news, outs):
            ref, _, _ = oracle.block_tensordot(na, p.a.dims, p.a.grid, nb, p.b.dims, p.b.grid,
                                               p.axes_a, p.axes_b)
            assert np.array_equal(o.cpu().numpy().astype(np.complex128), ref), rep
    # A call that differs only in a too small workspace size is planned
    # again (no replay) and refused.
    pb.wn = 256
    with pytest.raises(rn.RnError):
        with torch.cuda.stream(side):
            pb.run()
    side.synchronize()


@pytest.mark.parametrize("mode", ["fp64", "fp32_4m", "fp32_3m", "bf16x3"])
def test_batch_split_k_every_mode(ctx, mode):
    # Problems with few output tiles and a long K split K inside a batch
    # (partials reduced in ascending order afterwards): 16 x 16 and 32 x 64
    # outputs with K = 1024 and 512, beside one that does not split.
    r = rng.SplitMix64(9090)
    shapes = [(14, 14, 10), (14, 15, 9), (10, 9, 3)]
    for integer in (False, True):
        probs = [configs.make_problem(ra, rb, r.sample(ra, k), r.sample(rb, k),
                                      configs.split_first(ra), configs.split_first(rb),
                                      9100 + 7 * i, integer)
                 for i, (ra, rb, k) in enumerate(shapes)]
        _, res = run_batch(ctx, probs, mode)
        for p, (c, cd, cg) in zip(probs, res):
            ref, rd, rg = oracle.block_tensordot(p.a.data, p.a.dims, p.a.grid, p.b.data,
                                                 p.b.dims, p.b.grid, p.axes_a, p.axes_b)
            got = c.cpu().numpy().astype(np.complex128)
            if integer:
                assert np.array_equal(got, ref), mode
            else:
                parity.check(got, ref, parity.abs_product_blocked(p), 2 ** p.k, mode, "split-K")


@pytest.mark.parametrize("mode", ["fp64", "fp32_4m"])
def test_batch_more_problems_than_one_search_round(ctx, mode):
    # 4500 tiny problems (operand ranks 2-7, 0-3 contracted axes): the grouped
    # permute and GEMM launches hold more than 4096 jobs, so every workgroup
    # finds its job by the binary search over the prefix sums instead of the
    # two 64-wide probe rounds.  Gaussian integers: every output bit-exact.
    r = rng.SplitMix64(4500)
    probs = []
    while len(probs) < 4500:
        ra, rb, k = r.randint(2, 7), r.randint(2, 7), r.randint(0, 3)
        if k > min(ra, rb) or ra + rb - 2 * k > 8:
            continue
        axa, axb = r.sample(ra, k), r.sample(rb, k)
        probs.append(configs.make_problem(ra, rb, axa, axb, configs.split_first(ra, 1),
                                          configs.split_first(rb, 1), 90000 + len(probs),
                                          integer=True))
    log(f"{mode}: batch of {len(probs)} problems")
    _, res = run_batch(ctx, probs, mode)
    for i, (p, (c, cd, cg)) in enumerate(zip(probs, res)):
        ref, rd, rg = oracle.block_tensordot(p.a.data, p.a.dims, p.a.grid, p.b.data, p.b.dims,
                                             p.b.grid, p.axes_a, p.axes_b)
        assert cd == rd and cg == rg, i
        assert np.array_equal(c.cpu().numpy().astype(np.complex128), ref), (mode, i)


def test_empty_batch_enqueues_nothing(ctx):
    # n = 0 through the C ABI: OK, nothing launched, no workspace needed.
    import torch
    import paper_2201_06620_amd as rn
    s = torch.cuda.current_stream().cuda_stream
    assert rn.lib().rn_block_tensordot_batch(ctx.h, 0, None, None, None, None, None, None, 1,
                                             None, 0, s) == 0
    torch.cuda.synchronize()
