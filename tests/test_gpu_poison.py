"""GPU: no kernel reads memory it has not written.  Outputs and workspaces
are filled with NaN bytes (0xFF) before the call -- outside any captured
graph -- and the results must be bit-identical to a run whose outputs and
workspaces were zero-filled, with no NaN anywhere: ragged block tensordots
in every mode (with and without split-K and pair-split partials in the
workspace), a batch, and a sliced network with per-slice values.  Also
checks that the binding refuses mis-sized buffers before any launch."""
import sys

import numpy as np
import pytest

from workloads import circuits, configs, paths, rng

pytestmark = pytest.mark.gpu

MODES = ["fp64", "fp32_4m", "fp32_3m", "bf16x3"]


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2201_06620_amd as rn
    assert torch.cuda.is_available()
    return rn.Context(0)


def dt_of(mode):
    import torch
    return torch.complex128 if mode == "fp64" else torch.complex64


def filled(n, dtype, poison):
    """n elements of dtype, all bytes 0xFF (a NaN pattern) or all zero."""
    import torch
    t = torch.empty(n, dtype=dtype, device="cuda")
    t.view(torch.uint8).fill_(0xFF if poison else 0)
    return t


def problem(seed, ra, rb, k):
    r = rng.SplitMix64(seed)
    axa, axb = r.sample(ra, k), r.sample(rb, k)
    ga = [2 if r.below(3) == 0 else 1 for _ in range(ra)]
    gb = [2 if r.below(3) == 0 else 1 for _ in range(rb)]
    return configs.make_problem(ra, rb, axa, axb, ga, gb, seed)


def run_td(ctx, p, mode, poison):
    import torch
    a = torch.from_numpy(p.a.data).to(dt_of(mode)).cuda()
    b = torch.from_numpy(p.b.data).to(dt_of(mode)).cuda()
    cd, _, ws, _ = ctx.plan_block_tensordot(p.a.dims, p.a.grid, p.b.dims, p.b.grid, p.axes_a,
                                            p.axes_b, mode)
    n = int(np.prod(cd)) if cd else 1
    out = filled(n, dt_of(mode), poison)
    wsb = filled(max(ws, 1), torch.uint8, poison)
    torch.cuda.synchronize()
    c, _, _ = ctx.block_tensordot(a, p.a.dims, p.a.grid, b, p.b.dims, p.b.grid, p.axes_a,
                                  p.axes_b, mode, out=out, workspace=wsb)
    torch.cuda.synchronize()
    return c, ws


# Ragged shapes; (14, 14, 10) has a 16 x 16 output with K = 1024, which splits K.
SHAPES = [(13, 11, 6), (12, 9, 4), (14, 14, 10), (9, 16, 3)]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("shape", SHAPES)
def test_tensordot_poisoned_outputs_and_workspace(ctx, mode, shape):
    import torch
    ra, rb, k = shape
    p = problem(71000 + 37 * ra + rb + k, ra, rb, k)
    log(f"poison tensordot shape={shape} mode={mode}")
    clean, ws = run_td(ctx, p, mode, False)
    dirty, _ = run_td(ctx, p, mode, True)
    assert not torch.isnan(torch.view_as_real(dirty)).any()
    assert torch.equal(clean, dirty)
    log(f"  workspace {ws} bytes")


@pytest.mark.parametrize("mode", ["fp64", "fp32_4m"])
def test_pair_split_partials_poisoned(ctx, mode):
    import torch
    r = rng.SplitMix64(72000)
    ra, rb, k = 12, 12, 5
    axa, axb = r.sample(ra, k), r.sample(rb, k)
    ga, gb = [1] * ra, [1] * rb
    for i in range(3):
        ga[axa[i]] = gb[axb[i]] = 2
    p = configs.make_problem(ra, rb, axa, axb, ga, gb, 72000)
    ctx.set_option("pair_split_threshold", 8)
    try:
        clean, ws = run_td(ctx, p, mode, False)
        dirty, _ = run_td(ctx, p, mode, True)
    finally:
        ctx.set_option("pair_split_threshold", 0)
    assert not torch.isnan(torch.view_as_real(dirty)).any()
    assert torch.equal(clean, dirty)


@pytest.mark.parametrize("mode", ["fp32_4m", "bf16x3"])
def test_batch_poisoned(ctx, mode):
    import torch
    import paper_2201_06620_amd as rn
    r = rng.SplitMix64(73000)
    probs = []
    while len(probs) < 20:
        ra, rb, k = r.randint(3, 14), r.randint(3, 14), r.randint(0, 10)
        if k > min(ra, rb) or ra + rb - 2 * k > 14:
            continue
        probs.append(configs.make_problem(ra, rb, r.sample(ra, k), r.sample(rb, k),
                                          configs.split_first(ra), configs.split_first(rb),
                                          73000 + len(probs)))
    items = [(torch.from_numpy(p.a.data).to(dt_of(mode)).cuda(), p.a.dims, p.a.grid,
              torch.from_numpy(p.b.data).to(dt_of(mode)).cuda(), p.b.dims, p.b.grid,
              p.axes_a, p.axes_b) for p in probs]
    ws = rn.plan_batch_workspace(ctx, items, mode)
    results = []
    for poison in (False, True):
        pb = ctx.prepare_batch(items, mode, workspace=filled(max(ws, 1), torch.uint8, poison))
        for o in pb.outputs:
            o.view(torch.uint8).fill_(0xFF if poison else 0)
        torch.cuda.synchronize()
        results.append([o.clone() for o in pb.run()])
        torch.cuda.synchronize()
    for i, (c, d) in enumerate(zip(*results)):
        assert not torch.isnan(torch.view_as_real(d)).any(), i
        assert torch.equal(c, d), i


@pytest.mark.parametrize("mode", ["fp64", "fp32_4m"])
def test_network_poisoned(ctx, mode):
    import torch
    circ = circuits.random_circuit(3, 4, 8, seed=74)
    net = circuits.circuit_network(circ, circuits.random_bitstring(12, 75))
    path = paths.greedy_path(net.labels, 76, restarts=2)
    sliced = paths.greedy_slices(net.labels, path, 77, n_slices=3)
    ts = [torch.from_numpy(np.ascontiguousarray(t.reshape(-1))).to(dt_of(mode)).cuda()
          for t in net.tensors]
    ws, _, _ = ctx.contract_network_plan(ts, net.labels, path, sliced, mode)
    res = []
    for poison in (False, True):
        amp = filled(2, torch.float64, poison)
        sl = filled(2 << len(sliced), torch.float64, poison)
        wsb = filled(max(ws, 1), torch.uint8, poison)
        torch.cuda.synchronize()
        ctx.contract_network(ts, net.labels, path, sliced, mode, amp=amp, slices=sl,
                             workspace=wsb)
        torch.cuda.synchronize()
        res.append((amp.clone(), sl.clone()))
    (a0, s0), (a1, s1) = res
    assert not torch.isnan(a1).any() and not torch.isnan(s1).any()
    assert torch.equal(a0, a1) and torch.equal(s0, s1)


def test_binding_refuses_mis_sized_buffers(ctx):
    import torch
    import paper_2201_06620_amd as rn
    p = problem(75000, 8, 8, 3)
    a = torch.from_numpy(p.a.data).to(torch.complex64).cuda()
    b = torch.from_numpy(p.b.data).to(torch.complex64).cuda()
    with pytest.raises(rn.RnError):        # output one element short
        ctx.block_tensordot(a, p.a.dims, p.a.grid, b, p.b.dims, p.b.grid, p.axes_a, p.axes_b,
                            "fp32_4m", out=torch.empty(2 ** 10 - 1, dtype=torch.complex64,
                                                       device="cuda"))
    with pytest.raises(rn.RnError):        # complex64 operands in FP64 mode
        ctx.block_tensordot(a, p.a.dims, p.a.grid, b, p.b.dims, p.b.grid, p.axes_a, p.axes_b,
                            "fp64")
    with pytest.raises(rn.RnError):        # operand shorter than its dims
        ctx.block_tensordot(a[:-1], p.a.dims, p.a.grid, b, p.b.dims, p.b.grid, p.axes_a,
                            p.axes_b, "fp32_4m")
    t = torch.zeros(4, dtype=torch.complex128, device="cuda")
    with pytest.raises(rn.RnError):        # complex128 network tensors in an FP32 mode
        ctx.contract_network([t, t], [[1, 2], [1, 2]], [(0, 1)], [], "fp32_4m")
    t = torch.zeros(4, dtype=torch.complex64, device="cuda")
    with pytest.raises(rn.RnError):        # slices buffer shorter than 2 * 2^nsliced
        ctx.contract_network([t, t], [[1, 2], [1, 2]], [(0, 1)], [1], "fp32_4m",
                             slices=torch.zeros(3, dtype=torch.float64, device="cuda"))
