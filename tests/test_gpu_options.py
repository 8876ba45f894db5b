"""GPU parity under the handle options: the reduction-strategy switch and
slice-sum (slices viewed as blocks).

Same tolerances as the other parity tests (relative Frobenius error 1e-12
FP64, 1e-5 FP32, 1e-3 split BF16; amplitudes relative to
max(|a_ref|, 2^(-n/2))).  Gaussian-integer inputs make every mode exact, so
those cases compare bit for bit whatever the split count.
"""
import sys

import numpy as np
import pytest

import oracle
import parity
from workloads import circuits, configs, paths

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32_4m": 1e-5, "fp32_3m": 1e-5, "bf16x3": 1e-3}
MODES = ["fp64", "fp32_4m", "fp32_3m", "bf16x3"]


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture()
def ctx():
    import torch
    import paper_2201_06620_amd as rn
    assert torch.cuda.is_available()
    c = rn.Context(0)
    yield c
    c.close()


def dev(x, mode):
    import torch
    dt = torch.complex128 if mode == "fp64" else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(x)).to(dt).to("cuda")


def e_f(x, ref):
    return np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-300)


def run(ctx, p, mode):
    import torch
    c, cd, cg = ctx.block_tensordot(dev(p.a.data, mode), p.a.dims, p.a.grid,
                                    dev(p.b.data, mode), p.b.dims, p.b.grid,
                                    p.axes_a, p.axes_b, mode)
    torch.cuda.synchronize()
    return c.cpu().numpy().astype(np.complex128), cd, cg


def ws_of(ctx, p, mode):
    return ctx.plan_block_tensordot(p.a.dims, p.a.grid, p.b.dims, p.b.grid,
                                    p.axes_a, p.axes_b, mode)[2]


def blocked_k_problem(seed, integer=False, ra=16, rb=15, k=10, nblk=3):
    """k contracted axes, the first nblk of them split in two on both sides
    (B_k = 2^nblk coupled pairs), K = 2^k."""
    from workloads import rng
    r = rng.SplitMix64(seed)
    axa, axb = r.sample(ra, k), r.sample(rb, k)
    ga, gb = [1] * ra, [1] * rb
    for q in range(nblk):
        ga[axa[q]] = 2
        gb[axb[q]] = 2
    return configs.make_problem(ra, rb, axa, axb, ga, gb, seed, integer)


def test_options_roundtrip(ctx):
    import paper_2201_06620_amd as rn
    assert ctx.get_option("pair_split_threshold") == 0
    assert ctx.get_option("slice_sum") == 0
    assert ctx.get_option("graphs") in (0, 1)
    ctx.set_option("pair_split_threshold", 4)
    ctx.set_option("split_footprint", 1 << 20)
    ctx.set_option("slice_sum", 1)
    assert ctx.get_option("pair_split_threshold") == 4
    assert ctx.get_option("split_footprint") == 1 << 20
    assert ctx.get_option("slice_sum") == 1
    with pytest.raises(rn.RnError):
        ctx.set_option("slice_sum", 2)
    with pytest.raises(rn.RnError):
        ctx.set_option("pair_split_threshold", -1)


@pytest.mark.parametrize("mode", MODES)
def test_pair_split_matches_oracle(ctx, mode):
    p = blocked_k_problem(51000 + MODES.index(mode))
    log(f"pair split mode={mode} seed={p.seed}")
    ref, rd, rg = oracle.block_tensordot(p.a.data, p.a.dims, p.a.grid, p.b.data, p.b.dims,
                                         p.b.grid, p.axes_a, p.axes_b)
    # Threshold above B_k: one accumulator, no partials.
    ctx.set_option("pair_split_threshold", 1 << 20)
    ws_seq = ws_of(ctx, p, mode)
    c1, cd, cg = run(ctx, p, mode)
    assert cd == rd and cg == rg
    # Threshold at B_k: one partial per pair group; the workspace grows by the
    # partial sums, at most B_k of them.
    ctx.set_option("pair_split_threshold", 8)
    ws_split = ws_of(ctx, p, mode)
    c2, _, _ = run(ctx, p, mode)
    es = 16 if mode == "fp64" else 8
    m_n = int(np.prod(rd)) if rd else 1
    log(f"  ws sequential={ws_seq} split={ws_split}")
    assert ws_split > ws_seq
    assert ws_split - ws_seq <= 8 * m_n * es + 4096
    # A footprint cap below one partial turns the split off again.
    ctx.set_option("split_footprint", 1)
    assert ws_of(ctx, p, mode) == ws_seq
    absprod = parity.abs_product_blocked(p)
    for c in (c1, c2):
        parity.check(c, ref, absprod, 2 ** p.k, mode, "pair split")


@pytest.mark.parametrize("mode", MODES)
def test_pair_split_integers_bitwise(ctx, mode):
    p = blocked_k_problem(52000 + MODES.index(mode), integer=True)
    ref, _, _ = oracle.block_tensordot(p.a.data, p.a.dims, p.a.grid, p.b.data, p.b.dims,
                                       p.b.grid, p.axes_a, p.axes_b)
    ctx.set_option("pair_split_threshold", 2)
    c, _, _ = run(ctx, p, mode)
    assert np.array_equal(c, ref)


def gpu_amp(ctx, net, path, sliced, mode, slices=None):
    import torch
    dt = torch.complex128 if mode == "fp64" else torch.complex64
    ts = [torch.from_numpy(np.ascontiguousarray(t.reshape(-1))).to(dt).to("cuda")
          for t in net.tensors]
    amp = ctx.contract_network(ts, net.labels, path, sliced, mode, slices=slices)
    torch.cuda.synchronize()
    a = amp.cpu().numpy()
    return complex(a[0], a[1])


def amp_err(a, ref, n):
    return abs(a - ref) / max(abs(ref), 2.0 ** (-n / 2))


def net_flops(ctx, w, mode="fp64"):
    import torch
    dt = torch.complex128 if mode == "fp64" else torch.complex64
    ts = [torch.empty(t.size, dtype=dt, device="cuda") for t in w.network.tensors]
    return ctx.contract_network_plan(ts, w.network.labels, w.path, w.sliced, mode)[1]


@pytest.mark.parametrize("mode", MODES)
def test_slice_sum_config2(ctx, mode):
    w = configs.config2()
    log(f"slice-sum config2 mode={mode}")
    ref, _ = oracle.contract_network(w.network.tensors, w.network.labels, w.path, w.sliced)
    ref = complex(ref)
    batched_flops = net_flops(ctx, w)
    ctx.set_option("slice_sum", 1)
    sum_flops = net_flops(ctx, w)
    # Summing each sliced bond where it is contracted makes the work that of
    # the unsliced network on the same path.
    _, unsliced, _ = paths.path_stats(w.network.labels, w.path)
    naive = w.meta["flops_per_slice"] * (1 << len(w.sliced))
    log(f"  flops naive={naive:.4g} batched={batched_flops:.4g} slice-sum={sum_flops:.4g}")
    assert sum_flops == unsliced
    assert sum_flops <= batched_flops <= naive
    a = gpu_amp(ctx, w.network, w.path, w.sliced, mode)
    err = amp_err(a, ref, w.circuit.n)
    log(f"  amp={a} ref={ref} err={err:.3e}")
    assert err < TOL[mode]


def test_slice_sum_rejects_per_slice_buffer(ctx):
    import torch
    import paper_2201_06620_amd as rn
    w = configs.config2()
    ctx.set_option("slice_sum", 1)
    slices = torch.zeros(2 << len(w.sliced), dtype=torch.float64, device="cuda")
    with pytest.raises(rn.RnError):
        gpu_amp(ctx, w.network, w.path, w.sliced, "fp64", slices=slices)


@pytest.mark.parametrize("rows,cols,cycles,nsl", [(3, 3, 6, 2), (3, 4, 8, 4), (2, 5, 10, 6)])
def test_slice_sum_vs_statevector(ctx, rows, cols, cycles, nsl):
    log(f"slice-sum circuit {rows}x{cols} cycles={cycles} slices={nsl}")
    circ = circuits.random_circuit(rows, cols, cycles, seed=rows * 100 + cols * 10 + cycles + 1)
    psi = oracle.statevector(circ)
    ctx.set_option("slice_sum", 1)
    for trial in range(2):
        bits = circuits.random_bitstring(circ.n, seed=trial + 9)
        net = circuits.circuit_network(circ, bits)
        path = paths.greedy_path(net.labels, 5 + trial, restarts=2)
        sliced = paths.greedy_slices(net.labels, path, 6, n_slices=nsl)
        x = int("".join(map(str, bits)), 2)
        for mode in ("fp64", "fp32_4m"):
            a = gpu_amp(ctx, net, path, sliced, mode)
            assert amp_err(a, psi[x], circ.n) < TOL[mode]


def net_plan(ctx, w, mode="fp64"):
    import torch
    dt = torch.complex128 if mode == "fp64" else torch.complex64
    ts = [torch.empty(t.size, dtype=dt, device="cuda") for t in w.network.tensors]
    return ctx.contract_network_plan(ts, w.network.labels, w.path, w.sliced, mode)


@pytest.mark.parametrize("bits", [0, 1, 3])
def test_slice_passes_match_batched(ctx, bits):
    import torch
    w = configs.config2()
    ns = 1 << len(w.sliced)
    log(f"config2 with {bits} batched sliced bonds per pass")
    ref, _ = oracle.contract_network(w.network.tensors, w.network.labels, w.path, w.sliced)
    ref = complex(ref)
    full = torch.zeros(2 * ns, dtype=torch.float64, device="cuda")
    a_full = gpu_amp(ctx, w.network, w.path, w.sliced, "fp64", slices=full)
    ws_full, fl_full, _ = net_plan(ctx, w)
    ctx.set_option("batched_slice_bits", bits)
    ws_pass, fl_pass, _ = net_plan(ctx, w)
    log(f"  workspace all-batched={ws_full} passes={ws_pass}; flops {fl_full:.4g} {fl_pass:.4g}")
    assert ws_pass <= ws_full
    # Fixing a bond per pass re-does the work that does not depend on it.
    assert fl_pass >= fl_full
    part = torch.zeros(2 * ns, dtype=torch.float64, device="cuda")
    a = gpu_amp(ctx, w.network, w.path, w.sliced, "fp64", slices=part)
    sv_full = full.cpu().numpy()
    sv_part = part.cpu().numpy()
    # Per-slice values land at the same index either way.
    scale = np.abs(sv_full).max()
    assert np.abs(sv_part - sv_full).max() <= 1e-12 * scale
    assert amp_err(a, ref, w.circuit.n) < 1e-12
    assert amp_err(a_full, ref, w.circuit.n) < 1e-12
    # Slice-sum with passes: the fixed bonds still sum in FP64 across passes.
    ctx.set_option("slice_sum", 1)
    a2 = gpu_amp(ctx, w.network, w.path, w.sliced, "fp64")
    assert amp_err(a2, ref, w.circuit.n) < 1e-12


def test_network_footprint_cap(ctx):
    import paper_2201_06620_amd as rn
    w = configs.circuit_workload(3, 4, 10, 4242, n_slices=5, restarts=2)
    ref, _ = oracle.contract_network(w.network.tensors, w.network.labels, w.path, w.sliced)
    ref = complex(ref)
    ws_full, _, _ = net_plan(ctx, w)
    ctx.set_option("batched_slice_bits", 0)
    ws_min, _, _ = net_plan(ctx, w)
    log(f"  workspace all-batched={ws_full} one slice per pass={ws_min}")
    assert ws_min < ws_full
    ctx.set_option("batched_slice_bits", 64)
    cap = (ws_full + ws_min) // 2
    ctx.set_option("network_footprint", cap)
    ws_cap, _, _ = net_plan(ctx, w)
    assert ws_min <= ws_cap <= cap
    for mode in ("fp64", "fp32_4m"):
        a = gpu_amp(ctx, w.network, w.path, w.sliced, mode)
        assert amp_err(a, ref, w.circuit.n) < TOL[mode]
    ctx.set_option("network_footprint", ws_min - 1)
    with pytest.raises(rn.RnError) as ei:
        net_plan(ctx, w)
    assert ei.value.status == 5  # RN_ERR_OOM
