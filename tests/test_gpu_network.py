"""GPU parity: sliced network contraction against the oracle and the state vector.

Amplitude error is |a - a_ref| / max(|a_ref|, 2^(-n/2)) with the same
tolerances per mode as the block tensordot (1e-12 FP64, 1e-5 FP32,
1e-3 split BF16).
"""
import sys

import numpy as np
import pytest

import oracle
from workloads import circuits, configs, paths

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32_4m": 1e-5, "fp32_3m": 1e-5, "bf16x3": 1e-3}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2201_06620_amd as rn
    assert torch.cuda.is_available()
    return rn.Context(0)


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


@pytest.mark.parametrize("mode", ["fp64", "fp32_4m", "fp32_3m", "bf16x3"])
def test_config2_amplitude(ctx, mode):
    log(f"config2 network mode={mode}")
    w = configs.config2()
    ref, _ = oracle.contract_network(w.network.tensors, w.network.labels, w.path, w.sliced)
    ref = complex(ref)
    a = gpu_amp(ctx, w.network, w.path, w.sliced, mode)
    err = amp_err(a, ref, w.circuit.n)
    log(f"  amp={a} ref={ref} err={err:.3e}")
    assert err < TOL[mode]


@pytest.mark.parametrize("mode", ["fp64", "fp32_4m", "bf16x3"])
def test_config2_prepared_replay_equals_plain_call(ctx, mode):
    # The 20-qubit amplitude (subtrees of tiny steps, a large step whose split-K
    # partials the next permute sums) as a prepared call on a side stream --
    # direct, captured, then replayed from the graph's own parameter table --
    # gives the plain call's bits, per-slice values included.
    import torch
    w = configs.config2()
    dt = torch.complex128 if mode == "fp64" else torch.complex64
    ts = [torch.from_numpy(np.ascontiguousarray(t.reshape(-1))).to(dt).cuda()
          for t in w.network.tensors]
    ns = 1 << len(w.sliced)
    sl_c = torch.zeros(2 * ns, dtype=torch.float64, device="cuda")
    amp_c = ctx.contract_network(ts, w.network.labels, w.path, w.sliced, mode, slices=sl_c)
    torch.cuda.synchronize()
    prep = ctx.prepare_network(ts, w.network.labels, w.path, w.sliced, mode)
    s = torch.cuda.Stream()
    amp = torch.zeros(2, dtype=torch.float64, device="cuda")
    sl_p = torch.zeros_like(sl_c)
    for it in range(4):
        amp.fill_(float("nan"))
        sl_p.fill_(float("nan"))
        torch.cuda.synchronize()
        prep.run(amp=amp, slices=sl_p, stream=s)
        s.synchronize()
        assert np.array_equal(amp.cpu().numpy(), amp_c.cpu().numpy()), it
        assert np.array_equal(sl_p.cpu().numpy(), sl_c.cpu().numpy()), it
    del prep


def test_config2_per_slice_values(ctx):
    import torch
    w = configs.config2()
    ns = 1 << len(w.sliced)
    slices = torch.zeros(2 * ns, dtype=torch.float64, device="cuda")
    a = gpu_amp(ctx, w.network, w.path, w.sliced, "fp64", slices=slices)
    sv = slices.cpu().numpy()
    vals = sv[0::2] + 1j * sv[1::2]
    # Each slice equals the oracle run with that projection alone: contract
    # the network with the sliced bonds cut to one value by fixing them.
    for s in range(ns):
        net = w.network.copy()
        for i, lab in enumerate(w.sliced):
            bit = (s >> (len(w.sliced) - 1 - i)) & 1
            proj = np.zeros(2, dtype=np.complex128)
            proj[bit] = 1.0
            # Attach a projector on one side of the bond: replace the bond by
            # two labels joined through the projector vector outer product.
            for t_idx, labs in enumerate(net.labels):
                if lab in labs:
                    ax = labs.index(lab)
                    net.tensors[t_idx] = np.take(net.tensors[t_idx], [bit], axis=ax)
                    net.tensors[t_idx] = np.squeeze(net.tensors[t_idx], axis=ax)
                    net.labels[t_idx] = [x for x in labs if x != lab]
        ref, _ = oracle.contract_network(net.tensors, net.labels, w.path)
        assert abs(vals[s] - complex(ref)) < 1e-12 * max(abs(complex(ref)), 1e-6)
    assert abs(a - vals.sum()) < 1e-15


@pytest.mark.parametrize("rows,cols,cycles,nsl", [(3, 3, 6, 0), (3, 4, 8, 3), (2, 5, 10, 5)])
def test_small_circuits_vs_statevector(ctx, rows, cols, cycles, nsl):
    log(f"circuit {rows}x{cols} cycles={cycles} slices={nsl}")
    circ = circuits.random_circuit(rows, cols, cycles, seed=rows * 100 + cols * 10 + cycles)
    psi = oracle.statevector(circ)
    for trial in range(2):
        bits = circuits.random_bitstring(circ.n, seed=trial + 5)
        net = circuits.circuit_network(circ, bits)
        path = paths.greedy_path(net.labels, 3 + trial, restarts=2)
        sliced = paths.greedy_slices(net.labels, path, 4, n_slices=nsl) if nsl else []
        x = int("".join(map(str, bits)), 2)
        for mode in ("fp64", "fp32_4m"):
            a = gpu_amp(ctx, net, path, sliced, mode)
            assert amp_err(a, psi[x], circ.n) < TOL[mode]


def test_ghz_network(ctx):
    n = 8
    circ = circuits.ghz_circuit(n)
    for bits, expect in (([0] * n, 2 ** -0.5), ([1] * n, 2 ** -0.5), ([0, 1] * 4, 0.0)):
        net = circuits.circuit_network(circ, bits)
        path = paths.greedy_path(net.labels, 1, restarts=1)
        a = gpu_amp(ctx, net, path, [], "fp64")
        assert abs(a - expect) < 1e-15


def test_prepared_network_repeats_and_new_values(ctx):
    # A prepared call (plan cached on the handle, graph replayed on a side
    # stream) gives the oracle's amplitude, and follows new tensor values
    # written in place: another bitstring of the same circuit.
    import torch
    circ = circuits.random_circuit(3, 4, 8, seed=77)
    psi = oracle.statevector(circ)
    bits0 = circuits.random_bitstring(circ.n, seed=1)
    net0 = circuits.circuit_network(circ, bits0)
    path = paths.greedy_path(net0.labels, 9, restarts=2)
    sliced = paths.greedy_slices(net0.labels, path, 3, n_slices=3)
    ts = [torch.from_numpy(np.ascontiguousarray(t.reshape(-1))).cuda() for t in net0.tensors]
    prep = ctx.prepare_network(ts, net0.labels, path, sliced, "fp64")
    s = torch.cuda.Stream()
    amp = torch.zeros(2, dtype=torch.float64, device="cuda")
    for trial in range(4):
        bits = circuits.random_bitstring(circ.n, seed=1 + trial)
        net = circuits.circuit_network(circ, bits)
        assert net.labels == net0.labels
        for t_dev, t_new in zip(ts, net.tensors):
            t_dev.copy_(torch.from_numpy(np.ascontiguousarray(t_new.reshape(-1))))
        torch.cuda.synchronize()
        for _ in range(2):
            with torch.cuda.stream(s):
                prep.run(amp=amp)
            s.synchronize()
        a = amp.cpu().numpy()
        x = int("".join(map(str, bits)), 2)
        assert amp_err(complex(a[0], a[1]), psi[x], circ.n) < 1e-12
    # The prepared call (rn_network_execute) and the plain call
    # (rn_contract_network) give the same bits, per-slice values included.
    sl_p = torch.zeros(2 << len(sliced), dtype=torch.float64, device="cuda")
    sl_c = torch.zeros_like(sl_p)
    for _ in range(3):  # direct, captured, replayed; the stream passed explicitly
        prep.run(amp=amp, slices=sl_p, stream=s)
        s.synchronize()
    amp_c = ctx.contract_network(ts, net0.labels, path, sliced, "fp64", slices=sl_c)
    torch.cuda.synchronize()
    assert np.array_equal(amp.cpu().numpy(), amp_c.cpu().numpy())
    assert np.array_equal(sl_p.cpu().numpy(), sl_c.cpu().numpy())
    del prep  # rn_network_release


@pytest.mark.parametrize("mode", ["fp64", "fp32_4m"])
def test_degenerate_networks(ctx, mode):
    # A network that is one scalar (no step) returns that scalar; two vectors
    # sharing one bond (one step) return their dot product, with the bond
    # also sliced (two slices summed in FP64).
    import torch
    dt = torch.complex128 if mode == "fp64" else torch.complex64
    s = torch.tensor([1.25 - 0.5j], dtype=dt, device="cuda")
    amp = ctx.contract_network([s], [[]], [], [], mode)
    torch.cuda.synchronize()
    assert complex(*amp.cpu().numpy()) == 1.25 - 0.5j
    a = np.array([1.5 + 2j, -0.5 + 1j])
    b = np.array([2 - 1j, 4 + 0.25j])
    ta, tb = (torch.from_numpy(x).to(dt).cuda() for x in (a, b))
    for sliced in ([], [7]):
        amp = ctx.contract_network([ta, tb], [[7], [7]], [(0, 1)], sliced, mode)
        torch.cuda.synchronize()
        assert complex(*amp.cpu().numpy()) == complex(np.dot(a, b)), sliced
