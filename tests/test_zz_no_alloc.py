"""GPU: rn_block_tensordot_noalloc (the workspace is the library's fixed
device scratch array) called through the C ABI gives the same bits as
rn_block_tensordot with a caller workspace, and matches the oracle, on two
calls in a row (the second smaller, so it runs over what the first left in
the array), in every mode; plans that need more than the array holds are
refused before anything is enqueued."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import parity
from workloads import configs, rng

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


def problem(seed, ra, rb, k):
    r = rng.SplitMix64(seed)
    axa, axb = r.sample(ra, k), r.sample(rb, k)
    ga = [2 if r.below(3) == 0 else 1 for _ in range(ra)]
    gb = [2 if r.below(3) == 0 else 1 for _ in range(rb)]
    return configs.make_problem(ra, rb, axa, axb, ga, gb, seed)


def call_noalloc(ctx, p, mode, a, b, out):
    """rn_block_tensordot_noalloc through the C ABI; returns the status."""
    import torch
    import paper_2201_06620_amd as rn
    dt = rn.dtype_of_mode(mode)
    A = rn.descriptor(p.a.dims, p.a.grid, dt, a.data_ptr())
    B = rn.descriptor(p.b.dims, p.b.grid, dt, b.data_ptr())
    C = rn.RnTensor()
    axa = np.asarray(p.axes_a, dtype=np.int32)
    axb = np.asarray(p.axes_b, dtype=np.int32)
    pa = axa.ctypes.data if axa.size else None
    pb = axb.ctypes.data if axb.size else None
    L = rn.lib()
    st = L.rn_block_tensordot_plan(ctx.h, ctypes.byref(A), ctypes.byref(B), len(axa), pa, pb,
                                   rn.MODES[mode], ctypes.byref(C), None, None)
    assert st == 0
    C.data = out.data_ptr()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return L.rn_block_tensordot_noalloc(ctx.h, ctypes.byref(A), ctypes.byref(B), len(axa), pa,
                                        pb, ctypes.byref(C), rn.MODES[mode], stream)


@pytest.mark.parametrize("mode", MODES)
def test_noalloc_matches_workspace_call_twice(ctx, mode):
    import torch
    dt = torch.complex128 if mode == "fp64" else torch.complex64
    # First call: rank 18 x rank 16 with a workspace of 10-37 MiB (both
    # operands permuted, split-K partials); second: a smaller ragged one over
    # what the first left in the array.
    for ra, rb, k in ((18, 16, 8), (13, 11, 6)):
        p = problem(81000 + 31 * ra + rb + k, ra, rb, k)
        a = torch.from_numpy(p.a.data).to(dt).cuda()
        b = torch.from_numpy(p.b.data).to(dt).cuda()
        cd, cg, ws, _ = ctx.plan_block_tensordot(p.a.dims, p.a.grid, p.b.dims, p.b.grid,
                                                 p.axes_a, p.axes_b, mode)
        log(f"no-alloc {mode} shape {(ra, rb, k)}: workspace {ws} bytes")
        assert 0 < ws <= (1 << 26)
        n = int(np.prod(cd))
        ref_gpu, _, _ = ctx.block_tensordot(a, p.a.dims, p.a.grid, b, p.b.dims, p.b.grid,
                                            p.axes_a, p.axes_b, mode)
        out = torch.full((n,), float("nan"), dtype=dt, device="cuda")
        torch.cuda.synchronize()
        assert call_noalloc(ctx, p, mode, a, b, out) == 0
        torch.cuda.synchronize()
        assert torch.equal(out, ref_gpu), (mode, ra, rb, k)
        if ra + rb <= 35:
            ref, _, _ = oracle.block_tensordot(p.a.data, p.a.dims, p.a.grid, p.b.data,
                                               p.b.dims, p.b.grid, p.axes_a, p.axes_b)
            parity.check(out.cpu().numpy().astype(np.complex128), ref,
                         parity.abs_product_blocked(p), 2 ** k, mode, "no-alloc")


def test_noalloc_refuses_workspace_beyond_scratch(ctx):
    import torch
    import paper_2201_06620_amd as rn
    # Rank 24 x rank 24 complex64 with both operands permuted: 256 MiB of
    # workspace against the 64 MiB array.
    p = problem(82000, 24, 24, 12)
    cd, _, ws, _ = ctx.plan_block_tensordot(p.a.dims, p.a.grid, p.b.dims, p.b.grid, p.axes_a,
                                            p.axes_b, "fp32_4m")
    assert ws > (1 << 26)
    a = torch.zeros(2 ** 24, dtype=torch.complex64, device="cuda")
    b = torch.zeros(2 ** 24, dtype=torch.complex64, device="cuda")
    out = torch.full((int(np.prod(cd)),), 7.0, dtype=torch.complex64, device="cuda")
    st = call_noalloc(ctx, p, "fp32_4m", a, b, out)
    assert st == 4  # RN_ERR_WORKSPACE
    assert b"no-alloc scratch" in rn.lib().rn_last_error()
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())  # nothing ran
