"""GPU: repeated block tensordots on one shape reuse the binding's cached
plan (descriptors, axis arrays, C shape, workspace size).  A cached call on
new operands gives the same bits as a fresh handle's first call on them, and
the binding's no-alloc wrapper, cached too, gives the same bits as the
workspace call."""
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


def problem(seed, ra=14, rb=13, k=7):
    r = rng.SplitMix64(seed)
    axa, axb = r.sample(ra, k), r.sample(rb, k)
    ga = [2 if r.below(3) == 0 else 1 for _ in range(ra)]
    gb = [2 if r.below(3) == 0 else 1 for _ in range(rb)]
    return configs.make_problem(ra, rb, axa, axb, ga, gb, seed)


def dev(x, mode):
    import torch
    dt = torch.complex128 if mode == "fp64" else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(x)).to(dt).to("cuda")


@pytest.mark.parametrize("mode", MODES)
def test_cached_plan_on_new_operands(mode):
    import torch
    import paper_2201_06620_amd as rn
    p1, p2 = problem(91000 + MODES.index(mode)), problem(91100 + MODES.index(mode))
    # Same shape, grids and axes; different values.
    p2 = configs.make_problem(len(p1.a.dims), len(p1.b.dims), p1.axes_a, p1.axes_b, p1.a.grid,
                              p1.b.grid, p2.seed)
    log(f"plan cache {mode} seeds {p1.seed} {p2.seed}")
    ctx = rn.Context(0)
    outs = []
    for p in (p1, p2, p1):
        c, cd, cg = ctx.block_tensordot(dev(p.a.data, mode), p.a.dims, p.a.grid,
                                        dev(p.b.data, mode), p.b.dims, p.b.grid,
                                        p.axes_a, p.axes_b, mode)
        outs.append(c)
    assert len(ctx._plans) == 1
    fresh = rn.Context(0)
    c2, _, _ = fresh.block_tensordot(dev(p2.a.data, mode), p2.a.dims, p2.a.grid,
                                     dev(p2.b.data, mode), p2.b.dims, p2.b.grid,
                                     p2.axes_a, p2.axes_b, mode)
    torch.cuda.synchronize()
    assert torch.equal(outs[1], c2)
    assert torch.equal(outs[0], outs[2])
    assert not torch.equal(outs[0], outs[1])
    ref, _, _ = oracle.block_tensordot(p2.a.data, p2.a.dims, p2.a.grid, p2.b.data, p2.b.dims,
                                       p2.b.grid, p2.axes_a, p2.axes_b)
    parity.check(outs[1].cpu().numpy().astype(np.complex128), ref,
                 parity.abs_product_blocked(p2), 2 ** p2.k, mode, "cached plan")
    fresh.close()
    ctx.close()


@pytest.mark.parametrize("mode", MODES)
def test_binding_noalloc_matches_workspace_call(mode):
    import torch
    import paper_2201_06620_amd as rn
    ctx = rn.Context(0)
    for seed in (92000, 92001):
        p = problem(seed + 10 * MODES.index(mode), 12, 12, 6)
        log(f"binding no-alloc {mode} seed {p.seed}")
        a, b = dev(p.a.data, mode), dev(p.b.data, mode)
        ref, cd, cg = ctx.block_tensordot(a, p.a.dims, p.a.grid, b, p.b.dims, p.b.grid,
                                          p.axes_a, p.axes_b, mode)
        for _ in range(2):
            out = torch.full_like(ref, float("nan"))
            c, cd2, cg2 = ctx.block_tensordot_noalloc(a, p.a.dims, p.a.grid, b, p.b.dims,
                                                      p.b.grid, p.axes_a, p.axes_b, mode,
                                                      out=out)
            torch.cuda.synchronize()
            assert (cd2, cg2) == (cd, cg)
            assert torch.equal(c, ref)
    ctx.close()
