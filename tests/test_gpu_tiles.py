"""Every GEMM tile shape of every mode, forced through a tune file, against
the oracle: on normal inputs e_F and e_max within the mode's tolerance and
every entry within its rounding bound (tests/parity.py); bit-exact on
Gaussian integers and on odd nine-bit integers against units (nonzero
bfloat16 low parts on either side).  Shapes span several tiles with ragged
edges."""
import sys

import numpy as np
import pytest

import oracle
import parity
from workloads import configs, rng

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32_4m": 1e-5, "fp32_3m": 1e-5, "bf16x3": 1e-3}
MODE_ID = {"fp64": 0, "fp32_4m": 1, "fp32_3m": 2, "bf16x3": 3}


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2201_06620_amd as rn
    assert torch.cuda.is_available()
    return rn.Context(0)


def problem(ra, rb, k, seed, values):
    r = rng.SplitMix64(seed)
    return configs.make_problem(ra, rb, r.sample(ra, k), r.sample(rb, k), [1] * ra, [1] * rb,
                                seed, values=values)


def all_tiles():
    import paper_2201_06620_amd as rn
    out = []
    for mode in TOL:
        for t in range(rn.tile_count(mode)):
            out.append((mode, t))
    return out


@pytest.mark.parametrize("mode,tile", all_tiles())
@pytest.mark.parametrize("shape", [(16, 15, 7), (11, 12, 5), (10, 14, 7), (14, 9, 7),
                                   (8, 15, 8)])
def test_forced_tile(ctx, tmp_path, mode, tile, shape):
    import torch
    ra, rb, k = shape
    print(f"mode={mode} tile={tile} shape={shape}", flush=True)
    f = str(tmp_path / "t.txt")
    with open(f, "w") as fh:
        fh.write("rn_tune 1\n%d %d %d %d %d\n" % (MODE_ID[mode], ra - k, rb - k, k, tile))
    ctx.tune_clear()
    ctx.tune_load(f)
    dt = torch.complex128 if mode == "fp64" else torch.complex64
    try:
        for values in (("normal", "normal"), ("integer", "integer"), ("wide", "unit"),
                       ("unit", "wide")):
            p = problem(ra, rb, k, 300 + ra + rb + k, values)
            a = torch.from_numpy(p.a.data).to(dt).cuda()
            b = torch.from_numpy(p.b.data).to(dt).cuda()
            c, cd, cg = ctx.block_tensordot(a, p.a.dims, p.a.grid, b, p.b.dims, p.b.grid,
                                            p.axes_a, p.axes_b, mode)
            torch.cuda.synchronize()
            got = c.cpu().numpy().astype(np.complex128)
            ref, _, _ = oracle.block_tensordot(p.a.data, p.a.dims, p.a.grid, p.b.data,
                                               p.b.dims, p.b.grid, p.axes_a, p.axes_b)
            if values[0] != "normal":
                assert np.array_equal(got, ref), values
            else:
                parity.check(got, ref, parity.abs_product_blocked(p), 2 ** k, mode,
                             f"tile {tile} shape {shape}")
    finally:
        ctx.tune_clear()
