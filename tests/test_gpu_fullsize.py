"""Full-size parity of the rank-28 pairwise contraction: two rank-28 tensors
(all dims 2, 2^28 complex entries each), 14 contracted indices in seeded
random order, contracted through the same call and default tiles the
benchmark times.  The oracle computes sampled outputs one by one (two 32 x 32
blocks of C viewed as M x N, plus the corners): within each mode's tolerance
on complex normal inputs, and bit-exact on Gaussian-integer inputs, where
every partial sum is an integer below 2^24 and so exact in every mode.
"""
import sys

import numpy as np
import pytest

import oracle
from workloads import configs

pytestmark = pytest.mark.gpu

RANK, K = 28, 14
TOL = {"fp64": 1e-12, "fp32_4m": 1e-5, "fp32_3m": 1e-5, "bf16x3": 1e-3}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def sample_index():
    M = N = 2 ** (RANK - K)
    rs = np.random.default_rng(2828)
    idx = [0, N - 1, (M - 1) * N, M * N - 1]
    for _ in range(2):
        r0 = int(rs.integers(0, M // 32)) * 32
        c0 = int(rs.integers(0, N // 32)) * 32
        rr, cc = np.meshgrid(np.arange(r0, r0 + 32), np.arange(c0, c0 + 32), indexing="ij")
        idx.extend((rr * N + cc).reshape(-1).tolist())
    return np.unique(np.asarray(idx, dtype=np.int64))


def run_modes(p, idx, check):
    import torch
    import paper_2201_06620_amd as rn
    assert torch.cuda.is_available()
    ctx = rn.Context(0)
    dims = [2] * RANK
    A = p.a.data.reshape(dims)
    B = p.b.data.reshape(dims)
    log(f"oracle on {idx.size} sampled outputs")
    ref = oracle.tensordot_entries(A, B, p.axes_a, p.axes_b, idx)
    for dt, modes in ((torch.complex64, ("fp32_4m", "fp32_3m", "bf16x3")),
                      (torch.complex128, ("fp64",))):
        a = torch.from_numpy(p.a.data).to(dt).cuda()
        b = torch.from_numpy(p.b.data).to(dt).cuda()
        for mode in modes:
            log(f"mode {mode}: rank-{RANK} contraction, {K} contracted axes")
            c, cd, cg = ctx.block_tensordot(a, dims, None, b, dims, None, p.axes_a, p.axes_b,
                                            mode)
            torch.cuda.synchronize()
            assert cd == [2] * (2 * (RANK - K))
            got = c[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.complex128)
            check(mode, got, ref)
            del c
        del a, b
        torch.cuda.empty_cache()


def test_rank28_sampled_within_tolerance():
    log("generating rank-28 complex normal inputs")
    p = configs.config3()
    idx = sample_index()

    def check(mode, got, ref):
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        log(f"  e_F = {err:.3e}")
        assert err < TOL[mode], (mode, err)

    run_modes(p, idx, check)


def test_rank28_sampled_integers_bitwise():
    log("generating rank-28 Gaussian-integer inputs")
    p = configs.config3(integer=True)
    idx = sample_index()

    def check(mode, got, ref):
        assert np.array_equal(got, ref), mode

    run_modes(p, idx, check)
