"""Full-size parity of the rank-28 pairwise contraction: two rank-28 tensors
(all dims 2, 2^28 complex entries each), 14 contracted indices in seeded
random order, contracted through the same call and default tiles the
benchmark times, plus split BF16's opt-in Gauss tile (planar operands).  The oracle computes sampled outputs one by one (two 32 x 32
blocks of C viewed as M x N, plus the corners).  Complex normal inputs: e_F
and e_max within each mode's tolerance and every sampled entry within its
rounding bound (tests/parity.py).  Bit-exact on Gaussian-integer inputs,
where every partial sum is an integer below 2^24 and so exact in every mode,
and on odd nine-bit integers against units {0, +-1, +-i} (either operand
wide), whose bfloat16 split has nonzero low parts, so split BF16 is exact
only with both of its cross terms.
"""
import sys

import numpy as np
import pytest

import oracle
import parity
from workloads import configs

pytestmark = pytest.mark.gpu

RANK, K = 28, 14
TOL = {"fp64": 1e-12, "fp32_4m": 1e-5, "fp32_3m": 1e-5, "bf16x3": 1e-3}
BF16_GAUSS_TILE = 12  # split BF16, Gauss form on planar operands (opt-in tile)


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


def run_modes(p, idx, check, absprod=False):
    import tempfile
    from pathlib import Path
    import torch
    import paper_2201_06620_amd as rn
    assert torch.cuda.is_available()
    ctx = rn.Context(0)
    tmp_dir = Path(tempfile.mkdtemp())
    dims = [2] * RANK
    A = p.a.data.reshape(dims)
    B = p.b.data.reshape(dims)
    log(f"oracle on {idx.size} sampled outputs")
    ref = oracle.tensordot_entries(A, B, p.axes_a, p.axes_b, idx)
    if absprod:
        log("oracle (|A||B|) on the same outputs")
        ref = (ref, parity.abs_product_entries(A, B, p.axes_a, p.axes_b, idx))
    for dt, modes in ((torch.complex64, ("fp32_4m", "fp32_3m", "bf16x3", "bf16x3_gauss")),
                      (torch.complex128, ("fp64",))):
        a = torch.from_numpy(p.a.data).to(dt).cuda()
        b = torch.from_numpy(p.b.data).to(dt).cuda()
        for mode in modes:
            log(f"mode {mode}: rank-{RANK} contraction, {K} contracted axes")
            call = mode
            if mode == "bf16x3_gauss":  # the planar Gauss tile, through a tune file
                call = "bf16x3"
                tf = str(tmp_dir / "bf16_gauss_tune.txt")
                with open(tf, "w") as f:
                    f.write("rn_tune 1\n%d %d %d %d %d\n" % (rn.mode_id(call), RANK - K,
                                                             RANK - K, K, BF16_GAUSS_TILE))
                ctx.tune_load(tf)
            c, cd, cg = ctx.block_tensordot(a, dims, None, b, dims, None, p.axes_a, p.axes_b,
                                            call)
            ctx.tune_clear()
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
        ref, absprod = ref
        pm = "bf16x3" if mode == "bf16x3_gauss" else mode
        parity.check(got, ref, absprod, 2 ** K, pm, f"rank-28 sampled {mode}")

    run_modes(p, idx, check, absprod=True)


def test_rank28_sampled_integers_bitwise():
    log("generating rank-28 Gaussian-integer inputs")
    p = configs.config3(integer=True)
    idx = sample_index()

    def check(mode, got, ref):
        assert np.array_equal(got, ref), mode

    run_modes(p, idx, check)


@pytest.mark.parametrize("values", [("wide", "unit"), ("unit", "wide")])
def test_rank28_sampled_split_low_parts_bitwise(values):
    # Every partial sum is an integer below 2^24 (|term| <= 511 in 4M and
    # 1022 in Gauss, 2^14 terms), so every mode is exact; split BF16 only
    # with its lo*hi (wide A) or hi*lo (wide B) products.
    log(f"generating rank-28 inputs {values}")
    p = configs.config3(values=values)
    idx = sample_index()

    def check(mode, got, ref):
        assert np.array_equal(got, ref), mode

    run_modes(p, idx, check)


def unitary_rank28(seed):
    """A 2^14 x 2^14 unitary as a rank-28 tensor (row bits, then column
    bits): the Kronecker product of seven 4 x 4 unitaries Q_i, each the Q
    factor of a seeded complex normal matrix.  Also returns
    || |U|^T |U| ||_F = prod_i || |Q_i|^T |Q_i| ||_F (|U| is the Kronecker
    product of the |Q_i|), the scale of the terms the contraction sums."""
    rs = np.random.default_rng(seed)
    u = np.ones((1, 1), dtype=np.complex128)
    scale = 1.0
    qs = []
    for _ in range(7):
        q, _ = np.linalg.qr(rs.normal(size=(4, 4)) + 1j * rs.normal(size=(4, 4)))
        u = np.kron(u, q)
        qs.append(q)
        scale *= np.linalg.norm(np.abs(q).T @ np.abs(q))
    return u.reshape([2] * RANK), scale, rs, qs


def test_rank28_unitary_full_output():
    # Closed form at full size, every output checked: contracting a unitary
    # U with conj(U) over its row axes gives the identity over the column
    # axes, whatever order the axes are stored and paired in.  U's axes are
    # stored in a seeded random order and the 14 row axes paired in another,
    # so both operands take real permutes.  The exact result is the sum of
    # 2^14 terms that cancel to 0 or 1, so the error is measured against the
    # scale of those terms, || |U|^T |U| ||_F (normwise, as rounding error
    # bounds are stated), with the mode's tolerance; the error relative to
    # ||I||_F is logged too.  Entry by entry, |C - I|_ij must stay within the
    # mode's rounding bound g (tests/parity.py) times (|U|^T |U|)_ij, which
    # is the Kronecker product of the seven |Q_i|^T |Q_i| with its column
    # bits in the order C lists them.
    import torch
    import paper_2201_06620_amd as rn
    log("generating a rank-28 unitary")
    u, scale, rs, qs = unitary_rank28(2814)
    perm = rs.permutation(RANK)            # stored axis j holds original axis perm[j]
    pos = np.argsort(perm)                 # original axis -> stored position
    rows = rs.permutation(K)               # pairing order of the row axes
    axes = [int(pos[a]) for a in rows]
    t = np.ascontiguousarray(u.transpose(perm)).reshape(-1)
    tc = np.conj(t)
    del u
    ctx = rn.Context(0)
    dims = [2] * RANK
    n = 2 ** (RANK - K)
    log(f"scale || |U|^T |U| ||_F = {scale:.4g}, ||I||_F = {np.sqrt(n):.4g}")
    # C's axes: A's free (column) axes in stored order, then B's (the same).
    cols = [int(perm[j]) - K for j in range(RANK) if j not in set(axes)]
    w = torch.ones((1, 1), dtype=torch.float64, device="cuda")
    for q in qs:
        w = torch.kron(w, torch.from_numpy(np.abs(q).T @ np.abs(q)).cuda())
    # Row/column index of C -> the original column index it stands for.
    x = torch.arange(n, device="cuda")
    orig = torch.zeros_like(x)
    for pos_c, c in enumerate(cols):
        orig |= ((x >> (K - 1 - pos_c)) & 1) << (K - 1 - c)
    w = w[orig][:, orig].contiguous()
    eye = torch.eye(n, dtype=torch.complex128, device="cuda")
    errs = {}
    worst = {}
    for dt, modes in ((torch.complex64, ("fp32_4m", "fp32_3m", "bf16x3")),
                      (torch.complex128, ("fp64",))):
        a = torch.from_numpy(t).to(dt).cuda()
        b = torch.from_numpy(tc).to(dt).cuda()
        for mode in modes:
            log(f"mode {mode}: U . conj(U) over 14 row axes, full 2^28 output")
            c, cd, _ = ctx.block_tensordot(a, dims, None, b, dims, None, axes, axes, mode)
            assert cd == [2] * (2 * (RANK - K))
            m = c.view(n, n).to(torch.complex128)
            d = m.diagonal()
            err2 = (m.abs() ** 2).sum() - (d.abs() ** 2).sum() + ((d - 1).abs() ** 2).sum()
            err = float(err2.clamp(min=0).sqrt())
            errs[mode] = err / scale
            dev = (m - eye).abs()
            g = parity.bound_factor(mode, 2 ** K)
            over = int((dev > g * w).sum())
            hig = float((dev / (2 ** K * parity.UNIT[mode] * w)).max())
            worst[mode] = (over, hig)
            log(f"  ||C - I||_F / scale = {err / scale:.3e}   / ||I||_F = {err / np.sqrt(n):.3e}"
                f"   max higham = {hig:.3e} (bound {g / (2 ** K * parity.UNIT[mode]):.3g}),"
                f" over bound: {over}")
            del c, m, d, dev
        del a, b
        torch.cuda.empty_cache()
    for mode, e in errs.items():
        assert e < TOL[mode], (mode, e)
        assert worst[mode][0] == 0, (mode, worst[mode])


def test_outer_product_more_column_tiles_than_workgroups():
    # An outer product (no contracted axis, K = 1) of a 2-vector with a
    # rank-25 tensor runs on the skinny kernel with 2^21 column tiles of 16,
    # more than the 2^20 workgroups it launches, so every workgroup loops over
    # two tiles.  Gaussian-integer inputs make every product exact: sampled
    # outputs (the first and last tiles of both passes, plus random ones)
    # must be bit-identical to the oracle in every mode.
    import torch
    import paper_2201_06620_amd as rn
    rb = 25
    n = 2 ** rb
    rs = np.random.default_rng(2525)
    a = (rs.integers(-8, 9, 2) + 1j * rs.integers(-8, 9, 2)).astype(np.complex128)
    b = (rs.integers(-8, 9, n) + 1j * rs.integers(-8, 9, n)).astype(np.complex128)
    cols = np.concatenate([np.arange(64), np.arange(2 ** 24 - 64, 2 ** 24 + 64),
                           np.arange(n - 64, n), rs.integers(0, n, 256)])
    idx = np.unique(np.concatenate([cols, n + cols]).astype(np.int64))
    log(f"oracle on {idx.size} sampled outputs of a 2 x 2^{rb} outer product")
    ref = oracle.tensordot_entries(a, b.reshape([2] * rb), [], [], idx)
    ctx = rn.Context(0)
    for dt, modes in ((torch.complex64, ("fp32_4m", "fp32_3m", "bf16x3")),
                      (torch.complex128, ("fp64",))):
        ta = torch.from_numpy(a).to(dt).cuda()
        tb = torch.from_numpy(b).to(dt).cuda()
        for mode in modes:
            log(f"mode {mode}: outer product, 2^{rb + 1} outputs")
            c, cd, _ = ctx.block_tensordot(ta, [2], None, tb, [2] * rb, None, [], [], mode)
            torch.cuda.synchronize()
            assert cd == [2] * (rb + 1)
            got = c[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.complex128)
            assert np.array_equal(got, ref), mode
            del c
        del ta, tb
        torch.cuda.empty_cache()
