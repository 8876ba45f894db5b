"""Index bounds of the large GEMM tiles, checked on the CPU.

For every tile shape instantiated in the GEMM kernel files, the unguarded loads of
interior tiles, the LDS staging stores and the per-lane LDS fragment reads
are enumerated for all 256 threads (the same index arithmetic as the
kernels) and must stay inside the tile, its K chunk and its LDS arrays.  A
load by a thread past the tile would read rows beyond the matrix for the
last tile row or column, so the fast-path loads carry the same
`V % 256 == 0 || idx < V` guard that is modelled here.
"""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2201_06620_amd", "csrc")
SRC = "".join(open(os.path.join(CSRC, f)).read() for f in sorted(os.listdir(CSRC))
              if f.endswith(".hip"))


def instances(name):
    pat = name + r"(?:_grouped)?\s*<(\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+)>"
    return sorted(set(tuple(map(int, m)) for m in re.findall(pat, SRC)))


def thread_loads(rows, bk, per_load):
    """(row, first k) of each load a thread issues for one stage of a tile
    with `rows` rows and `bk` complex k, `per_load` complex per load."""
    v = rows * bk // per_load
    for j in range((v + 255) // 256):
        for tid in range(256):
            idx = tid + 256 * j
            if v % 256 == 0 or idx < v:
                yield idx // (bk // per_load), (idx % (bk // per_load)) * per_load


def test_fp32_large_tiles():
    shapes = instances("cgemm_f32_big")
    assert shapes
    for wm_, wn_, tm, tn, bk in shapes:
        bm, bn, ldr = wm_ * tm * 32, wn_ * tn * 32, 2 * bk + 4
        for rows in (bm, bn):
            for r, c in thread_loads(rows, bk, 2):
                assert r < rows and c + 1 < bk
                assert r * ldr + bk + c + 1 < rows * ldr  # planar staging store
        for lane in range(64):
            kh = lane >> 5
            for w in range(4):
                wm, wn = w // wn_, w % wn_
                for kq in range(0, bk, 4):
                    for i in range(tm):
                        o = (wm * tm * 32 + lane % 32 + i * 32) * ldr + kh * bk + kq
                        assert o % 4 == 0 and o + 3 < bm * ldr
                    for j in range(tn):
                        for half in (kh, 1 - kh):
                            o = (wn * tn * 32 + lane % 32 + j * 32) * ldr + half * bk + kq
                            assert o % 4 == 0 and o + 3 < bn * ldr


def test_fp64_large_tiles():
    shapes = instances("cgemm_f64_big")
    assert shapes
    for wm_, wn_, tm, tn, bk in shapes:
        bm, bn, ldr, hb = wm_ * tm * 16, wn_ * tn * 16, 2 * bk + 2, bk // 2
        for rows in (bm, bn):
            for r, c in thread_loads(rows, bk, 1):
                assert r < rows and c < bk
                assert r * ldr + (c & 1) * hb + (c >> 1) + bk < rows * ldr
        for lane in range(64):
            kc, half = lane >> 5, (lane >> 4) & 1
            for w in range(4):
                wm, wn = w // wn_, w % wn_
                for s2 in range(0, hb, 2):
                    for i in range(tm):
                        o = (wm * tm * 16 + lane % 16 + i * 16) * ldr + half * bk + kc * hb + s2
                        assert o % 2 == 0 and o + 1 < bm * ldr
                    for j in range(tn):
                        for h in (half, 1 - half):
                            o = (wn * tn * 16 + lane % 16 + j * 16) * ldr + h * bk + kc * hb + s2
                            assert o % 2 == 0 and o + 1 < bn * ldr


def bf16_swz(bk, r):
    return (((r >> 1) ^ (r >> 3)) & 3) if bk == 16 else (((r >> 2) ^ (r >> 3)) & 1)


def bf16_chunk_at(bk, r, word):
    return r * bk + (((word >> 2) ^ bf16_swz(bk, r)) << 2)


def test_bf16x3_tiles():
    shapes = instances("cgemm_bf16x3_ri")
    assert shapes
    for wm_, wn_, tm, tn, bk in shapes:
        bm, bn = wm_ * tm * 32, wn_ * tn * 32
        for rows in (bm, bn):
            for r, c in thread_loads(rows, bk, 4):
                assert r < rows and c + 3 < bk
                o = bf16_chunk_at(bk, r, c)
                assert o % 4 == 0 and r * bk <= o and o + 3 < (r + 1) * bk
        for lane in range(64):
            kq = (lane >> 5) * 4
            for w in range(4):
                wm, wn = w // wn_, w % wn_
                for kk in range(0, bk, 8):
                    for i in range(tm):
                        o = bf16_chunk_at(bk, wm * tm * 32 + lane % 32 + i * 32, kk + kq)
                        assert o % 4 == 0 and o + 3 < bm * bk
                    for j in range(tn):
                        o = bf16_chunk_at(bk, wn * tn * 32 + lane % 32 + j * 32, kk + kq)
                        assert o % 4 == 0 and o + 3 < bn * bk


def test_bf16x3_swizzle_spreads_banks():
    # For 32 banks (8 chunks per 128 bytes, 8 lanes of a 128-bit access per
    # cycle) and 64 banks (16 chunks, 16 lanes): the rows of one fragment
    # read, and the chunks of one staging store, fall on distinct chunks.
    for bk in (8, 16):
        cpr = bk // 4
        for group, nchunk in ((8, 8), (16, 16)):
            for r0 in range(0, 128, group):
                for q in range(cpr):
                    got = {(bf16_chunk_at(bk, r0 + l, 4 * q) // 4) % nchunk for l in range(group)}
                    assert len(got) == group
            for t0 in range(0, 256, group):
                got = {(bf16_chunk_at(bk, t // cpr, 4 * (t % cpr)) // 4) % nchunk
                       for t in range(t0, t0 + group)}
                assert len(got) == group


def test_guard_matters():
    # Without the guard, the 256 x 64 split-BF16 tile (B stage of 128 loads
    # of four complex) would send threads 128..255 to B rows 64..127.
    rows, bk, per = 64, 8, 4
    v = rows * bk // per
    assert v % 256 != 0
    unguarded = [(tid // (bk // per)) for tid in range(256)]
    assert max(unguarded) >= rows
    assert max(r for r, _ in thread_loads(rows, bk, per)) < rows


def find_job_model(prefix, n, w):
    """The grouped launches' two-round search (64 lanes per round)."""
    if n <= 4096:
        s = (n + 63) >> 6
        lanes = [j for j in range(64) if j * s < n and prefix[j * s] <= w]
        base = max(lanes) * s
        lanes = [j for j in range(64) if j < s and base + j < n and prefix[base + j] <= w]
        return base + max(lanes)
    lo, hi = 0, n - 1
    while lo < hi:
        mid = (lo + hi + 1) >> 1
        if prefix[mid] <= w:
            lo = mid
        else:
            hi = mid - 1
    return lo


def test_find_job_matches_definition():
    import random
    rnd = random.Random(7)
    for n in [1, 2, 3, 63, 64, 65, 127, 500, 4095, 4096, 4097, 6000]:
        sizes = [rnd.choice([0, 0, 1, 2, 5, 40]) for _ in range(n)]
        sizes[-1] = max(sizes[-1], 1)
        prefix = [0]
        for c in sizes:
            prefix.append(prefix[-1] + c)
        total = prefix[-1]
        for w in sorted(set([0, total - 1] + [rnd.randrange(total) for _ in range(50)])):
            want = max(i for i in range(n) if prefix[i] <= w)
            got = find_job_model(prefix, n, w)
            assert got == want
            assert prefix[got] <= w < prefix[got + 1]


def test_fp32_3m_large_tiles():
    shapes = instances("cgemm_f32_3mbig")
    assert shapes
    for wm_, wn_, tm, tn, bk in shapes:
        bm, bn, hb, ldr = wm_ * tm * 32, wn_ * tn * 32, bk // 2, 3 * bk + 4
        assert ldr % 4 == 0 and (ldr // 4) % 2 == 1  # odd number of 16-byte chunks
        for rows in (bm, bn):
            for r, c in thread_loads(rows, bk, 2):
                assert r < rows and c + 1 < bk and c % 2 == 0
                e = c >> 1
                for o in (e, hb + e, bk + e, bk + hb + e, 2 * bk + e, 2 * bk + hb + e):
                    assert 0 <= o < 3 * bk
        for lane in range(64):
            kh = lane >> 5
            for w in range(4):
                wm, wn = w // wn_, w % wn_
                for s4 in range(0, hb, 4):
                    for plane in range(3):
                        for i in range(tm):
                            row = wm * tm * 32 + lane % 32 + i * 32
                            o = row * ldr + kh * hb + s4 + plane * bk
                            assert o % 4 == 0 and row * ldr <= o and o + 3 < (row + 1) * ldr
                        for j in range(tn):
                            row = wn * tn * 32 + lane % 32 + j * 32
                            o = row * ldr + kh * hb + s4 + plane * bk
                            assert o % 4 == 0 and row * ldr <= o and o + 3 < (row + 1) * ldr


def dl_swz(r):
    return (r ^ (r >> 3)) & 7


def dl_swz16(r):
    return r & 15


def test_fp32_direct_lds_tiles():
    # Direct-to-LDS tile: a wave's copy writes 64 consecutive 16-byte slots;
    # slot s of a stage holds logical chunk (s % cpr) ^ swz(row) of row
    # s / cpr, with cpr = BK / 2 chunks per row (8 or 16).
    shapes = instances("cgemm_f32_dl")
    assert shapes
    for wm_, wn_, tm, tn, bk in shapes:
        assert bk in (16, 32)
        cpr = bk // 2
        swz = dl_swz if cpr == 8 else dl_swz16
        bm, bn = wm_ * tm * 32, wn_ * tn * 32
        for rows in (bm, bn):
            v = rows * cpr
            assert v % 256 == 0
            seen = set()
            for j in range(v // 256):
                for tid in range(256):
                    wave, lane = tid >> 6, tid & 63
                    s = tid + 256 * j
                    dst = 256 * j + 64 * wave + lane  # slot the copy writes
                    assert dst == s and 0 <= dst < v
                    r, c = s // cpr, (s % cpr) ^ swz(s // cpr)
                    assert r < rows and 0 <= 2 * c and 2 * c + 1 < bk
                    seen.add((r, c))
                    # the edge path stores the same logical chunk at the same slot
                    assert r * cpr + ((c ^ swz(r)) % cpr) == s
            assert len(seen) == v  # every chunk of the stage exactly once
        for lane in range(64):
            kh = lane >> 5
            for w in range(4):
                wm, wn = w // wn_, w % wn_
                for g in range(cpr // 2):
                    for base, t, n in ((wm * tm * 32, tm, bm), (wn * tn * 32, tn, bn)):
                        for i in range(t):
                            r = base + (lane & 31) + 32 * i
                            slot = r * cpr + ((2 * g + kh) ^ swz(r))
                            assert r < n and r * cpr <= slot < r * cpr + cpr
                            # the slot holds logical chunk 2g + kh of row r
                            assert ((slot % cpr) ^ swz(r)) == 2 * g + kh


def test_fp32_direct_lds_reads_spread_banks():
    # 128-bit fragment reads: 8 (32 banks) or 16 (64 banks) consecutive lanes
    # read consecutive rows at one logical chunk; their slots must fall on
    # distinct 16-byte bank groups, for rows of 8 and of 16 chunks.
    for cpr, swz in ((8, dl_swz), (16, dl_swz16)):
        for group, nchunk in ((8, 8), (16, 16)):
            for r0 in range(0, 256, group):
                for c in range(cpr):
                    got = {(r * cpr + (c ^ swz(r))) % nchunk for r in range(r0, r0 + group)}
                    assert len(got) == group


def test_fp64_direct_lds_tiles():
    # FP64 direct-to-LDS tile: one chunk is one complex, 8 per row; lane / 16
    # picks the chunk 4g + lane / 16 of a 16-row fragment.
    shapes = instances("cgemm_f64_dl")
    assert shapes
    for wm_, wn_, tm, tn, bk in shapes:
        assert bk == 8
        bm, bn = wm_ * tm * 16, wn_ * tn * 16
        for rows in (bm, bn):
            v = rows * 8
            assert v % 256 == 0
            seen = set()
            for j in range(v // 256):
                for tid in range(256):
                    s = tid + 256 * j
                    assert 256 * j + 64 * (tid >> 6) + (tid & 63) == s < v
                    r, c = s >> 3, (s & 7) ^ dl_swz(s >> 3)
                    assert r < rows and 0 <= c < bk
                    seen.add((r, c))
            assert len(seen) == v
        for lane in range(64):
            kq = lane >> 4
            for w in range(4):
                wm, wn = w // wn_, w % wn_
                for g in range(bk // 4):
                    for base, t, n in ((wm * tm * 16, tm, bm), (wn * tn * 16, tn, bn)):
                        for i in range(t):
                            r = base + (lane & 15) + 16 * i
                            slot = r * 8 + ((4 * g + kq) ^ dl_swz(r))
                            assert r < n and r * 8 <= slot < r * 8 + 8
                            assert ((slot & 7) ^ dl_swz(r)) == 4 * g + kq


def test_fp32_3m_direct_lds_tiles():
    # Same staging and fragment reads as the FP32-4M direct-to-LDS tile.
    shapes = instances("cgemm_f32_3mdl")
    assert shapes
    for wm_, wn_, tm, tn, bk in shapes:
        assert bk == 16
        bm, bn = wm_ * tm * 32, wn_ * tn * 32
        for rows in (bm, bn):
            assert (rows * 8) % 256 == 0
        for lane in range(64):
            kh = lane >> 5
            for w in range(4):
                wm, wn = w // wn_, w % wn_
                for g in range(4):
                    for base, t, n in ((wm * tm * 32, tm, bm), (wn * tn * 32, tn, bn)):
                        for i in range(t):
                            r = base + (lane & 31) + 32 * i
                            slot = r * 8 + ((2 * g + kh) ^ dl_swz(r))
                            assert r < n and r * 8 <= slot < r * 8 + 8


def test_bf16x3_direct_lds_tiles():
    # Slot s of a stage (one part, hi or lo) is row s / 4, stored chunk s % 4,
    # holding logical chunk (s % 4) ^ swz(row): the word offset 4 s equals
    # the Re/Im-split tile's chunk_at(row, 4 * logical chunk).
    shapes = instances("cgemm_bf16x3_dl")
    assert shapes
    for wm_, wn_, tm, tn, bk in shapes:
        assert bk == 16
        cpr = bk // 4
        bm, bn = wm_ * tm * 32, wn_ * tn * 32
        for rows in (bm, bn):
            v = rows * cpr
            assert v % 256 == 0
            seen = set()
            for j in range(v // 256):
                for tid in range(256):
                    s = tid + 256 * j
                    assert 256 * j + 64 * (tid >> 6) + (tid & 63) == s < v
                    r, q = s // cpr, (s % cpr) ^ bf16_swz(bk, s // cpr)
                    assert r < rows and 0 <= q < cpr
                    assert bf16_chunk_at(bk, r, 4 * q) == 4 * s
                    seen.add((r, q))
            assert len(seen) == v


def test_fp64_3m_direct_lds_tiles():
    # Same staging and fragment reads as the FP64 4M direct-to-LDS tile.
    shapes = instances("cgemm_f64_3mdl")
    assert shapes
    for wm_, wn_, tm, tn, bk in shapes:
        assert bk == 8
        bm, bn = wm_ * tm * 16, wn_ * tn * 16
        for rows in (bm, bn):
            assert (rows * 8) % 256 == 0
        for lane in range(64):
            kq = lane >> 4
            for w in range(4):
                wm, wn = w // wn_, w % wn_
                for g in range(bk // 4):
                    for base, t, n in ((wm * tm * 16, tm, bm), (wn * tn * 16, tn, bn)):
                        for i in range(t):
                            r = base + (lane & 15) + 16 * i
                            slot = r * 8 + ((4 * g + kq) ^ dl_swz(r))
                            assert r < n and r * 8 <= slot < r * 8 + 8


def test_fp64_gauss_tile_index():
    # bench.py selects the FP64 Gauss tile by index through a tune file: it
    # is the last FP64 tile before the four skinny ones.
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    table = SRC[SRC.index("kF64Tiles[] = {"):]
    table = table[:table.index("};")]
    entries = re.findall(r"\{\d+, \d+, \d+\}", table)
    assert bench.FP64_GAUSS_TILE == len(entries) - 5
    launch = SRC[SRC.index("void launch_tiles_f64(int tile"):]
    launch = launch[:launch.index("void launch_tiles_f64_grouped(")]
    assert re.search(r"else\s+cgemm_f64_3mdl<2, 2, 2, 2, 8>", launch)
    assert "tile == %d" % (bench.FP64_GAUSS_TILE - 1) in launch


def gauss_f(r):
    return (((r >> 2) ^ (r >> 4)) & 1) | (((r >> 3) & 1) << 1)


def test_bf16_gauss_planar_tiles():
    # Planar split-BF16 Gauss tile: per operand and stage, R LDS rows of 12
    # chunks (chunk j = 2 plane + half); slot s = tid + NT j (NT threads) is row s / 12,
    # stored chunk s % 12 holding logical chunk (s % 12) ^ f(row), at LDS
    # word 4 s.  Every (row, logical chunk) is filled once and stays in its
    # group of four; the fragment read of lane l (row l % 32 of a subtile,
    # plane q, half l / 32) finds the word its slot was copied to; the
    # global chunk (8 elements from 8 j in the row's 96-element stage group)
    # stays inside the group.
    shapes = instances("cgemm_bf16g_dl")
    assert shapes
    for wm_, wn_, tm, tn, bk in shapes:
        assert bk == 16
        nt = 64 * wm_ * wn_  # four or eight waves
        assert nt in (256, 512)
        for rows, sub, nsub in ((wm_ * tm * 32, tm, wm_), (wn_ * tn * 32, tn, wn_)):
            v = 12 * rows
            assert v % nt == 0
            where = {}
            for j in range(v // nt):
                for tid in range(nt):
                    s = tid + nt * j
                    assert nt * j + 64 * (tid >> 6) + (tid & 63) == s < v
                    r, ch = s // 12, (s % 12) ^ gauss_f(s // 12)
                    assert 0 <= ch < 12 and ch // 4 == (s % 12) // 4
                    assert 8 * ch + 8 <= 6 * bk
                    where[(r, ch)] = 4 * s
            assert len(where) == v
            for w in range(nsub):
                for i in range(sub):
                    for lane in range(64):
                        r = w * sub * 32 + i * 32 + (lane & 31)
                        for q in range(6):
                            ch = 2 * q + (lane >> 5)
                            word = r * 48 + ((ch ^ gauss_f(r)) << 2)
                            assert word == where[(r, ch)] and word + 4 <= 48 * rows


def test_bf16_gauss_reads_spread_banks():
    # 128-bit fragment reads of 16 (64 banks) or 32 (128 banks) consecutive
    # lanes: consecutive rows of 12 chunks at one logical chunk; their
    # 16-byte slots must fall on distinct bank groups.
    for group in (16, 32):
        for r0 in range(0, 256, group):
            for ch in range(12):
                got = {(12 * r + (ch ^ gauss_f(r))) % group for r in range(r0, r0 + group)}
                assert len(got) == group


def test_bf16_gauss_group_layout_formula():
    # The permute's address 6 (oo - w) + q W + w (w = oo % W) equals the
    # kernel's r 6K + 6W (k / W) + q W + k % W for oo = r K + k, W = min(16, K).
    for K in (1, 2, 4, 8, 16, 32, 64):
        W = min(16, K)
        seen = set()
        for r in range(3):
            for k in range(K):
                oo = r * K + k
                w = oo % W
                for q in range(6):
                    a = 6 * (oo - w) + q * W + w
                    assert a == r * 6 * K + 6 * W * (k // W) + q * W + k % W
                    seen.add(a)
        assert seen == set(range(3 * 6 * K))


def test_bf16_interleaved_layout_matches_tile_reads():
    # Permute kind 3 writes element oo = r K + k (K a multiple of 16) at word
    # 2 (oo - oo % 16) + oo % 16 (hi) and 16 words later (lo).  The
    # direct-to-LDS tile reads the 16-byte chunk of words c .. c + 3 of a
    # stage k0 (a multiple of 16) at row * 2K + 2 k0 + c (hi, A) and the
    # same plus 16 (lo, A2 = A + 16 words).  Every (row, k, part) must be
    # read from where it was written, and the writes must tile 2 M K words.
    assert "KIND == 3" in SRC and "kmul * k0" in SRC
    for K in (16, 32, 64):
        M = 3
        written = {}
        for r in range(M):
            for k in range(K):
                oo = r * K + k
                base = 2 * (oo - oo % 16) + oo % 16
                written[(r, k, 0)] = base
                written[(r, k, 1)] = base + 16
        assert sorted(written.values()) == list(range(2 * M * K))
        for r in range(M):
            for k0 in range(0, K, 16):
                for c in range(0, 16, 4):
                    for part in (0, 1):
                        w0 = r * 2 * K + 2 * k0 + c + 16 * part
                        for t in range(4):
                            assert written[(r, k0 + c + t, part)] == w0 + t
