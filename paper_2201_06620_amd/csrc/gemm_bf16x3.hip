// Complex GEMM tiles of the split-BF16x3 mode (operands split into bf16
// hi + lo, products lo*hi + hi*lo + hi*hi on v_mfma_f32_32x32x16_bf16,
// FP32 accumulation) and their launcher.
#include "kcommon.hpp"

namespace rn {

// ---------------------------------------------------------------------------
// Split BF16 x3, 4M embedding, v_mfma_f32_32x32x16_bf16.
// Operands are bf16 complex pairs packed as uint32 (re low, im high), hi and
// lo parts in separate arrays.  Per 16 real k: lo*hi + hi*lo + hi*hi into
// one FP32 accumulator.
// ---------------------------------------------------------------------------
template <int WM, int WN, int TM, int TN, int BK>
__device__ __forceinline__ void cgemm_bf16x3_body(const GemmParams& p, int tm, int tn, int split,
                                                int b) {
  static_assert(WM * WN == 4, "four waves");
  static_assert(BK % 8 == 0, "eight complex k per MFMA");
  constexpr int BM = WM * TM * 32;
  constexpr int BN = WN * TN * 16;
  constexpr int LDK = BK + 4;       // uint32 per padded row
  constexpr int AV = BM * BK / 4;   // uint4 loads (4 complex) per array
  constexpr int BV = BN * BK / 4;
  constexpr int NA = (AV + 255) / 256;
  constexpr int NB = (BV + 255) / 256;
  __shared__ __align__(16) uint32_t Ah[2][BM * LDK];
  __shared__ __align__(16) uint32_t Al[2][BM * LDK];
  __shared__ __align__(16) uint32_t Bh[2][BN * LDK];
  __shared__ __align__(16) uint32_t Bl[2][BN * LDK];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t row0 = int64_t(tm) * BM;
  const int64_t col0 = int64_t(tn) * BN;
  const int64_t ao = batch_off(p.a_bs, p.nbb, b), bo = batch_off(p.b_bs, p.nbb, b);
  const uint32_t* __restrict__ Agh = reinterpret_cast<const uint32_t*>(p.A) + ao;
  const uint32_t* __restrict__ Agl = reinterpret_cast<const uint32_t*>(p.A2) + ao;
  const uint32_t* __restrict__ Bgh = reinterpret_cast<const uint32_t*>(p.B) + bo;
  const uint32_t* __restrict__ Bgl = reinterpret_cast<const uint32_t*>(p.B2) + bo;
  const int64_t kbeg = int64_t(split) * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int nk = (int)((kend - kbeg + BK - 1) / BK);

  uint4 rah[NA], ral[NA], rbh[NB], rbl[NB];
  auto ld4 = [&](const uint32_t* src, int64_t gk) -> uint4 {
    if (gk + 3 < kend) return *reinterpret_cast<const uint4*>(src);
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (gk < kend) v.x = src[0];
    if (gk + 1 < kend) v.y = src[1];
    if (gk + 2 < kend) v.z = src[2];
    return v;
  };
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      int idx = tid + 256 * j;
      uint4 h = make_uint4(0u, 0u, 0u, 0u), l = h;
      if (idx < AV) {
        int r = idx / (BK / 4), c = (idx % (BK / 4)) * 4;
        int64_t gr = row0 + r, gk = k0 + c;
        if (gr < p.M && gk < kend) {
          h = ld4(Agh + gr * p.lda + gk, gk);
          l = ld4(Agl + gr * p.lda + gk, gk);
        }
      }
      rah[j] = h;
      ral[j] = l;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      int idx = tid + 256 * j;
      uint4 h = make_uint4(0u, 0u, 0u, 0u), l = h;
      if (idx < BV) {
        int r = idx / (BK / 4), c = (idx % (BK / 4)) * 4;
        int64_t gr = col0 + r, gk = k0 + c;
        if (gr < p.N && gk < kend) {
          h = ld4(Bgh + gr * p.ldb + gk, gk);
          l = ld4(Bgl + gr * p.ldb + gk, gk);
        }
      }
      rbh[j] = h;
      rbl[j] = l;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      int idx = tid + 256 * j;
      if (idx < AV) {
        int r = idx / (BK / 4), c = (idx % (BK / 4)) * 4;
        *reinterpret_cast<uint4*>(&Ah[buf][r * LDK + c]) = rah[j];
        *reinterpret_cast<uint4*>(&Al[buf][r * LDK + c]) = ral[j];
      }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      int idx = tid + 256 * j;
      if (idx < BV) {
        int r = idx / (BK / 4), c = (idx % (BK / 4)) * 4;
        *reinterpret_cast<uint4*>(&Bh[buf][r * LDK + c]) = rbh[j];
        *reinterpret_cast<uint4*>(&Bl[buf][r * LDK + c]) = rbl[j];
      }
    }
  };

  v16f acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  // 32x32x16 bf16 roles: A row = lane % 32, real k = 8*(lane/32) + 0..7,
  // i.e. complex k 4*(lane/32) + 0..3 in interleaved (re, im) order; B real
  // column n = lane % 32 reads the same four complex b's of complex column
  // n / 2 and turns each packed (b_r, b_i) into (b_r, -b_i) for n even or
  // (b_i, b_r) for n odd.
  const int kq = (lane >> 5) * 4;
  const bool odd = lane & 1;
  const int arow = wm * TM * 32 + (lane & 31);
  const int bcol = wn * TN * 16 + ((lane & 31) >> 1);
  auto bfix = [&](v4u w) -> v4u {
    if (odd) return (w >> 16) | (w << 16);
    return w ^ 0x80000000u;
  };

  if (nk > 0) {
    gload(kbeg);
    sstore(0);
  }
  __syncthreads();
  for (int it = 0; it < nk; ++it) {
    const int buf = it & 1;
    if (it + 1 < nk) gload(kbeg + int64_t(it + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 8) {
      v8bf ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        int o = (arow + i * 32) * LDK + kk + kq;
        ah[i] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v4u*>(&Ah[buf][o]));
        al[i] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v4u*>(&Al[buf][o]));
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        int o = (bcol + j * 16) * LDK + kk + kq;
        bh[j] = __builtin_bit_cast(v8bf, bfix(*reinterpret_cast<const v4u*>(&Bh[buf][o])));
        bl[j] = __builtin_bit_cast(v8bf, bfix(*reinterpret_cast<const v4u*>(&Bl[buf][o])));
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
    }
    if (it + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

  const int khalf = lane >> 5;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        int64_t row = row0 + wm * TM * 32 + i * 32 + 8 * (e >> 2) + 4 * khalf + (e & 3);
        int n = wn * TN * 32 + j * 32 + (lane & 31);
        store_out<float>(p, b, split, row, col0 + (n >> 1), n & 1, acc[i][j][e]);
      }
}

template <int WM, int WN, int TM, int TN, int BK>
__device__ __forceinline__ void cgemm_bf16x3_ri_body(const GemmParams& p, int tm, int tn,
                                                     int split, int b) {
  static_assert(WM * WN == 4, "four waves");
  static_assert(BK % 8 == 0, "eight complex k per MFMA");
  constexpr int BM = WM * TM * 32;
  constexpr int BN = WN * TN * 32;  // complex columns
  // LDS rows of BK words (BK / 4 chunks of 16 bytes), unpadded: chunk q of
  // row r sits at chunk q ^ swz(r), which puts the rows one 128-bit read
  // touches (consecutive rows, same chunk) and the chunks one staging store
  // writes (whole consecutive rows) on distinct bank groups, for 32 or 64
  // four-byte banks.
  constexpr int LDK = BK;
  static_assert(BK == 8 || BK == 16, "swizzle defined for 2 or 4 chunks per row");
  auto swz = [](int r) -> int {
    return BK == 16 ? (((r >> 1) ^ (r >> 3)) & 3) : (((r >> 2) ^ (r >> 3)) & 1);
  };
  auto chunk_at = [&](int r, int word) -> int {  // word: multiple of 4 within the row
    return r * LDK + ((((word >> 2) ^ swz(r))) << 2);
  };
  constexpr int AV = BM * BK / 4;
  constexpr int BV = BN * BK / 4;
  constexpr int NA = (AV + 255) / 256;
  constexpr int NB = (BV + 255) / 256;
  __shared__ __align__(16) uint32_t Ah[2][BM * LDK];
  __shared__ __align__(16) uint32_t Al[2][BM * LDK];
  __shared__ __align__(16) uint32_t Bh[2][BN * LDK];
  __shared__ __align__(16) uint32_t Bl[2][BN * LDK];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t row0 = int64_t(tm) * BM;
  const int64_t col0 = int64_t(tn) * BN;
  const int64_t ao = batch_off(p.a_bs, p.nbb, b), bo = batch_off(p.b_bs, p.nbb, b);
  const uint32_t* __restrict__ Agh = reinterpret_cast<const uint32_t*>(p.A) + ao;
  const uint32_t* __restrict__ Agl = reinterpret_cast<const uint32_t*>(p.A2) + ao;
  const uint32_t* __restrict__ Bgh = reinterpret_cast<const uint32_t*>(p.B) + bo;
  const uint32_t* __restrict__ Bgl = reinterpret_cast<const uint32_t*>(p.B2) + bo;
  const int64_t kbeg = int64_t(split) * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int nk = (int)((kend - kbeg + BK - 1) / BK);

  const bool interior = row0 + BM <= p.M && col0 + BN <= p.N && (kend - kbeg) % BK == 0;
  uint4 rah[NA], ral[NA], rbh[NB], rbl[NB];
  // Interior tiles: unguarded loads (see the FP32 large tile).
  auto gload_fast = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      int idx = tid + 256 * j;
      if (AV % 256 == 0 || idx < AV) {  // threads past the tile load nothing
        int64_t o = (row0 + idx / (BK / 4)) * p.lda + k0 + (idx % (BK / 4)) * 4;
        rah[j] = *reinterpret_cast<const uint4*>(Agh + o);
        ral[j] = *reinterpret_cast<const uint4*>(Agl + o);
      }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      int idx = tid + 256 * j;
      if (BV % 256 == 0 || idx < BV) {
        int64_t o = (col0 + idx / (BK / 4)) * p.ldb + k0 + (idx % (BK / 4)) * 4;
        rbh[j] = *reinterpret_cast<const uint4*>(Bgh + o);
        rbl[j] = *reinterpret_cast<const uint4*>(Bgl + o);
      }
    }
  };
  auto ld4 = [&](const uint32_t* src, int64_t gk) -> uint4 {
    if (gk + 3 < kend) return *reinterpret_cast<const uint4*>(src);
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (gk < kend) v.x = src[0];
    if (gk + 1 < kend) v.y = src[1];
    if (gk + 2 < kend) v.z = src[2];
    return v;
  };
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      int idx = tid + 256 * j;
      uint4 h = make_uint4(0u, 0u, 0u, 0u), l = h;
      if (idx < AV) {
        int r = idx / (BK / 4), c = (idx % (BK / 4)) * 4;
        int64_t gr = row0 + r, gk = k0 + c;
        if (gr < p.M && gk < kend) {
          h = ld4(Agh + gr * p.lda + gk, gk);
          l = ld4(Agl + gr * p.lda + gk, gk);
        }
      }
      rah[j] = h;
      ral[j] = l;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      int idx = tid + 256 * j;
      uint4 h = make_uint4(0u, 0u, 0u, 0u), l = h;
      if (idx < BV) {
        int r = idx / (BK / 4), c = (idx % (BK / 4)) * 4;
        int64_t gr = col0 + r, gk = k0 + c;
        if (gr < p.N && gk < kend) {
          h = ld4(Bgh + gr * p.ldb + gk, gk);
          l = ld4(Bgl + gr * p.ldb + gk, gk);
        }
      }
      rbh[j] = h;
      rbl[j] = l;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      int idx = tid + 256 * j;
      if (AV % 256 == 0 || idx < AV) {
        int r = idx / (BK / 4), c = (idx % (BK / 4)) * 4;
        *reinterpret_cast<uint4*>(&Ah[buf][chunk_at(r, c)]) = rah[j];
        *reinterpret_cast<uint4*>(&Al[buf][chunk_at(r, c)]) = ral[j];
      }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      int idx = tid + 256 * j;
      if (BV % 256 == 0 || idx < BV) {
        int r = idx / (BK / 4), c = (idx % (BK / 4)) * 4;
        *reinterpret_cast<uint4*>(&Bh[buf][chunk_at(r, c)]) = rbh[j];
        *reinterpret_cast<uint4*>(&Bl[buf][chunk_at(r, c)]) = rbl[j];
      }
    }
  };

  v16f cr[TM][TN], ci[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) cr[i][j][e] = ci[i][j][e] = 0.f;

  // A row = lane % 32 and complex k 4*(lane/32) + 0..3 (interleaved re, im
  // = 8 real k); B complex column = lane % 32, same complex k.  Packed b
  // (b_r | b_i << 16) becomes (b_r, -b_i) for the real-part tile and
  // (b_i, b_r) for the imaginary-part tile.
  const int kq = (lane >> 5) * 4;
  const int arow = wm * TM * 32 + (lane & 31);
  const int bcol = wn * TN * 32 + (lane & 31);

  auto mainloop = [&](auto tag) {
  constexpr bool FAST = decltype(tag)::value;
  if (nk > 0) {
    if constexpr (FAST) gload_fast(kbeg); else gload(kbeg);
    sstore(0);
  }
  __syncthreads();
  for (int it = 0; it < nk; ++it) {
    const int buf = it & 1;
    if constexpr (FAST) {
      gload_fast(kbeg + int64_t(it + 1 < nk ? it + 1 : it) * BK);
      __builtin_amdgcn_sched_barrier(0);
    } else if (it + 1 < nk) {
      gload(kbeg + int64_t(it + 1) * BK);
    }
#pragma unroll
    for (int kk = 0; kk < BK; kk += 8) {
      v8bf ah[TM], al[TM];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        int o = chunk_at(arow + i * 32, kk + kq);
        ah[i] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v4u*>(&Ah[buf][o]));
        al[i] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v4u*>(&Al[buf][o]));
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        int o = chunk_at(bcol + j * 32, kk + kq);
        const v4u wh = *reinterpret_cast<const v4u*>(&Bh[buf][o]);
        const v4u wl = *reinterpret_cast<const v4u*>(&Bl[buf][o]);
        const v8bf bhr = __builtin_bit_cast(v8bf, wh ^ 0x80000000u);
        const v8bf blr = __builtin_bit_cast(v8bf, wl ^ 0x80000000u);
        const v8bf bhi = __builtin_bit_cast(v8bf, (wh >> 16) | (wh << 16));
        const v8bf bli = __builtin_bit_cast(v8bf, (wl >> 16) | (wl << 16));
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bhr, cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bhi, ci[i][j], 0, 0, 0);
          cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], blr, cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bli, ci[i][j], 0, 0, 0);
          cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bhr, cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bhi, ci[i][j], 0, 0, 0);
        }
      }
    }
    if (FAST || it + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }
  };
  if (interior) mainloop(BoolTag<true>{}); else mainloop(BoolTag<false>{});

  const int khalf = lane >> 5;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        int64_t row = row0 + wm * TM * 32 + i * 32 + 8 * (e >> 2) + 4 * khalf + (e & 3);
        int64_t col = col0 + wn * TN * 32 + j * 32 + (lane & 31);
        store_out<float>(p, b, split, row, col, 0, cr[i][j][e]);
        store_out<float>(p, b, split, row, col, 1, ci[i][j][e]);
      }
}

// Split-BF16x3 with direct-to-LDS staging: the LDS layout of the Re/Im-split
// BF16 tile (interleaved bf16 pairs, BK / 4 chunks of 16 bytes per row,
// chunk q of row r at q ^ swz(r)) filled by global_load_lds_dwordx4 on
// interior tiles (a wave writes 64 consecutive slots; slot s of a stage is
// row s / (BK / 4), stored chunk s % (BK / 4)).  One array per buffer and the
// stage loop unrolled by two, as in the FP32 direct-to-LDS tile.  The
// operands are either two arrays (hi, lo) or one row-interleaved array
// (p.ilv: per 16 k of a row, 16 hi words then 16 lo words), where a stage of
// a row is one 128-byte line rather than a 64-byte half line of each array.
template <int WM, int WN, int TM, int TN, int BK>
__device__ __forceinline__ void cgemm_bf16x3_dl_body(const GemmParams& p, int tm, int tn,
                                                     int split, int b) {
  static_assert(WM * WN == 4, "four waves");
  static_assert(BK == 16, "four 16-byte chunks per LDS row");
  constexpr int BM = WM * TM * 32;
  constexpr int BN = WN * TN * 32;  // complex columns
  constexpr int CPR = BK / 4;       // chunks per row
  constexpr int LDK = BK;           // words per row
  auto swz = [](int r) -> int { return ((r >> 1) ^ (r >> 3)) & 3; };
  auto chunk_at = [&](int r, int word) -> int {  // word: multiple of 4 within the row
    return r * LDK + ((((word >> 2) ^ swz(r))) << 2);
  };
  constexpr int AV = BM * CPR;  // chunks per stage and part
  constexpr int BV = BN * CPR;
  static_assert(AV % 256 == 0 && BV % 256 == 0, "whole waves of chunks");
  constexpr int NA = AV / 256;
  constexpr int NB = BV / 256;
  __shared__ __align__(16) uint32_t Ah0[BM * LDK], Ah1[BM * LDK], Al0[BM * LDK], Al1[BM * LDK];
  __shared__ __align__(16) uint32_t Bh0[BN * LDK], Bh1[BN * LDK], Bl0[BN * LDK], Bl1[BN * LDK];
  auto pick = [](auto t, uint32_t* x0, uint32_t* x1) -> uint32_t* {
    if constexpr (decltype(t)::value) return x1; else return x0;
  };

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t row0 = int64_t(tm) * BM;
  const int64_t col0 = int64_t(tn) * BN;
  const int64_t ao = batch_off(p.a_bs, p.nbb, b), bo = batch_off(p.b_bs, p.nbb, b);
  const uint32_t* __restrict__ Agh = reinterpret_cast<const uint32_t*>(p.A) + ao;
  const uint32_t* __restrict__ Agl = reinterpret_cast<const uint32_t*>(p.A2) + ao;
  const uint32_t* __restrict__ Bgh = reinterpret_cast<const uint32_t*>(p.B) + bo;
  const uint32_t* __restrict__ Bgl = reinterpret_cast<const uint32_t*>(p.B2) + bo;
  const int64_t kbeg = int64_t(split) * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int nk = (int)((kend - kbeg + BK - 1) / BK);
  const bool interior = row0 + BM <= p.M && col0 + BN <= p.N && (kend - kbeg) % BK == 0;
  // Row-interleaved operands (p.ilv): the 16 k of a stage start at word 2 k0
  // of the row, hi then lo (A2 = A + 16 words); otherwise at word k0.
  const int64_t kmul = 1 + p.ilv;

  auto dma = [&](auto buf, int64_t k0) {
    uint32_t* ah = pick(buf, Ah0, Ah1);
    uint32_t* al = pick(buf, Al0, Al1);
    uint32_t* bh = pick(buf, Bh0, Bh1);
    uint32_t* bl = pick(buf, Bl0, Bl1);
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int s = tid + 256 * j, r = s / CPR, q = (s % CPR) ^ swz(r);
      const int64_t o = (row0 + r) * p.lda + kmul * k0 + 4 * q;
      const int d = 4 * (256 * j + 64 * wave);
      __builtin_amdgcn_global_load_lds(Agh + o, (__attribute__((address_space(3))) void*)(ah + d),
                                       16, 0, 0);
      __builtin_amdgcn_global_load_lds(Agl + o, (__attribute__((address_space(3))) void*)(al + d),
                                       16, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int s = tid + 256 * j, r = s / CPR, q = (s % CPR) ^ swz(r);
      const int64_t o = (col0 + r) * p.ldb + kmul * k0 + 4 * q;
      const int d = 4 * (256 * j + 64 * wave);
      __builtin_amdgcn_global_load_lds(Bgh + o, (__attribute__((address_space(3))) void*)(bh + d),
                                       16, 0, 0);
      __builtin_amdgcn_global_load_lds(Bgl + o, (__attribute__((address_space(3))) void*)(bl + d),
                                       16, 0, 0);
    }
  };
  uint4 rah[NA], ral[NA], rbh[NB], rbl[NB];
  auto ld4 = [&](const uint32_t* src, int64_t gk) -> uint4 {
    if (gk + 3 < kend) return *reinterpret_cast<const uint4*>(src);
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (gk < kend) v.x = src[0];
    if (gk + 1 < kend) v.y = src[1];
    if (gk + 2 < kend) v.z = src[2];
    return v;
  };
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int s = tid + 256 * j, r = s / CPR, c = (s % CPR) * 4;
      const int64_t gr = row0 + r, gk = k0 + c, o = gr * p.lda + kmul * k0 + c;
      uint4 h = make_uint4(0u, 0u, 0u, 0u), l = h;
      if (gr < p.M && gk < kend) {
        h = ld4(Agh + o, gk);
        l = ld4(Agl + o, gk);
      }
      rah[j] = h;
      ral[j] = l;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int s = tid + 256 * j, r = s / CPR, c = (s % CPR) * 4;
      const int64_t gr = col0 + r, gk = k0 + c, o = gr * p.ldb + kmul * k0 + c;
      uint4 h = make_uint4(0u, 0u, 0u, 0u), l = h;
      if (gr < p.N && gk < kend) {
        h = ld4(Bgh + o, gk);
        l = ld4(Bgl + o, gk);
      }
      rbh[j] = h;
      rbl[j] = l;
    }
  };
  auto sstore = [&](auto buf) {
    uint32_t* ah = pick(buf, Ah0, Ah1);
    uint32_t* al = pick(buf, Al0, Al1);
    uint32_t* bh = pick(buf, Bh0, Bh1);
    uint32_t* bl = pick(buf, Bl0, Bl1);
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int s = tid + 256 * j, r = s / CPR, c = (s % CPR) * 4;
      *reinterpret_cast<uint4*>(ah + chunk_at(r, c)) = rah[j];
      *reinterpret_cast<uint4*>(al + chunk_at(r, c)) = ral[j];
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int s = tid + 256 * j, r = s / CPR, c = (s % CPR) * 4;
      *reinterpret_cast<uint4*>(bh + chunk_at(r, c)) = rbh[j];
      *reinterpret_cast<uint4*>(bl + chunk_at(r, c)) = rbl[j];
    }
  };

  v16f cr[TM][TN], ci[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) cr[i][j][e] = ci[i][j][e] = 0.f;

  // As in the Re/Im-split BF16 tile: A row lane % 32, complex k
  // 4 * (lane / 32) + 0..3 of each group of eight; packed b becomes
  // (b_r, -b_i) for the real tile and (b_i, b_r) for the imaginary tile.
  const int kq = (lane >> 5) * 4;
  const int arow = wm * TM * 32 + (lane & 31);
  const int bcol = wn * TN * 32 + (lane & 31);

  auto stage = [&](auto fast, auto cur, int it) {
    constexpr bool FAST = decltype(fast)::value;
    constexpr bool CUR = decltype(cur)::value;
    const uint32_t* ahs = pick(cur, Ah0, Ah1);
    const uint32_t* als = pick(cur, Al0, Al1);
    const uint32_t* bhs = pick(cur, Bh0, Bh1);
    const uint32_t* bls = pick(cur, Bl0, Bl1);
    if constexpr (FAST) {
      dma(BoolTag<!CUR>{}, kbeg + int64_t(it + 1 < nk ? it + 1 : it) * BK);
      __builtin_amdgcn_sched_barrier(0);
    } else if (it + 1 < nk) {
      gload(kbeg + int64_t(it + 1) * BK);
    }
#pragma unroll
    for (int kk = 0; kk < BK; kk += 8) {
      v8bf ah[TM], al[TM];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int o = chunk_at(arow + i * 32, kk + kq);
        ah[i] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v4u*>(ahs + o));
        al[i] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v4u*>(als + o));
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int o = chunk_at(bcol + j * 32, kk + kq);
        const v4u wh = *reinterpret_cast<const v4u*>(bhs + o);
        const v4u wl = *reinterpret_cast<const v4u*>(bls + o);
        const v8bf bhr = __builtin_bit_cast(v8bf, wh ^ 0x80000000u);
        const v8bf blr = __builtin_bit_cast(v8bf, wl ^ 0x80000000u);
        const v8bf bhi = __builtin_bit_cast(v8bf, (wh >> 16) | (wh << 16));
        const v8bf bli = __builtin_bit_cast(v8bf, (wl >> 16) | (wl << 16));
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bhr, cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bhi, ci[i][j], 0, 0, 0);
          cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], blr, cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bli, ci[i][j], 0, 0, 0);
          cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bhr, cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bhi, ci[i][j], 0, 0, 0);
        }
      }
    }
    if constexpr (FAST) {
      __builtin_amdgcn_s_waitcnt(0);  // this wave's copies have landed
    } else if (it + 1 < nk) {
      sstore(BoolTag<!CUR>{});
    }
    __syncthreads();
  };

  auto mainloop = [&](auto fast) {
    constexpr bool FAST = decltype(fast)::value;
    if (nk > 0) {
      if constexpr (FAST) {
        dma(BoolTag<false>{}, kbeg);
        __builtin_amdgcn_s_waitcnt(0);
      } else {
        gload(kbeg);
        sstore(BoolTag<false>{});
      }
    }
    __syncthreads();
    for (int it = 0; it < nk; it += 2) {
      stage(fast, BoolTag<false>{}, it);
      if (it + 1 < nk) stage(fast, BoolTag<true>{}, it + 1);
    }
  };
  if (interior) mainloop(BoolTag<true>{}); else mainloop(BoolTag<false>{});

  const int khalf = lane >> 5;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        int64_t row = row0 + wm * TM * 32 + i * 32 + 8 * (e >> 2) + 4 * khalf + (e & 3);
        int64_t col = col0 + wn * TN * 32 + j * 32 + (lane & 31);
        store_out<float>(p, b, split, row, col, 0, cr[i][j][e]);
        store_out<float>(p, b, split, row, col, 1, ci[i][j][e]);
      }
}

RN_GEMM_ENTRY(cgemm_bf16x3)
RN_GEMM_ENTRY(cgemm_bf16x3_ri)
// Column groups of 4 row tiles: on the rank-28 pair 444-445 against 435-439
// useful TFLOP/s with groups of 8 (2: 419, 16: 401, in one timing run).
RN_GEMM_ENTRY_OCC_GM(cgemm_bf16x3_dl, 2, 4)

// Split-BF16x3 in the Gauss (3M) form, direct-to-LDS.  Operands come from
// permute kind 2 in the planar-group layout: per row, per group of W = min(16,
// K) consecutive k, six planes of W bf16 each -- re hi, im hi, (re + im) hi,
// re lo, im lo, (re + im) lo -- so row r, plane q, k sits at element
// r * 6K + 6W (k / W) + q W + k % W, and a stage of 16 k of one row is 192
// contiguous bytes.  Per 16 complex k and 32 x 32 subtile, T1 = Ar.Br,
// T2 = Ai.Bi and T3 = (Ar + Ai).(Br + Bi), each lo*hi + hi*lo + hi*hi on
// v_mfma_f32_32x32x16_bf16 (nine MFMAs where the 4M form needs twelve);
// C = (T1 - T2) + i ((T3 - T1) - T2).  LDS per buffer and operand: R rows of
// 12 chunks of 16 bytes (chunk j = 2 * plane + half), logical chunk j of row
// r stored at j ^ f(r) (f < 4 keeps it in its group of four), which puts 16
// or 32 consecutive rows read at one chunk on distinct bank groups; slot s
// of a stage is row s / 12, stored chunk s % 12, and a wave's copies fill 64
// consecutive slots (about five rows of 192 contiguous bytes each).  Four
// waves (128 x 64) or eight (128 x 128, two waves per SIMD, one workgroup
// per CU) per workgroup.  Unbatched problems only.
template <int WM, int WN, int TM, int TN, int BK>
__device__ __forceinline__ void cgemm_bf16g_dl_body(const GemmParams& p, int tm, int tn,
                                                    int split, int b) {
  static_assert(WM * WN == 4 || WM * WN == 8, "four or eight waves");
  static_assert(BK == 16, "one MFMA k-step of 16 per stage");
  constexpr int NT = 64 * WM * WN;   // threads
  constexpr int BM = WM * TM * 32;
  constexpr int BN = WN * TN * 32;
  constexpr int RWD = 48;            // words per LDS row (12 chunks)
  constexpr int AW = BM * RWD;       // words per buffer
  constexpr int BW = BN * RWD;
  constexpr int NA = 12 * BM / NT;   // 16-byte slots per thread and stage
  constexpr int NB = 12 * BN / NT;
  static_assert((12 * BM) % NT == 0 && (12 * BN) % NT == 0, "whole waves of slots");
  auto f = [](int r) -> int { return (((r >> 2) ^ (r >> 4)) & 1) | (((r >> 3) & 1) << 1); };
  __shared__ __align__(16) uint32_t A0[AW], A1[AW], B0[BW], B1[BW];
  auto pick = [](auto t, uint32_t* x0, uint32_t* x1) -> uint32_t* {
    if constexpr (decltype(t)::value) return x1; else return x0;
  };
  (void)b;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t row0 = int64_t(tm) * BM;
  const int64_t col0 = int64_t(tn) * BN;
  const uint16_t* __restrict__ Ag = reinterpret_cast<const uint16_t*>(p.A);
  const uint16_t* __restrict__ Bg = reinterpret_cast<const uint16_t*>(p.B);
  const int64_t rsA = 6 * p.lda, rsB = 6 * p.ldb;  // elements per row
  const int64_t W = min(p.K, int64_t(16));          // k per plane group
  const int64_t kbeg = int64_t(split) * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int nk = (int)((kend - kbeg + BK - 1) / BK);
  const bool interior = row0 + BM <= p.M && col0 + BN <= p.N && (kend - kbeg) % BK == 0 &&
                        kbeg % BK == 0 && p.K % BK == 0;

  auto dma = [&](auto buf, int64_t k0) {
    uint32_t* a = pick(buf, A0, A1);
    uint32_t* bb = pick(buf, B0, B1);
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int s = tid + NT * j, r = s / 12, ch = (s % 12) ^ f(r);
      const uint16_t* src = Ag + (row0 + r) * rsA + 6 * k0 + 8 * ch;
      __builtin_amdgcn_global_load_lds(src,
                                       (__attribute__((address_space(3))) void*)(a + 4 * (NT * j + 64 * wave)),
                                       16, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int s = tid + NT * j, r = s / 12, ch = (s % 12) ^ f(r);
      const uint16_t* src = Bg + (col0 + r) * rsB + 6 * k0 + 8 * ch;
      __builtin_amdgcn_global_load_lds(src,
                                       (__attribute__((address_space(3))) void*)(bb + 4 * (NT * j + 64 * wave)),
                                       16, 0, 0);
    }
  };
  // Edge tiles: the same slots through registers, element by element, zero
  // outside M, N or the K chunk.
  uint4 ra[NA], rb[NB];
  auto ld8 = [&](const uint16_t* X, int64_t gr, int64_t rs, int q, int64_t gk) -> uint4 {
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t k = gk + e;
      if (k < kend)
        w[e >> 1] |= uint32_t(X[gr * rs + 6 * W * (k / W) + q * W + (k % W)]) << (16 * (e & 1));
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
  };
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int s = tid + NT * j, r = s / 12, ch = (s % 12) ^ f(r);
      ra[j] = row0 + r < p.M ? ld8(Ag, row0 + r, rsA, ch >> 1, k0 + 8 * (ch & 1))
                             : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int s = tid + NT * j, r = s / 12, ch = (s % 12) ^ f(r);
      rb[j] = col0 + r < p.N ? ld8(Bg, col0 + r, rsB, ch >> 1, k0 + 8 * (ch & 1))
                             : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto sstore = [&](auto buf) {
    uint32_t* a = pick(buf, A0, A1);
    uint32_t* bb = pick(buf, B0, B1);
#pragma unroll
    for (int j = 0; j < NA; ++j) *reinterpret_cast<uint4*>(a + 4 * (tid + NT * j)) = ra[j];
#pragma unroll
    for (int j = 0; j < NB; ++j) *reinterpret_cast<uint4*>(bb + 4 * (tid + NT * j)) = rb[j];
  };

  v16f t1[TM][TN], t2[TM][TN], t3[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) t1[i][j][e] = t2[i][j][e] = t3[i][j][e] = 0.f;

  // Lane l reads row l % 32 of its subtile, half l / 32 (k 0-7 or 8-15 of
  // the stage), in each of the six planes.
  const int hf = lane >> 5;
  auto frag = [&](const uint32_t* x, int q, int r) -> v8bf {
    return __builtin_bit_cast(
        v8bf, *reinterpret_cast<const v4u*>(x + r * RWD + (((2 * q + hf) ^ f(r)) << 2)));
  };

  auto stage = [&](auto fast, auto cur, int it) {
    constexpr bool FAST = decltype(fast)::value;
    constexpr bool CUR = decltype(cur)::value;
    const uint32_t* as = pick(cur, A0, A1);
    const uint32_t* bs = pick(cur, B0, B1);
    if constexpr (FAST) {
      dma(BoolTag<!CUR>{}, kbeg + int64_t(it + 1 < nk ? it + 1 : it) * BK);
      __builtin_amdgcn_sched_barrier(0);
    } else if (it + 1 < nk) {
      gload(kbeg + int64_t(it + 1) * BK);
    }
    // Planes: 0 re hi, 1 im hi, 2 (re + im) hi, 3 re lo, 4 im lo, 5 (re + im) lo.
    v8bf a[TM][6], bv[TN][6];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int q = 0; q < 6; ++q) a[i][q] = frag(as, q, wm * TM * 32 + i * 32 + (lane & 31));
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int q = 0; q < 6; ++q) bv[j][q] = frag(bs, q, wn * TN * 32 + j * 32 + (lane & 31));
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        t1[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][3], bv[j][0], t1[i][j], 0, 0, 0);
        t2[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][4], bv[j][1], t2[i][j], 0, 0, 0);
        t3[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][5], bv[j][2], t3[i][j], 0, 0, 0);
        t1[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], bv[j][3], t1[i][j], 0, 0, 0);
        t2[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][1], bv[j][4], t2[i][j], 0, 0, 0);
        t3[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][2], bv[j][5], t3[i][j], 0, 0, 0);
        t1[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][0], bv[j][0], t1[i][j], 0, 0, 0);
        t2[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][1], bv[j][1], t2[i][j], 0, 0, 0);
        t3[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i][2], bv[j][2], t3[i][j], 0, 0, 0);
      }
    if constexpr (FAST) {
      __builtin_amdgcn_s_waitcnt(0);  // this wave's copies have landed
    } else if (it + 1 < nk) {
      sstore(BoolTag<!CUR>{});
    }
    __syncthreads();
  };

  auto mainloop = [&](auto fast) {
    constexpr bool FAST = decltype(fast)::value;
    if (nk > 0) {
      if constexpr (FAST) {
        dma(BoolTag<false>{}, kbeg);
        __builtin_amdgcn_s_waitcnt(0);
      } else {
        gload(kbeg);
        sstore(BoolTag<false>{});
      }
    }
    __syncthreads();
    for (int it = 0; it < nk; it += 2) {
      stage(fast, BoolTag<false>{}, it);
      if (it + 1 < nk) stage(fast, BoolTag<true>{}, it + 1);
    }
  };
  if (interior) mainloop(BoolTag<true>{}); else mainloop(BoolTag<false>{});

  const int khalf = lane >> 5;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t row = row0 + wm * TM * 32 + i * 32 + 8 * (e >> 2) + 4 * khalf + (e & 3);
        const int64_t col = col0 + wn * TN * 32 + j * 32 + (lane & 31);
        const float x1 = t1[i][j][e], x2 = t2[i][j][e];
        store_out<float>(p, 0, split, row, col, 0, x1 - x2);
        store_out<float>(p, 0, split, row, col, 1, (t3[i][j][e] - x1) - x2);
      }
}

// Entry with 64 * WM * WN threads (four or eight waves), two waves per SIMD.
template <int WM, int WN, int TM, int TN, int BK>
__global__ __launch_bounds__(64 * WM * WN, 2) void cgemm_bf16g_dl(GemmParams p) {
  int tm, tn;
  tile_coords(p.tiles_m, p.tiles_n, tm, tn);
  cgemm_bf16g_dl_body<WM, WN, TM, TN, BK>(p, tm, tn, blockIdx.y, blockIdx.z);
}

// MFMA tile `tile` (index into this mode's tile table, not the one-thread
// or skinny kernels) over `grid` workgroups; errors via hipGetLastError.
void launch_tiles_bf16x3(int tile, dim3 grid, const GemmParams& p, hipStream_t s) {
  if (tile == 1)
    cgemm_bf16x3<2, 2, 2, 2, 16><<<grid, 256, 0, s>>>(p);
  else if (tile == 2)
    cgemm_bf16x3<2, 2, 1, 1, 16><<<grid, 256, 0, s>>>(p);
  else if (tile == 3)
    cgemm_bf16x3<2, 2, 4, 2, 8><<<grid, 256, 0, s>>>(p);
  else if (tile == 4)
    cgemm_bf16x3<2, 2, 2, 4, 8><<<grid, 256, 0, s>>>(p);
  else if (tile == 5)
    cgemm_bf16x3_ri<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(p);
  else if (tile == 6)
    cgemm_bf16x3_ri<2, 2, 2, 2, 8><<<grid, 256, 0, s>>>(p);
  else if (tile == 7)
    cgemm_bf16x3_ri<2, 2, 4, 1, 8><<<grid, 256, 0, s>>>(p);
  else if (tile == 8)
    cgemm_bf16x3_ri<2, 2, 2, 2, 16><<<grid, 256, 0, s>>>(p);
  else if (tile == 9)
    cgemm_bf16x3_dl<2, 2, 2, 2, 16><<<grid, 256, 0, s>>>(p);
  else if (tile == 11)  // planar operands (Gauss form), four waves
    cgemm_bf16g_dl<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(p);
  else if (tile == 12)  // planar operands (Gauss form), eight waves
    cgemm_bf16g_dl<2, 4, 2, 1, 16><<<grid, 512, 0, s>>>(p);
  else
    cgemm_bf16x3_dl<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(p);
}

void launch_tiles_bf16x3_grouped(int tile, dim3 grid, const GroupTable& t, hipStream_t s) {
  if (tile == 1) cgemm_bf16x3_grouped<2, 2, 2, 2, 16><<<grid, 256, 0, s>>>(t);
  else if (tile == 2) cgemm_bf16x3_grouped<2, 2, 1, 1, 16><<<grid, 256, 0, s>>>(t);
  else if (tile == 3) cgemm_bf16x3_grouped<2, 2, 4, 2, 8><<<grid, 256, 0, s>>>(t);
  else if (tile == 4) cgemm_bf16x3_grouped<2, 2, 2, 4, 8><<<grid, 256, 0, s>>>(t);
  else if (tile == 5) cgemm_bf16x3_ri_grouped<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(t);
  else if (tile == 6) cgemm_bf16x3_ri_grouped<2, 2, 2, 2, 8><<<grid, 256, 0, s>>>(t);
  else if (tile == 7) cgemm_bf16x3_ri_grouped<2, 2, 4, 1, 8><<<grid, 256, 0, s>>>(t);
  else if (tile == 8) cgemm_bf16x3_ri_grouped<2, 2, 2, 2, 16><<<grid, 256, 0, s>>>(t);
  else if (tile == 9) cgemm_bf16x3_dl_grouped<2, 2, 2, 2, 16><<<grid, 256, 0, s>>>(t);
  else cgemm_bf16x3_dl_grouped<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(t);
}

}  // namespace rn
