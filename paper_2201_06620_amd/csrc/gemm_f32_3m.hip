// Complex GEMM tiles of the FP32-3M mode (Gauss: 3 real products per
// complex product, v_mfma_f32_32x32x2f32) and their launcher.
#include "kcommon.hpp"

namespace rn {

// ---------------------------------------------------------------------------
// FP32, 3M (Gauss): T1 = Ar.Br, T2 = Ai.Bi, T3 = (Ar + Ai).(Br + Bi);
// Re C = T1 - T2, Im C = (T3 - T1) - T2.  v_mfma_f32_32x32x2_f32 with the
// two k of one instruction = two consecutive complex k: lane halves read
// different complex elements and use both parts, so the operands stay
// interleaved in memory and LDS (no planar copy) and each 32x32 tile is 32
// complex columns.  6 real flops per complex multiply-add are executed.
// ---------------------------------------------------------------------------
template <int WM, int WN, int TM, int TN, int BK>
__device__ __forceinline__ void cgemm_f32_3m_body(const GemmParams& p, int tm, int tn, int split,
                                                int b) {
  static_assert(WM * WN == 4, "four waves");
  static_assert(BK % 2 == 0, "two complex k per MFMA");
  constexpr int BM = WM * TM * 32;
  constexpr int BN = WN * TN * 32;  // complex columns
  constexpr int LDK = BK + 1;
  constexpr int AV = BM * BK / 2;
  constexpr int BV = BN * BK / 2;
  constexpr int NA = (AV + 255) / 256;
  constexpr int NB = (BV + 255) / 256;
  __shared__ float2 As[2][BM * LDK];
  __shared__ float2 Bs[2][BN * LDK];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t row0 = int64_t(tm) * BM;
  const int64_t col0 = int64_t(tn) * BN;
  const float2* __restrict__ Ag =
      reinterpret_cast<const float2*>(p.A) + batch_off(p.a_bs, p.nbb, b);
  const float2* __restrict__ Bg =
      reinterpret_cast<const float2*>(p.B) + batch_off(p.b_bs, p.nbb, b);
  const int64_t kbeg = int64_t(split) * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int nk = (int)((kend - kbeg + BK - 1) / BK);

  float4 ra[NA], rb[NB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      int idx = tid + 256 * j;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (idx < AV) {
        int r = idx / (BK / 2), c = (idx % (BK / 2)) * 2;
        int64_t gr = row0 + r, gk = k0 + c;
        if (gr < p.M) {
          const float2* src = Ag + gr * p.lda + gk;
          if (gk + 1 < kend) {
            v = *reinterpret_cast<const float4*>(src);
          } else if (gk < kend) {
            float2 t = src[0];
            v.x = t.x;
            v.y = t.y;
          }
        }
      }
      ra[j] = v;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      int idx = tid + 256 * j;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (idx < BV) {
        int r = idx / (BK / 2), c = (idx % (BK / 2)) * 2;
        int64_t gr = col0 + r, gk = k0 + c;
        if (gr < p.N) {
          const float2* src = Bg + gr * p.ldb + gk;
          if (gk + 1 < kend) {
            v = *reinterpret_cast<const float4*>(src);
          } else if (gk < kend) {
            float2 t = src[0];
            v.x = t.x;
            v.y = t.y;
          }
        }
      }
      rb[j] = v;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      int idx = tid + 256 * j;
      if (idx < AV) {
        int r = idx / (BK / 2), c = (idx % (BK / 2)) * 2;
        As[buf][r * LDK + c] = make_float2(ra[j].x, ra[j].y);
        As[buf][r * LDK + c + 1] = make_float2(ra[j].z, ra[j].w);
      }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      int idx = tid + 256 * j;
      if (idx < BV) {
        int r = idx / (BK / 2), c = (idx % (BK / 2)) * 2;
        Bs[buf][r * LDK + c] = make_float2(rb[j].x, rb[j].y);
        Bs[buf][r * LDK + c + 1] = make_float2(rb[j].z, rb[j].w);
      }
    }
  };

  v16f t1[TM][TN], t2[TM][TN], t3[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) t1[i][j][e] = t2[i][j][e] = t3[i][j][e] = 0.f;

  const int kh = lane >> 5;
  const int arow = wm * TM * 32 + (lane & 31);
  const int bcol = wn * TN * 32 + (lane & 31);

  if (nk > 0) {
    gload(kbeg);
    sstore(0);
  }
  __syncthreads();
  for (int it = 0; it < nk; ++it) {
    const int buf = it & 1;
    if (it + 1 < nk) gload(kbeg + int64_t(it + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      float ar[TM], ai[TM], as[TM], br[TN], bi[TN], bs[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        float2 a = As[buf][(arow + i * 32) * LDK + kk + kh];
        ar[i] = a.x;
        ai[i] = a.y;
        as[i] = a.x + a.y;
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        float2 v = Bs[buf][(bcol + j * 32) * LDK + kk + kh];
        br[j] = v.x;
        bi[j] = v.y;
        bs[j] = v.x + v.y;
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          t1[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[i], br[j], t1[i][j], 0, 0, 0);
          t2[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[i], bi[j], t2[i][j], 0, 0, 0);
          t3[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(as[i], bs[j], t3[i][j], 0, 0, 0);
        }
    }
    if (it + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        int64_t row = row0 + wm * TM * 32 + i * 32 + 8 * (e >> 2) + 4 * kh + (e & 3);
        int64_t col = col0 + wn * TN * 32 + j * 32 + (lane & 31);
        float a = t1[i][j][e], c = t2[i][j][e];
        store_out<float>(p, b, split, row, col, 0, a - c);
        store_out<float>(p, b, split, row, col, 1, (t3[i][j][e] - a) - c);
      }
}

// FP32-3M (Gauss) with the direct-to-LDS staging of the FP32-4M tile: the
// same interleaved, swizzled LDS rows; a lane's chunk [a_r, a_i, a_r', a_i']
// feeds T1 = Ar Br, T2 = Ai Bi and T3 = (Ar + Ai)(Br + Bi) for its two complex
// k (the sums formed after the fragment read), six MFMAs per tile and chunk
// where 4M takes eight.
template <int WM, int WN, int TM, int TN, int BK>
__device__ __forceinline__ void cgemm_f32_3mdl_body(const GemmParams& p, int tm, int tn,
                                                  int split, int b) {
  static_assert(WM * WN == 4, "four waves");
  static_assert(BK == 16, "eight 16-byte chunks per LDS row");
  constexpr int BM = WM * TM * 32;
  constexpr int BN = WN * TN * 32;  // complex columns
  constexpr int CPR = BK / 2;       // chunks per row
  constexpr int AV = BM * CPR;      // chunks per stage
  constexpr int BV = BN * CPR;
  static_assert(AV % 256 == 0 && BV % 256 == 0, "whole waves of chunks");
  constexpr int NA = AV / 256;
  constexpr int NB = BV / 256;
  // One array per buffer: with the buffer known at compile time in every
  // stage, the compiler can tell the copies into one buffer from the
  // fragment reads of the other and does not wait for the copies first.
  __shared__ __align__(16) float4 Ad0[AV], Ad1[AV];
  __shared__ __align__(16) float4 Bd0[BV], Bd1[BV];
  auto abuf = [&](auto t) -> float4* { if constexpr (decltype(t)::value) return Ad1; else return Ad0; };
  auto bbuf = [&](auto t) -> float4* { if constexpr (decltype(t)::value) return Bd1; else return Bd0; };

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t row0 = int64_t(tm) * BM;
  const int64_t col0 = int64_t(tn) * BN;
  const float2* __restrict__ Ag =
      reinterpret_cast<const float2*>(p.A) + batch_off(p.a_bs, p.nbb, b);
  const float2* __restrict__ Bg =
      reinterpret_cast<const float2*>(p.B) + batch_off(p.b_bs, p.nbb, b);
  const int64_t kbeg = int64_t(split) * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int nk = (int)((kend - kbeg + BK - 1) / BK);
  const bool interior = row0 + BM <= p.M && col0 + BN <= p.N && (kend - kbeg) % BK == 0;

  // Slot s = 256 j + tid of a stage: row s / 8, stored chunk s % 8, which
  // holds logical chunk (s % 8) ^ dl_swz(row).
  auto dma = [&](auto buf, int64_t k0) {
    float4* As = abuf(buf);
    float4* Bs = bbuf(buf);
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int s = tid + 256 * j, r = s >> 3, c = (s & 7) ^ dl_swz(r);
      __builtin_amdgcn_global_load_lds(
          Ag + (row0 + r) * p.lda + k0 + 2 * c,
          (__attribute__((address_space(3))) void*)(As + 256 * j + 64 * wave), 16, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int s = tid + 256 * j, r = s >> 3, c = (s & 7) ^ dl_swz(r);
      __builtin_amdgcn_global_load_lds(
          Bg + (col0 + r) * p.ldb + k0 + 2 * c,
          (__attribute__((address_space(3))) void*)(Bs + 256 * j + 64 * wave), 16, 0, 0);
    }
  };
  float4 ra[NA], rb[NB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int s = tid + 256 * j, r = s >> 3, c = s & 7;
      const int64_t gr = row0 + r, gk = k0 + 2 * c;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (gr < p.M) {
        const float2* src = Ag + gr * p.lda + gk;
        if (gk + 1 < kend) {
          v = *reinterpret_cast<const float4*>(src);
        } else if (gk < kend) {
          const float2 t = src[0];
          v.x = t.x;
          v.y = t.y;
        }
      }
      ra[j] = v;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int s = tid + 256 * j, r = s >> 3, c = s & 7;
      const int64_t gr = col0 + r, gk = k0 + 2 * c;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (gr < p.N) {
        const float2* src = Bg + gr * p.ldb + gk;
        if (gk + 1 < kend) {
          v = *reinterpret_cast<const float4*>(src);
        } else if (gk < kend) {
          const float2 t = src[0];
          v.x = t.x;
          v.y = t.y;
        }
      }
      rb[j] = v;
    }
  };
  auto sstore = [&](auto buf) {
    float4* As = abuf(buf);
    float4* Bs = bbuf(buf);
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int s = tid + 256 * j, r = s >> 3;
      As[r * CPR + ((s & 7) ^ dl_swz(r))] = ra[j];
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int s = tid + 256 * j, r = s >> 3;
      Bs[r * CPR + ((s & 7) ^ dl_swz(r))] = rb[j];
    }
  };

  v16f t1[TM][TN], t2[TM][TN], t3[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) t1[i][j][e] = t2[i][j][e] = t3[i][j][e] = 0.f;

  const int kh = lane >> 5;
  const int arow = wm * TM * 32 + (lane & 31);
  const int brow = wn * TN * 32 + (lane & 31);

  // One K stage computed from buffer CUR while the next stage fills the
  // other buffer.
  auto stage = [&](auto fast, auto cur, int it) {
    constexpr bool FAST = decltype(fast)::value;
    constexpr bool CUR = decltype(cur)::value;
    const float4* As = abuf(cur);
    const float4* Bs = bbuf(cur);
    // Fast path: always fill the other buffer (the last stage copies itself
    // again), so the stage has no branch.
    if constexpr (FAST) {
      dma(BoolTag<!CUR>{}, kbeg + int64_t(it + 1 < nk ? it + 1 : it) * BK);
      __builtin_amdgcn_sched_barrier(0);
    } else if (it + 1 < nk) {
      gload(kbeg + int64_t(it + 1) * BK);
    }
#pragma unroll
    for (int g = 0; g < CPR / 2; ++g) {
      float4 a4[TM], b4[TN];
      float2 as[TM], bs[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int r = arow + 32 * i;
        a4[i] = As[r * CPR + ((2 * g + kh) ^ dl_swz(r))];
        as[i] = make_float2(a4[i].x + a4[i].y, a4[i].z + a4[i].w);
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int r = brow + 32 * j;
        b4[j] = Bs[r * CPR + ((2 * g + kh) ^ dl_swz(r))];
        bs[j] = make_float2(b4[j].x + b4[j].y, b4[j].z + b4[j].w);
      }
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            const float ar = q ? a4[i].z : a4[i].x, ai = q ? a4[i].w : a4[i].y;
            const float br = q ? b4[j].z : b4[j].x, bi = q ? b4[j].w : b4[j].y;
            const float sa = q ? as[i].y : as[i].x, sb = q ? bs[j].y : bs[j].x;
            t1[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, br, t1[i][j], 0, 0, 0);
            t2[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, bi, t2[i][j], 0, 0, 0);
            t3[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(sa, sb, t3[i][j], 0, 0, 0);
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

#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        int64_t row = row0 + wm * TM * 32 + i * 32 + 8 * (e >> 2) + 4 * kh + (e & 3);
        int64_t col = col0 + wn * TN * 32 + j * 32 + (lane & 31);
        const float a = t1[i][j][e], c = t2[i][j][e], d = t3[i][j][e];
        store_out<float>(p, b, split, row, col, 0, a - c);
        store_out<float>(p, b, split, row, col, 1, (d - a) - c);
      }
}

// Large-tile FP32-3M (Gauss): T1 = Ar Br, T2 = Ai Bi, T3 = (Ar + Ai)(Br + Bi)
// as three real MFMA GEMMs whose K is the complex K (lane / 32 picks the
// complex k of an instruction).  Each LDS row holds three planes (re, im,
// re + im; the sums formed once while staging), each ordered [even k | odd
// k], so the values one lane needs for four consecutive instructions are
// adjacent and come in one 128-bit read; rows padded to an odd number of
// 16-byte chunks.  Interior tiles use the pinned fast path of the FP32 large
// tile.
template <int WM, int WN, int TM, int TN, int BK>
__device__ __forceinline__ void cgemm_f32_3mbig_body(const GemmParams& p, int tm, int tn,
                                                     int split, int b) {
  static_assert(WM * WN == 4, "four waves");
  static_assert(BK % 8 == 0, "four instructions (eight complex k) per 128-bit read");
  constexpr int BM = WM * TM * 32;
  constexpr int BN = WN * TN * 32;
  constexpr int HB = BK / 2;
  constexpr int LDR = 3 * BK + 4;  // floats per row: 3 planes + pad (odd chunk count)
  constexpr int AV = BM * BK / 2;  // float4 loads (two complex) per stage
  constexpr int BV = BN * BK / 2;
  constexpr int NA = (AV + 255) / 256;
  constexpr int NB = (BV + 255) / 256;
  __shared__ __align__(16) float As0[2 * BM * LDR];
  __shared__ __align__(16) float Bs0[2 * BN * LDR];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t row0 = int64_t(tm) * BM;
  const int64_t col0 = int64_t(tn) * BN;
  const float2* __restrict__ Ag =
      reinterpret_cast<const float2*>(p.A) + batch_off(p.a_bs, p.nbb, b);
  const float2* __restrict__ Bg =
      reinterpret_cast<const float2*>(p.B) + batch_off(p.b_bs, p.nbb, b);
  const int64_t kbeg = int64_t(split) * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int nk = (int)((kend - kbeg + BK - 1) / BK);
  const bool interior = row0 + BM <= p.M && col0 + BN <= p.N && (kend - kbeg) % BK == 0;

  float4 ra[NA], rb[NB];
  auto gload_fast = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      int idx = tid + 256 * j;
      if (AV % 256 == 0 || idx < AV) {  // threads past the tile load nothing
        int r = idx / (BK / 2), c = (idx % (BK / 2)) * 2;
        ra[j] = *reinterpret_cast<const float4*>(Ag + (row0 + r) * p.lda + k0 + c);
      }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      int idx = tid + 256 * j;
      if (BV % 256 == 0 || idx < BV) {
        int r = idx / (BK / 2), c = (idx % (BK / 2)) * 2;
        rb[j] = *reinterpret_cast<const float4*>(Bg + (col0 + r) * p.ldb + k0 + c);
      }
    }
  };
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      int idx = tid + 256 * j;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (idx < AV) {
        int r = idx / (BK / 2), c = (idx % (BK / 2)) * 2;
        int64_t gr = row0 + r, gk = k0 + c;
        if (gr < p.M) {
          const float2* src = Ag + gr * p.lda + gk;
          if (gk + 1 < kend) {
            v = *reinterpret_cast<const float4*>(src);
          } else if (gk < kend) {
            float2 t = src[0];
            v.x = t.x;
            v.y = t.y;
          }
        }
      }
      ra[j] = v;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      int idx = tid + 256 * j;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (idx < BV) {
        int r = idx / (BK / 2), c = (idx % (BK / 2)) * 2;
        int64_t gr = col0 + r, gk = k0 + c;
        if (gr < p.N) {
          const float2* src = Bg + gr * p.ldb + gk;
          if (gk + 1 < kend) {
            v = *reinterpret_cast<const float4*>(src);
          } else if (gk < kend) {
            float2 t = src[0];
            v.x = t.x;
            v.y = t.y;
          }
        }
      }
      rb[j] = v;
    }
  };
  // Complex k = c (even) and c + 1 go to index c / 2 of the even and odd
  // halves of each plane.
  auto put = [](float* row, int c, const float4& v) {
    const int e = c >> 1;
    row[e] = v.x;
    row[HB + e] = v.z;
    row[BK + e] = v.y;
    row[BK + HB + e] = v.w;
    row[2 * BK + e] = v.x + v.y;
    row[2 * BK + HB + e] = v.z + v.w;
  };
  auto sstore = [&](int buf) {
    float* As = As0 + buf * BM * LDR;
    float* Bs = Bs0 + buf * BN * LDR;
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      int idx = tid + 256 * j;
      if (AV % 256 == 0 || idx < AV) put(As + (idx / (BK / 2)) * LDR, (idx % (BK / 2)) * 2, ra[j]);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      int idx = tid + 256 * j;
      if (BV % 256 == 0 || idx < BV) put(Bs + (idx / (BK / 2)) * LDR, (idx % (BK / 2)) * 2, rb[j]);
    }
  };

  v16f t1[TM][TN], t2[TM][TN], t3[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) t1[i][j][e] = t2[i][j][e] = t3[i][j][e] = 0.f;

  const int kh = lane >> 5;
  const int aoff = (wm * TM * 32 + (lane & 31)) * LDR + kh * HB;
  const int boff = (wn * TN * 32 + (lane & 31)) * LDR + kh * HB;

  auto mainloop = [&](auto tag) {
    constexpr bool FAST = decltype(tag)::value;
    if (nk > 0) {
      if constexpr (FAST) gload_fast(kbeg); else gload(kbeg);
      sstore(0);
    }
    __syncthreads();
    for (int it = 0; it < nk; ++it) {
      const int buf = it & 1;
      const float* As = As0 + buf * BM * LDR;
      const float* Bs = Bs0 + buf * BN * LDR;
      if constexpr (FAST) {
        gload_fast(kbeg + int64_t(it + 1 < nk ? it + 1 : it) * BK);
        __builtin_amdgcn_sched_barrier(0);
      } else if (it + 1 < nk) {
        gload(kbeg + int64_t(it + 1) * BK);
      }
#pragma unroll
      for (int s4 = 0; s4 < HB; s4 += 4) {
        float4 ar[TM], ai[TM], as[TM], br[TN], bi[TN], bs[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          const float* a = As + aoff + i * 32 * LDR + s4;
          ar[i] = *reinterpret_cast<const float4*>(a);
          ai[i] = *reinterpret_cast<const float4*>(a + BK);
          as[i] = *reinterpret_cast<const float4*>(a + 2 * BK);
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const float* v = Bs + boff + j * 32 * LDR + s4;
          br[j] = *reinterpret_cast<const float4*>(v);
          bi[j] = *reinterpret_cast<const float4*>(v + BK);
          bs[j] = *reinterpret_cast<const float4*>(v + 2 * BK);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
              auto pick = [q](const float4& v) {
                return q == 0 ? v.x : q == 1 ? v.y : q == 2 ? v.z : v.w;
              };
              t1[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(pick(ar[i]), pick(br[j]), t1[i][j],
                                                              0, 0, 0);
              t2[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(pick(ai[i]), pick(bi[j]), t2[i][j],
                                                              0, 0, 0);
              t3[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(pick(as[i]), pick(bs[j]), t3[i][j],
                                                              0, 0, 0);
            }
      }
      if (FAST || it + 1 < nk) sstore(buf ^ 1);
      __syncthreads();
    }
  };
  if (interior) mainloop(BoolTag<true>{}); else mainloop(BoolTag<false>{});

#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        int64_t row = row0 + wm * TM * 32 + i * 32 + 8 * (e >> 2) + 4 * kh + (e & 3);
        int64_t col = col0 + wn * TN * 32 + j * 32 + (lane & 31);
        const float a = t1[i][j][e], c = t2[i][j][e], d = t3[i][j][e];
        store_out<float>(p, b, split, row, col, 0, a - c);
        store_out<float>(p, b, split, row, col, 1, (d - a) - c);
      }
}

RN_GEMM_ENTRY(cgemm_f32_3m)
RN_GEMM_ENTRY_OCC(cgemm_f32_3mdl, 2)
RN_GEMM_ENTRY(cgemm_f32_3mbig)

// MFMA tile `tile` (index into this mode's tile table, not the one-thread
// or skinny kernels) over `grid` workgroups; errors via hipGetLastError.
void launch_tiles_f32_3m(int tile, dim3 grid, const GemmParams& p, hipStream_t s) {
  if (tile == 1)
    cgemm_f32_3m<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(p);
  else if (tile == 2)
    cgemm_f32_3m<2, 2, 1, 1, 16><<<grid, 256, 0, s>>>(p);
  else if (tile == 3)
    cgemm_f32_3mbig<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(p);
  else if (tile == 4)
    cgemm_f32_3mbig<2, 2, 1, 2, 16><<<grid, 256, 0, s>>>(p);
  else if (tile == 5)
    cgemm_f32_3mdl<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(p);
  else
    cgemm_f32_3mdl<2, 2, 1, 2, 16><<<grid, 256, 0, s>>>(p);
}

void launch_tiles_f32_3m_grouped(int tile, dim3 grid, const GroupTable& t, hipStream_t s) {
  if (tile == 1) cgemm_f32_3m_grouped<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(t);
  else if (tile == 2) cgemm_f32_3m_grouped<2, 2, 1, 1, 16><<<grid, 256, 0, s>>>(t);
  else if (tile == 3) cgemm_f32_3mbig_grouped<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(t);
  else if (tile == 4) cgemm_f32_3mbig_grouped<2, 2, 1, 2, 16><<<grid, 256, 0, s>>>(t);
  else if (tile == 5) cgemm_f32_3mdl_grouped<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(t);
  else cgemm_f32_3mdl_grouped<2, 2, 1, 2, 16><<<grid, 256, 0, s>>>(t);
}

}  // namespace rn
