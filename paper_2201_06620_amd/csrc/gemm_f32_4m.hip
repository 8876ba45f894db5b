// Complex GEMM tiles of the FP32-4M mode (4 real products per complex
// product, v_mfma_f32_32x32x2f32) and their launcher.
#include "kcommon.hpp"

namespace rn {

// ---------------------------------------------------------------------------
// FP32, 4M embedding, v_mfma_f32_32x32x2_f32.
// WM x WN waves; each wave owns TM x TN MFMA tiles of 32 x 32 real outputs.
// ---------------------------------------------------------------------------
template <int WM, int WN, int TM, int TN, int BK>
__device__ __forceinline__ void cgemm_f32_4m_body(const GemmParams& p, int tm, int tn, int split,
                                                int b) {
  static_assert(WM * WN == 4, "four waves");
  constexpr int BM = WM * TM * 32;
  constexpr int BN = WN * TN * 16;  // complex columns
  constexpr int LDK = BK + 1;       // padded LDS row, complex elements
  constexpr int AV = BM * BK / 2;   // float4 (two complex) loads per A chunk
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

  v16f acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  // Lane roles in the 32x32x2 MFMA: A operand row = lane % 32, k = lane / 32
  // (k 0 = real part, k 1 = imaginary part of the complex a); B operand real
  // column n = lane % 32 (complex column n / 2, part n & 1), same k.
  const int khalf = lane >> 5;
  const int par = lane & 1;
  const bool b_take_re = (khalf == par);
  const uint32_t b_sign = (khalf == 1 && par == 0) ? 0x80000000u : 0u;
  const int arow = wm * TM * 32 + (lane & 31);
  const int bcol = wn * TN * 16 + ((lane & 31) >> 1);

  if (nk > 0) {
    gload(kbeg);
    sstore(0);
  }
  __syncthreads();
  for (int it = 0; it < nk; ++it) {
    const int buf = it & 1;
    if (it + 1 < nk) gload(kbeg + int64_t(it + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      float af[TM], bf[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        float2 a = As[buf][(arow + i * 32) * LDK + kk];
        af[i] = khalf ? a.y : a.x;
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        float2 bv = Bs[buf][(bcol + j * 16) * LDK + kk];
        float v = b_take_re ? bv.x : bv.y;
        bf[j] = __uint_as_float(__float_as_uint(v) ^ b_sign);
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    if (it + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

  // 32x32 accumulator layout: lane holds real column lane % 32 and rows
  // 8*(e/4) + 4*(lane/32) + e%4 for e = 0..15.
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

// ---------------------------------------------------------------------------
// Re/Im-split variants of the 4M kernels.  Each 32x32 MFMA tile covers 32
// complex columns and comes in a pair: one accumulates the real parts and
// one the imaginary parts of C.  For the real part, B's embedded rows are
// (b_r, -b_i) per complex k; for the imaginary part (b_i, b_r).  All lanes
// of one MFMA then apply the same transform to the same complex B values,
// so a B fragment is read from LDS once for both tiles and no lane diverges.
// ---------------------------------------------------------------------------
template <int WM, int WN, int TM, int TN, int BK>
__device__ __forceinline__ void cgemm_f32_ri_body(const GemmParams& p, int tm, int tn, int split,
                                                  int b) {
  static_assert(WM * WN == 4, "four waves");
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

  v16f cr[TM][TN], ci[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) cr[i][j][e] = ci[i][j][e] = 0.f;

  // Lane roles: A row = lane % 32, real k = lane / 32 (0: re, 1: im part of
  // complex a); B complex column = lane % 32, same real k.
  const int kh = lane >> 5;
  const uint32_t neg = kh ? 0x80000000u : 0u;
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
    for (int kk = 0; kk < BK; ++kk) {
      float af[TM], br[TN], bi[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        float2 a = As[buf][(arow + i * 32) * LDK + kk];
        af[i] = kh ? a.y : a.x;
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        float2 v = Bs[buf][(bcol + j * 32) * LDK + kk];
        // Real-part row: (b_r, -b_i); imaginary-part row: (b_i, b_r).
        br[j] = __uint_as_float(__float_as_uint(kh ? v.y : v.x) ^ neg);
        bi[j] = kh ? v.x : v.y;
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i], br[j], cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i], bi[j], ci[i][j], 0, 0, 0);
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
        store_out<float>(p, b, split, row, col, 0, cr[i][j][e]);
        store_out<float>(p, b, split, row, col, 1, ci[i][j][e]);
      }
}

// ---------------------------------------------------------------------------
// Re/Im-split tiles with planar LDS rows.  While staging a chunk into LDS,
// each row of A is stored as [a_r(0..BK-1) | a_i(0..BK-1)] and each row of B
// as [b_r(0..BK-1) | -b_i(0..BK-1)], so the MFMA lane whose real k is the
// imaginary half reads the second half directly: no per-fragment select.
// The real-part tile uses B rows as stored; the imaginary-part tile needs
// (b_i, b_r), read from the other half with one sign flip on the first.
// ---------------------------------------------------------------------------
template <int WM, int WN, int TM, int TN, int BK>
__device__ __forceinline__ void cgemm_f32_rp_body(const GemmParams& p, int tm, int tn, int split,
                                                  int b) {
  static_assert(WM * WN == 4, "four waves");
  constexpr int BM = WM * TM * 32;
  constexpr int BN = WN * TN * 32;  // complex columns
  constexpr int LDR = 2 * BK + 1;   // floats per padded LDS row
  constexpr int AV = BM * BK / 2;
  constexpr int BV = BN * BK / 2;
  constexpr int NA = (AV + 255) / 256;
  constexpr int NB = (BV + 255) / 256;
  __shared__ float As[2][BM * LDR];
  __shared__ float Bs[2][BN * LDR];

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
        float* row = &As[buf][r * LDR];
        row[c] = ra[j].x;
        row[c + 1] = ra[j].z;
        row[BK + c] = ra[j].y;
        row[BK + c + 1] = ra[j].w;
      }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      int idx = tid + 256 * j;
      if (idx < BV) {
        int r = idx / (BK / 2), c = (idx % (BK / 2)) * 2;
        float* row = &Bs[buf][r * LDR];
        row[c] = rb[j].x;
        row[c + 1] = rb[j].z;
        row[BK + c] = -rb[j].y;
        row[BK + c + 1] = -rb[j].w;
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

  const int kh = lane >> 5;
  const int aoff = (wm * TM * 32 + (lane & 31)) * LDR + kh * BK;
  const int boff_r = (wn * TN * 32 + (lane & 31)) * LDR + kh * BK;
  const int boff_i = (wn * TN * 32 + (lane & 31)) * LDR + (1 - kh) * BK;
  const uint32_t flip = kh ? 0u : 0x80000000u;  // Im row: (-(-b_i), b_r)

  if (nk > 0) {
    gload(kbeg);
    sstore(0);
  }
  __syncthreads();
  for (int it = 0; it < nk; ++it) {
    const int buf = it & 1;
    if (it + 1 < nk) gload(kbeg + int64_t(it + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      float af[TM], br[TN], bi[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) af[i] = As[buf][aoff + i * 32 * LDR + kk];
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        br[j] = Bs[buf][boff_r + j * 32 * LDR + kk];
        bi[j] = __uint_as_float(__float_as_uint(Bs[buf][boff_i + j * 32 * LDR + kk]) ^ flip);
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i], br[j], cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i], bi[j], ci[i][j], 0, 0, 0);
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
        store_out<float>(p, b, split, row, col, 0, cr[i][j][e]);
        store_out<float>(p, b, split, row, col, 1, ci[i][j][e]);
      }
}

// Large-tile FP32-4M: each wave owns TM x TN Re/Im tile pairs (up to 16
// accumulators), LDS rows padded to a multiple of 16 bytes so a lane reads
// four consecutive k of its row in one 128-bit LDS read, and staging writes
// are 64-bit.  Rows [a_r | a_i] and [b_r | -b_i] as in the planar tile; the
// padding of 4 floats puts 16 consecutive rows on distinct 16-byte bank
// groups.
template <int WM, int WN, int TM, int TN, int BK>
__device__ __forceinline__ void cgemm_f32_big_body(const GemmParams& p, int tm, int tn,
                                                   int split, int b) {
  static_assert(WM * WN == 4, "four waves");
  static_assert(BK % 4 == 0, "k in groups of four");
  constexpr int BM = WM * TM * 32;
  constexpr int BN = WN * TN * 32;  // complex columns
  constexpr int LDR = 2 * BK + 4;   // floats per LDS row, 16-byte multiple
  constexpr int AV = BM * BK / 2;   // float4 loads (two complex) per stage
  constexpr int BV = BN * BK / 2;
  constexpr int NA = (AV + 255) / 256;
  constexpr int NB = (BV + 255) / 256;
  extern __shared__ float4 big_lds[];
  float* As0 = reinterpret_cast<float*>(big_lds);
  float* Bs0 = As0 + 2 * BM * LDR;

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

  // Interior tiles (whole tile inside M x N, K chunk a multiple of BK) load
  // without guards, so no load sits behind a divergent branch and the loads
  // of the next stage stay in flight across the MFMA phase.
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
  auto sstore = [&](int buf) {
    float* As = As0 + buf * BM * LDR;
    float* Bs = Bs0 + buf * BN * LDR;
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      int idx = tid + 256 * j;
      if (AV % 256 == 0 || idx < AV) {
        int r = idx / (BK / 2), c = (idx % (BK / 2)) * 2;
        float* row = As + r * LDR;
        row[c] = ra[j].x;
        row[c + 1] = ra[j].z;
        row[BK + c] = ra[j].y;
        row[BK + c + 1] = ra[j].w;
      }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      int idx = tid + 256 * j;
      if (BV % 256 == 0 || idx < BV) {
        int r = idx / (BK / 2), c = (idx % (BK / 2)) * 2;
        float* row = Bs + r * LDR;
        row[c] = rb[j].x;
        row[c + 1] = rb[j].z;
        row[BK + c] = -rb[j].y;
        row[BK + c + 1] = -rb[j].w;
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

  const int kh = lane >> 5;
  const int aoff = (wm * TM * 32 + (lane & 31)) * LDR + kh * BK;
  const int boff_r = (wn * TN * 32 + (lane & 31)) * LDR + kh * BK;
  const int boff_i = (wn * TN * 32 + (lane & 31)) * LDR + (1 - kh) * BK;
  const uint32_t flip = kh ? 0u : 0x80000000u;  // Im row: (-(-b_i), b_r)

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
    // Fast path: always prefetch (the last stage re-reads itself), so the
    // loop body has no branch and the loads stay in flight over the MFMAs.
    if constexpr (FAST) {
      gload_fast(kbeg + int64_t(it + 1 < nk ? it + 1 : it) * BK);
      // Keep the loads at the top of the stage: the scheduler would
      // otherwise sink them next to their LDS stores, exposing their latency.
      __builtin_amdgcn_sched_barrier(0);
    } else if (it + 1 < nk) {
      gload(kbeg + int64_t(it + 1) * BK);
    }
#pragma unroll
    for (int kq = 0; kq < BK; kq += 4) {
      float4 a4[TM], r4[TN], i4[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        a4[i] = *reinterpret_cast<const float4*>(As + aoff + i * 32 * LDR + kq);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        r4[j] = *reinterpret_cast<const float4*>(Bs + boff_r + j * 32 * LDR + kq);
        float4 t = *reinterpret_cast<const float4*>(Bs + boff_i + j * 32 * LDR + kq);
        t.x = __uint_as_float(__float_as_uint(t.x) ^ flip);
        t.y = __uint_as_float(__float_as_uint(t.y) ^ flip);
        t.z = __uint_as_float(__float_as_uint(t.z) ^ flip);
        t.w = __uint_as_float(__float_as_uint(t.w) ^ flip);
        i4[j] = t;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            const float av = q == 0 ? a4[i].x : q == 1 ? a4[i].y : q == 2 ? a4[i].z : a4[i].w;
            const float bv = q == 0 ? r4[j].x : q == 1 ? r4[j].y : q == 2 ? r4[j].z : r4[j].w;
            const float cv = q == 0 ? i4[j].x : q == 1 ? i4[j].y : q == 2 ? i4[j].z : i4[j].w;
            cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, cr[i][j], 0, 0, 0);
            ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, cv, ci[i][j], 0, 0, 0);
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
        store_out<float>(p, b, split, row, col, 0, cr[i][j][e]);
        store_out<float>(p, b, split, row, col, 1, ci[i][j][e]);
      }
}

// Dynamic LDS bytes of the large FP32 tile.
template <int WM, int WN, int TM, int TN, int BK>
constexpr size_t big_lds_bytes() {
  return size_t(2) * (WM * TM * 32 + WN * TN * 32) * (2 * BK + 4) * sizeof(float);
}

// Large-tile FP32-4M with direct-to-LDS staging: interior tiles copy each
// 16-byte chunk (two complex) of A and B from global memory straight into
// LDS (global_load_lds_dwordx4: a wave writes 64 consecutive chunks), so no
// VGPRs hold the next stage and no LDS stores are issued.  LDS rows keep the
// interleaved (re, im) order of the operands, 8 chunks per row (16 complex
// k), unpadded; logical chunk c of row r sits at chunk c ^ dl_swz(r), so the
// 128-bit fragment reads of 8 (or 16) consecutive rows fall on distinct bank
// groups.  A lane reads chunk 2g + kh of its row (kh = lane / 32) and feeds
// its four floats to four MFMAs; the B lane that meets it in an instruction
// reads the same logical chunk of its column and supplies b_r or -b_i (real
// accumulator) and b_i or b_r (imaginary accumulator), i.e. the 4M
// embedding with the real k of an instruction taken from consecutive floats.
// Edge tiles stage through registers into the same layout, zero-filled.
template <int WM, int WN, int TM, int TN, int BK>
__device__ __forceinline__ void cgemm_f32_dl_body(const GemmParams& p, int tm, int tn,
                                                  int split, int b) {
  static_assert(WM * WN == 4, "four waves");
  static_assert(BK == 16 || BK == 32, "eight or sixteen 16-byte chunks per LDS row");
  constexpr int BM = WM * TM * 32;
  constexpr int BN = WN * TN * 32;  // complex columns
  constexpr int CPR = BK / 2;       // chunks per row
  auto swz = [](int r) -> int { return CPR == 8 ? dl_swz(r) : dl_swz16(r); };
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

  // Slot s = 256 j + tid of a stage: row s / CPR, stored chunk s % CPR,
  // which holds logical chunk (s % CPR) ^ swz(row).
  auto dma = [&](auto buf, int64_t k0) {
    float4* As = abuf(buf);
    float4* Bs = bbuf(buf);
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int s = tid + 256 * j, r = s / CPR, c = (s % CPR) ^ swz(r);
      __builtin_amdgcn_global_load_lds(
          Ag + (row0 + r) * p.lda + k0 + 2 * c,
          (__attribute__((address_space(3))) void*)(As + 256 * j + 64 * wave), 16, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int s = tid + 256 * j, r = s / CPR, c = (s % CPR) ^ swz(r);
      __builtin_amdgcn_global_load_lds(
          Bg + (col0 + r) * p.ldb + k0 + 2 * c,
          (__attribute__((address_space(3))) void*)(Bs + 256 * j + 64 * wave), 16, 0, 0);
    }
  };
  float4 ra[NA], rb[NB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int s = tid + 256 * j, r = s / CPR, c = s % CPR;
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
      const int s = tid + 256 * j, r = s / CPR, c = s % CPR;
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
      const int s = tid + 256 * j, r = s / CPR;
      As[r * CPR + ((s % CPR) ^ swz(r))] = ra[j];
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int s = tid + 256 * j, r = s / CPR;
      Bs[r * CPR + ((s % CPR) ^ swz(r))] = rb[j];
    }
  };

  v16f cr[TM][TN], ci[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) cr[i][j][e] = ci[i][j][e] = 0.f;

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
      float4 a4[TM], b4[TN], n4[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int r = arow + 32 * i;
        a4[i] = As[r * CPR + ((2 * g + kh) ^ swz(r))];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int r = brow + 32 * j;
        b4[j] = Bs[r * CPR + ((2 * g + kh) ^ swz(r))];
        n4[j] = make_float4(b4[j].x, -b4[j].y, b4[j].z, -b4[j].w);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            const float av = q == 0 ? a4[i].x : q == 1 ? a4[i].y : q == 2 ? a4[i].z : a4[i].w;
            const float bv = q == 0 ? n4[j].x : q == 1 ? n4[j].y : q == 2 ? n4[j].z : n4[j].w;
            const float cv = q == 0 ? b4[j].y : q == 1 ? b4[j].x : q == 2 ? b4[j].w : b4[j].z;
            cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, cr[i][j], 0, 0, 0);
            ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, cv, ci[i][j], 0, 0, 0);
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
        store_out<float>(p, b, split, row, col, 0, cr[i][j][e]);
        store_out<float>(p, b, split, row, col, 1, ci[i][j][e]);
      }
}

RN_GEMM_ENTRY(cgemm_f32_4m)
RN_GEMM_ENTRY(cgemm_f32_ri)
RN_GEMM_ENTRY(cgemm_f32_rp)
RN_GEMM_ENTRY(cgemm_f32_big)
// Two waves per SIMD for the 128 x 128 tiles, three for 128 x 64 (48 KiB of
// LDS: three workgroups per CU), four for the 64 x 64 and 128 x 32 tiles.
RN_GEMM_ENTRY_OCC(cgemm_f32_dl, (TM * TN * WM * WN <= 4 ? 4 : TM * TN * WM * WN <= 8 ? 3 : 2))

// The large FP32 tiles take more than 64 KiB of dynamic LDS; raise each
// kernel's limit once per process.
static void big_tiles_setup() {
  static const bool once = [] {
    hipFuncSetAttribute(reinterpret_cast<const void*>(&cgemm_f32_big<2, 2, 2, 2, 16>),
                        hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)big_lds_bytes<2, 2, 2, 2, 16>());
    hipFuncSetAttribute(reinterpret_cast<const void*>(&cgemm_f32_big_grouped<2, 2, 2, 2, 16>),
                        hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)big_lds_bytes<2, 2, 2, 2, 16>());
    hipFuncSetAttribute(reinterpret_cast<const void*>(&cgemm_f32_big<1, 4, 4, 1, 16>),
                        hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)big_lds_bytes<1, 4, 4, 1, 16>());
    hipFuncSetAttribute(reinterpret_cast<const void*>(&cgemm_f32_big_grouped<1, 4, 4, 1, 16>),
                        hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)big_lds_bytes<1, 4, 4, 1, 16>());
    return true;
  }();
  (void)once;
}

// MFMA tile `tile` (index into this mode's tile table, not the one-thread
// or skinny kernels) over `grid` workgroups; errors via hipGetLastError.
void launch_tiles_f32_4m(int tile, dim3 grid, const GemmParams& p, hipStream_t s) {
  if (tile == 1)
    cgemm_f32_4m<2, 2, 2, 2, 16><<<grid, 256, 0, s>>>(p);
  else if (tile == 2)
    cgemm_f32_4m<2, 2, 1, 1, 16><<<grid, 256, 0, s>>>(p);
  else if (tile == 3)
    cgemm_f32_4m<2, 2, 4, 2, 8><<<grid, 256, 0, s>>>(p);
  else if (tile == 4)
    cgemm_f32_4m<2, 2, 2, 4, 8><<<grid, 256, 0, s>>>(p);
  else if (tile == 5)
    cgemm_f32_ri<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(p);
  else if (tile == 6)
    cgemm_f32_ri<2, 2, 2, 2, 8><<<grid, 256, 0, s>>>(p);
  else if (tile == 7)
    cgemm_f32_rp<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(p);
  else if (tile == 8)
    cgemm_f32_rp<2, 2, 2, 2, 8><<<grid, 256, 0, s>>>(p);
  else if (tile == 9)
    cgemm_f32_rp<1, 4, 4, 1, 16><<<grid, 256, 0, s>>>(p);
  else if (tile == 10) {
    big_tiles_setup();
    cgemm_f32_big<2, 2, 2, 2, 16><<<grid, 256, big_lds_bytes<2, 2, 2, 2, 16>(), s>>>(p);
  } else if (tile == 11) {
    cgemm_f32_big<2, 2, 2, 1, 16><<<grid, 256, big_lds_bytes<2, 2, 2, 1, 16>(), s>>>(p);
  } else if (tile == 12) {
    cgemm_f32_big<2, 2, 2, 1, 8><<<grid, 256, big_lds_bytes<2, 2, 2, 1, 8>(), s>>>(p);
  } else if (tile == 13) {
    cgemm_f32_big<2, 2, 2, 2, 8><<<grid, 256, big_lds_bytes<2, 2, 2, 2, 8>(), s>>>(p);
  } else if (tile == 14) {
    big_tiles_setup();
    cgemm_f32_big<1, 4, 4, 1, 16><<<grid, 256, big_lds_bytes<1, 4, 4, 1, 16>(), s>>>(p);
  } else if (tile == 15) {
    cgemm_f32_dl<1, 4, 4, 1, 16><<<grid, 256, 0, s>>>(p);
  } else if (tile == 16) {
    cgemm_f32_dl<2, 2, 2, 2, 16><<<grid, 256, 0, s>>>(p);
  } else if (tile == 17) {
    cgemm_f32_dl<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(p);
  } else if (tile == 18) {
    cgemm_f32_dl<2, 2, 1, 1, 16><<<grid, 256, 0, s>>>(p);
  } else if (tile == 19) {
    cgemm_f32_dl<4, 1, 1, 1, 16><<<grid, 256, 0, s>>>(p);
  } else if (tile == 20) {
    cgemm_f32_dl<2, 2, 1, 1, 32><<<grid, 256, 0, s>>>(p);
  } else {
    cgemm_f32_dl<4, 1, 1, 1, 32><<<grid, 256, 0, s>>>(p);
  }
}

void launch_tiles_f32_4m_grouped(int tile, dim3 grid, const GroupTable& t, hipStream_t s) {
  if (tile == 1) cgemm_f32_4m_grouped<2, 2, 2, 2, 16><<<grid, 256, 0, s>>>(t);
  else if (tile == 2) cgemm_f32_4m_grouped<2, 2, 1, 1, 16><<<grid, 256, 0, s>>>(t);
  else if (tile == 3) cgemm_f32_4m_grouped<2, 2, 4, 2, 8><<<grid, 256, 0, s>>>(t);
  else if (tile == 4) cgemm_f32_4m_grouped<2, 2, 2, 4, 8><<<grid, 256, 0, s>>>(t);
  else if (tile == 5) cgemm_f32_ri_grouped<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(t);
  else if (tile == 6) cgemm_f32_ri_grouped<2, 2, 2, 2, 8><<<grid, 256, 0, s>>>(t);
  else if (tile == 7) cgemm_f32_rp_grouped<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(t);
  else if (tile == 8) cgemm_f32_rp_grouped<2, 2, 2, 2, 8><<<grid, 256, 0, s>>>(t);
  else if (tile == 9) cgemm_f32_rp_grouped<1, 4, 4, 1, 16><<<grid, 256, 0, s>>>(t);
  else if (tile == 10) {
    big_tiles_setup();
    cgemm_f32_big_grouped<2, 2, 2, 2, 16>
        <<<grid, 256, big_lds_bytes<2, 2, 2, 2, 16>(), s>>>(t);
  } else if (tile == 11) {
    cgemm_f32_big_grouped<2, 2, 2, 1, 16>
        <<<grid, 256, big_lds_bytes<2, 2, 2, 1, 16>(), s>>>(t);
  } else if (tile == 12) {
    cgemm_f32_big_grouped<2, 2, 2, 1, 8>
        <<<grid, 256, big_lds_bytes<2, 2, 2, 1, 8>(), s>>>(t);
  } else if (tile == 13) {
    cgemm_f32_big_grouped<2, 2, 2, 2, 8>
        <<<grid, 256, big_lds_bytes<2, 2, 2, 2, 8>(), s>>>(t);
  } else if (tile == 14) {
    big_tiles_setup();
    cgemm_f32_big_grouped<1, 4, 4, 1, 16>
        <<<grid, 256, big_lds_bytes<1, 4, 4, 1, 16>(), s>>>(t);
  } else if (tile == 15) {
    cgemm_f32_dl_grouped<1, 4, 4, 1, 16><<<grid, 256, 0, s>>>(t);
  } else if (tile == 16) {
    cgemm_f32_dl_grouped<2, 2, 2, 2, 16><<<grid, 256, 0, s>>>(t);
  } else if (tile == 17) {
    cgemm_f32_dl_grouped<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(t);
  } else if (tile == 18) {
    cgemm_f32_dl_grouped<2, 2, 1, 1, 16><<<grid, 256, 0, s>>>(t);
  } else if (tile == 19) {
    cgemm_f32_dl_grouped<4, 1, 1, 1, 16><<<grid, 256, 0, s>>>(t);
  } else if (tile == 20) {
    cgemm_f32_dl_grouped<2, 2, 1, 1, 32><<<grid, 256, 0, s>>>(t);
  } else {
    cgemm_f32_dl_grouped<4, 1, 1, 1, 32><<<grid, 256, 0, s>>>(t);
  }
}

}  // namespace rn
