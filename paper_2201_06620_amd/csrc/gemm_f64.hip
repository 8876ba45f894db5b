// Complex GEMM tiles of the FP64 mode (v_mfma_f64_16x16x4f64; 4 real
// products per complex product, or 3 in the Gauss tile) and their launcher.
#include "kcommon.hpp"

namespace rn {

// ---------------------------------------------------------------------------
// FP64, 4M embedding, v_mfma_f64_16x16x4_f64 (4 real k = 2 complex k).
// ---------------------------------------------------------------------------
template <int WM, int WN, int TM, int TN, int BK>
__device__ __forceinline__ void cgemm_f64_4m_body(const GemmParams& p, int tm, int tn, int split,
                                                int b) {
  static_assert(WM * WN == 4, "four waves");
  static_assert(BK % 2 == 0, "two complex k per MFMA");
  constexpr int BM = WM * TM * 16;
  constexpr int BN = WN * TN * 8;  // complex columns
  constexpr int LDK = BK + 1;
  constexpr int AV = BM * BK;  // double2 loads
  constexpr int BV = BN * BK;
  constexpr int NA = (AV + 255) / 256;
  constexpr int NB = (BV + 255) / 256;
  __shared__ double2 As[2][BM * LDK];
  __shared__ double2 Bs[2][BN * LDK];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t row0 = int64_t(tm) * BM;
  const int64_t col0 = int64_t(tn) * BN;
  const double2* __restrict__ Ag =
      reinterpret_cast<const double2*>(p.A) + batch_off(p.a_bs, p.nbb, b);
  const double2* __restrict__ Bg =
      reinterpret_cast<const double2*>(p.B) + batch_off(p.b_bs, p.nbb, b);
  const int64_t kbeg = int64_t(split) * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int nk = (int)((kend - kbeg + BK - 1) / BK);

  double2 ra[NA], rb[NB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      int idx = tid + 256 * j;
      double2 v = make_double2(0.0, 0.0);
      if (idx < AV) {
        int r = idx / BK, c = idx % BK;
        int64_t gr = row0 + r, gk = k0 + c;
        if (gr < p.M && gk < kend) v = Ag[gr * p.lda + gk];
      }
      ra[j] = v;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      int idx = tid + 256 * j;
      double2 v = make_double2(0.0, 0.0);
      if (idx < BV) {
        int r = idx / BK, c = idx % BK;
        int64_t gr = col0 + r, gk = k0 + c;
        if (gr < p.N && gk < kend) v = Bg[gr * p.ldb + gk];
      }
      rb[j] = v;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      int idx = tid + 256 * j;
      if (idx < AV) As[buf][(idx / BK) * LDK + idx % BK] = ra[j];
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      int idx = tid + 256 * j;
      if (idx < BV) Bs[buf][(idx / BK) * LDK + idx % BK] = rb[j];
    }
  };

  v4d acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[i][j][e] = 0.0;

  // 16x16x4 f64 roles: A row = lane % 16, real k = lane / 16, i.e. complex k
  // lane / 32 and part (lane / 16) & 1; B real column n = lane % 16 (complex
  // column n / 2, part n & 1), same real k.
  const int kc = lane >> 5;
  const int kpart = (lane >> 4) & 1;
  const int par = lane & 1;
  const bool b_take_re = (kpart == par);
  const bool b_neg = (kpart == 1 && par == 0);
  const int arow = wm * TM * 16 + (lane & 15);
  const int bcol = wn * TN * 8 + ((lane & 15) >> 1);

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
      double af[TM], bf[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        double2 a = As[buf][(arow + i * 16) * LDK + kk + kc];
        af[i] = kpart ? a.y : a.x;
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        double2 bv = Bs[buf][(bcol + j * 8) * LDK + kk + kc];
        double v = b_take_re ? bv.x : bv.y;
        bf[j] = b_neg ? -v : v;
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    if (it + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

  // 16x16 f64 accumulator layout (unlike the f32 16x16 one): lane holds
  // real column lane % 16 and rows 4*e + lane/16 for e = 0..3.
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int64_t row = row0 + wm * TM * 16 + i * 16 + 4 * e + (lane >> 4);
        int n = wn * TN * 16 + j * 16 + (lane & 15);
        store_out<double>(p, b, split, row, col0 + (n >> 1), n & 1, acc[i][j][e]);
      }
}

// FP64 counterpart: v_mfma_f64_16x16x4_f64, 16 complex columns per tile
// pair, 2 complex k per instruction (real k = lane / 16: complex k lane / 32,
// half (lane / 16) & 1).
template <int WM, int WN, int TM, int TN, int BK>
__device__ __forceinline__ void cgemm_f64_rp_body(const GemmParams& p, int tm, int tn, int split,
                                                  int b) {
  static_assert(WM * WN == 4, "four waves");
  static_assert(BK % 2 == 0, "two complex k per MFMA");
  constexpr int BM = WM * TM * 16;
  constexpr int BN = WN * TN * 16;  // complex columns
  constexpr int LDR = 2 * BK + 1;   // doubles per padded LDS row
  constexpr int AV = BM * BK;
  constexpr int BV = BN * BK;
  constexpr int NA = (AV + 255) / 256;
  constexpr int NB = (BV + 255) / 256;
  __shared__ double As[2][BM * LDR];
  __shared__ double Bs[2][BN * LDR];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t row0 = int64_t(tm) * BM;
  const int64_t col0 = int64_t(tn) * BN;
  const double2* __restrict__ Ag =
      reinterpret_cast<const double2*>(p.A) + batch_off(p.a_bs, p.nbb, b);
  const double2* __restrict__ Bg =
      reinterpret_cast<const double2*>(p.B) + batch_off(p.b_bs, p.nbb, b);
  const int64_t kbeg = int64_t(split) * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int nk = (int)((kend - kbeg + BK - 1) / BK);

  double2 ra[NA], rb[NB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      int idx = tid + 256 * j;
      double2 v = make_double2(0.0, 0.0);
      if (idx < AV) {
        int r = idx / BK, c = idx % BK;
        int64_t gr = row0 + r, gk = k0 + c;
        if (gr < p.M && gk < kend) v = Ag[gr * p.lda + gk];
      }
      ra[j] = v;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      int idx = tid + 256 * j;
      double2 v = make_double2(0.0, 0.0);
      if (idx < BV) {
        int r = idx / BK, c = idx % BK;
        int64_t gr = col0 + r, gk = k0 + c;
        if (gr < p.N && gk < kend) v = Bg[gr * p.ldb + gk];
      }
      rb[j] = v;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      int idx = tid + 256 * j;
      if (idx < AV) {
        int r = idx / BK, c = idx % BK;
        As[buf][r * LDR + c] = ra[j].x;
        As[buf][r * LDR + BK + c] = ra[j].y;
      }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      int idx = tid + 256 * j;
      if (idx < BV) {
        int r = idx / BK, c = idx % BK;
        Bs[buf][r * LDR + c] = rb[j].x;
        Bs[buf][r * LDR + BK + c] = -rb[j].y;
      }
    }
  };

  v4d cr[TM][TN], ci[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) cr[i][j][e] = ci[i][j][e] = 0.0;

  const int kc = lane >> 5;
  const int half = (lane >> 4) & 1;
  const int aoff = (wm * TM * 16 + (lane & 15)) * LDR + half * BK + kc;
  const int boff_r = (wn * TN * 16 + (lane & 15)) * LDR + half * BK + kc;
  const int boff_i = (wn * TN * 16 + (lane & 15)) * LDR + (1 - half) * BK + kc;
  const bool negi = (half == 0);

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
      double af[TM], br[TN], bi[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) af[i] = As[buf][aoff + i * 16 * LDR + kk];
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        br[j] = Bs[buf][boff_r + j * 16 * LDR + kk];
        double v = Bs[buf][boff_i + j * 16 * LDR + kk];
        bi[j] = negi ? -v : v;
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], br[j], cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bi[j], ci[i][j], 0, 0, 0);
        }
    }
    if (it + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

  // 16x16 f64 accumulator layout: column lane % 16, rows 4*e + lane/16.
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int64_t row = row0 + wm * TM * 16 + i * 16 + 4 * e + (lane >> 4);
        int64_t col = col0 + wn * TN * 16 + j * 16 + (lane & 15);
        store_out<double>(p, b, split, row, col, 0, cr[i][j][e]);
        store_out<double>(p, b, split, row, col, 1, ci[i][j][e]);
      }
}

// Large-tile FP64: v_mfma_f64_16x16x4f64 (two complex k per instruction:
// lane / 32 picks the complex k, (lane / 16) & 1 the real or imaginary
// half).  LDS rows hold [re of even k | re of odd k | im of even k | im of
// odd k], so the values one lane needs for two consecutive instructions are
// adjacent and come in one 128-bit read; rows padded to 16-byte multiples.
// Interior tiles load without guards and pin the next stage's loads to the
// top of the stage, as in the FP32 large tile.
template <int WM, int WN, int TM, int TN, int BK>
__device__ __forceinline__ void cgemm_f64_big_body(const GemmParams& p, int tm, int tn,
                                                   int split, int b) {
  static_assert(WM * WN == 4, "four waves");
  static_assert(BK % 4 == 0, "two instructions per 128-bit read");
  constexpr int BM = WM * TM * 16;
  constexpr int BN = WN * TN * 16;  // complex columns
  constexpr int LDR = 2 * BK + 2;   // doubles per LDS row, 16-byte multiple
  constexpr int HB = BK / 2;
  constexpr int AV = BM * BK;       // complex loads per stage
  constexpr int BV = BN * BK;
  constexpr int NA = (AV + 255) / 256;
  constexpr int NB = (BV + 255) / 256;
  extern __shared__ double2 big64_lds[];
  double* As0 = reinterpret_cast<double*>(big64_lds);
  double* Bs0 = As0 + 2 * BM * LDR;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t row0 = int64_t(tm) * BM;
  const int64_t col0 = int64_t(tn) * BN;
  const double2* __restrict__ Ag =
      reinterpret_cast<const double2*>(p.A) + batch_off(p.a_bs, p.nbb, b);
  const double2* __restrict__ Bg =
      reinterpret_cast<const double2*>(p.B) + batch_off(p.b_bs, p.nbb, b);
  const int64_t kbeg = int64_t(split) * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int nk = (int)((kend - kbeg + BK - 1) / BK);
  const bool interior = row0 + BM <= p.M && col0 + BN <= p.N && (kend - kbeg) % BK == 0;

  double2 ra[NA], rb[NB];
  auto gload_fast = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      int idx = tid + 256 * j;
      if (AV % 256 == 0 || idx < AV)  // threads past the tile load nothing
        ra[j] = Ag[(row0 + idx / BK) * p.lda + k0 + idx % BK];
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      int idx = tid + 256 * j;
      if (BV % 256 == 0 || idx < BV) rb[j] = Bg[(col0 + idx / BK) * p.ldb + k0 + idx % BK];
    }
  };
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      int idx = tid + 256 * j;
      double2 v = make_double2(0.0, 0.0);
      if (idx < AV) {
        int64_t gr = row0 + idx / BK, gk = k0 + idx % BK;
        if (gr < p.M && gk < kend) v = Ag[gr * p.lda + gk];
      }
      ra[j] = v;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      int idx = tid + 256 * j;
      double2 v = make_double2(0.0, 0.0);
      if (idx < BV) {
        int64_t gr = col0 + idx / BK, gk = k0 + idx % BK;
        if (gr < p.N && gk < kend) v = Bg[gr * p.ldb + gk];
      }
      rb[j] = v;
    }
  };
  // Complex k = c goes to position (c & 1) * HB + c / 2 of each half.
  auto sstore = [&](int buf) {
    double* As = As0 + buf * BM * LDR;
    double* Bs = Bs0 + buf * BN * LDR;
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      int idx = tid + 256 * j;
      if (AV % 256 == 0 || idx < AV) {
        int r = idx / BK, c = idx % BK;
        double* row = As + r * LDR + (c & 1) * HB + (c >> 1);
        row[0] = ra[j].x;
        row[BK] = ra[j].y;
      }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      int idx = tid + 256 * j;
      if (BV % 256 == 0 || idx < BV) {
        int r = idx / BK, c = idx % BK;
        double* row = Bs + r * LDR + (c & 1) * HB + (c >> 1);
        row[0] = rb[j].x;
        row[BK] = -rb[j].y;
      }
    }
  };

  v4d cr[TM][TN], ci[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) cr[i][j][e] = ci[i][j][e] = 0.0;

  const int kc = lane >> 5;
  const int half = (lane >> 4) & 1;
  const int aoff = (wm * TM * 16 + (lane & 15)) * LDR + half * BK + kc * HB;
  const int boff_r = (wn * TN * 16 + (lane & 15)) * LDR + half * BK + kc * HB;
  const int boff_i = (wn * TN * 16 + (lane & 15)) * LDR + (1 - half) * BK + kc * HB;
  const bool negi = (half == 0);

  auto mainloop = [&](auto tag) {
    constexpr bool FAST = decltype(tag)::value;
    if (nk > 0) {
      if constexpr (FAST) gload_fast(kbeg); else gload(kbeg);
      sstore(0);
    }
    __syncthreads();
    for (int it = 0; it < nk; ++it) {
      const int buf = it & 1;
      const double* As = As0 + buf * BM * LDR;
      const double* Bs = Bs0 + buf * BN * LDR;
      if constexpr (FAST) {
        gload_fast(kbeg + int64_t(it + 1 < nk ? it + 1 : it) * BK);
        __builtin_amdgcn_sched_barrier(0);
      } else if (it + 1 < nk) {
        gload(kbeg + int64_t(it + 1) * BK);
      }
#pragma unroll
      for (int s2 = 0; s2 < HB; s2 += 2) {
        double2 a2[TM], r2[TN], i2[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
          a2[i] = *reinterpret_cast<const double2*>(As + aoff + i * 16 * LDR + s2);
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          r2[j] = *reinterpret_cast<const double2*>(Bs + boff_r + j * 16 * LDR + s2);
          double2 t = *reinterpret_cast<const double2*>(Bs + boff_i + j * 16 * LDR + s2);
          i2[j] = negi ? make_double2(-t.x, -t.y) : t;
        }
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
              const double av = q == 0 ? a2[i].x : a2[i].y;
              const double bv = q == 0 ? r2[j].x : r2[j].y;
              const double cv = q == 0 ? i2[j].x : i2[j].y;
              cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, cr[i][j], 0, 0, 0);
              ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, cv, ci[i][j], 0, 0, 0);
            }
      }
      if (FAST || it + 1 < nk) sstore(buf ^ 1);
      __syncthreads();
    }
  };
  if (interior) mainloop(BoolTag<true>{}); else mainloop(BoolTag<false>{});

  // 16x16 f64 accumulator layout: column lane % 16, rows 4*e + lane/16.
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int64_t row = row0 + wm * TM * 16 + i * 16 + 4 * e + (lane >> 4);
        int64_t col = col0 + wn * TN * 16 + j * 16 + (lane & 15);
        store_out<double>(p, b, split, row, col, 0, cr[i][j][e]);
        store_out<double>(p, b, split, row, col, 1, ci[i][j][e]);
      }
}

template <int WM, int WN, int TM, int TN, int BK>
constexpr size_t big64_lds_bytes() {
  return size_t(2) * (WM * TM * 16 + WN * TN * 16) * (2 * BK + 2) * sizeof(double);
}

// Large-tile FP64 with direct-to-LDS staging, as the FP32 direct-LDS tile:
// one 16-byte chunk is one complex (re, im), 8 chunks (BK = 8 complex k)
// per LDS row, unpadded and XOR-swizzled by dl_swz.  In
// v_mfma_f64_16x16x4f64 lane / 16 picks the real k; here it picks the
// complex k (chunk 4g + lane / 16) and the two floats of the chunk feed two
// instructions: a_r with b_r (real) and b_i (imaginary), then a_i with -b_i
// and b_r.
template <int WM, int WN, int TM, int TN, int BK>
__device__ __forceinline__ void cgemm_f64_dl_body(const GemmParams& p, int tm, int tn,
                                                  int split, int b) {
  static_assert(WM * WN == 4, "four waves");
  static_assert(BK == 8, "eight 16-byte chunks per LDS row");
  constexpr int BM = WM * TM * 16;
  constexpr int BN = WN * TN * 16;  // complex columns
  constexpr int CPR = BK;           // chunks (complex) per row
  constexpr int AV = BM * CPR;      // chunks per stage
  constexpr int BV = BN * CPR;
  static_assert(AV % 256 == 0 && BV % 256 == 0, "whole waves of chunks");
  constexpr int NA = AV / 256;
  constexpr int NB = BV / 256;
  __shared__ __align__(16) double2 Ad0[AV], Ad1[AV];
  __shared__ __align__(16) double2 Bd0[BV], Bd1[BV];
  auto abuf = [&](auto t) -> double2* { if constexpr (decltype(t)::value) return Ad1; else return Ad0; };
  auto bbuf = [&](auto t) -> double2* { if constexpr (decltype(t)::value) return Bd1; else return Bd0; };

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t row0 = int64_t(tm) * BM;
  const int64_t col0 = int64_t(tn) * BN;
  const double2* __restrict__ Ag =
      reinterpret_cast<const double2*>(p.A) + batch_off(p.a_bs, p.nbb, b);
  const double2* __restrict__ Bg =
      reinterpret_cast<const double2*>(p.B) + batch_off(p.b_bs, p.nbb, b);
  const int64_t kbeg = int64_t(split) * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int nk = (int)((kend - kbeg + BK - 1) / BK);
  const bool interior = row0 + BM <= p.M && col0 + BN <= p.N && (kend - kbeg) % BK == 0;

  auto dma = [&](auto buf, int64_t k0) {
    double2* As = abuf(buf);
    double2* Bs = bbuf(buf);
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int s = tid + 256 * j, r = s >> 3, c = (s & 7) ^ dl_swz(r);
      __builtin_amdgcn_global_load_lds(
          Ag + (row0 + r) * p.lda + k0 + c,
          (__attribute__((address_space(3))) void*)(As + 256 * j + 64 * wave), 16, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int s = tid + 256 * j, r = s >> 3, c = (s & 7) ^ dl_swz(r);
      __builtin_amdgcn_global_load_lds(
          Bg + (col0 + r) * p.ldb + k0 + c,
          (__attribute__((address_space(3))) void*)(Bs + 256 * j + 64 * wave), 16, 0, 0);
    }
  };
  double2 ra[NA], rb[NB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int s = tid + 256 * j;
      const int64_t gr = row0 + (s >> 3), gk = k0 + (s & 7);
      ra[j] = (gr < p.M && gk < kend) ? Ag[gr * p.lda + gk] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int s = tid + 256 * j;
      const int64_t gr = col0 + (s >> 3), gk = k0 + (s & 7);
      rb[j] = (gr < p.N && gk < kend) ? Bg[gr * p.ldb + gk] : make_double2(0.0, 0.0);
    }
  };
  auto sstore = [&](auto buf) {
    double2* As = abuf(buf);
    double2* Bs = bbuf(buf);
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

  v4d cr[TM][TN], ci[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) cr[i][j][e] = ci[i][j][e] = 0.0;

  const int kq = lane >> 4;
  const int arow = wm * TM * 16 + (lane & 15);
  const int brow = wn * TN * 16 + (lane & 15);

  auto stage = [&](auto fast, auto cur, int it) {
    constexpr bool FAST = decltype(fast)::value;
    constexpr bool CUR = decltype(cur)::value;
    const double2* As = abuf(cur);
    const double2* Bs = bbuf(cur);
    if constexpr (FAST) {
      dma(BoolTag<!CUR>{}, kbeg + int64_t(it + 1 < nk ? it + 1 : it) * BK);
      __builtin_amdgcn_sched_barrier(0);
    } else if (it + 1 < nk) {
      gload(kbeg + int64_t(it + 1) * BK);
    }
#pragma unroll
    for (int g = 0; g < CPR / 4; ++g) {
      double2 a2[TM], b2[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int r = arow + 16 * i;
        a2[i] = As[r * CPR + ((4 * g + kq) ^ dl_swz(r))];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int r = brow + 16 * j;
        b2[j] = Bs[r * CPR + ((4 * g + kq) ^ dl_swz(r))];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[i].x, b2[j].x, cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[i].x, b2[j].y, ci[i][j], 0, 0, 0);
        }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[i].y, -b2[j].y, cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[i].y, b2[j].x, ci[i][j], 0, 0, 0);
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

  // 16x16 f64 accumulator layout: column lane % 16, rows 4*e + lane/16.
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int64_t row = row0 + wm * TM * 16 + i * 16 + 4 * e + (lane >> 4);
        int64_t col = col0 + wn * TN * 16 + j * 16 + (lane & 15);
        store_out<double>(p, b, split, row, col, 0, cr[i][j][e]);
        store_out<double>(p, b, split, row, col, 1, ci[i][j][e]);
      }
}

// FP64 Gauss (3M) with the direct-to-LDS staging of the FP64 tile: the chunk
// (a_r, a_i) a lane reads feeds T1 = Ar Br, T2 = Ai Bi and
// T3 = (Ar + Ai)(Br + Bi), three instructions per tile and complex k where
// the 4M tile takes four; Re = T1 - T2, Im = T3 - T1 - T2.  Three
// accumulators per 16 x 16 tile: 64 x 64 is the largest tile without spills
// in the loop; it runs three waves per SIMD (32 KiB of LDS per workgroup).
// An alternative FP64 tile (the FP64 default stays the 4M one).
template <int WM, int WN, int TM, int TN, int BK>
__device__ __forceinline__ void cgemm_f64_3mdl_body(const GemmParams& p, int tm, int tn,
                                                  int split, int b) {
  static_assert(WM * WN == 4, "four waves");
  static_assert(BK == 8, "eight 16-byte chunks per LDS row");
  constexpr int BM = WM * TM * 16;
  constexpr int BN = WN * TN * 16;  // complex columns
  constexpr int CPR = BK;           // chunks (complex) per row
  constexpr int AV = BM * CPR;      // chunks per stage
  constexpr int BV = BN * CPR;
  static_assert(AV % 256 == 0 && BV % 256 == 0, "whole waves of chunks");
  constexpr int NA = AV / 256;
  constexpr int NB = BV / 256;
  __shared__ __align__(16) double2 Ad0[AV], Ad1[AV];
  __shared__ __align__(16) double2 Bd0[BV], Bd1[BV];
  auto abuf = [&](auto t) -> double2* { if constexpr (decltype(t)::value) return Ad1; else return Ad0; };
  auto bbuf = [&](auto t) -> double2* { if constexpr (decltype(t)::value) return Bd1; else return Bd0; };

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t row0 = int64_t(tm) * BM;
  const int64_t col0 = int64_t(tn) * BN;
  const double2* __restrict__ Ag =
      reinterpret_cast<const double2*>(p.A) + batch_off(p.a_bs, p.nbb, b);
  const double2* __restrict__ Bg =
      reinterpret_cast<const double2*>(p.B) + batch_off(p.b_bs, p.nbb, b);
  const int64_t kbeg = int64_t(split) * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int nk = (int)((kend - kbeg + BK - 1) / BK);
  const bool interior = row0 + BM <= p.M && col0 + BN <= p.N && (kend - kbeg) % BK == 0;

  auto dma = [&](auto buf, int64_t k0) {
    double2* As = abuf(buf);
    double2* Bs = bbuf(buf);
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int s = tid + 256 * j, r = s >> 3, c = (s & 7) ^ dl_swz(r);
      __builtin_amdgcn_global_load_lds(
          Ag + (row0 + r) * p.lda + k0 + c,
          (__attribute__((address_space(3))) void*)(As + 256 * j + 64 * wave), 16, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int s = tid + 256 * j, r = s >> 3, c = (s & 7) ^ dl_swz(r);
      __builtin_amdgcn_global_load_lds(
          Bg + (col0 + r) * p.ldb + k0 + c,
          (__attribute__((address_space(3))) void*)(Bs + 256 * j + 64 * wave), 16, 0, 0);
    }
  };
  double2 ra[NA], rb[NB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int s = tid + 256 * j;
      const int64_t gr = row0 + (s >> 3), gk = k0 + (s & 7);
      ra[j] = (gr < p.M && gk < kend) ? Ag[gr * p.lda + gk] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int s = tid + 256 * j;
      const int64_t gr = col0 + (s >> 3), gk = k0 + (s & 7);
      rb[j] = (gr < p.N && gk < kend) ? Bg[gr * p.ldb + gk] : make_double2(0.0, 0.0);
    }
  };
  auto sstore = [&](auto buf) {
    double2* As = abuf(buf);
    double2* Bs = bbuf(buf);
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

  v4d t1[TM][TN], t2[TM][TN], t3[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) t1[i][j][e] = t2[i][j][e] = t3[i][j][e] = 0.0;

  const int kq = lane >> 4;
  const int arow = wm * TM * 16 + (lane & 15);
  const int brow = wn * TN * 16 + (lane & 15);

  auto stage = [&](auto fast, auto cur, int it) {
    constexpr bool FAST = decltype(fast)::value;
    constexpr bool CUR = decltype(cur)::value;
    const double2* As = abuf(cur);
    const double2* Bs = bbuf(cur);
    if constexpr (FAST) {
      dma(BoolTag<!CUR>{}, kbeg + int64_t(it + 1 < nk ? it + 1 : it) * BK);
      __builtin_amdgcn_sched_barrier(0);
    } else if (it + 1 < nk) {
      gload(kbeg + int64_t(it + 1) * BK);
    }
#pragma unroll
    for (int g = 0; g < CPR / 4; ++g) {
      double2 a2[TM], b2[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int r = arow + 16 * i;
        a2[i] = As[r * CPR + ((4 * g + kq) ^ dl_swz(r))];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int r = brow + 16 * j;
        b2[j] = Bs[r * CPR + ((4 * g + kq) ^ dl_swz(r))];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          t1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[i].x, b2[j].x, t1[i][j], 0, 0, 0);
          t2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[i].y, b2[j].y, t2[i][j], 0, 0, 0);
          t3[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[i].x + a2[i].y, b2[j].x + b2[j].y,
                                                          t3[i][j], 0, 0, 0);
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

  // 16x16 f64 accumulator layout: column lane % 16, rows 4*e + lane/16.
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int64_t row = row0 + wm * TM * 16 + i * 16 + 4 * e + (lane >> 4);
        int64_t col = col0 + wn * TN * 16 + j * 16 + (lane & 15);
        const double a = t1[i][j][e], c = t2[i][j][e], d = t3[i][j][e];
        store_out<double>(p, b, split, row, col, 0, a - c);
        store_out<double>(p, b, split, row, col, 1, (d - a) - c);
      }
}

RN_GEMM_ENTRY(cgemm_f64_4m)
RN_GEMM_ENTRY(cgemm_f64_rp)
RN_GEMM_ENTRY_OCC(cgemm_f64_big, 2)
RN_GEMM_ENTRY_OCC(cgemm_f64_dl, 2)
RN_GEMM_ENTRY_OCC(cgemm_f64_3mdl, 3)

// MFMA tile `tile` (index into this mode's tile table, not the one-thread
// or skinny kernels) over `grid` workgroups; errors via hipGetLastError.
void launch_tiles_f64(int tile, dim3 grid, const GemmParams& p, hipStream_t s) {
  if (tile == 1)
    cgemm_f64_4m<2, 2, 4, 4, 8><<<grid, 256, 0, s>>>(p);
  else if (tile == 2)
    cgemm_f64_4m<2, 2, 2, 2, 8><<<grid, 256, 0, s>>>(p);
  else if (tile == 3)
    cgemm_f64_rp<2, 2, 4, 2, 8><<<grid, 256, 0, s>>>(p);
  else if (tile == 4)
    cgemm_f64_rp<2, 2, 2, 2, 8><<<grid, 256, 0, s>>>(p);
  else if (tile == 5)
    cgemm_f64_big<2, 2, 4, 2, 8><<<grid, 256, big64_lds_bytes<2, 2, 4, 2, 8>(), s>>>(p);
  else if (tile == 6)
    cgemm_f64_big<2, 2, 2, 4, 8><<<grid, 256, big64_lds_bytes<2, 2, 2, 4, 8>(), s>>>(p);
  else if (tile == 7)
    cgemm_f64_big<2, 2, 2, 2, 8><<<grid, 256, big64_lds_bytes<2, 2, 2, 2, 8>(), s>>>(p);
  else if (tile == 8)
    cgemm_f64_dl<2, 2, 4, 2, 8><<<grid, 256, 0, s>>>(p);
  else if (tile == 9)
    cgemm_f64_dl<2, 2, 2, 4, 8><<<grid, 256, 0, s>>>(p);
  else
    cgemm_f64_3mdl<2, 2, 2, 2, 8><<<grid, 256, 0, s>>>(p);
}

void launch_tiles_f64_grouped(int tile, dim3 grid, const GroupTable& t, hipStream_t s) {
  if (tile == 1) cgemm_f64_4m_grouped<2, 2, 4, 4, 8><<<grid, 256, 0, s>>>(t);
  else if (tile == 2) cgemm_f64_4m_grouped<2, 2, 2, 2, 8><<<grid, 256, 0, s>>>(t);
  else if (tile == 3) cgemm_f64_rp_grouped<2, 2, 4, 2, 8><<<grid, 256, 0, s>>>(t);
  else if (tile == 4) cgemm_f64_rp_grouped<2, 2, 2, 2, 8><<<grid, 256, 0, s>>>(t);
  else if (tile == 5)
    cgemm_f64_big_grouped<2, 2, 4, 2, 8>
        <<<grid, 256, big64_lds_bytes<2, 2, 4, 2, 8>(), s>>>(t);
  else if (tile == 6)
    cgemm_f64_big_grouped<2, 2, 2, 4, 8>
        <<<grid, 256, big64_lds_bytes<2, 2, 2, 4, 8>(), s>>>(t);
  else if (tile == 7)
    cgemm_f64_big_grouped<2, 2, 2, 2, 8>
        <<<grid, 256, big64_lds_bytes<2, 2, 2, 2, 8>(), s>>>(t);
  else if (tile == 8)
    cgemm_f64_dl_grouped<2, 2, 4, 2, 8><<<grid, 256, 0, s>>>(t);
  else if (tile == 9)
    cgemm_f64_dl_grouped<2, 2, 2, 4, 8><<<grid, 256, 0, s>>>(t);
  else
    cgemm_f64_3mdl_grouped<2, 2, 2, 2, 8><<<grid, 256, 0, s>>>(t);
}

}  // namespace rn
