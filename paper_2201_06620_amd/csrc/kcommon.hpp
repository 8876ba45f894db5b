// Device-side definitions shared by the kernel files: GEMM parameters,
// output maps, tile order, bf16 helpers, the grouped-launch job lookup, the
// GEMM entry-point macros and the per-mode tile launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <utility>

#include "rn_internal.hpp"

namespace rn {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// Largest grid of one launch: HIP counts the work-items of a grid dimension
// in 32 bits, and every kernel here runs 256 per workgroup.
constexpr int64_t kMaxGrid = ((int64_t(1) << 32) - 1) / 256;

__device__ __forceinline__ int lds_pad(int x) { return x + (x >> 5); }

__device__ __forceinline__ uint32_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

// hi = nearest bfloat16 of x; lo = nearest bfloat16 of the exact residual
// x - hi (Henry, Tang and Heinecke, "Leveraging the bfloat16 artificial
// intelligence datatype for higher-precision computations", ARITH 2019).
__device__ __forceinline__ void bf16_split(float x, uint32_t& hi, uint32_t& lo) {
  hi = bf16_rne(x);
  float r = x - __uint_as_float(hi << 16);
  lo = bf16_rne(r);
}


// Job of global workgroup index w in a grouped launch: the largest i < n
// with prefix[i] <= w (prefix is non-decreasing, prefix[0] = 0).  Every
// wave searches on its own with two rounds of 64 parallel probes (n up to
// 4096), so a workgroup pays two dependent loads instead of a
// log2(n)-deep binary search through global memory.
__device__ __forceinline__ int find_job(const int32_t* __restrict__ prefix, int n, int w) {
  if (n <= 4096) {
    const int lane = threadIdx.x & 63;
    const int S = (n + 63) >> 6;
    int idx = lane * S;
    bool pred = idx < n && prefix[idx] <= w;
    unsigned long long m = __ballot(pred);
    const int base = (63 - __clzll(m)) * S;
    idx = base + lane;
    pred = lane < S && idx < n && prefix[idx] <= w;
    m = __ballot(pred);
    return base + (63 - __clzll(m));
  }
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= w) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ===========================================================================
// Complex GEMM: C[M x N] = A[M x K] * B[N x K]^T (both operands K-contiguous),
// batched over slices, optionally split along K into partial sums.
// ===========================================================================
struct GemmParams {
  const void* A;
  const void* B;
  const void* A2;
  const void* B2;
  void* C;
  void* partial;
  int64_t M, N, K, lda, ldb;
  int64_t crh, crl, cch, ccl;
  int crs, ccs;
  int nbb;
  int splitk;
  int ilv;   // split-BF16 operands row-interleaved (hi, lo per 16 k); lda counts words
  int pad_;
  int64_t kchunk;
  int tiles_m, tiles_n;
  int64_t a_bs[RN_MAX_SLICED], b_bs[RN_MAX_SLICED], c_bs[RN_MAX_SLICED];
};

__device__ __forceinline__ int64_t batch_off(const int64_t* st, int nbb, int b) {
  int64_t o = 0;
  for (int i = 0; i < nbb; ++i)
    if ((b >> i) & 1) o += st[i];
  return o;
}

__device__ __forceinline__ int64_t map2(int64_t x, int sh, int64_t hi, int64_t lo) {
  return (x >> sh) * hi + (x & ((int64_t(1) << sh) - 1)) * lo;
}

template <bool B>
struct BoolTag {
  static constexpr bool value = B;
};

// Output element (row, col, part) of tile results: either straight into C
// through the two-level maps, or into the split-K partial buffer.
template <typename R>
__device__ __forceinline__ void store_out(const GemmParams& p, int b, int split, int64_t row,
                                          int64_t col, int part, R v) {
  if (row >= p.M || col >= p.N) return;
  if (p.splitk > 1) {
    int64_t nb = int64_t(1) << p.nbb;
    int64_t idx = ((int64_t(split) * nb + b) * p.M + row) * p.N + col;
    reinterpret_cast<R*>(p.partial)[2 * idx + part] = v;
  } else {
    int64_t off = batch_off(p.c_bs, p.nbb, b) + map2(row, p.crs, p.crh, p.crl) +
                  map2(col, p.ccs, p.cch, p.ccl);
    reinterpret_cast<R*>(p.C)[2 * off + part] = v;
  }
}

// Workgroup -> output tile.  Hardware hands consecutive workgroups to the 8
// XCDs round-robin; renumbering them so each XCD receives one contiguous run
// of logical tiles, and walking tiles in column groups of GROUP_M row tiles,
// keeps the A row panels and B column panels a group shares inside one L2.
template <int GROUP_M = 8>
__device__ __forceinline__ void tile_coords(int tiles_m, int tiles_n, int& tm, int& tn) {
  int nwg = gridDim.x;
  int bid = blockIdx.x;
  if ((nwg & 7) == 0) bid = (bid & 7) * (nwg >> 3) + (bid >> 3);
  int group_size = GROUP_M * tiles_n;
  int g = bid / group_size;
  int first_m = g * GROUP_M;
  int gm = min(tiles_m - first_m, GROUP_M);
  int r = bid % group_size;
  tm = first_m + r % gm;
  tn = r / gm;
}

// Chunk swizzle of the direct-to-LDS tiles: logical 16-byte chunk c of LDS
// row r is stored at chunk c ^ dl_swz(r) (rows of 8 chunks) or
// c ^ dl_swz16(r) (rows of 16 chunks).
__device__ __forceinline__ int dl_swz(int r) { return (r ^ (r >> 3)) & 7; }
// Rows of 16 chunks (BK = 32): 256-byte rows start on the same bank, so the
// low four row bits alone spread 8 or 16 consecutive rows.
__device__ __forceinline__ int dl_swz16(int r) { return r & 15; }

// ---------------------------------------------------------------------------
// Kernel entry points.  Single problem: the grid is (tiles, splits, slice
// batch).  Grouped: many problems in one launch; workgroup w serves problem
// i with prefix[i] <= w < prefix[i+1] (problems ordered by decreasing work,
// so the largest start first) and takes that problem's local tile.
// ---------------------------------------------------------------------------
struct GroupTable {
  const GemmParams* probs;
  const int32_t* prefix;  // n + 1 entries
  int n;
};

__device__ __forceinline__ int group_find(const GroupTable& g, int bid) {
  return find_job(g.prefix, g.n, bid);
}

#define RN_GEMM_ENTRY(NAME)                                                              \
  template <int WM, int WN, int TM, int TN, int BK>                                     \
  __global__ __launch_bounds__(256) void NAME(GemmParams p) {                           \
    int tm, tn;                                                                         \
    tile_coords(p.tiles_m, p.tiles_n, tm, tn);                                          \
    NAME##_body<WM, WN, TM, TN, BK>(p, tm, tn, blockIdx.y, blockIdx.z);                 \
  }                                                                                     \
  template <int WM, int WN, int TM, int TN, int BK>                                     \
  __global__ __launch_bounds__(256) void NAME##_grouped(GroupTable g) {                 \
    const int i = group_find(g, blockIdx.x);                                            \
    const GemmParams p = g.probs[i]; /* by value: uniform scalar loads, once */         \
    const int local = blockIdx.x - g.prefix[i];                                         \
    const int per = p.tiles_m * p.tiles_n; /* tiles per K split */                      \
    NAME##_body<WM, WN, TM, TN, BK>(p, (local % per) / p.tiles_n, local % p.tiles_n,    \
                                    local / per, 0);                                    \
  }

// Entry points whose register use is capped for WAVES waves per SIMD, and
// whose single-problem tiles are walked in column groups of GROUP_M row tiles.
#define RN_GEMM_ENTRY_OCC_GM(NAME, WAVES, GROUP_M)                                                  \
  template <int WM, int WN, int TM, int TN, int BK>                                     \
  __global__ __launch_bounds__(256, WAVES) void NAME(GemmParams p) {                           \
    int tm, tn;                                                                         \
    tile_coords<GROUP_M>(p.tiles_m, p.tiles_n, tm, tn);                                 \
    NAME##_body<WM, WN, TM, TN, BK>(p, tm, tn, blockIdx.y, blockIdx.z);                 \
  }                                                                                     \
  template <int WM, int WN, int TM, int TN, int BK>                                     \
  __global__ __launch_bounds__(256, WAVES) void NAME##_grouped(GroupTable g) {                 \
    const int i = group_find(g, blockIdx.x);                                            \
    const GemmParams p = g.probs[i]; /* by value: uniform scalar loads, once */         \
    const int local = blockIdx.x - g.prefix[i];                                         \
    const int per = p.tiles_m * p.tiles_n; /* tiles per K split */                      \
    NAME##_body<WM, WN, TM, TN, BK>(p, (local % per) / p.tiles_n, local % p.tiles_n,    \
                                    local / per, 0);                                    \
  }
#define RN_GEMM_ENTRY_OCC(NAME, WAVES) RN_GEMM_ENTRY_OCC_GM(NAME, WAVES, 8)
// Per-mode tile launchers (one kernel file per mode).
void launch_tiles_f32_4m(int tile, dim3 grid, const GemmParams& p, hipStream_t s);
void launch_tiles_f32_4m_grouped(int tile, dim3 grid, const GroupTable& t, hipStream_t s);
void launch_tiles_f32_3m(int tile, dim3 grid, const GemmParams& p, hipStream_t s);
void launch_tiles_f32_3m_grouped(int tile, dim3 grid, const GroupTable& t, hipStream_t s);
void launch_tiles_f64(int tile, dim3 grid, const GemmParams& p, hipStream_t s);
void launch_tiles_f64_grouped(int tile, dim3 grid, const GroupTable& t, hipStream_t s);
void launch_tiles_bf16x3(int tile, dim3 grid, const GemmParams& p, hipStream_t s);
void launch_tiles_bf16x3_grouped(int tile, dim3 grid, const GroupTable& t, hipStream_t s);

}  // namespace rn
