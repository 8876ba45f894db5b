// HIP kernels for gfx950 (MI355X): index permutation, complex GEMM on MFMA,
// split-K reduction and FP64 reductions.
//
// Terminology: a "complex column" is one complex output element per row; in
// the 4M real embedding a complex m x k matrix A is the real m x 2k matrix of
// its interleaved (re, im) values, and a complex k x n matrix B becomes the
// real 2k x 2n matrix whose 2x2 cell for b is [[b_r, b_i], [-b_i, b_r]].  One
// real GEMM then yields C already interleaved, with 8*M*N*K real flops.  The
// embedding of B is never stored: each lane builds its B operand from the
// complex value in LDS (select re or im, flip a sign), or, in the
// direct-to-LDS tiles, the pairing of MFMA operands does it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <utility>
#include <cstdint>
#include <cstring>
#include <vector>

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

// Block count of a grouped launch, or -1 when the groups add up to more than
// one launch can hold (the launch then reports hipErrorInvalidConfiguration
// instead of wrapping its 32-bit prefix sums).
static int grouped_blocks(int64_t total) { return total <= kMaxGrid ? (int)total : -1; }
static int32_t prefix_entry(int64_t total) { return (int32_t)std::min(total, kMaxGrid); }

// ===========================================================================
// Index permutation (TTGT relayout).  Output bit o of the linear element
// index reads input bit src[o]; input bits outside src are fixed by in_base
// (slice projection).  A workgroup moves one tile: the set S of bits made of
// the lowest output bits and the lowest input bits, so both the global reads
// (input order) and the global writes (output order) run over contiguous
// runs of >= 512 bytes, while the transpose between the two orders happens
// in LDS.  The remaining bits index the tiles.
// ===========================================================================
struct PermParams {
  const void* in;
  void* out;
  void* out2;
  int64_t in_base;
  int64_t ntiles;
  int nS;        // tile bits
  int nO;        // outer bits
  int8_t ls_in[16];   // load order q -> input bit
  int8_t ss_out[16];  // store order q -> output bit
  int8_t ss_lds[16];  // store order q -> load-order position
  int8_t os_in[48];   // outer bit q -> input bit
  int8_t os_out[48];  // outer bit q -> output bit
  // Offsets of element j * 256 of a tile (bits >= 8 of the tile index).
  int64_t hi_in[16];
  int64_t hi_out[16];
  int32_t hi_lds[16];
};

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

// Thread-fixed low parts of the tile-local index u = tid + 256 * j.
__device__ __forceinline__ void perm_lo(const PermParams& p, int tid, int64_t& in_lo,
                                        int64_t& out_lo, int& lds_lo) {
  const int lo_bits = p.nS < 8 ? p.nS : 8;
  in_lo = out_lo = 0;
  lds_lo = 0;
  for (int q = 0; q < lo_bits; ++q) {
    if ((tid >> q) & 1) {
      in_lo += int64_t(1) << p.ls_in[q];
      out_lo += int64_t(1) << p.ss_out[q];
      lds_lo += 1 << p.ss_lds[q];
    }
  }
}

// One tile t of a permutation.  E elements per thread (tile = 256 * E
// elements, or fewer for a tile smaller than one workgroup); with PRED the
// tile may hold fewer than 256 * E elements.  All loads of a tile are
// issued before any is consumed, so each thread keeps E reads in flight.
template <typename T, int KIND, int E, bool PRED>
__device__ __forceinline__ void permute_tile(const PermParams& p, int64_t t, T* tile,
                                             int64_t in_lo, int64_t out_lo, int lds_lo) {
  const T* __restrict__ in = reinterpret_cast<const T*>(p.in);
  const int tid = threadIdx.x;
  const int tsize = 1 << p.nS;
  const bool active = tid < tsize;
  int64_t ib = p.in_base, ob = 0;
  for (int q = 0; q < p.nO; ++q) {
    if ((t >> q) & 1) {
      ib += int64_t(1) << p.os_in[q];
      ob += int64_t(1) << p.os_out[q];
    }
  }
  T v[E];
  if (active) {
#pragma unroll
    for (int j = 0; j < E; ++j)
      if (!PRED || (j << 8) < tsize) v[j] = in[ib + in_lo + p.hi_in[j]];
#pragma unroll
    for (int j = 0; j < E; ++j)
      if (!PRED || (j << 8) < tsize) tile[lds_pad(tid + (j << 8))] = v[j];
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int j = 0; j < E; ++j)
      if (!PRED || (j << 8) < tsize) v[j] = tile[lds_pad(lds_lo + p.hi_lds[j])];
#pragma unroll
    for (int j = 0; j < E; ++j) {
      if (PRED && (j << 8) >= tsize) continue;
      const int64_t oo = ob + out_lo + p.hi_out[j];
      if constexpr (KIND == 0) {
        reinterpret_cast<T*>(p.out)[oo] = v[j];
      } else {
        uint32_t hr, lr, hi_, li_;
        bf16_split(v[j].x, hr, lr);
        bf16_split(v[j].y, hi_, li_);
        reinterpret_cast<uint32_t*>(p.out)[oo] = hr | (hi_ << 16);
        reinterpret_cast<uint32_t*>(p.out2)[oo] = lr | (li_ << 16);
      }
    }
  }
  __syncthreads();
}

template <typename T, int KIND, int E>
__global__ __launch_bounds__(256) void permute_kernel(PermParams p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* tile = reinterpret_cast<T*>(smem_raw);
  int64_t in_lo, out_lo;
  int lds_lo;
  perm_lo(p, threadIdx.x, in_lo, out_lo, lds_lo);
  for (int64_t t = blockIdx.x; t < p.ntiles; t += gridDim.x)
    permute_tile<T, KIND, E, false>(p, t, tile, in_lo, out_lo, lds_lo);
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

// Many permutations in one launch: workgroup w moves one tile of job i,
// prefix[i] <= w < prefix[i+1].  The job's parameters are copied into LDS
// first: the tile code reads them many times, and from the table in global
// memory each read would be a dependent scalar load.
struct PermTable {
  const PermParams* jobs;
  const int32_t* prefix;
  int n;
};
static_assert(sizeof(PermParams) % 4 == 0 && sizeof(PermParams) <= 4 * 256,
              "parameters copied by one word per thread");

template <typename T, int KIND, int E>
__global__ __launch_bounds__(256) void permute_grouped(PermTable g) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ PermParams sp;
  T* tile = reinterpret_cast<T*>(smem_raw);
  const int bid = blockIdx.x;
  const int lo = find_job(g.prefix, g.n, bid);
  if (threadIdx.x < sizeof(PermParams) / 4)
    reinterpret_cast<uint32_t*>(&sp)[threadIdx.x] =
        reinterpret_cast<const uint32_t*>(&g.jobs[lo])[threadIdx.x];
  __syncthreads();
  int64_t in_lo, out_lo;
  int lds_lo;
  perm_lo(sp, threadIdx.x, in_lo, out_lo, lds_lo);
  permute_tile<T, KIND, E, true>(sp, bid - g.prefix[lo], tile, in_lo, out_lo, lds_lo);
}

template <typename T, int KIND>
static void launch_perm_e(const PermParams& p, int e, unsigned grid, size_t lds, hipStream_t s) {
  switch (e) {
    case 1: permute_kernel<T, KIND, 1><<<grid, 256, lds, s>>>(p); break;
    case 2: permute_kernel<T, KIND, 2><<<grid, 256, lds, s>>>(p); break;
    case 4: permute_kernel<T, KIND, 4><<<grid, 256, lds, s>>>(p); break;
    case 8: permute_kernel<T, KIND, 8><<<grid, 256, lds, s>>>(p); break;
    default: permute_kernel<T, KIND, 16><<<grid, 256, lds, s>>>(p); break;
  }
}

// Tile choice and offset tables of one permutation (host).
static void perm_setup(const PermLaunch& L, PermParams& p) {
  const int R = L.perm.nbits;
  p = PermParams{};
  p.in = L.in;
  p.out = L.out;
  p.out2 = L.out2;
  p.in_base = L.in_base;
  const int tlow = (L.in_es == 16) ? 5 : 6;
  bool inS[64] = {false};
  if (R <= 2 * tlow) {
    for (int o = 0; o < R; ++o) inS[o] = true;
  } else {
    for (int o = 0; o < tlow; ++o) inS[o] = true;
    // Output bits ordered by their input position: the lowest tlow of them
    // are the input-contiguous bits.
    int ord[64];
    for (int o = 0; o < R; ++o) ord[o] = o;
    std::sort(ord, ord + R, [&](int a, int b) { return L.perm.src[a] < L.perm.src[b]; });
    for (int q = 0; q < tlow; ++q) inS[ord[q]] = true;
    // Where the low input and output bits overlap, grow the tile with the
    // next input bits up to 2 * tlow bits, so it is never a sliver (tiny
    // tiles made a batch of many permutations dispatch-bound).
    int nsel = 0;
    for (int o = 0; o < R; ++o) nsel += inS[o] ? 1 : 0;
    for (int q = tlow; q < R && nsel < 2 * tlow; ++q)
      if (!inS[ord[q]]) {
        inS[ord[q]] = true;
        ++nsel;
      }
  }
  int ls[16], ss[16], nS = 0, nO = 0;
  for (int o = 0; o < R; ++o) {
    if (inS[o]) {
      ss[nS++] = o;
    } else {
      p.os_in[nO] = L.perm.src[o];
      p.os_out[nO] = (int8_t)o;
      ++nO;
    }
  }
  for (int q = 0; q < nS; ++q) ls[q] = ss[q];
  std::sort(ls, ls + nS, [&](int a, int b) { return L.perm.src[a] < L.perm.src[b]; });
  for (int q = 0; q < nS; ++q) {
    p.ls_in[q] = L.perm.src[ls[q]];
    p.ss_out[q] = (int8_t)ss[q];
    for (int r = 0; r < nS; ++r)
      if (ls[r] == ss[q]) p.ss_lds[q] = (int8_t)r;
  }
  p.nS = nS;
  p.nO = nO;
  p.ntiles = int64_t(1) << nO;
  const int tsize = 1 << nS;
  const int E = tsize >= 256 ? tsize / 256 : 1;
  for (int j = 0; j < E; ++j) {
    int64_t hi = 0, ho = 0;
    int hl = 0;
    for (int q = 8; q < nS; ++q) {
      if ((j >> (q - 8)) & 1) {
        hi += int64_t(1) << p.ls_in[q];
        ho += int64_t(1) << p.ss_out[q];
        hl += 1 << p.ss_lds[q];
      }
    }
    p.hi_in[j] = hi;
    p.hi_out[j] = ho;
    p.hi_lds[j] = hl;
  }
}

hipError_t launch_permute(const PermLaunch& L, hipStream_t s) {
  if (L.perm.nbits > 48) return hipErrorInvalidValue;
  PermParams p;
  perm_setup(L, p);
  const int tsize = 1 << p.nS;
  const int E = tsize >= 256 ? tsize / 256 : 1;
  size_t lds = size_t(tsize + (tsize >> 5) + 1) * L.in_es;
  // Up to 64 workgroups per CU, each looping over a few tiles: a 2^28-element
  // complex64 relayout measured 0.84 ms here against 0.86-0.89 ms with 2, 4 or
  // 16 per CU and 0.89 ms with one tile per workgroup.
  unsigned grid = (unsigned)std::min<int64_t>(p.ntiles, 256 * 64);
  if (L.kind == 1)
    launch_perm_e<float2, 1>(p, E, grid, lds, s);
  else if (L.in_es == 16)
    launch_perm_e<double2, 0>(p, E, grid, lds, s);
  else
    launch_perm_e<float2, 0>(p, E, grid, lds, s);
  return hipGetLastError();
}

size_t grouped_perm_build(const std::vector<PermLaunch>& jobs, std::vector<char>& table,
                          GroupedLaunch& G) {
  G = GroupedLaunch{};
  G.n = (int)jobs.size();
  if (jobs.empty()) return 0;
  G.kind = jobs[0].kind;
  G.es = jobs[0].in_es;
  std::vector<PermParams> ps(jobs.size());
  std::vector<int32_t> prefix(jobs.size() + 1, 0);
  int max_tsize = 1;
  int64_t total = 0;
  for (size_t i = 0; i < jobs.size(); ++i) {
    perm_setup(jobs[i], ps[i]);
    max_tsize = std::max(max_tsize, 1 << ps[i].nS);
    total += ps[i].ntiles;
    prefix[i + 1] = prefix_entry(total);
  }
  G.blocks = grouped_blocks(total);
  G.lds = size_t(max_tsize + (max_tsize >> 5) + 1) * G.es;
  G.params_off = 0;
  G.prefix_off = (jobs.size() * sizeof(PermParams) + 255) & ~size_t(255);
  size_t bytes = (G.prefix_off + prefix.size() * sizeof(int32_t) + 255) & ~size_t(255);
  table.resize(bytes);
  memcpy(table.data(), ps.data(), jobs.size() * sizeof(PermParams));
  memcpy(table.data() + G.prefix_off, prefix.data(), prefix.size() * sizeof(int32_t));
  return bytes;
}

hipError_t launch_permute_grouped(const GroupedLaunch& G, const void* table_dev, hipStream_t s) {
  if (G.n == 0 || G.blocks == 0) return hipSuccess;
  if (G.blocks < 0) return hipErrorInvalidConfiguration;
  PermTable t;
  t.jobs = reinterpret_cast<const PermParams*>(static_cast<const char*>(table_dev) + G.params_off);
  t.prefix = reinterpret_cast<const int32_t*>(static_cast<const char*>(table_dev) + G.prefix_off);
  t.n = G.n;
  const unsigned grid = (unsigned)G.blocks;
  if (G.kind == 1)
    permute_grouped<float2, 1, 16><<<grid, 256, G.lds, s>>>(t);
  else if (G.es == 16)
    permute_grouped<double2, 0, 4><<<grid, 256, G.lds, s>>>(t);
  else
    permute_grouped<float2, 0, 16><<<grid, 256, G.lds, s>>>(t);
  return hipGetLastError();
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
__device__ __forceinline__ void tile_coords(int tiles_m, int tiles_n, int& tm, int& tn) {
  int nwg = gridDim.x;
  int bid = blockIdx.x;
  if ((nwg & 7) == 0) bid = (bid & 7) * (nwg >> 3) + (bid >> 3);
  const int GROUP_M = 8;
  int group_size = GROUP_M * tiles_n;
  int g = bid / group_size;
  int first_m = g * GROUP_M;
  int gm = min(tiles_m - first_m, GROUP_M);
  int r = bid % group_size;
  tm = first_m + r % gm;
  tn = r / gm;
}

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
// stage loop unrolled by two, as in the FP32 direct-to-LDS tile.
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

  auto dma = [&](auto buf, int64_t k0) {
    uint32_t* ah = pick(buf, Ah0, Ah1);
    uint32_t* al = pick(buf, Al0, Al1);
    uint32_t* bh = pick(buf, Bh0, Bh1);
    uint32_t* bl = pick(buf, Bl0, Bl1);
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int s = tid + 256 * j, r = s / CPR, q = (s % CPR) ^ swz(r);
      const int64_t o = (row0 + r) * p.lda + k0 + 4 * q;
      const int d = 4 * (256 * j + 64 * wave);
      __builtin_amdgcn_global_load_lds(Agh + o, (__attribute__((address_space(3))) void*)(ah + d),
                                       16, 0, 0);
      __builtin_amdgcn_global_load_lds(Agl + o, (__attribute__((address_space(3))) void*)(al + d),
                                       16, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int s = tid + 256 * j, r = s / CPR, q = (s % CPR) ^ swz(r);
      const int64_t o = (col0 + r) * p.ldb + k0 + 4 * q;
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
      const int64_t gr = row0 + r, gk = k0 + c;
      uint4 h = make_uint4(0u, 0u, 0u, 0u), l = h;
      if (gr < p.M && gk < kend) {
        h = ld4(Agh + gr * p.lda + gk, gk);
        l = ld4(Agl + gr * p.lda + gk, gk);
      }
      rah[j] = h;
      ral[j] = l;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int s = tid + 256 * j, r = s / CPR, c = (s % CPR) * 4;
      const int64_t gr = col0 + r, gk = k0 + c;
      uint4 h = make_uint4(0u, 0u, 0u, 0u), l = h;
      if (gr < p.N && gk < kend) {
        h = ld4(Bgh + gr * p.ldb + gk, gk);
        l = ld4(Bgl + gr * p.ldb + gk, gk);
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
__device__ __forceinline__ int dl_swz(int r) { return (r ^ (r >> 3)) & 7; }
// Rows of 16 chunks (BK = 32): 256-byte rows start on the same bank, so the
// low four row bits alone spread 8 or 16 consecutive rows.
__device__ __forceinline__ int dl_swz16(int r) { return r & 15; }

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

// ---------------------------------------------------------------------------
// Small problems: one thread per complex output, sequential K loop (FP64,
// FP32 or split BF16 products).  Used when a tile would be mostly empty.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

template <int MODE>
__device__ __forceinline__ void cgemm_small_body(const GemmParams& p, int64_t blk, int split,
                                                 int b) {
  const int64_t e = blk * 256 + threadIdx.x;
  if (e >= p.M * p.N) return;
  const int64_t row = e / p.N, col = e % p.N;
  const int64_t kbeg = int64_t(split) * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int64_t ao = batch_off(p.a_bs, p.nbb, b) + row * p.lda;
  const int64_t bo = batch_off(p.b_bs, p.nbb, b) + col * p.ldb;
  if constexpr (MODE == RN_FP64) {
    const double2* A = reinterpret_cast<const double2*>(p.A) + ao;
    const double2* B = reinterpret_cast<const double2*>(p.B) + bo;
    double re = 0.0, im = 0.0;
    for (int64_t k = kbeg; k < kend; ++k) {
      double2 a = A[k], bb = B[k];
      re = fma(a.x, bb.x, re);
      re = fma(-a.y, bb.y, re);
      im = fma(a.x, bb.y, im);
      im = fma(a.y, bb.x, im);
    }
    store_out<double>(p, b, split, row, col, 0, re);
    store_out<double>(p, b, split, row, col, 1, im);
  } else if constexpr (MODE == RN_FP32_3M) {
    const float2* A = reinterpret_cast<const float2*>(p.A) + ao;
    const float2* B = reinterpret_cast<const float2*>(p.B) + bo;
    float t1 = 0.f, t2 = 0.f, t3 = 0.f;
    for (int64_t k = kbeg; k < kend; ++k) {
      float2 a = A[k], bb = B[k];
      t1 = fmaf(a.x, bb.x, t1);
      t2 = fmaf(a.y, bb.y, t2);
      t3 = fmaf(a.x + a.y, bb.x + bb.y, t3);
    }
    store_out<float>(p, b, split, row, col, 0, t1 - t2);
    store_out<float>(p, b, split, row, col, 1, (t3 - t1) - t2);
  } else if constexpr (MODE == RN_FP32_4M) {
    const float2* A = reinterpret_cast<const float2*>(p.A) + ao;
    const float2* B = reinterpret_cast<const float2*>(p.B) + bo;
    float re = 0.f, im = 0.f;
    for (int64_t k = kbeg; k < kend; ++k) {
      float2 a = A[k], bb = B[k];
      re = fmaf(a.x, bb.x, re);
      re = fmaf(-a.y, bb.y, re);
      im = fmaf(a.x, bb.y, im);
      im = fmaf(a.y, bb.x, im);
    }
    store_out<float>(p, b, split, row, col, 0, re);
    store_out<float>(p, b, split, row, col, 1, im);
  } else {
    const uint32_t* Ah = reinterpret_cast<const uint32_t*>(p.A) + ao;
    const uint32_t* Al = reinterpret_cast<const uint32_t*>(p.A2) + ao;
    const uint32_t* Bh = reinterpret_cast<const uint32_t*>(p.B) + bo;
    const uint32_t* Bl = reinterpret_cast<const uint32_t*>(p.B2) + bo;
    float re = 0.f, im = 0.f;
    for (int64_t k = kbeg; k < kend; ++k) {
      uint32_t ah = Ah[k], al = Al[k], bh = Bh[k], bl = Bl[k];
      float ahr = bf_lo(ah), ahi = bf_hi(ah), alr = bf_lo(al), ali = bf_hi(al);
      float bhr = bf_lo(bh), bhi = bf_hi(bh), blr = bf_lo(bl), bli = bf_hi(bl);
      // lo*hi + hi*lo + hi*hi, each a complex product of bf16 values (exact
      // in FP32), accumulated in FP32.
      re = fmaf(alr, bhr, re); re = fmaf(-ali, bhi, re);
      im = fmaf(alr, bhi, im); im = fmaf(ali, bhr, im);
      re = fmaf(ahr, blr, re); re = fmaf(-ahi, bli, re);
      im = fmaf(ahr, bli, im); im = fmaf(ahi, blr, im);
      re = fmaf(ahr, bhr, re); re = fmaf(-ahi, bhi, re);
      im = fmaf(ahr, bhi, im); im = fmaf(ahi, bhr, im);
    }
    store_out<float>(p, b, split, row, col, 0, re);
    store_out<float>(p, b, split, row, col, 1, im);
  }
}

// ---------------------------------------------------------------------------
// Skinny problems (at most 8 output rows after orienting, see
// skinny_orient): memory-bound, so the GEMM streams each B row once.  A
// workgroup owns 16 output columns (4 per wave).  Lane l of every wave
// handles k = k0 + l + 64 u (u < U) of each K chunk, so it loads its A
// values for the chunk once into registers and reuses them for all four
// columns; the 4 x U loads of B per chunk are issued together.  Per-(column,
// row) partial sums are combined across the wave by a fixed xor-shuffle
// tree at the end.
// ---------------------------------------------------------------------------
constexpr int kSkinnyRows = 8;
constexpr int kSkinnyCols = 16;

template <typename R>
__device__ __forceinline__ R wave_sum(R v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Operand element of each mode: complex128, complex64, or the bf16 hi/lo
// words of one complex (re in the low half, im in the high half).
template <int MODE>
struct SkinnyElem {
  using T = typename std::conditional<MODE == RN_FP64, double2,
                                      typename std::conditional<MODE == RN_BF16X3, uint2,
                                                                float2>::type>::type;
};

template <int MODE>
__device__ __forceinline__ typename SkinnyElem<MODE>::T skinny_load(const void* X, const void* X2,
                                                                   int64_t i) {
  if constexpr (MODE == RN_FP64) {
    return reinterpret_cast<const double2*>(X)[i];
  } else if constexpr (MODE == RN_BF16X3) {
    return make_uint2(reinterpret_cast<const uint32_t*>(X)[i],
                      reinterpret_cast<const uint32_t*>(X2)[i]);
  } else {
    return reinterpret_cast<const float2*>(X)[i];
  }
}

template <int MODE>
__device__ __forceinline__ typename SkinnyElem<MODE>::T skinny_zero() {
  if constexpr (MODE == RN_FP64) return make_double2(0.0, 0.0);
  else if constexpr (MODE == RN_BF16X3) return make_uint2(0u, 0u);
  else return make_float2(0.f, 0.f);
}

// acc[0..NT) += a * b in the mode's arithmetic (the same per-term formulas
// as the one-thread kernel).
template <int MODE, typename R, typename E>
__device__ __forceinline__ void skinny_mac(R* acc, const E& a, const E& bb) {
  if constexpr (MODE == RN_FP64) {
    acc[0] = fma(a.x, bb.x, acc[0]);
    acc[0] = fma(-a.y, bb.y, acc[0]);
    acc[1] = fma(a.x, bb.y, acc[1]);
    acc[1] = fma(a.y, bb.x, acc[1]);
  } else if constexpr (MODE == RN_BF16X3) {
    const float ahr = bf_lo(a.x), ahi = bf_hi(a.x), alr = bf_lo(a.y), ali = bf_hi(a.y);
    const float bhr = bf_lo(bb.x), bhi = bf_hi(bb.x), blr = bf_lo(bb.y), bli = bf_hi(bb.y);
    float re = acc[0], im = acc[1];
    re = fmaf(alr, bhr, re); re = fmaf(-ali, bhi, re);
    im = fmaf(alr, bhi, im); im = fmaf(ali, bhr, im);
    re = fmaf(ahr, blr, re); re = fmaf(-ahi, bli, re);
    im = fmaf(ahr, bli, im); im = fmaf(ahi, blr, im);
    re = fmaf(ahr, bhr, re); re = fmaf(-ahi, bhi, re);
    im = fmaf(ahr, bhi, im); im = fmaf(ahi, bhr, im);
    acc[0] = re;
    acc[1] = im;
  } else if constexpr (MODE == RN_FP32_3M) {
    acc[0] = fmaf(a.x, bb.x, acc[0]);
    acc[1] = fmaf(a.y, bb.y, acc[1]);
    acc[2] = fmaf(a.x + a.y, bb.x + bb.y, acc[2]);
  } else {
    acc[0] = fmaf(a.x, bb.x, acc[0]);
    acc[0] = fmaf(-a.y, bb.y, acc[0]);
    acc[1] = fmaf(a.x, bb.y, acc[1]);
    acc[1] = fmaf(a.y, bb.x, acc[1]);
  }
}

template <int MODE, int MR>
__device__ __forceinline__ void cgemm_skinny_body(const GemmParams& p, int64_t tn, int split,
                                                  int b) {
  using R = typename std::conditional<MODE == RN_FP64, double, float>::type;
  using E = typename SkinnyElem<MODE>::T;
  constexpr int CPW = kSkinnyCols / 4;
  constexpr int NT = (MODE == RN_FP32_3M) ? 3 : 2;  // partial sums per (column, row)
  constexpr int U = (MODE == RN_FP64) ? 2 : 4;      // k per lane per chunk
  constexpr int KC = 64 * U;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t kbeg = int64_t(split) * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int64_t ao = batch_off(p.a_bs, p.nbb, b), bo = batch_off(p.b_bs, p.nbb, b);
  const int M = (int)p.M;
  const int64_t n0 = int64_t(tn) * kSkinnyCols + wave * CPW;
  R acc[CPW][MR][NT];
#pragma unroll
  for (int c = 0; c < CPW; ++c)
#pragma unroll
    for (int m = 0; m < MR; ++m)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[c][m][t] = R(0);

  for (int64_t k0 = kbeg; k0 < kend; k0 += KC) {
    E av[MR][U];
#pragma unroll
    for (int m = 0; m < MR; ++m)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t k = k0 + lane + 64 * u;
        av[m][u] = (m < M && k < kend) ? skinny_load<MODE>(p.A, p.A2, ao + m * p.lda + k)
                                       : skinny_zero<MODE>();
      }
    E bv[CPW][U];
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t k = k0 + lane + 64 * u;
        const int64_t n = n0 + c;
        bv[c][u] = (n < p.N && k < kend) ? skinny_load<MODE>(p.B, p.B2, bo + n * p.ldb + k)
                                         : skinny_zero<MODE>();
      }
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int m = 0; m < MR; ++m) skinny_mac<MODE>(acc[c][m], av[m][u], bv[c][u]);
  }
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int64_t n = n0 + c;
#pragma unroll
    for (int m = 0; m < MR; ++m) {
      if (m >= M) break;
      R t[NT];
#pragma unroll
      for (int q = 0; q < NT; ++q) t[q] = wave_sum(acc[c][m][q]);
      if (lane == 0 && n < p.N) {
        R re = t[0], im = t[1];
        if constexpr (MODE == RN_FP32_3M) {
          re = t[0] - t[1];
          im = (t[2] - t[0]) - t[1];
        }
        store_out<R>(p, b, split, m, n, 0, re);
        store_out<R>(p, b, split, m, n, 1, im);
      }
    }
  }
}

// Column tiles run grid-stride, so an outer product (K = 1) with billions of
// columns still fits one launch.
template <int MODE, int MR>
__global__ __launch_bounds__(256) void cgemm_skinny(GemmParams p) {
  for (int64_t tn = blockIdx.x; tn < p.tiles_n; tn += gridDim.x)
    cgemm_skinny_body<MODE, MR>(p, tn, blockIdx.y, blockIdx.z);
}

template <int MODE>
static void launch_skinny_m(int mr, dim3 grid, const GemmParams& p, hipStream_t s) {
  switch (mr) {
    case 1: cgemm_skinny<MODE, 1><<<grid, 256, 0, s>>>(p); break;
    case 2: cgemm_skinny<MODE, 2><<<grid, 256, 0, s>>>(p); break;
    case 4: cgemm_skinny<MODE, 4><<<grid, 256, 0, s>>>(p); break;
    default: cgemm_skinny<MODE, 8><<<grid, 256, 0, s>>>(p); break;
  }
}
static void launch_skinny(rn_mode mode, int mr, dim3 grid, const GemmParams& p, hipStream_t s) {
  switch (mode) {
    case RN_FP64: launch_skinny_m<RN_FP64>(mr, grid, p, s); break;
    case RN_FP32_3M: launch_skinny_m<RN_FP32_3M>(mr, grid, p, s); break;
    case RN_BF16X3: launch_skinny_m<RN_BF16X3>(mr, grid, p, s); break;
    default: launch_skinny_m<RN_FP32_4M>(mr, grid, p, s); break;
  }
}

// Orient a skinny problem so that its short side is M: C^T = B A^T runs
// with the operands, strides and output maps exchanged.
static void skinny_orient(GemmParams& p) {
  if (p.M <= p.N) return;
  std::swap(p.A, p.B);
  std::swap(p.A2, p.B2);
  std::swap(p.M, p.N);
  std::swap(p.lda, p.ldb);
  std::swap(p.crs, p.ccs);
  std::swap(p.crh, p.cch);
  std::swap(p.crl, p.ccl);
  for (int i = 0; i < RN_MAX_SLICED; ++i) std::swap(p.a_bs[i], p.b_bs[i]);
}

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

// Entry points whose register use is capped for WAVES waves per SIMD.
#define RN_GEMM_ENTRY_OCC(NAME, WAVES)                                                              \
  template <int WM, int WN, int TM, int TN, int BK>                                     \
  __global__ __launch_bounds__(256, WAVES) void NAME(GemmParams p) {                           \
    int tm, tn;                                                                         \
    tile_coords(p.tiles_m, p.tiles_n, tm, tn);                                          \
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

RN_GEMM_ENTRY(cgemm_f32_4m)
RN_GEMM_ENTRY(cgemm_f32_3m)
RN_GEMM_ENTRY(cgemm_f64_4m)
RN_GEMM_ENTRY(cgemm_bf16x3)
RN_GEMM_ENTRY(cgemm_f32_ri)
RN_GEMM_ENTRY(cgemm_bf16x3_ri)
RN_GEMM_ENTRY(cgemm_f32_rp)
RN_GEMM_ENTRY(cgemm_f64_rp)
RN_GEMM_ENTRY(cgemm_f32_big)
RN_GEMM_ENTRY(cgemm_f32_3mbig)
// Two waves per SIMD for the 128 x 128 tiles, three for 128 x 64 (48 KiB of
// LDS: three workgroups per CU), four for the 64 x 64 and 128 x 32 tiles.
RN_GEMM_ENTRY_OCC(cgemm_f32_dl, (TM * TN * WM * WN <= 4 ? 4 : TM * TN * WM * WN <= 8 ? 3 : 2))
RN_GEMM_ENTRY_OCC(cgemm_f64_dl, 2)
RN_GEMM_ENTRY_OCC(cgemm_f64_3mdl, 3)
RN_GEMM_ENTRY_OCC(cgemm_f32_3mdl, 2)
RN_GEMM_ENTRY_OCC(cgemm_bf16x3_dl, 2)
RN_GEMM_ENTRY_OCC(cgemm_f64_big, 2)

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

template <int MODE>
__global__ __launch_bounds__(256) void cgemm_small(GemmParams p) {
  cgemm_small_body<MODE>(p, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <int MODE>
__global__ __launch_bounds__(256) void cgemm_small_grouped(GroupTable g) {
  const int i = group_find(g, blockIdx.x);
  const GemmParams p = g.probs[i];
  cgemm_small_body<MODE>(p, blockIdx.x - g.prefix[i], 0, 0);
}

template <int MODE, int MR>
__global__ __launch_bounds__(256) void cgemm_skinny_grouped(GroupTable g) {
  const int i = group_find(g, blockIdx.x);
  const GemmParams p = g.probs[i];
  cgemm_skinny_body<MODE, MR>(p, blockIdx.x - g.prefix[i], 0, 0);
}

template <int MODE>
static void launch_skinny_grouped_m(int mr, dim3 grid, const GroupTable& t, hipStream_t s) {
  switch (mr) {
    case 1: cgemm_skinny_grouped<MODE, 1><<<grid, 256, 0, s>>>(t); break;
    case 2: cgemm_skinny_grouped<MODE, 2><<<grid, 256, 0, s>>>(t); break;
    case 4: cgemm_skinny_grouped<MODE, 4><<<grid, 256, 0, s>>>(t); break;
    default: cgemm_skinny_grouped<MODE, 8><<<grid, 256, 0, s>>>(t); break;
  }
}
static void launch_skinny_grouped(rn_mode mode, int mr, dim3 grid, const GroupTable& t,
                                  hipStream_t s) {
  switch (mode) {
    case RN_FP64: launch_skinny_grouped_m<RN_FP64>(mr, grid, t, s); break;
    case RN_FP32_3M: launch_skinny_grouped_m<RN_FP32_3M>(mr, grid, t, s); break;
    case RN_BF16X3: launch_skinny_grouped_m<RN_BF16X3>(mr, grid, t, s); break;
    default: launch_skinny_grouped_m<RN_FP32_4M>(mr, grid, t, s); break;
  }
}

// Split-K reduction: C = sum over splits of the partials, in ascending split
// order, written through the two-level maps.
// Sum of output e's partials (split s at complex index s * total + e) in
// ascending split order, which fixes the rounding.  Eight splits are loaded
// before any is added, so a long split list costs an eighth of the chain of
// dependent loads.
template <typename R>
__device__ __forceinline__ void splitk_sum(const void* partial, int splitk, int64_t total,
                                           int64_t e, R& re, R& im) {
  using V = typename std::conditional<std::is_same<R, double>::value, double2, float2>::type;
  const V* __restrict__ pv = reinterpret_cast<const V*>(partial);
  re = R(0);
  im = R(0);
  int s = 0;
  for (; s + 8 <= splitk; s += 8) {
    V v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = pv[int64_t(s + u) * total + e];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      re += v[u].x;
      im += v[u].y;
    }
  }
  for (; s < splitk; ++s) {
    const V v = pv[int64_t(s) * total + e];
    re += v.x;
    im += v.y;
  }
}

template <typename R>
__global__ __launch_bounds__(256) void splitk_reduce(GemmParams p) {
  const int64_t nb = int64_t(1) << p.nbb;
  const int64_t total = nb * p.M * p.N;
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * 256) {
    const int64_t b = e / (p.M * p.N);
    const int64_t rc = e % (p.M * p.N);
    const int64_t row = rc / p.N, col = rc % p.N;
    R re, im;
    splitk_sum<R>(p.partial, p.splitk, total, e, re, im);
    int64_t off = batch_off(p.c_bs, p.nbb, (int)b) + map2(row, p.crs, p.crh, p.crl) +
                  map2(col, p.ccs, p.cch, p.ccl);
    reinterpret_cast<R*>(p.C)[2 * off] = re;
    reinterpret_cast<R*>(p.C)[2 * off + 1] = im;
  }
}

// Grouped form: workgroup w serves problem i with prefix[i] <= w <
// prefix[i+1], 256 outputs each; partials summed in ascending split order.
template <typename R>
__global__ __launch_bounds__(256) void splitk_reduce_grouped(GroupTable g) {
  const int i = group_find(g, blockIdx.x);
  // By reference: a copy of the parameters (with their stride arrays) would
  // live in scratch memory, per thread, for a few loads.
  const GemmParams& p = g.probs[i];
  const int64_t nb = int64_t(1) << p.nbb;
  const int64_t total = nb * p.M * p.N;
  const int64_t e = int64_t(blockIdx.x - g.prefix[i]) * 256 + threadIdx.x;
  if (e >= total) return;
  const int64_t b = e / (p.M * p.N);
  const int64_t rc = e % (p.M * p.N);
  const int64_t row = rc / p.N, col = rc % p.N;
  R re, im;
  splitk_sum<R>(p.partial, p.splitk, total, e, re, im);
  const int64_t off = batch_off(p.c_bs, p.nbb, (int)b) + map2(row, p.crs, p.crh, p.crl) +
                      map2(col, p.ccs, p.cch, p.ccl);
  reinterpret_cast<R*>(p.C)[2 * off] = re;
  reinterpret_cast<R*>(p.C)[2 * off + 1] = im;
}

// ---------------------------------------------------------------------------
// Tile configurations and dispatch.
// ---------------------------------------------------------------------------
struct TileCfg {
  int bm, bn;  // rows, complex columns
  int bk;      // complex k per LDS stage
};

// Index 0 = small-problem kernel; the rest are MFMA tile shapes per mode.
static const TileCfg kF32Tiles[] = {{1, 1, 1},    {128, 64, 16}, {64, 32, 16},
                                    {256, 64, 8},  {128, 128, 8}, {128, 64, 16},
                                    {128, 128, 8}, {128, 64, 16}, {128, 128, 8},
                                    {128, 128, 16}, {128, 128, 16}, {128, 64, 16},
                                    {128, 64, 8},   {128, 128, 8},  {128, 128, 16},
                                    {128, 128, 16}, {128, 128, 16}, {128, 64, 16},
                                    {64, 64, 16},   {128, 32, 16},  {64, 64, 32},
                                    {128, 32, 32},  {1, 16, 64},    {2, 16, 64},
                                    {4, 16, 64},    {8, 16, 64}};
static const TileCfg kF64Tiles[] = {{1, 1, 1},   {128, 64, 8}, {64, 32, 8},  {128, 64, 8},
                                    {64, 64, 8},  {128, 64, 8}, {64, 128, 8}, {64, 64, 8},
                                    {128, 64, 8}, {64, 128, 8}, {64, 64, 8},  {1, 16, 64},
                                    {2, 16, 64},  {4, 16, 64},  {8, 16, 64}};
static const TileCfg kBF16Tiles[] = {{1, 1, 1},      {128, 64, 16},  {64, 32, 16},
                                     {256, 64, 8},   {128, 128, 8},  {128, 64, 16},
                                     {128, 128, 8},  {256, 64, 8},   {128, 128, 16},
                                     {128, 128, 16}, {128, 64, 16},  {1, 16, 64},
                                     {2, 16, 64},    {4, 16, 64},    {8, 16, 64}};
static const TileCfg k3MTiles[] = {{1, 1, 1},    {128, 64, 16}, {64, 64, 16}, {128, 64, 16},
                                   {64, 128, 16}, {128, 64, 16}, {64, 128, 16}, {1, 16, 64},
                                   {2, 16, 64},   {4, 16, 64},   {8, 16, 64}};

static const TileCfg& tile_of(rn_mode mode, int t) {
  if (mode == RN_FP64) return kF64Tiles[t];
  if (mode == RN_BF16X3) return kBF16Tiles[t];
  if (mode == RN_FP32_3M) return k3MTiles[t];
  return kF32Tiles[t];
}

// Default tile shape when the autotuner has no entry: the one-thread kernel
// for tiny problems, the skinny kernel for outputs with at most 8 rows or
// columns, otherwise the largest tile the output fills (the direct-to-LDS
// tiles, measured fastest on large pairs).
static int tile_count_of(rn_mode mode);

// The last four tiles of every mode are the skinny kernel for at most 1, 2,
// 4 and 8 rows on the short output side; 0 for any other tile.
static int skinny_rows(rn_mode mode, int tile) {
  const int first = tile_count_of(mode) - 4;
  return (tile >= first && tile < first + 4) ? (1 << (tile - first)) : 0;
}
static int skinny_tile(rn_mode mode, int64_t rows) {
  int t = tile_count_of(mode) - 4;
  while (skinny_rows(mode, t) < rows) ++t;
  return t;
}

static int choose_tile(rn_mode mode, int64_t M, int64_t N, int64_t K) {
  // The one-thread kernel loops over K alone: only for short K.  Long K with
  // a narrow output goes to the skinny kernel, whose lanes stride over K.
  if (M * N * K <= (int64_t(1) << 15) && K <= 256) return 0;
  if (std::min(M, N) <= kSkinnyRows) return skinny_tile(mode, std::min(M, N));
  if (M * N * K <= (int64_t(1) << 15)) return 0;
  if (M < 16 || N < 8) return 0;
  if (M >= 128 && N >= 64 && M * N >= (int64_t(1) << 18)) {
    // Direct-to-LDS tiles, except the 128 x 64 split-BF16 Re/Im tile.
    if (mode == RN_FP32_4M) return N >= 128 ? 15 : 17;
    if (mode == RN_FP64) return N >= 128 ? 9 : 8;
    if (mode == RN_BF16X3) return N >= 128 ? 9 : 5;
    return N >= 128 ? 6 : 5;  // FP32-3M
  }
  return 2;
}

int choose_splitk(rn_mode mode, int64_t M, int64_t N, int64_t K, int64_t batch) {
  int t = choose_tile(mode, M, N, K);
  const TileCfg& c = tile_of(mode, t);
  int64_t tiles = ((M + c.bm - 1) / c.bm) * ((N + c.bn - 1) / c.bn) * batch;
  if (skinny_rows(mode, t))  // skinny: one workgroup per 16 long-side entries
    tiles = ((std::max(M, N) + kSkinnyCols - 1) / kSkinnyCols) * batch;
  int64_t minchunk = (t == 0) ? 64 : 4 * c.bk;
  int s = 1;
  while (s < 64 && tiles * s < 1024 && K / (2 * s) >= minchunk) s *= 2;
  return s;
}

static void fill_params(const GemmLaunch& g, GemmParams& p) {
  p = GemmParams{};
  p.A = g.A;
  p.B = g.B;
  p.A2 = g.A2;
  p.B2 = g.B2;
  p.C = g.C;
  p.partial = g.partial;
  p.M = g.M;
  p.N = g.N;
  p.K = g.K;
  p.lda = g.lda;
  p.ldb = g.ldb;
  p.crs = g.crow.shift;
  p.crh = g.crow.hi;
  p.crl = g.crow.lo;
  p.ccs = g.ccol.shift;
  p.cch = g.ccol.hi;
  p.ccl = g.ccol.lo;
  p.nbb = g.nbb;
  for (int i = 0; i < g.nbb; ++i) {
    p.a_bs[i] = g.a_bstride[i];
    p.b_bs[i] = g.b_bstride[i];
    p.c_bs[i] = g.c_bstride[i];
  }
  p.splitk = g.splitk;
  p.kchunk = (g.K + g.splitk - 1) / g.splitk;
}

static int tile_count_of(rn_mode mode) {
  if (mode == RN_FP64) return (int)(sizeof(kF64Tiles) / sizeof(kF64Tiles[0]));
  if (mode == RN_BF16X3) return (int)(sizeof(kBF16Tiles) / sizeof(kBF16Tiles[0]));
  if (mode == RN_FP32_3M) return (int)(sizeof(k3MTiles) / sizeof(k3MTiles[0]));
  return (int)(sizeof(kF32Tiles) / sizeof(kF32Tiles[0]));
}

int gemm_tile_count(rn_mode mode) { return tile_count_of(mode); }

// The skinny tiles run problems whose shorter output side has at most their
// row count.
bool gemm_tile_valid(rn_mode mode, int tile, int64_t M, int64_t N) {
  if (tile < 0 || tile >= tile_count_of(mode)) return false;
  if (const int mr = skinny_rows(mode, tile)) return std::min(M, N) <= mr;
  return true;
}

bool gemm_tile_splits(rn_mode mode, int tile) {
  return tile > 0 && tile < tile_count_of(mode) && !skinny_rows(mode, tile);
}

int gemm_default_tile(rn_mode mode, int64_t M, int64_t N, int64_t K) {
  return choose_tile(mode, M, N, K);
}

hipError_t launch_gemm(const GemmLaunch& g, hipStream_t s, Profiler* prof) {
  GemmParams p;
  fill_params(g, p);
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  const int tile = gemm_tile_valid(g.mode, g.tile, g.M, g.N)
                       ? g.tile
                       : choose_tile(g.mode, g.M, g.N, g.K);
  const TileCfg& c = tile_of(g.mode, tile);
  const unsigned nbatch = 1u << g.nbb;
  const int ev = prof ? prof->begin(1, s) : -1;
  if (const int mr = skinny_rows(g.mode, tile)) {
    skinny_orient(p);
    const int64_t tiles = (p.N + kSkinnyCols - 1) / kSkinnyCols;
    if (tiles > INT32_MAX) return hipErrorInvalidConfiguration;
    p.tiles_m = 1;
    p.tiles_n = (int)tiles;
    dim3 grid((unsigned)std::min<int64_t>(tiles, int64_t(1) << 20), (unsigned)g.splitk, nbatch);
    launch_skinny(g.mode, mr, grid, p, s);
  } else if (tile == 0) {
    if ((g.M * g.N + 255) / 256 > kMaxGrid) return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)((g.M * g.N + 255) / 256), (unsigned)g.splitk, nbatch);
    if (g.mode == RN_FP64)
      cgemm_small<RN_FP64><<<grid, 256, 0, s>>>(p);
    else if (g.mode == RN_FP32_3M)
      cgemm_small<RN_FP32_3M><<<grid, 256, 0, s>>>(p);
    else if (g.mode == RN_BF16X3)
      cgemm_small<RN_BF16X3><<<grid, 256, 0, s>>>(p);
    else
      cgemm_small<RN_FP32_4M><<<grid, 256, 0, s>>>(p);
  } else {
    const int64_t tm = (g.M + c.bm - 1) / c.bm, tn = (g.N + c.bn - 1) / c.bn;
    if (tm * tn > kMaxGrid) return hipErrorInvalidConfiguration;
    p.tiles_m = (int)tm;
    p.tiles_n = (int)tn;
    dim3 grid((unsigned)(tm * tn), (unsigned)g.splitk, nbatch);
    if (g.mode == RN_FP64) {
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
    } else if (g.mode == RN_FP32_3M) {
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
    } else if (g.mode == RN_BF16X3) {
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
      else
        cgemm_bf16x3_dl<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(p);
    } else {
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
  }
  hipError_t e = hipGetLastError();
  if (prof) prof->end(ev, s);
  if (e != hipSuccess || g.splitk <= 1) return e;
  int64_t total = int64_t(nbatch) * g.M * g.N;
  unsigned rg = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
  const int ev2 = prof ? prof->begin(2, s) : -1;
  if (g.mode == RN_FP64)
    splitk_reduce<double><<<rg, 256, 0, s>>>(p);
  else
    splitk_reduce<float><<<rg, 256, 0, s>>>(p);
  e = hipGetLastError();
  if (prof) prof->end(ev2, s);
  return e;
}

// Upper bound of the parameter tables of one grouped batch of n problems,
// whatever the tile choice (at most one GEMM group per tile shape).
size_t grouped_table_bound(rn_mode mode, int n) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  // Permutes: up to two per problem, split over one table per tile shape
  // (each table padded to 256 bytes twice).
  const size_t groups = size_t(gemm_tile_count(mode));
  size_t b = 2 * size_t(n) * sizeof(PermParams) + (2 * size_t(n) + groups) * sizeof(int32_t) +
             2 * 256 * groups;
  // One GEMM group per tile shape, plus the split-K reduction's table.
  b += size_t(gemm_tile_count(mode) + 1) *
       (al(size_t(n) * sizeof(GemmParams)) + al((size_t(n) + 1) * sizeof(int32_t)));
  return b;
}

size_t grouped_gemm_build(const std::vector<GemmLaunch>& probs, int tile,
                          std::vector<char>& table, GroupedLaunch& G) {
  G = GroupedLaunch{};
  G.n = (int)probs.size();
  G.tile = tile;
  if (probs.empty()) return 0;
  G.mode = probs[0].mode;
  const TileCfg& c = tile_of(G.mode, tile);
  std::vector<GemmParams> ps(probs.size());
  std::vector<int32_t> prefix(probs.size() + 1, 0);
  int64_t total = 0;
  // The MFMA tiles also split K (splitk > 1: partials reduced afterwards by
  // splitk_reduce_grouped); the skinny and one-thread kernels do not.
  const bool can_split = tile != 0 && !skinny_rows(G.mode, tile);
  for (size_t i = 0; i < probs.size(); ++i) {
    fill_params(probs[i], ps[i]);
    if (!can_split || probs[i].splitk <= 1 || !probs[i].partial) {
      ps[i].splitk = 1;
      ps[i].partial = nullptr;
    }
    ps[i].kchunk = (probs[i].K + ps[i].splitk - 1) / ps[i].splitk;
    int64_t blocks;
    if (skinny_rows(G.mode, tile)) {
      skinny_orient(ps[i]);
      blocks = (ps[i].N + kSkinnyCols - 1) / kSkinnyCols;
      ps[i].tiles_m = 1;
      ps[i].tiles_n = (int)std::min<int64_t>(blocks, INT32_MAX);
    } else if (tile == 0) {
      blocks = (probs[i].M * probs[i].N + 255) / 256;
    } else {
      const int64_t tm = (probs[i].M + c.bm - 1) / c.bm, tn = (probs[i].N + c.bn - 1) / c.bn;
      ps[i].tiles_m = (int)std::min<int64_t>(tm, INT32_MAX);
      ps[i].tiles_n = (int)std::min<int64_t>(tn, INT32_MAX);
      blocks = tm * tn * ps[i].splitk;
    }
    total += blocks;
    prefix[i + 1] = prefix_entry(total);
  }
  G.blocks = grouped_blocks(total);
  G.params_off = 0;
  G.prefix_off = (probs.size() * sizeof(GemmParams) + 255) & ~size_t(255);
  size_t bytes = (G.prefix_off + prefix.size() * sizeof(int32_t) + 255) & ~size_t(255);
  table.resize(bytes);
  memcpy(table.data(), ps.data(), probs.size() * sizeof(GemmParams));
  memcpy(table.data() + G.prefix_off, prefix.data(), prefix.size() * sizeof(int32_t));
  return bytes;
}

hipError_t launch_gemm_grouped(const GroupedLaunch& G, const void* table_dev, hipStream_t s) {
  if (G.n == 0 || G.blocks == 0) return hipSuccess;
  if (G.blocks < 0) return hipErrorInvalidConfiguration;
  GroupTable t;
  t.probs = reinterpret_cast<const GemmParams*>(static_cast<const char*>(table_dev) + G.params_off);
  t.prefix = reinterpret_cast<const int32_t*>(static_cast<const char*>(table_dev) + G.prefix_off);
  t.n = G.n;
  const dim3 grid((unsigned)G.blocks);
  const int tile = G.tile;
  if (const int mr = skinny_rows(G.mode, tile)) {
    launch_skinny_grouped(G.mode, mr, grid, t, s);
    return hipGetLastError();
  }
  switch (G.mode) {
    case RN_FP64:
      if (tile == 0) cgemm_small_grouped<RN_FP64><<<grid, 256, 0, s>>>(t);
      else if (tile == 1) cgemm_f64_4m_grouped<2, 2, 4, 4, 8><<<grid, 256, 0, s>>>(t);
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
      break;
    case RN_FP32_3M:
      if (tile == 0) cgemm_small_grouped<RN_FP32_3M><<<grid, 256, 0, s>>>(t);
      else if (tile == 1) cgemm_f32_3m_grouped<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(t);
      else if (tile == 2) cgemm_f32_3m_grouped<2, 2, 1, 1, 16><<<grid, 256, 0, s>>>(t);
      else if (tile == 3) cgemm_f32_3mbig_grouped<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(t);
      else if (tile == 4) cgemm_f32_3mbig_grouped<2, 2, 1, 2, 16><<<grid, 256, 0, s>>>(t);
      else if (tile == 5) cgemm_f32_3mdl_grouped<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(t);
      else cgemm_f32_3mdl_grouped<2, 2, 1, 2, 16><<<grid, 256, 0, s>>>(t);
      break;
    case RN_BF16X3:
      if (tile == 0) cgemm_small_grouped<RN_BF16X3><<<grid, 256, 0, s>>>(t);
      else if (tile == 1) cgemm_bf16x3_grouped<2, 2, 2, 2, 16><<<grid, 256, 0, s>>>(t);
      else if (tile == 2) cgemm_bf16x3_grouped<2, 2, 1, 1, 16><<<grid, 256, 0, s>>>(t);
      else if (tile == 3) cgemm_bf16x3_grouped<2, 2, 4, 2, 8><<<grid, 256, 0, s>>>(t);
      else if (tile == 4) cgemm_bf16x3_grouped<2, 2, 2, 4, 8><<<grid, 256, 0, s>>>(t);
      else if (tile == 5) cgemm_bf16x3_ri_grouped<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(t);
      else if (tile == 6) cgemm_bf16x3_ri_grouped<2, 2, 2, 2, 8><<<grid, 256, 0, s>>>(t);
      else if (tile == 7) cgemm_bf16x3_ri_grouped<2, 2, 4, 1, 8><<<grid, 256, 0, s>>>(t);
      else if (tile == 8) cgemm_bf16x3_ri_grouped<2, 2, 2, 2, 16><<<grid, 256, 0, s>>>(t);
      else if (tile == 9) cgemm_bf16x3_dl_grouped<2, 2, 2, 2, 16><<<grid, 256, 0, s>>>(t);
      else cgemm_bf16x3_dl_grouped<2, 2, 2, 1, 16><<<grid, 256, 0, s>>>(t);
      break;
    default:
      if (tile == 0) cgemm_small_grouped<RN_FP32_4M><<<grid, 256, 0, s>>>(t);
      else if (tile == 1) cgemm_f32_4m_grouped<2, 2, 2, 2, 16><<<grid, 256, 0, s>>>(t);
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
      break;
  }
  return hipGetLastError();
}

// Reduction of the split-K partials of a grouped batch: one table entry per
// problem that was split (the GEMM parameters, with its partial buffer).
size_t grouped_reduce_build(const std::vector<GemmLaunch>& probs, std::vector<char>& table,
                            GroupedLaunch& G) {
  G = GroupedLaunch{};
  std::vector<GemmParams> ps;
  std::vector<int32_t> prefix(1, 0);
  int64_t total = 0;
  for (const GemmLaunch& g : probs) {
    if (g.splitk <= 1 || !g.partial || g.M <= 0 || g.N <= 0) continue;
    GemmParams p;
    fill_params(g, p);
    ps.push_back(p);
    total += ((int64_t(1) << g.nbb) * g.M * g.N + 255) / 256;
    prefix.push_back(prefix_entry(total));
  }
  G.n = (int)ps.size();
  if (ps.empty()) return 0;
  G.mode = probs[0].mode;
  G.blocks = grouped_blocks(total);
  G.params_off = 0;
  G.prefix_off = (ps.size() * sizeof(GemmParams) + 255) & ~size_t(255);
  size_t bytes = (G.prefix_off + prefix.size() * sizeof(int32_t) + 255) & ~size_t(255);
  table.assign(bytes, 0);
  memcpy(table.data(), ps.data(), ps.size() * sizeof(GemmParams));
  memcpy(table.data() + G.prefix_off, prefix.data(), prefix.size() * sizeof(int32_t));
  return bytes;
}

hipError_t launch_reduce_grouped(const GroupedLaunch& G, const void* table_dev, hipStream_t s) {
  if (G.n == 0 || G.blocks == 0) return hipSuccess;
  if (G.blocks < 0) return hipErrorInvalidConfiguration;
  GroupTable t;
  t.probs = reinterpret_cast<const GemmParams*>(static_cast<const char*>(table_dev) + G.params_off);
  t.prefix = reinterpret_cast<const int32_t*>(static_cast<const char*>(table_dev) + G.prefix_off);
  t.n = G.n;
  if (G.mode == RN_FP64)
    splitk_reduce_grouped<double><<<dim3((unsigned)G.blocks), 256, 0, s>>>(t);
  else
    splitk_reduce_grouped<float><<<dim3((unsigned)G.blocks), 256, 0, s>>>(t);
  return hipGetLastError();
}

// ===========================================================================
// Small network steps, evaluated straight from the stored layouts.  One
// workgroup computes 256 consecutive outputs of one slice batch; the K-part
// offsets of both operands are tabulated in LDS once per workgroup.  All
// independent small steps of one dependency level of the path share one
// launch.
// ===========================================================================
static_assert(sizeof(DirectStep) % 4 == 0 && sizeof(DirectStep) <= 4 * 256,
              "step copied by one word per thread");
struct DirectTable {
  const DirectStep* steps;
  const int32_t* prefix;
  int n;
  int nout;
  int64_t pass;
};

template <int MODE>
__global__ __launch_bounds__(256) void direct_grouped(DirectTable g) {
  __shared__ int32_t koa[kDirectMaxK];
  __shared__ int32_t kob[kDirectMaxK];
  const int bid = blockIdx.x;
  const int lo = find_job(g.prefix, g.n, bid);
  // The step's bit maps are read per output; copy them into LDS once.
  __shared__ __align__(16) uint32_t d_raw[sizeof(DirectStep) / 4];
  if (threadIdx.x < sizeof(DirectStep) / 4)
    d_raw[threadIdx.x] = reinterpret_cast<const uint32_t*>(&g.steps[lo])[threadIdx.x];
  __syncthreads();
  const DirectStep& d = *reinterpret_cast<const DirectStep*>(d_raw);
  const int local = bid - g.prefix[lo];
  const int b = local / d.blocks_per_batch;
  const int64_t e = int64_t(local % d.blocks_per_batch) * 256 + threadIdx.x;
  for (int k = threadIdx.x; k < d.K; k += 256) {
    int32_t oa = 0, ob = 0;
    for (int i = 0; i < d.kbits; ++i)
      if ((k >> i) & 1) {
        oa += int32_t(1) << d.ak[i];
        ob += int32_t(1) << d.bk[i];
      }
    koa[k] = oa;
    kob[k] = ob;
  }
  __syncthreads();
  if (e >= d.M * d.N) return;
  const int64_t m = e >> d.nbits, n = e & (d.N - 1);
  int64_t ao = 0, bo = 0;
  for (int i = 0; i < d.nbb; ++i)
    if ((b >> i) & 1) {
      ao += d.a_bs[i];
      bo += d.b_bs[i];
    }
  for (int i = 0; i < g.nout; ++i)
    if ((g.pass >> (g.nout - 1 - i)) & 1) {
      if (d.a_pp[i]) ao += int64_t(1) << (d.a_pp[i] - 1);
      if (d.b_pp[i]) bo += int64_t(1) << (d.b_pp[i] - 1);
    }
  for (int i = 0; i < d.mbits; ++i)
    if ((m >> i) & 1) ao += int64_t(1) << d.am[i];
  for (int i = 0; i < d.nbits; ++i)
    if ((n >> i) & 1) bo += int64_t(1) << d.bn[i];
  const int64_t co = int64_t(b) * d.M * d.N + e;
  if constexpr (MODE == RN_FP64) {
    const double2* A = reinterpret_cast<const double2*>(d.A) + ao;
    const double2* B = reinterpret_cast<const double2*>(d.B) + bo;
    double re = 0.0, im = 0.0;
    for (int k = 0; k < d.K; ++k) {
      double2 a = A[koa[k]], bb = B[kob[k]];
      re = fma(a.x, bb.x, re);
      re = fma(-a.y, bb.y, re);
      im = fma(a.x, bb.y, im);
      im = fma(a.y, bb.x, im);
    }
    reinterpret_cast<double2*>(d.C)[co] = make_double2(re, im);
  } else {
    const float2* A = reinterpret_cast<const float2*>(d.A) + ao;
    const float2* B = reinterpret_cast<const float2*>(d.B) + bo;
    float re = 0.f, im = 0.f;
    if constexpr (MODE == RN_FP32_3M) {
      float t1 = 0.f, t2 = 0.f, t3 = 0.f;
      for (int k = 0; k < d.K; ++k) {
        float2 a = A[koa[k]], bb = B[kob[k]];
        t1 = fmaf(a.x, bb.x, t1);
        t2 = fmaf(a.y, bb.y, t2);
        t3 = fmaf(a.x + a.y, bb.x + bb.y, t3);
      }
      re = t1 - t2;
      im = (t3 - t1) - t2;
    } else if constexpr (MODE == RN_BF16X3) {
      for (int k = 0; k < d.K; ++k) {
        float2 a = A[koa[k]], bb = B[kob[k]];
        uint32_t h0, l0, h1, l1, h2, l2, h3, l3;
        bf16_split(a.x, h0, l0);
        bf16_split(a.y, h1, l1);
        bf16_split(bb.x, h2, l2);
        bf16_split(bb.y, h3, l3);
        const float ahr = __uint_as_float(h0 << 16), alr = __uint_as_float(l0 << 16);
        const float ahi = __uint_as_float(h1 << 16), ali = __uint_as_float(l1 << 16);
        const float bhr = __uint_as_float(h2 << 16), blr = __uint_as_float(l2 << 16);
        const float bhi = __uint_as_float(h3 << 16), bli = __uint_as_float(l3 << 16);
        re = fmaf(alr, bhr, re); re = fmaf(-ali, bhi, re);
        im = fmaf(alr, bhi, im); im = fmaf(ali, bhr, im);
        re = fmaf(ahr, blr, re); re = fmaf(-ahi, bli, re);
        im = fmaf(ahr, bli, im); im = fmaf(ahi, blr, im);
        re = fmaf(ahr, bhr, re); re = fmaf(-ahi, bhi, re);
        im = fmaf(ahr, bhi, im); im = fmaf(ahi, bhr, im);
      }
    } else {
      for (int k = 0; k < d.K; ++k) {
        float2 a = A[koa[k]], bb = B[kob[k]];
        re = fmaf(a.x, bb.x, re);
        re = fmaf(-a.y, bb.y, re);
        im = fmaf(a.x, bb.y, im);
        im = fmaf(a.y, bb.x, im);
      }
    }
    reinterpret_cast<float2*>(d.C)[co] = make_float2(re, im);
  }
}

size_t grouped_perm_bound(int n) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  return al(size_t(n) * sizeof(PermParams)) + al((size_t(n) + 1) * sizeof(int32_t));
}

size_t grouped_direct_bound(int n) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  return al(size_t(n) * sizeof(DirectStep)) + al((size_t(n) + 1) * sizeof(int32_t));
}

size_t grouped_direct_build(const std::vector<DirectStep>& steps, rn_mode mode,
                            std::vector<char>& table, GroupedLaunch& G) {
  G = GroupedLaunch{};
  G.n = (int)steps.size();
  G.mode = mode;
  if (steps.empty()) return 0;
  std::vector<int32_t> prefix(steps.size() + 1, 0);
  int64_t total = 0;
  for (size_t i = 0; i < steps.size(); ++i) {
    total += int64_t(steps[i].blocks_per_batch) << steps[i].nbb;
    prefix[i + 1] = prefix_entry(total);
  }
  G.blocks = grouped_blocks(total);
  G.params_off = 0;
  G.prefix_off = (steps.size() * sizeof(DirectStep) + 255) & ~size_t(255);
  size_t bytes = (G.prefix_off + prefix.size() * sizeof(int32_t) + 255) & ~size_t(255);
  table.assign(bytes, 0);
  memcpy(table.data(), steps.data(), steps.size() * sizeof(DirectStep));
  memcpy(table.data() + G.prefix_off, prefix.data(), prefix.size() * sizeof(int32_t));
  return bytes;
}

hipError_t launch_direct_grouped(const GroupedLaunch& G, const void* table_dev, int64_t pass,
                                 int nout, hipStream_t s) {
  if (G.n == 0 || G.blocks == 0) return hipSuccess;
  if (G.blocks < 0) return hipErrorInvalidConfiguration;
  if (nout < 0 || nout > RN_MAX_SLICED) return hipErrorInvalidValue;
  DirectTable t;
  t.pass = pass;
  t.nout = nout;
  t.steps = reinterpret_cast<const DirectStep*>(static_cast<const char*>(table_dev) + G.params_off);
  t.prefix = reinterpret_cast<const int32_t*>(static_cast<const char*>(table_dev) + G.prefix_off);
  t.n = G.n;
  switch (G.mode) {
    case RN_FP64: direct_grouped<RN_FP64><<<G.blocks, 256, 0, s>>>(t); break;
    case RN_FP32_3M: direct_grouped<RN_FP32_3M><<<G.blocks, 256, 0, s>>>(t); break;
    case RN_BF16X3: direct_grouped<RN_BF16X3><<<G.blocks, 256, 0, s>>>(t); break;
    default: direct_grouped<RN_FP32_4M><<<G.blocks, 256, 0, s>>>(t); break;
  }
  return hipGetLastError();
}

// ===========================================================================
// C += P over n complex elements (streamed contraction: the partial of one
// block pair added to its output block).
// ===========================================================================
template <typename T>
__global__ __launch_bounds__(256) void add_into(T* __restrict__ c, const T* __restrict__ p,
                                                int64_t n) {
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    T a = c[i], b = p[i];
    a.x += b.x;
    a.y += b.y;
    c[i] = a;
  }
}

hipError_t launch_add_into(void* c, const void* p, int64_t n, int es, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 256 * 32);
  if (es == 16)
    add_into<double2><<<grid, 256, 0, s>>>(static_cast<double2*>(c),
                                           static_cast<const double2*>(p), n);
  else
    add_into<float2><<<grid, 256, 0, s>>>(static_cast<float2*>(c), static_cast<const float2*>(p),
                                          n);
  return hipGetLastError();
}

// ===========================================================================
// FP64 reductions.  Deterministic: every element goes to a fixed lane, lanes
// combine in a fixed butterfly order (cross-lane shuffles), waves in a fixed
// order through LDS, blocks in ascending order in a second pass.
// ===========================================================================
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  return t;
}

constexpr int kRedBlocks = 2048;  // partials; the handle's reduction scratch holds 4096

// Each thread keeps four independent loads in flight per round: a block
// reads four consecutive 256-element pieces of one 1024-element chunk (the
// chunks dealt round robin over the blocks), so the loads stay close in
// memory; four partial sums, added in a fixed order.
template <typename T>
__global__ __launch_bounds__(256) void norm2_partial(const T* x, int64_t n, double* part) {
  __shared__ double sh[4];
  const int64_t stride = int64_t(kRedBlocks) * 1024;
  double s4[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t i = int64_t(blockIdx.x) * 1024 + threadIdx.x;
  for (; i + 768 < n; i += stride) {
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = x[i + 256 * u];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double re = (double)v[u].x, im = (double)v[u].y;
      s4[u] += re * re + im * im;
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (i + 256 * u < n) {
      const double re = (double)x[i + 256 * u].x, im = (double)x[i + 256 * u].y;
      s4[u] += re * re + im * im;
    }
  double s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void sum_partials(const double* part, int n, double* out) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[0] = s;
}

hipError_t launch_norm2(const void* x, int64_t n, int dtype, double* out, double* scratch,
                        hipStream_t s) {
  if (dtype == RN_C128)
    norm2_partial<double2><<<kRedBlocks, 256, 0, s>>>(reinterpret_cast<const double2*>(x), n,
                                                     scratch);
  else
    norm2_partial<float2><<<kRedBlocks, 256, 0, s>>>(reinterpret_cast<const float2*>(x), n,
                                                    scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  sum_partials<<<1, 256, 0, s>>>(scratch, kRedBlocks, out);
  return hipGetLastError();
}

// Complex sum of n values in FP64 by one workgroup: lane t accumulates
// values t, t + 256, ... in ascending order, then the fixed tree.
template <typename T>
__global__ __launch_bounds__(256) void csum_kernel(const T* v, int64_t n, double* out,
                                                   double* each) {
  __shared__ double sh[4];
  double re = 0.0, im = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    double r = (double)v[i].x, m = (double)v[i].y;
    re += r;
    im += m;
    if (each) {
      each[2 * i] = r;
      each[2 * i + 1] = m;
    }
  }
  re = block_sum(re, sh);
  __syncthreads();
  im = block_sum(im, sh);
  if (threadIdx.x == 0) {
    out[0] = re;
    out[1] = im;
  }
}

hipError_t launch_sum_c128(const double* vals, int64_t n, double* out, hipStream_t s) {
  csum_kernel<double2><<<1, 256, 0, s>>>(reinterpret_cast<const double2*>(vals), n, out,
                                         nullptr);
  return hipGetLastError();
}

hipError_t launch_sum_slices(const void* vals, int es, int64_t n, double* out_sum,
                             double* out_each, hipStream_t s) {
  if (es == 16)
    csum_kernel<double2><<<1, 256, 0, s>>>(reinterpret_cast<const double2*>(vals), n, out_sum,
                                           out_each);
  else
    csum_kernel<float2><<<1, 256, 0, s>>>(reinterpret_cast<const float2*>(vals), n, out_sum,
                                          out_each);
  return hipGetLastError();
}

}  // namespace rn
