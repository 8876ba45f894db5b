// HIP kernels for gfx950 (MI355X): index permutation, GEMM dispatch (the
// MFMA tiles live in one file per mode, gemm_*.hip), the one-thread and
// skinny GEMM kernels, split-K reduction, small network steps and FP64
// reductions.
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

#include "kcommon.hpp"

namespace rn {

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
  int64_t gw;  // KIND 2: k per plane group (W = min(16, K), a power of two)
  int64_t sstride;  // nsum > 1: elements between the input's split-K partials
  int nsum;         // partials summed (ascending) per element read
  int nt_store;     // copy: non-temporal stores (outputs beyond the caches)
};

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

// Streaming accesses of the permutes: every element is read once, so loads
// are non-temporal; stores too when the launch's outputs are larger than the
// 256 MiB memory-side cache (a smaller output is read next by the GEMM, which
// then finds it there: non-temporal stores cost the FP64 20-qubit amplitude
// 7 us).  Measured: 2 GiB complex64 relayout 0.84 -> 0.80 ms.
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  typedef typename std::conditional<sizeof(T) == 8, float, double>::type S;
  typedef S nv __attribute__((ext_vector_type(2)));
  const nv t = __builtin_nontemporal_load(reinterpret_cast<const nv*>(p));
  T v;
  v.x = t.x;
  v.y = t.y;
  return v;
}
template <typename T>
__device__ __forceinline__ void st_stream(T* p, const T& v) {
  typedef typename std::conditional<sizeof(T) == 8, float, double>::type S;
  typedef S nv __attribute__((ext_vector_type(2)));
  const nv t = {v.x, v.y};
  __builtin_nontemporal_store(t, reinterpret_cast<nv*>(p));
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
      if (!PRED || (j << 8) < tsize) v[j] = ld_stream(in + ib + in_lo + p.hi_in[j]);
    // Unreduced split-K partials: add the others in ascending split order.
    for (int q = 1; q < p.nsum; ++q) {
#pragma unroll
      for (int j = 0; j < E; ++j)
        if (!PRED || (j << 8) < tsize) {
          const T w = in[ib + in_lo + p.hi_in[j] + q * p.sstride];
          v[j].x += w.x;
          v[j].y += w.y;
        }
    }
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
        if (p.nt_store)
          st_stream(reinterpret_cast<T*>(p.out) + oo, v[j]);
        else
          reinterpret_cast<T*>(p.out)[oo] = v[j];
      } else if constexpr (KIND == 1) {
        uint32_t hr, lr, hi_, li_;
        bf16_split(v[j].x, hr, lr);
        bf16_split(v[j].y, hi_, li_);
        reinterpret_cast<uint32_t*>(p.out)[oo] = hr | (hi_ << 16);
        reinterpret_cast<uint32_t*>(p.out2)[oo] = lr | (li_ << 16);
      } else if constexpr (KIND == 3) {
        // Row-interleaved split: element oo = r K + k of the K-contiguous
        // operand (K a multiple of 16) goes to word 2 (oo - oo % 16) + oo % 16
        // (hi) and 16 words later (lo), so each 16 k of a row are one line.
        uint32_t hr, lr, hi_, li_;
        bf16_split(v[j].x, hr, lr);
        bf16_split(v[j].y, hi_, li_);
        uint32_t* o = reinterpret_cast<uint32_t*>(p.out) + 2 * (oo & ~int64_t(15)) + (oo & 15);
        o[0] = hr | (hi_ << 16);
        o[16] = lr | (li_ << 16);
      } else {
        // Planar-group split for the Gauss form: element oo = r K + k of the
        // K-contiguous operand goes to 6 (oo - w) + q W + w, w = oo % W, in
        // plane q = re hi, im hi, (re + im) hi, re lo, im lo, (re + im) lo
        // (the sum rounded once in FP32); one output array.
        uint32_t hr, lr, hi_, li_, hs, ls;
        bf16_split(v[j].x, hr, lr);
        bf16_split(v[j].y, hi_, li_);
        bf16_split(v[j].x + v[j].y, hs, ls);
        const int64_t w = oo & (p.gw - 1);
        uint16_t* o = reinterpret_cast<uint16_t*>(p.out) + 6 * (oo - w) + w;
        o[0] = (uint16_t)hr;
        o[p.gw] = (uint16_t)hi_;
        o[2 * p.gw] = (uint16_t)hs;
        o[3 * p.gw] = (uint16_t)lr;
        o[4 * p.gw] = (uint16_t)li_;
        o[5 * p.gw] = (uint16_t)ls;
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
  p.gw = L.gw;
  p.nsum = L.nsum;
  p.nt_store = (int64_t(L.in_es) << R) > (int64_t(256) << 20) ? 1 : 0;
  p.sstride = L.sstride;
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
  if (L.kind == 2 && (L.in_es != 8 || L.gw < 1 || L.gw > 16 || (L.gw & (L.gw - 1))))
    return hipErrorInvalidValue;
  if (L.kind == 3 && (L.in_es != 8 || L.perm.nbits < 4)) return hipErrorInvalidValue;
  if (L.kind == 1)
    launch_perm_e<float2, 1>(p, E, grid, lds, s);
  else if (L.kind == 3)
    launch_perm_e<float2, 3>(p, E, grid, lds, s);
  else if (L.kind == 2)
    launch_perm_e<float2, 2>(p, E, grid, lds, s);
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
  int64_t total = 0, out_bytes = 0;
  for (size_t i = 0; i < jobs.size(); ++i) {
    perm_setup(jobs[i], ps[i]);
    max_tsize = std::max(max_tsize, 1 << ps[i].nS);
    total += ps[i].ntiles;
    prefix[i + 1] = prefix_entry(total);
    out_bytes += int64_t(jobs[i].in_es) << jobs[i].perm.nbits;
  }
  // The launch's outputs together decide: beyond the memory-side cache, they
  // are evicted before the GEMMs read them anyway.
  for (PermParams& q : ps) q.nt_store = out_bytes > (int64_t(256) << 20) ? 1 : 0;
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
// Split-BF16 tiles 11 and 12 are the Gauss form on planar operands (permute
// kind 2): only the single block tensordot runs them (see gemm_tile_planar).
static const TileCfg kBF16Tiles[] = {{1, 1, 1},      {128, 64, 16},  {64, 32, 16},
                                     {256, 64, 8},   {128, 128, 8},  {128, 64, 16},
                                     {128, 128, 8},  {256, 64, 8},   {128, 128, 16},
                                     {128, 128, 16}, {128, 64, 16},  {128, 64, 16},
                                     {128, 128, 16}, {1, 16, 64},    {2, 16, 64},
                                     {4, 16, 64},    {8, 16, 64}};
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

static int choose_tile(rn_mode mode, int64_t M, int64_t N, int64_t K, int64_t batch = 1) {
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
  // FP64, mid-size outputs batched over many slices (a sliced network's
  // late steps): 64 x 64 tiles, measured faster than 64 x 32 there (FP32-4M
  // measured no faster with them).
  if (mode == RN_FP64 && M * N * batch >= (int64_t(1) << 18) && M >= 32 && N >= 32) return 10;
  return 2;
}

int choose_splitk(rn_mode mode, int64_t M, int64_t N, int64_t K, int64_t batch) {
  int t = choose_tile(mode, M, N, K, batch);
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
  p.ilv = g.interleaved ? 1 : 0;
}

static int tile_count_of(rn_mode mode) {
  if (mode == RN_FP64) return (int)(sizeof(kF64Tiles) / sizeof(kF64Tiles[0]));
  if (mode == RN_BF16X3) return (int)(sizeof(kBF16Tiles) / sizeof(kBF16Tiles[0]));
  if (mode == RN_FP32_3M) return (int)(sizeof(k3MTiles) / sizeof(k3MTiles[0]));
  return (int)(sizeof(kF32Tiles) / sizeof(kF32Tiles[0]));
}

int gemm_tile_count(rn_mode mode) { return tile_count_of(mode); }

bool gemm_tile_planar(rn_mode mode, int tile) {
  return mode == RN_BF16X3 && (tile == 11 || tile == 12);
}

// The split-BF16 direct-to-LDS tiles (9, 10).
bool gemm_tile_interleaved(rn_mode mode, int tile) {
  return mode == RN_BF16X3 && (tile == 9 || tile == 10);
}

// The skinny tiles run problems whose shorter output side has at most their
// row count; planar-operand tiles need the planar permute and are not valid
// for a GEMM on packed operands.
bool gemm_tile_valid(rn_mode mode, int tile, int64_t M, int64_t N) {
  if (tile < 0 || tile >= tile_count_of(mode)) return false;
  if (gemm_tile_planar(mode, tile)) return false;
  if (const int mr = skinny_rows(mode, tile)) return std::min(M, N) <= mr;
  return true;
}

// No shape defaults to a planar tile: on the rank-28 pair the Gauss tiles
// ran at 352 useful TFLOP/s against 407 for the 4M 128 x 128 tile; a tune
// entry selects them.
int gemm_planar_default(rn_mode mode, int64_t M, int64_t N, int64_t K) {
  (void)mode;
  (void)M;
  (void)N;
  (void)K;
  return -1;
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
  if (g.planar != gemm_tile_planar(g.mode, g.tile) || (g.planar && g.nbb != 0))
    return hipErrorInvalidValue;  // planar operands need a planar tile, unbatched
  const int tile = g.planar || gemm_tile_valid(g.mode, g.tile, g.M, g.N)
                       ? g.tile
                       : choose_tile(g.mode, g.M, g.N, g.K, int64_t(1) << g.nbb);
  // Interleaved operands: a tile that reads them, whole 16-k groups per split.
  if (g.interleaved && (!gemm_tile_interleaved(g.mode, tile) || g.nbb != 0 || g.K % 16 != 0 ||
                        p.kchunk % 16 != 0 || g.lda != 2 * g.K || g.ldb != 2 * g.K))
    return hipErrorInvalidValue;
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
    switch (g.mode) {
      case RN_FP64: launch_tiles_f64(tile, grid, p, s); break;
      case RN_FP32_3M: launch_tiles_f32_3m(tile, grid, p, s); break;
      case RN_BF16X3: launch_tiles_bf16x3(tile, grid, p, s); break;
      default: launch_tiles_f32_4m(tile, grid, p, s); break;
    }
  }
  hipError_t e = hipGetLastError();
  if (prof) prof->end(ev, s);
  if (e != hipSuccess || g.splitk <= 1 || g.partial_only) return e;
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
  if (tile == 0) {
    switch (G.mode) {
      case RN_FP64: cgemm_small_grouped<RN_FP64><<<grid, 256, 0, s>>>(t); break;
      case RN_FP32_3M: cgemm_small_grouped<RN_FP32_3M><<<grid, 256, 0, s>>>(t); break;
      case RN_BF16X3: cgemm_small_grouped<RN_BF16X3><<<grid, 256, 0, s>>>(t); break;
      default: cgemm_small_grouped<RN_FP32_4M><<<grid, 256, 0, s>>>(t); break;
    }
    return hipGetLastError();
  }
  switch (G.mode) {
    case RN_FP64: launch_tiles_f64_grouped(tile, grid, t, s); break;
    case RN_FP32_3M: launch_tiles_f32_3m_grouped(tile, grid, t, s); break;
    case RN_BF16X3: launch_tiles_bf16x3_grouped(tile, grid, t, s); break;
    default: launch_tiles_f32_4m_grouped(tile, grid, t, s); break;
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
// launch, and so do subtrees of tiny steps, each run whole by one workgroup.
// ===========================================================================
static_assert(sizeof(DirectStep) % 4 == 0 && sizeof(DirectStep) <= 4 * 256,
              "step copied by one word per thread");
static_assert(sizeof(TinyStep) % 4 == 0, "tiny steps copied by words");
struct DirectTable {
  const DirectStep* steps;
  const TinyStep* tiny;
  const int32_t* maps;
  const DirectJob* jobs;
  const int32_t* prefix;
  int n;  // jobs
  int nout;
  int64_t pass;
};

// K-part offsets of both operands of step d, for k < K.
__device__ __forceinline__ void direct_ktab(const DirectStep& d, int32_t* koa, int32_t* kob) {
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
}

// The K terms of one output, in k order.  Eight operand pairs are loaded
// before any is used (the loads are independent, so their memory latency is
// paid once per eight terms, not per term); past K the index is clamped, so
// the extra loads stay in bounds and their terms are skipped.
template <typename T, typename F>
__device__ __forceinline__ void direct_kloop(const T* A, const T* B, int K, const int32_t* koa,
                                             const int32_t* kob, F&& term) {
  constexpr int U = 8;
  for (int k0 = 0; k0 < K; k0 += U) {
    T a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = min(k0 + u, K - 1);
      a[u] = A[koa[k]];
      b[u] = B[kob[k]];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k0 + u < K) term(a[u], b[u]);
  }
}

// C[co] = sum_k A[ao + koa[k]] * B[bo + kob[k]] in the mode's arithmetic.
template <int MODE>
__device__ __forceinline__ void direct_dot(const void* Av, const void* Bv, int64_t ao, int64_t bo,
                                           int K, const int32_t* koa, const int32_t* kob,
                                           void* C, int64_t co) {
  if constexpr (MODE == RN_FP64) {
    const double2* A = reinterpret_cast<const double2*>(Av) + ao;
    const double2* B = reinterpret_cast<const double2*>(Bv) + bo;
    double re = 0.0, im = 0.0;
    direct_kloop(A, B, K, koa, kob, [&](double2 a, double2 bb) {
      re = fma(a.x, bb.x, re);
      re = fma(-a.y, bb.y, re);
      im = fma(a.x, bb.y, im);
      im = fma(a.y, bb.x, im);
    });
    reinterpret_cast<double2*>(C)[co] = make_double2(re, im);
  } else {
    const float2* A = reinterpret_cast<const float2*>(Av) + ao;
    const float2* B = reinterpret_cast<const float2*>(Bv) + bo;
    float re = 0.f, im = 0.f;
    if constexpr (MODE == RN_FP32_3M) {
      float t1 = 0.f, t2 = 0.f, t3 = 0.f;
      direct_kloop(A, B, K, koa, kob, [&](float2 a, float2 bb) {
        t1 = fmaf(a.x, bb.x, t1);
        t2 = fmaf(a.y, bb.y, t2);
        t3 = fmaf(a.x + a.y, bb.x + bb.y, t3);
      });
      re = t1 - t2;
      im = (t3 - t1) - t2;
    } else if constexpr (MODE == RN_BF16X3) {
      direct_kloop(A, B, K, koa, kob, [&](float2 a, float2 bb) {
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
      });
    } else {
      direct_kloop(A, B, K, koa, kob, [&](float2 a, float2 bb) {
        re = fmaf(a.x, bb.x, re);
        re = fmaf(-a.y, bb.y, re);
        im = fmaf(a.x, bb.y, im);
        im = fmaf(a.y, bb.x, im);
      });
    }
    reinterpret_cast<float2*>(C)[co] = make_float2(re, im);
  }
}

// Output e (< M*N) of slice batch b of step d.
template <int MODE>
__device__ __forceinline__ void direct_out(const DirectStep& d, int b, int64_t e, int nout,
                                           int64_t pass, const int32_t* koa,
                                           const int32_t* kob) {
  const int64_t m = e >> d.nbits, n = e & (d.N - 1);
  int64_t ao = 0, bo = 0;
  for (int i = 0; i < d.nbb; ++i)
    if ((b >> i) & 1) {
      ao += d.a_bs[i];
      bo += d.b_bs[i];
    }
  for (int i = 0; i < nout; ++i)
    if ((pass >> (nout - 1 - i)) & 1) {
      if (d.a_pp[i]) ao += int64_t(1) << (d.a_pp[i] - 1);
      if (d.b_pp[i]) bo += int64_t(1) << (d.b_pp[i] - 1);
    }
  for (int i = 0; i < d.mbits; ++i)
    if ((m >> i) & 1) ao += int64_t(1) << d.am[i];
  for (int i = 0; i < d.nbits; ++i)
    if ((n >> i) & 1) bo += int64_t(1) << d.bn[i];
  direct_dot<MODE>(d.A, d.B, ao, bo, (int)d.K, koa, kob, d.C, int64_t(b) * d.M * d.N + e);
}

// Output u (slice batch major, then row, then column: also its index in C)
// of tiny step d, with d's maps at mp.
template <int MODE>
__device__ __forceinline__ void tiny_out(const TinyStep& d, int u, const int32_t* mp, int nout,
                                         int64_t pass) {
  const int sh = d.mbits + d.nbits;
  const int b = u >> sh, e = u & ((1 << sh) - 1);
  const int M = 1 << d.mbits, N = 1 << d.nbits, K = d.K;
  const int32_t* bat = mp + M + N + 2 * K;
  int64_t ao = mp[e >> d.nbits] + bat[b];
  int64_t bo = mp[M + (e & (N - 1))] + bat[(1 << d.nbb) + b];
  for (int i = 0; i < nout; ++i)
    if ((pass >> (nout - 1 - i)) & 1) {
      if (d.a_pp[i]) ao += int64_t(1) << (d.a_pp[i] - 1);
      if (d.b_pp[i]) bo += int64_t(1) << (d.b_pp[i] - 1);
    }
  direct_dot<MODE>(d.A, d.B, ao, bo, K, mp + M + N, mp + M + N + K, d.C, u);
}

constexpr int kDirectW = sizeof(DirectStep) / 4, kTinyW = sizeof(TinyStep) / 4;
constexpr int kDirectLdsWords =
    std::max<int>(kDirectW + 2 * (int)kDirectMaxK, kClusterMaxSteps * kTinyW + kClusterMapWords);

// dst[i] = src[i] for i < n by the workgroup's 256 threads.
__device__ __forceinline__ void copy_words(uint32_t* dst, const uint32_t* __restrict__ src, int n) {
  constexpr int U = 8;
  for (int i0 = threadIdx.x; i0 < n; i0 += 256 * U) {
    uint32_t v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + 256 * u;
      v[u] = i < n ? src[i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + 256 * u;
      if (i < n) dst[i] = v[u];
    }
  }
}

template <int MODE>
__global__ __launch_bounds__(256) void direct_grouped(DirectTable g) {
  __shared__ __align__(16) uint32_t lds[kDirectLdsWords];
  const int bid = blockIdx.x;
  const int j = find_job(g.prefix, g.n, bid);
  const DirectJob job = g.jobs[j];
  if (job.count == 1) {
    // The step's bit maps are read per output; copy them into LDS once.
    const uint32_t* src = reinterpret_cast<const uint32_t*>(g.steps + job.first);
    if (threadIdx.x < kDirectW) lds[threadIdx.x] = src[threadIdx.x];
    __syncthreads();
    const DirectStep& d = *reinterpret_cast<const DirectStep*>(lds);
    int32_t* koa = reinterpret_cast<int32_t*>(lds + kDirectW);
    int32_t* kob = koa + kDirectMaxK;
    const int local = bid - g.prefix[j];
    const int b = local / d.blocks_per_batch;
    const int64_t e = int64_t(local % d.blocks_per_batch) * 256 + threadIdx.x;
    direct_ktab(d, koa, kob);
    __syncthreads();
    if (e < d.M * d.N) direct_out<MODE>(d, b, e, g.nout, g.pass, koa, kob);
    return;
  }
  // A subtree: its steps and maps into LDS, then one height at a time (the
  // steps of a height are independent), the height's outputs dealt round
  // robin over the workgroup; the barrier after a height makes its results
  // visible to the next one.
  const TinyStep* ts = reinterpret_cast<const TinyStep*>(lds);
  int32_t* map = reinterpret_cast<int32_t*>(lds + kClusterMaxSteps * kTinyW);
  {
    // Eight loads in flight per thread before their stores (a loop of
    // load-then-store pays one memory latency per word a thread copies).
    const uint32_t* src = reinterpret_cast<const uint32_t*>(g.tiny + job.first);
    copy_words(lds, src, job.count * kTinyW);
    copy_words(reinterpret_cast<uint32_t*>(map),
               reinterpret_cast<const uint32_t*>(g.maps + job.map_first), job.map_words);
  }
  __syncthreads();
  for (int q = 0; q < job.count;) {
    const int r = ts[q].run_end, total = ts[q].run_total;
    const uint8_t* sel = reinterpret_cast<const uint8_t*>(map + ts[q].sel);
    for (int t = threadIdx.x; t < total; t += 256) {
      const TinyStep& d = ts[sel[t]];  // the step output t belongs to
      tiny_out<MODE>(d, t - d.ooff, map + d.map, g.nout, g.pass);
    }
    __syncthreads();
    q = r;
  }
}

size_t grouped_perm_bound(int n) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  return al(size_t(n) * sizeof(PermParams)) + al((size_t(n) + 1) * sizeof(int32_t));
}

size_t grouped_direct_bound(int n, int64_t map_words) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  return al(size_t(n) * sizeof(DirectStep)) + al(size_t(n) * sizeof(TinyStep)) +
         al(size_t(map_words) * sizeof(int32_t)) + al(size_t(n) * sizeof(DirectJob)) +
         al((size_t(n) + 1) * sizeof(int32_t));
}

size_t grouped_direct_build(const std::vector<DirectStep>& steps,
                            const std::vector<TinyStep>& tiny, const std::vector<int32_t>& maps,
                            const std::vector<DirectJob>& jobs, rn_mode mode,
                            std::vector<char>& table, GroupedLaunch& G) {
  G = GroupedLaunch{};
  G.n = (int)jobs.size();
  G.mode = mode;
  if (jobs.empty()) return 0;
  std::vector<int32_t> prefix(jobs.size() + 1, 0);
  int64_t total = 0;
  for (size_t i = 0; i < jobs.size(); ++i) {
    const DirectJob& jb = jobs[i];
    bool ok = jb.count >= 1 && jb.first >= 0;
    if (ok && jb.count == 1) ok = size_t(jb.first) < steps.size();
    if (ok && jb.count > 1)
      ok = jb.count <= kClusterMaxSteps && size_t(jb.first) + size_t(jb.count) <= tiny.size() &&
           jb.map_first >= 0 && jb.map_words >= 0 && jb.map_words <= kClusterMapWords &&
           size_t(jb.map_first) + size_t(jb.map_words) <= maps.size();
    if (!ok) {
      G.blocks = -1;  // refused at launch
      return 0;
    }
    total += jb.count == 1 ? int64_t(steps[jb.first].blocks_per_batch) << steps[jb.first].nbb : 1;
    prefix[i + 1] = prefix_entry(total);
  }
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  G.blocks = grouped_blocks(total);
  G.params_off = 0;
  G.tiny_off = al(steps.size() * sizeof(DirectStep));
  G.maps_off = G.tiny_off + al(tiny.size() * sizeof(TinyStep));
  G.jobs_off = G.maps_off + al(maps.size() * sizeof(int32_t));
  G.prefix_off = G.jobs_off + al(jobs.size() * sizeof(DirectJob));
  const size_t bytes = G.prefix_off + al(prefix.size() * sizeof(int32_t));
  table.assign(bytes, 0);
  if (!steps.empty()) memcpy(table.data(), steps.data(), steps.size() * sizeof(DirectStep));
  if (!tiny.empty()) memcpy(table.data() + G.tiny_off, tiny.data(), tiny.size() * sizeof(TinyStep));
  if (!maps.empty()) memcpy(table.data() + G.maps_off, maps.data(), maps.size() * sizeof(int32_t));
  memcpy(table.data() + G.jobs_off, jobs.data(), jobs.size() * sizeof(DirectJob));
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
  t.jobs = reinterpret_cast<const DirectJob*>(static_cast<const char*>(table_dev) + G.jobs_off);
  t.tiny = reinterpret_cast<const TinyStep*>(static_cast<const char*>(table_dev) + G.tiny_off);
  t.maps = reinterpret_cast<const int32_t*>(static_cast<const char*>(table_dev) + G.maps_off);
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
    for (int u = 0; u < 4; ++u) v[u] = ld_stream(x + i + 256 * u);  // read once
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
