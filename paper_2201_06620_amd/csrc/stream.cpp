// Streamed block tensordot: operands in host memory, output in HBM.
//
// This is the commutative reduction of Section IV.A on one device: the
// coupled block pairs of an output block are brought in one at a time and
// added into that block, so device memory holds C plus a couple of operand
// blocks (Eq. 2 per block in flight) instead of both whole operands.
//
// Order: output block rows r (A-free block coordinates) outermost, then the
// pairs p, then the output block columns s.  The A block (r, p) is copied
// once and used for every column of the row; the B blocks (p, s) stream.
// Copies run on the handle's copy stream into double-buffered staging, the
// permutes, GEMMs and block additions on the caller's stream; events order
// the two, so copies of later blocks overlap the GEMMs of earlier ones.
// Pair 0 of a block writes C directly; every later pair's product goes to a
// partial buffer that is then added into the block, in ascending pair order.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "rn_internal.hpp"

namespace rn {
namespace {

struct StreamPlan {
  TdPlan td;  // validation, C descriptor, mode
  int es = 16;
  // Block bookkeeping of A and B (block-major storage).
  int64_t blkA = 1, blkB = 1;        // elements per stored block
  int64_t Mb = 1, Nb = 1, Kb = 1;    // GEMM sizes of one block pair
  int mbits = 0, nbits = 0, kbits = 0;
  BitPerm permA, permB;              // stored block -> [Mb x Kb] / [Nb x Kb]
  bool permuteA = false, permuteB = false;
  // Block counts: rows (A-free), columns (B-free), pairs.
  int64_t rows = 1, cols = 1, pairs = 1;
  // Per-axis block bits and the block-index stride of each axis.
  std::vector<int> freeA, freeB;     // axis indices
  int64_t strideA[RN_MAX_RANK], strideB[RN_MAX_RANK];  // block-index strides
  int gbA[RN_MAX_RANK], gbB[RN_MAX_RANK];              // log2 grid per axis
  // Workspace (byte offsets).
  int64_t off_stA[2], off_stB[2], off_pa = -1, off_pa2 = -1, off_pb = -1, off_pb2 = -1;
  int64_t off_part = 0;
  int64_t ws = 0;
  double h2d = 0;
};

int64_t al256(int64_t x) { return (x + 255) & ~int64_t(255); }

rn_status plan_stream(const rn_tensor* A, const rn_tensor* B, int32_t k, const int32_t* axesA,
                      const int32_t* axesB, rn_mode mode, StreamPlan* S) {
  StreamPlan& p = *S;
  rn_status st = plan_tensordot(A, B, k, axesA, axesB, mode, &p.td, false);
  if (st != RN_OK) return st;
  p.es = p.td.es;
  Layout LA, LB;
  if ((st = make_layout(A, "A", &LA)) != RN_OK) return st;
  if ((st = make_layout(B, "B", &LB)) != RN_OK) return st;
  for (int i = 0; i < k; ++i)
    if (LA.cbits[axesA[i]] != LB.cbits[axesB[i]])
      return fail(RN_ERR_UNSUPPORTED,
                  "streamed contraction needs equal grids on paired axes (pair " +
                      std::to_string(i) + ")");
  std::vector<bool> conA(LA.rank, false), conB(LB.rank, false);
  for (int i = 0; i < k; ++i) {
    conA[axesA[i]] = true;
    conB[axesB[i]] = true;
  }
  auto inner = [](const Layout& L, int j) { return L.abits[j] - L.cbits[j]; };
  // Inner bit position of (axis j, bit t) inside one stored block.
  auto ipos = [&](const Layout& L, int j, int t) {
    int pos = t;
    for (int q = j + 1; q < L.rank; ++q) pos += inner(L, q);
    return pos;
  };
  // Block-index strides (row-major over block coordinates).
  auto strides = [](const Layout& L, int64_t* out) {
    int64_t sacc = 1;
    for (int j = L.rank - 1; j >= 0; --j) {
      out[j] = sacc;
      sacc <<= L.cbits[j];
    }
  };
  strides(LA, p.strideA);
  strides(LB, p.strideB);
  for (int j = 0; j < LA.rank; ++j) p.gbA[j] = LA.cbits[j];
  for (int j = 0; j < LB.rank; ++j) p.gbB[j] = LB.cbits[j];
  int ib = 0;
  for (int j = 0; j < LA.rank; ++j) ib += inner(LA, j);
  p.blkA = int64_t(1) << ib;
  ib = 0;
  for (int j = 0; j < LB.rank; ++j) ib += inner(LB, j);
  p.blkB = int64_t(1) << ib;
  // K bits: pair i's inner bits, pair 0 most significant.
  int o = 0;
  BitPerm pa, pb;
  for (int i = k - 1; i >= 0; --i) {
    int e = inner(LA, axesA[i]);
    for (int t = 0; t < e; ++t) {
      pa.src[o] = (int8_t)ipos(LA, axesA[i], t);
      pb.src[o] = (int8_t)ipos(LB, axesB[i], t);
      ++o;
    }
  }
  p.kbits = o;
  int oa = o, ob = o;
  for (int j = LA.rank - 1; j >= 0; --j) {
    if (conA[j]) continue;
    for (int t = 0; t < inner(LA, j); ++t) pa.src[oa++] = (int8_t)ipos(LA, j, t);
  }
  for (int j = LB.rank - 1; j >= 0; --j) {
    if (conB[j]) continue;
    for (int t = 0; t < inner(LB, j); ++t) pb.src[ob++] = (int8_t)ipos(LB, j, t);
  }
  pa.nbits = oa;
  pb.nbits = ob;
  p.mbits = oa - o;
  p.nbits = ob - o;
  p.Mb = int64_t(1) << p.mbits;
  p.Nb = int64_t(1) << p.nbits;
  p.Kb = int64_t(1) << p.kbits;
  p.permA = pa;
  p.permB = pb;
  const bool split_prec = mode == RN_BF16X3;
  p.permuteA = split_prec || !pa.identity();
  p.permuteB = split_prec || !pb.identity();
  p.freeA.clear();
  p.freeB.clear();
  int rb = 0, cb = 0, pbits = 0;
  for (int j = 0; j < LA.rank; ++j)
    if (!conA[j]) {
      p.freeA.push_back(j);
      rb += LA.cbits[j];
    }
  for (int j = 0; j < LB.rank; ++j)
    if (!conB[j]) {
      p.freeB.push_back(j);
      cb += LB.cbits[j];
    }
  for (int i = 0; i < k; ++i) pbits += LA.cbits[axesA[i]];
  p.rows = int64_t(1) << rb;
  p.cols = int64_t(1) << cb;
  p.pairs = int64_t(1) << pbits;
  // Workspace: two staging slots per operand, the permuted blocks, and one
  // partial output block.
  int64_t off = 0;
  for (int q = 0; q < 2; ++q) {
    p.off_stA[q] = off;
    off = al256(off + p.blkA * p.es);
    p.off_stB[q] = off;
    off = al256(off + p.blkB * p.es);
  }
  const int pes = split_prec ? 4 : p.es;
  if (p.permuteA) {
    p.off_pa = off;
    off = al256(off + p.blkA * pes);
    if (split_prec) {
      p.off_pa2 = off;
      off = al256(off + p.blkA * pes);
    }
  }
  if (p.permuteB) {
    p.off_pb = off;
    off = al256(off + p.blkB * pes);
    if (split_prec) {
      p.off_pb2 = off;
      off = al256(off + p.blkB * pes);
    }
  }
  p.off_part = off;
  off = al256(off + (p.pairs > 1 ? p.Mb * p.Nb * p.es : 0));
  p.ws = off;
  p.h2d = double(p.rows) * double(p.pairs) * double(p.blkA * p.es + p.cols * p.blkB * p.es);
  return RN_OK;
}

// Block index of A block (row r, pair q) and B block (pair q, column c).
int64_t a_block(const StreamPlan& p, const int32_t* axesA, int k, int64_t r, int64_t q) {
  int64_t idx = 0;
  for (int f = (int)p.freeA.size() - 1; f >= 0; --f) {
    int j = p.freeA[f];
    idx += (r & ((int64_t(1) << p.gbA[j]) - 1)) * p.strideA[j];
    r >>= p.gbA[j];
  }
  for (int i = k - 1; i >= 0; --i) {
    int j = axesA[i];
    idx += (q & ((int64_t(1) << p.gbA[j]) - 1)) * p.strideA[j];
    q >>= p.gbA[j];
  }
  return idx;
}

int64_t b_block(const StreamPlan& p, const int32_t* axesB, int k, int64_t q, int64_t c) {
  int64_t idx = 0;
  for (int f = (int)p.freeB.size() - 1; f >= 0; --f) {
    int j = p.freeB[f];
    idx += (c & ((int64_t(1) << p.gbB[j]) - 1)) * p.strideB[j];
    c >>= p.gbB[j];
  }
  for (int i = k - 1; i >= 0; --i) {
    int j = axesB[i];
    idx += (q & ((int64_t(1) << p.gbB[j]) - 1)) * p.strideB[j];
    q >>= p.gbB[j];
  }
  return idx;
}

}  // namespace
}  // namespace rn

using namespace rn;

extern "C" {

rn_status rn_block_tensordot_streamed_plan(rn_handle h, const rn_tensor* A, const rn_tensor* B,
                                           int32_t k, const int32_t* axesA,
                                           const int32_t* axesB, rn_mode mode, rn_tensor* C,
                                           size_t* ws_bytes, double* flops, double* h2d_bytes) {
  (void)h;
  StreamPlan S;
  rn_status st = plan_stream(A, B, k, axesA, axesB, mode, &S);
  if (st != RN_OK) return st;
  if (C) {
    C->rank = S.td.crank;
    C->dtype = mode == RN_FP64 ? RN_C128 : RN_C64;
    for (int j = 0; j < RN_MAX_RANK; ++j) {
      C->dims[j] = j < S.td.crank ? S.td.cdims[j] : 0;
      C->grid[j] = j < S.td.crank ? S.td.cgrid[j] : 0;
    }
  }
  if (ws_bytes) *ws_bytes = (size_t)S.ws;
  if (flops) *flops = S.td.flops;
  if (h2d_bytes) *h2d_bytes = S.h2d;
  return RN_OK;
}

rn_status rn_block_tensordot_streamed(rn_handle h, const rn_tensor* A, const rn_tensor* B,
                                      int32_t k, const int32_t* axesA, const int32_t* axesB,
                                      rn_tensor* C, rn_mode mode, void* ws, size_t ws_bytes,
                                      void* stream) {
  if (!h) return fail(RN_ERR_INVALID, "null handle");
  StreamPlan S;
  rn_status st = plan_stream(A, B, k, axesA, axesB, mode, &S);
  if (st != RN_OK) return st;
  if ((st = check_c(S.td, C)) != RN_OK) return st;
  if (!A->data || !B->data || !C->data) return fail(RN_ERR_INVALID, "null tensor data");
  if ((int64_t)ws_bytes < S.ws || !ws)
    return fail(RN_ERR_WORKSPACE,
                "workspace smaller than planned (" + std::to_string(S.ws) + " bytes needed)");
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return fail(RN_ERR_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
  if (!h->copy_stream) {
    if ((e = hipStreamCreateWithFlags(&h->copy_stream, hipStreamNonBlocking)) != hipSuccess)
      return fail(RN_ERR_HIP, std::string("copy stream: ") + hipGetErrorString(e));
    for (hipEvent_t& ev : h->copy_ev)
      if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
        return fail(RN_ERR_HIP, std::string("copy events: ") + hipGetErrorString(e));
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipStream_t cs = h->copy_stream;
  hipEvent_t* a_ready = h->copy_ev;      // [2]
  hipEvent_t* a_free = h->copy_ev + 2;   // [2]
  hipEvent_t* b_ready = h->copy_ev + 4;  // [2]
  hipEvent_t* b_free = h->copy_ev + 6;   // [2]
  hipEvent_t start = h->copy_ev[8];
  char* w = static_cast<char*>(ws);
  const bool split_prec = mode == RN_BF16X3;
  const char* ha = static_cast<const char*>(A->data);
  const char* hb = static_cast<const char*>(B->data);
  char* cdev = static_cast<char*>(C->data);
  const int tile = tuned_tile(h, mode, S.mbits, S.nbits, S.kbits);
  Profiler* prof = &h->prof;
  auto hip_err = [](hipError_t err, const char* what) {
    return fail(RN_ERR_HIP, std::string(what) + ": " + hipGetErrorString(err));
  };
  // Event record / wait, stopping at the first failure.
  auto rec = [&](hipEvent_t ev, hipStream_t st) { if (e == hipSuccess) e = hipEventRecord(ev, st); };
  auto wait = [&](hipStream_t st, hipEvent_t ev) {
    if (e == hipSuccess) e = hipStreamWaitEvent(st, ev, 0);
  };
  // Copies start after whatever the caller queued before this call.
  if ((e = hipEventRecord(start, s)) != hipSuccess) return hip_err(e, "event record");
  if ((e = hipStreamWaitEvent(cs, start, 0)) != hipSuccess) return hip_err(e, "stream wait");
  // The first use of each slot must not wait on a stale record: mark all
  // free on the caller's stream now.
  for (int q = 0; q < 2; ++q) {
    rec(a_free[q], s);
    rec(b_free[q], s);
  }
  if (e != hipSuccess) return hip_err(e, "event record");
  int64_t na = 0, nb = 0;  // A blocks and B blocks brought in so far
  for (int64_t r = 0; r < S.rows; ++r) {
    for (int64_t q = 0; q < S.pairs; ++q) {
      const int sa = (int)(na & 1);
      ++na;
      char* stA = w + S.off_stA[sa];
      const int64_t ai = a_block(S, axesA, k, r, q);
      if ((e = hipStreamWaitEvent(cs, a_free[sa], 0)) != hipSuccess) return hip_err(e, "wait");
      if ((e = hipMemcpyAsync(stA, ha + ai * S.blkA * S.es, S.blkA * S.es,
                              hipMemcpyHostToDevice, cs)) != hipSuccess)
        return hip_err(e, "copy A block");
      rec(a_ready[sa], cs);
      wait(s, a_ready[sa]);
      if (e != hipSuccess) return hip_err(e, "copy event");
      const void* am = stA;
      const void* am2 = nullptr;
      if (S.permuteA) {
        PermLaunch L;
        L.in = stA;
        L.out = w + S.off_pa;
        L.out2 = split_prec ? w + S.off_pa2 : nullptr;
        L.perm = S.permA;
        L.in_es = S.es;
        L.kind = split_prec ? 1 : 0;
        int ev = prof->begin(0, s);
        e = launch_permute(L, s);
        prof->end(ev, s);
        if (e != hipSuccess) return hip_err(e, "permute A block");
        am = L.out;
        am2 = L.out2;
        rec(a_free[sa], s);
      }
      for (int64_t c = 0; c < S.cols; ++c) {
        const int sb = (int)(nb & 1);
        ++nb;
        char* stB = w + S.off_stB[sb];
        const int64_t bi = b_block(S, axesB, k, q, c);
        if ((e = hipStreamWaitEvent(cs, b_free[sb], 0)) != hipSuccess) return hip_err(e, "wait");
        if ((e = hipMemcpyAsync(stB, hb + bi * S.blkB * S.es, S.blkB * S.es,
                                hipMemcpyHostToDevice, cs)) != hipSuccess)
          return hip_err(e, "copy B block");
        rec(b_ready[sb], cs);
        wait(s, b_ready[sb]);
        if (e != hipSuccess) return hip_err(e, "copy event");
        const void* bm = stB;
        const void* bm2 = nullptr;
        if (S.permuteB) {
          PermLaunch L;
          L.in = stB;
          L.out = w + S.off_pb;
          L.out2 = split_prec ? w + S.off_pb2 : nullptr;
          L.perm = S.permB;
          L.in_es = S.es;
          L.kind = split_prec ? 1 : 0;
          int ev = prof->begin(0, s);
          e = launch_permute(L, s);
          prof->end(ev, s);
          if (e != hipSuccess) return hip_err(e, "permute B block");
          bm = L.out;
          bm2 = L.out2;
          rec(b_free[sb], s);
        }
        // Output block (r, c): C's block index is row-major over
        // [A-free block coords | B-free block coords], i.e. r * cols + c.
        char* cblk = cdev + (r * S.cols + c) * S.Mb * S.Nb * S.es;
        GemmLaunch g;
        g.mode = mode;
        g.A = am;
        g.B = bm;
        g.A2 = am2;
        g.B2 = bm2;
        g.C = q == 0 ? cblk : w + S.off_part;
        g.M = S.Mb;
        g.N = S.Nb;
        g.K = S.Kb;
        g.lda = S.Kb;
        g.ldb = S.Kb;
        g.crow.lo = S.Nb;
        g.ccol.lo = 1;
        g.tile = tile;
        if ((e = launch_gemm(g, s, prof)) != hipSuccess) return hip_err(e, "complex GEMM");
        if (!S.permuteB) rec(b_free[sb], s);
        if (e != hipSuccess) return hip_err(e, "event record");
        if (q > 0) {
          int ev = prof->begin(2, s);
          e = launch_add_into(cblk, w + S.off_part, S.Mb * S.Nb, S.es, s);
          prof->end(ev, s);
          if (e != hipSuccess) return hip_err(e, "block add");
        }
      }
      if (!S.permuteA) rec(a_free[sa], s);
      if (e != hipSuccess) return hip_err(e, "event record");
    }
  }
  return RN_OK;
}

}  // extern "C"
