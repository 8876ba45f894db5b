// C ABI entry points: argument checks, planning, and kernel enqueue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "rn_internal.hpp"

namespace rn {
const std::string& last_error();

static rn_status hip_fail(hipError_t e, const char* what) {
  return fail(RN_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

static char* ws_at(void* ws, int64_t off) { return static_cast<char*>(ws) + off; }

// Enqueue one planned block tensordot: permutes (unless the stored layout
// already is the GEMM layout), then the GEMM with its K loop over pairs.
int Profiler::begin(int cls, hipStream_t s) {
  if (!on) return -1;
  Rec r;
  r.cls = cls;
  for (hipEvent_t* e : {&r.a, &r.b}) {
    if (!pool.empty()) {
      *e = pool.back();
      pool.pop_back();
    } else if (hipEventCreate(e) != hipSuccess) {
      return -1;
    }
  }
  hipEventRecord(r.a, s);
  recs.push_back(r);
  return (int)recs.size() - 1;
}

void Profiler::end(int idx, hipStream_t s) {
  if (idx >= 0 && idx < (int)recs.size()) hipEventRecord(recs[idx].b, s);
}

rn_status enqueue_tensordot(const TdPlan& P, const rn_tensor* A, const rn_tensor* B,
                            const rn_tensor* C, void* ws, hipStream_t s, Profiler* prof,
                            int tile) {
  const bool split_prec = (P.mode == RN_BF16X3);
  // Split BF16 on a plan sized for it: the planar Gauss tile when tuned to
  // it, or by default for large outputs; else the packed form.
  bool planar = false;
  if (split_prec && P.planar_ok) {
    if (gemm_tile_planar(P.mode, tile)) {
      planar = true;
    } else if (!gemm_tile_valid(P.mode, tile, P.M, P.N)) {
      const int t = gemm_planar_default(P.mode, P.M, P.N, P.K);
      if (t >= 0) {
        planar = true;
        tile = t;
      }
    }
  }
  if (!planar && gemm_tile_planar(P.mode, tile)) tile = -1;  // plan without planar room
  // Packed split BF16 for a direct-to-LDS tile, on a plan made for the
  // single block tensordot: row-interleaved hi and lo (permute kind 3, one
  // 128-byte line per 16 k of a row, measured 8-9 % faster on the rank-28
  // pair than two arrays), in the room the plan keeps for both arrays.
  const int rt = planar || gemm_tile_valid(P.mode, tile, P.M, P.N)
                     ? tile
                     : gemm_default_tile(P.mode, P.M, P.N, P.K);
  const bool ilv = split_prec && P.planar_ok && !planar && P.K % 16 == 0 &&
                   gemm_tile_interleaved(P.mode, rt);
  const int pkind = planar ? 2 : ilv ? 3 : split_prec ? 1 : 0;
  const void* am = A->data;
  const void* bm = B->data;
  const void* am2 = nullptr;
  const void* bm2 = nullptr;
  hipError_t e;
  if (P.permuteA) {
    PermLaunch L;
    L.in = A->data;
    L.out = ws_at(ws, P.off_a);
    L.out2 = split_prec && !planar && !ilv ? ws_at(ws, P.off_a2) : nullptr;
    L.perm = P.permA;
    L.in_es = P.es;
    L.kind = pkind;
    L.gw = std::min<int64_t>(P.K, 16);
    int ev = prof ? prof->begin(0, s) : -1;
    e = launch_permute(L, s);
    if (prof) prof->end(ev, s);
    if (e != hipSuccess) return hip_fail(e, "permute A");
    am = L.out;
    am2 = ilv ? static_cast<const uint32_t*>(am) + 16 : L.out2;
  }
  if (P.permuteB) {
    PermLaunch L;
    L.in = B->data;
    L.out = ws_at(ws, P.off_b);
    L.out2 = split_prec && !planar && !ilv ? ws_at(ws, P.off_b2) : nullptr;
    L.perm = P.permB;
    L.in_es = P.es;
    L.kind = pkind;
    L.gw = std::min<int64_t>(P.K, 16);
    int ev = prof ? prof->begin(0, s) : -1;
    e = launch_permute(L, s);
    if (prof) prof->end(ev, s);
    if (e != hipSuccess) return hip_fail(e, "permute B");
    bm = L.out;
    bm2 = ilv ? static_cast<const uint32_t*>(bm) + 16 : L.out2;
  }
  GemmLaunch g;
  g.mode = P.mode;
  g.A = am;
  g.B = bm;
  g.A2 = am2;
  g.B2 = bm2;
  g.C = C->data;
  g.M = P.M;
  g.N = P.N;
  g.K = P.K;
  g.lda = ilv ? 2 * P.K : P.K;
  g.ldb = ilv ? 2 * P.K : P.K;
  g.crow = P.crow;
  g.ccol = P.ccol;
  g.splitk = P.splitk;
  g.partial = P.splitk > 1 ? ws_at(ws, P.off_part) : nullptr;
  g.tile = tile;
  g.planar = planar;
  g.interleaved = ilv;
  if (planar && P.splitk > 1 && !gemm_tile_splits(P.mode, tile)) g.splitk = 1;
  if ((e = launch_gemm(g, s, prof)) != hipSuccess) return hip_fail(e, "complex GEMM");
  return RN_OK;
}

static rn_status bind_device(rn_handle h) {
  if (!h) return fail(RN_ERR_INVALID, "null handle");
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  return RN_OK;
}

static void fill_c(const TdPlan& P, int dtype, rn_tensor* C) {
  C->rank = P.crank;
  C->dtype = dtype;
  for (int j = 0; j < RN_MAX_RANK; ++j) {
    C->dims[j] = j < P.crank ? P.cdims[j] : 0;
    C->grid[j] = j < P.crank ? P.cgrid[j] : 0;
  }
}

}  // namespace rn

using namespace rn;

extern "C" {

rn_status rn_create(rn_handle* h, int device) {
  if (!h) return fail(RN_ERR_INVALID, "null handle pointer");
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= n) return fail(RN_ERR_INVALID, "device index out of range");
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  rn_status st = noalloc_init(device);
  if (st != RN_OK) return st;
  rn_ctx* c = new rn_ctx();
  c->device = device;
  const char* g = getenv("RN_GRAPHS");
  c->graphs_enabled = !(g && g[0] == '0');
  const char* tp = getenv("RN_TUNE_CACHE");
  if (tp && tp[0]) {
    c->tune_path = tp;
    FILE* f = fopen(tp, "r");
    if (f) {
      fclose(f);
      rn_tune_load(c, tp);
    }
  }
  e = hipMalloc(&c->red_scratch, 4096 * sizeof(double));
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "hipMalloc (reduction scratch)");
  }
  *h = c;
  return RN_OK;
}

rn_status rn_destroy(rn_handle h) {
  if (!h) return RN_OK;
  hipSetDevice(h->device);
  if (h->red_scratch) hipFree(h->red_scratch);
  for (auto& r : h->prof.recs) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  for (hipEvent_t e : h->prof.pool) hipEventDestroy(e);
  if (!h->graphs.empty()) hipDeviceSynchronize();  // a replay may still run
  for (auto& g : h->graphs) {
    hipGraphExecDestroy(g.exec);
    if (g.pinned) hipHostFree(g.pinned);
    if (g.table) hipFree(g.table);
  }
  if (h->pinned_done) {
    hipEventSynchronize(h->pinned_done);
    hipEventDestroy(h->pinned_done);
  }
  if (h->pinned) hipHostFree(h->pinned);
  if (h->copy_stream) {
    hipStreamSynchronize(h->copy_stream);
    hipStreamDestroy(h->copy_stream);
  }
  for (hipEvent_t e : h->copy_ev)
    if (e) hipEventDestroy(e);
  for (int i = 0; i < 3; ++i) {
    if (h->aux_streams[i]) {
      hipStreamSynchronize(h->aux_streams[i]);
      hipStreamDestroy(h->aux_streams[i]);
    }
    if (h->aux_join[i]) hipEventDestroy(h->aux_join[i]);
  }
  if (h->aux_fork) hipEventDestroy(h->aux_fork);
  delete h;
  return RN_OK;
}

const char* rn_status_str(rn_status s) {
  switch (s) {
    case RN_OK: return "ok";
    case RN_ERR_INVALID: return "invalid argument";
    case RN_ERR_SHAPE: return "shape mismatch";
    case RN_ERR_GRID: return "grid mismatch";
    case RN_ERR_WORKSPACE: return "workspace too small";
    case RN_ERR_OOM: return "exceeds memory budget";
    case RN_ERR_HIP: return "HIP runtime error";
    case RN_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* rn_last_error(void) { return last_error().c_str(); }

rn_status rn_block_tensordot_plan(rn_handle h, const rn_tensor* A, const rn_tensor* B, int32_t k,
                                  const int32_t* axesA, const int32_t* axesB, rn_mode mode,
                                  rn_tensor* C, size_t* ws_bytes, double* flops) {
  TdPlan P;
  rn_status st =
      plan_tensordot(A, B, k, axesA, axesB, mode, &P, true, h ? &h->split : nullptr, true);
  if (st != RN_OK) return st;
  if (C) fill_c(P, A->dtype, C);
  if (ws_bytes) *ws_bytes = P.ws_bytes;
  if (flops) *flops = P.flops;
  return RN_OK;
}

rn_status rn_block_tensordot(rn_handle h, const rn_tensor* A, const rn_tensor* B, int32_t k,
                             const int32_t* axesA, const int32_t* axesB, rn_tensor* C,
                             rn_mode mode, void* ws, size_t ws_bytes, void* stream) {
  if (!h) return fail(RN_ERR_INVALID, "null handle");
  TdPlan P;
  rn_status st;
  if ((st = plan_tensordot(A, B, k, axesA, axesB, mode, &P, true, &h->split, true)) != RN_OK)
    return st;
  if ((st = check_c(P, C)) != RN_OK) return st;
  if (!A->data || !B->data) return fail(RN_ERR_INVALID, "null operand data");
  if (C->data == A->data || C->data == B->data) return fail(RN_ERR_INVALID, "C aliases an operand");
  if (ws_bytes < P.ws_bytes || (P.ws_bytes > 0 && !ws))
    return fail(RN_ERR_WORKSPACE, "workspace smaller than planned (" +
                                      std::to_string(P.ws_bytes) + " bytes needed)");
  if ((st = bind_device(h)) != RN_OK) return st;
  return enqueue_tensordot(P, A, B, C, ws, static_cast<hipStream_t>(stream), &h->prof,
                           tuned_tile(h, P.mode, P.mbits, P.nbits, P.kbits));
}

rn_status rn_block_pairs(rn_handle h, const rn_tensor* A, const rn_tensor* B, int32_t k,
                         const int32_t* axesA, const int32_t* axesB, int64_t cblock,
                         int64_t* pairs, int64_t cap, int64_t* npairs) {
  (void)h;
  TdPlan P;
  rn_status st = plan_tensordot(A, B, k, axesA, axesB, RN_FP64, &P);
  if (st == RN_ERR_INVALID && A && B && A->dtype == RN_C64 && B->dtype == RN_C64)
    st = plan_tensordot(A, B, k, axesA, axesB, RN_FP32_4M, &P);
  if (st != RN_OK) return st;
  int64_t nblk = 1;
  for (int j = 0; j < P.crank; ++j) nblk *= P.cgrid[j];
  if (cblock < 0 || cblock >= nblk) return fail(RN_ERR_INVALID, "C block index out of range");
  int64_t np = int64_t(1) << P.pairbits;
  if (npairs) *npairs = np;
  if (!pairs) return RN_OK;
  // Block coordinates of this C block (row-major over C's grid).
  int64_t cb[2 * RN_MAX_RANK];
  int64_t rest = cblock;
  for (int j = P.crank - 1; j >= 0; --j) {
    cb[j] = rest % P.cgrid[j];
    rest /= P.cgrid[j];
  }
  bool ca[RN_MAX_RANK] = {false}, cbm[RN_MAX_RANK] = {false};
  for (int i = 0; i < k; ++i) {
    ca[axesA[i]] = true;
    cbm[axesB[i]] = true;
  }
  int nfa = 0;
  for (int j = 0; j < A->rank; ++j) nfa += !ca[j];
  for (int64_t p = 0; p < np && p < cap; ++p) {
    // Refined contracted block coordinates of pair p, row-major over pairs.
    int64_t pc[RN_MAX_RANK], r = p;
    for (int i = k - 1; i >= 0; --i) {
      int64_t g = int64_t(1) << P.pair_cbits[i];
      pc[i] = r % g;
      r /= g;
    }
    int64_t coordA[RN_MAX_RANK], coordB[RN_MAX_RANK];
    int fi = 0;
    for (int j = 0; j < A->rank; ++j)
      if (!ca[j]) coordA[j] = cb[fi++];
    fi = nfa;
    for (int j = 0; j < B->rank; ++j)
      if (!cbm[j]) coordB[j] = cb[fi++];
    for (int i = 0; i < k; ++i) {
      // A refined coordinate covers 2^(refined - stored) refined blocks per
      // stored block.
      int ga = 0, gb = 0;
      for (int64_t v = A->grid[axesA[i]]; v > 1; v >>= 1) ++ga;
      for (int64_t v = B->grid[axesB[i]]; v > 1; v >>= 1) ++gb;
      coordA[axesA[i]] = pc[i] >> (P.pair_cbits[i] - ga);
      coordB[axesB[i]] = pc[i] >> (P.pair_cbits[i] - gb);
    }
    int64_t la = 0, lb = 0;
    for (int j = 0; j < A->rank; ++j) la = la * A->grid[j] + coordA[j];
    for (int j = 0; j < B->rank; ++j) lb = lb * B->grid[j] + coordB[j];
    pairs[2 * p] = la;
    pairs[2 * p + 1] = lb;
  }
  return RN_OK;
}

rn_status rn_block_footprint(const rn_tensor* A, const rn_tensor* B, int32_t k,
                             const int32_t* axesA, const int32_t* axesB, double* eq1_elems,
                             double* eq2_elems) {
  TdPlan P;
  rn_mode mode = (A && A->dtype == RN_C128) ? RN_FP64 : RN_FP32_4M;
  rn_status st = plan_tensordot(A, B, k, axesA, axesB, mode, &P);
  if (st != RN_OK) return st;
  double mb = double(int64_t(1) << P.Mi), nb = double(int64_t(1) << P.Ni);
  double kb = double(int64_t(1) << (P.kbits - P.pairbits));
  double bk = double(int64_t(1) << P.pairbits);
  if (eq1_elems) *eq1_elems = bk * kb * (mb + nb) + mb * nb;
  if (eq2_elems) *eq2_elems = kb * (mb + nb) + mb * nb;
  return RN_OK;
}

rn_status rn_norm2(rn_handle h, const rn_tensor* T, double* out_dev, void* stream) {
  rn_status st = bind_device(h);
  if (st != RN_OK) return st;
  Layout L;
  if ((st = make_layout(T, "T", &L)) != RN_OK) return st;
  if (!T->data || !out_dev) return fail(RN_ERR_INVALID, "null pointer");
  if (T->dtype != RN_C64 && T->dtype != RN_C128) return fail(RN_ERR_INVALID, "bad dtype");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int ev = h->prof.begin(3, s);
  hipError_t e = launch_norm2(T->data, int64_t(1) << L.total, T->dtype, out_dev,
                              static_cast<double*>(h->red_scratch), s);
  h->prof.end(ev, s);
  return e == hipSuccess ? RN_OK : hip_fail(e, "norm2");
}

rn_status rn_sum_c128(rn_handle h, int64_t n, const double* vals_dev, double* out_dev,
                      void* stream) {
  rn_status st = bind_device(h);
  if (st != RN_OK) return st;
  if (n < 0 || n > (int64_t(1) << 20)) return fail(RN_ERR_INVALID, "n out of range");
  if ((n > 0 && !vals_dev) || !out_dev) return fail(RN_ERR_INVALID, "null pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int ev = h->prof.begin(3, s);
  hipError_t e = launch_sum_c128(vals_dev, n, out_dev, s);
  h->prof.end(ev, s);
  return e == hipSuccess ? RN_OK : hip_fail(e, "sum");
}

rn_status rn_set_option(rn_handle h, rn_option opt, int64_t value) {
  if (!h) return fail(RN_ERR_INVALID, "null handle");
  switch (opt) {
    case RN_OPT_GRAPHS: h->graphs_enabled = value != 0; return RN_OK;
    case RN_OPT_PAIR_SPLIT_THRESHOLD:
      if (value < 0) return fail(RN_ERR_INVALID, "threshold must be >= 0");
      h->split.pair_threshold = value;
      return RN_OK;
    case RN_OPT_SPLIT_FOOTPRINT:
      if (value < 0) return fail(RN_ERR_INVALID, "footprint must be >= 0");
      h->split.footprint = value;
      return RN_OK;
    case RN_OPT_SLICE_SUM:
      if (value != 0 && value != 1) return fail(RN_ERR_INVALID, "slice sum mode is 0 or 1");
      h->net.slice_sum = value != 0;
      return RN_OK;
    case RN_OPT_BATCHED_SLICE_BITS:
      if (value < 0) return fail(RN_ERR_INVALID, "batched slice bits must be >= 0");
      h->net.batch_bits = (int)std::min<int64_t>(value, 64);
      return RN_OK;
    case RN_OPT_NETWORK_FOOTPRINT:
      if (value < 0) return fail(RN_ERR_INVALID, "footprint must be >= 0");
      h->net.footprint = value;
      return RN_OK;
  }
  return fail(RN_ERR_INVALID, "unknown option");
}

rn_status rn_get_option(rn_handle h, rn_option opt, int64_t* value) {
  if (!h || !value) return fail(RN_ERR_INVALID, "null argument");
  switch (opt) {
    case RN_OPT_GRAPHS: *value = h->graphs_enabled ? 1 : 0; return RN_OK;
    case RN_OPT_PAIR_SPLIT_THRESHOLD: *value = h->split.pair_threshold; return RN_OK;
    case RN_OPT_SPLIT_FOOTPRINT: *value = h->split.footprint; return RN_OK;
    case RN_OPT_SLICE_SUM: *value = h->net.slice_sum ? 1 : 0; return RN_OK;
    case RN_OPT_BATCHED_SLICE_BITS: *value = h->net.batch_bits; return RN_OK;
    case RN_OPT_NETWORK_FOOTPRINT: *value = h->net.footprint; return RN_OK;
  }
  return fail(RN_ERR_INVALID, "unknown option");
}

rn_status rn_profile_enable(rn_handle h, int on) {
  if (!h) return fail(RN_ERR_INVALID, "null handle");
  h->prof.on = on != 0;
  return RN_OK;
}

rn_status rn_profile_read(rn_handle h, double ms[4], int64_t count[4]) {
  if (!h || !ms || !count) return fail(RN_ERR_INVALID, "null pointer");
  rn_status st = bind_device(h);
  if (st != RN_OK) return st;
  for (int c = 0; c < 4; ++c) {
    ms[c] = 0.0;
    count[c] = 0;
  }
  for (auto& r : h->prof.recs) {
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float t = 0.f;
    e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    ms[r.cls] += t;
    count[r.cls] += 1;
    h->prof.pool.push_back(r.a);
    h->prof.pool.push_back(r.b);
  }
  h->prof.recs.clear();
  return RN_OK;
}
}  // extern "C"
