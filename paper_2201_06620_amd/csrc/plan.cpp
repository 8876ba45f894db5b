// Planner of one block tensordot (host, integer work only).
//
// Follows the four steps of block tensor contraction (Section II.C): the
// output blocks are indexed by the free-axis block coordinates, the coupled
// pairs by the contracted block coordinates on the refined grid, and each
// pair's local contraction plus the sum over pairs becomes one complex GEMM
// whose K index runs over (pair, element-within-pair).  Because every dim
// and grid count is a power of two, the block-major layouts of A, B and C
// are bit permutations of dense row-major layouts; the planner derives
//   * the bit permutation taking A's stored layout to a row-major
//     M x K matrix and B's to a row-major N x K matrix, and
//   * the two-level maps taking GEMM (row, col) to C's block-major offset.
#include <algorithm>
#include <cstring>

#include "rn_internal.hpp"

namespace rn {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }
const std::string& last_error() { return g_err; }

rn_status fail(rn_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

static int log2_exact(int64_t v) {
  if (v < 1 || (v & (v - 1))) return -1;
  int r = 0;
  while ((int64_t(1) << r) < v) ++r;
  return r;
}

int Layout::phys_pos(int axis, int t) const {
  int inner_total = 0;
  for (int j = 0; j < rank; ++j) inner_total += abits[j] - cbits[j];
  int e = abits[axis] - cbits[axis];
  int pos = 0;
  if (t < e) {
    for (int j = axis + 1; j < rank; ++j) pos += abits[j] - cbits[j];
    return pos + t;
  }
  pos = inner_total;
  for (int j = axis + 1; j < rank; ++j) pos += cbits[j];
  return pos + (t - e);
}

rn_status make_layout(const rn_tensor* T, const char* name, Layout* L) {
  if (!T) return fail(RN_ERR_INVALID, std::string(name) + ": null descriptor");
  if (T->rank < 0 || T->rank > RN_MAX_RANK)
    return fail(RN_ERR_INVALID, std::string(name) + ": rank out of range");
  L->rank = T->rank;
  L->total = 0;
  for (int j = 0; j < T->rank; ++j) {
    int a = log2_exact(T->dims[j]);
    int g = log2_exact(T->grid[j]);
    if (T->dims[j] < 1 || T->grid[j] < 1)
      return fail(RN_ERR_SHAPE, std::string(name) + ": dims and grid must be >= 1");
    if (a < 0)
      return fail(RN_ERR_UNSUPPORTED, std::string(name) + ": dims must be powers of two");
    if (g < 0)
      return fail(RN_ERR_UNSUPPORTED, std::string(name) + ": grid counts must be powers of two");
    if (g > a) return fail(RN_ERR_GRID, std::string(name) + ": grid count exceeds dim");
    L->abits[j] = a;
    L->cbits[j] = g;
    L->total += a;
  }
  if (L->total > 40)
    return fail(RN_ERR_UNSUPPORTED, std::string(name) + ": more than 2^40 elements");
  return RN_OK;
}

bool BitPerm::identity() const {
  for (int o = 0; o < nbits; ++o)
    if (src[o] != o) return false;
  return true;
}

static int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

rn_status plan_tensordot(const rn_tensor* A, const rn_tensor* B, int32_t k,
                         const int32_t* axesA, const int32_t* axesB, rn_mode mode,
                         TdPlan* P, bool allow_splitk, const SplitPolicy* policy,
                         bool planar_ok) {
  Layout LA, LB;
  rn_status st;
  if ((st = make_layout(A, "A", &LA)) != RN_OK) return st;
  if ((st = make_layout(B, "B", &LB)) != RN_OK) return st;
  if (mode < RN_FP64 || mode > RN_BF16X3) return fail(RN_ERR_INVALID, "unknown mode");
  int want = (mode == RN_FP64) ? RN_C128 : RN_C64;
  if (A->dtype != want || B->dtype != want)
    return fail(RN_ERR_INVALID, mode == RN_FP64 ? "RN_FP64 needs RN_C128 operands"
                                                 : "this mode needs RN_C64 operands");
  if (k < 0 || k > A->rank || k > B->rank) return fail(RN_ERR_INVALID, "k out of range");
  if (k > 0 && (!axesA || !axesB)) return fail(RN_ERR_INVALID, "null axes");
  bool ca[RN_MAX_RANK] = {false}, cb[RN_MAX_RANK] = {false};
  for (int i = 0; i < k; ++i) {
    int a = axesA[i], b = axesB[i];
    if (a < 0 || a >= A->rank || b < 0 || b >= B->rank)
      return fail(RN_ERR_INVALID, "axis out of range");
    if (ca[a] || cb[b]) return fail(RN_ERR_INVALID, "repeated axis");
    ca[a] = cb[b] = true;
    if (A->dims[a] != B->dims[b]) return fail(RN_ERR_SHAPE, "paired dims differ");
  }
  TdPlan p;
  p.mode = mode;
  p.es = (mode == RN_FP64) ? 16 : 8;
  p.k = k;
  std::vector<int> fa, fb;
  for (int j = 0; j < A->rank; ++j)
    if (!ca[j]) fa.push_back(j);
  for (int j = 0; j < B->rank; ++j)
    if (!cb[j]) fb.push_back(j);

  // Common refinement of the contracted pairs: lcm of two powers of two.
  for (int i = 0; i < k; ++i) {
    p.axA[i] = axesA[i];
    p.axB[i] = axesB[i];
    p.pair_cbits[i] = std::max(LA.cbits[axesA[i]], LB.cbits[axesB[i]]);
  }

  // K bits, least significant first: inner bits of pair k-1 .. pair 0, then
  // block bits of pair k-1 .. pair 0 (K = [pair | element], both row-major
  // in pairing order).
  std::vector<int> kA, kB;
  for (int i = k - 1; i >= 0; --i) {
    int a = LA.abits[axesA[i]], inner = a - p.pair_cbits[i];
    for (int t = 0; t < inner; ++t) {
      kA.push_back(LA.phys_pos(axesA[i], t));
      kB.push_back(LB.phys_pos(axesB[i], t));
    }
  }
  p.pairbits = 0;
  for (int i = k - 1; i >= 0; --i) {
    int a = LA.abits[axesA[i]], inner = a - p.pair_cbits[i];
    for (int t = inner; t < a; ++t) {
      kA.push_back(LA.phys_pos(axesA[i], t));
      kB.push_back(LB.phys_pos(axesB[i], t));
      ++p.pairbits;
    }
  }
  // M bits (A free axes) and N bits (B free axes): inner bits, then block
  // bits, each in reverse axis order -- the restriction of C's block-major
  // layout to that operand's free axes.
  auto free_bits = [](const Layout& L, const std::vector<int>& fr, std::vector<int>& out,
                      int& inner_cnt, int& block_cnt) {
    inner_cnt = block_cnt = 0;
    for (int q = (int)fr.size() - 1; q >= 0; --q) {
      int j = fr[q], e = L.abits[j] - L.cbits[j];
      for (int t = 0; t < e; ++t) out.push_back(L.phys_pos(j, t));
      inner_cnt += e;
    }
    for (int q = (int)fr.size() - 1; q >= 0; --q) {
      int j = fr[q], e = L.abits[j] - L.cbits[j];
      for (int t = e; t < L.abits[j]; ++t) out.push_back(L.phys_pos(j, t));
      block_cnt += L.cbits[j];
    }
  };
  std::vector<int> mA, nB;
  free_bits(LA, fa, mA, p.Mi, p.Mb);
  free_bits(LB, fb, nB, p.Ni, p.Nb);
  p.kbits = (int)kA.size();
  p.mbits = (int)mA.size();
  p.nbits = (int)nB.size();
  if (p.mbits + p.nbits > 40) return fail(RN_ERR_UNSUPPORTED, "output over 2^40 elements");
  p.M = int64_t(1) << p.mbits;
  p.N = int64_t(1) << p.nbits;
  p.K = int64_t(1) << p.kbits;

  p.permA.nbits = p.kbits + p.mbits;
  for (int o = 0; o < p.kbits; ++o) p.permA.src[o] = (int8_t)kA[o];
  for (int o = 0; o < p.mbits; ++o) p.permA.src[p.kbits + o] = (int8_t)mA[o];
  p.permB.nbits = p.kbits + p.nbits;
  for (int o = 0; o < p.kbits; ++o) p.permB.src[o] = (int8_t)kB[o];
  for (int o = 0; o < p.nbits; ++o) p.permB.src[p.kbits + o] = (int8_t)nB[o];

  // C block-major bits, most significant first: [Mb | Nb | Mi | Ni].
  p.crow.shift = p.Mi;
  p.crow.hi = int64_t(1) << (p.Nb + p.Mi + p.Ni);
  p.crow.lo = int64_t(1) << p.Ni;
  p.ccol.shift = p.Ni;
  p.ccol.hi = int64_t(1) << (p.Mi + p.Ni);
  p.ccol.lo = 1;

  p.crank = (int)(fa.size() + fb.size());
  for (size_t q = 0; q < fa.size(); ++q) {
    p.cdims[q] = A->dims[fa[q]];
    p.cgrid[q] = A->grid[fa[q]];
  }
  for (size_t q = 0; q < fb.size(); ++q) {
    p.cdims[fa.size() + q] = B->dims[fb[q]];
    p.cgrid[fa.size() + q] = B->grid[fb[q]];
  }

  // Workspace.
  bool split_prec = (mode == RN_BF16X3);
  p.permuteA = split_prec || !p.permA.identity();
  p.permuteB = split_prec || !p.permB.identity();
  int64_t off = 0;
  // Split BF16: hi and lo arrays of 4 bytes per complex (packed pairs); when
  // the planar Gauss form may run, one region of 12 bytes per complex holds
  // either its six planes or the two packed arrays.
  p.planar_ok = split_prec && planar_ok;
  int64_t abytes = p.M * p.K * (split_prec ? 4 : p.es);
  int64_t bbytes = p.N * p.K * (split_prec ? 4 : p.es);
  auto operand = [&](int64_t bytes, int64_t& o1, int64_t& o2) {
    o1 = off;
    if (p.planar_ok) {
      o2 = off + align256(bytes);
      off = align256(std::max(o1 + 3 * bytes, o2 + bytes));
      return;
    }
    off = align256(off + bytes);
    if (split_prec) {
      o2 = off;
      off = align256(off + bytes);
    }
  };
  if (p.permuteA) operand(abytes, p.off_a, p.off_a2);
  if (p.permuteB) operand(bbytes, p.off_b, p.off_b2);
  p.splitk = allow_splitk ? choose_splitk(mode, p.M, p.N, p.K, 1) : 1;
  const int64_t bk = int64_t(1) << p.pairbits;
  if (allow_splitk && policy && policy->pair_threshold > 0) {
    if (bk >= policy->pair_threshold && bk >= 2) {
      // One partial per group of pairs: split count a power of two <= B_k,
      // so every split boundary is a pair boundary; chunks of at least 64
      // keep each split's K range a whole number of MFMA K-steps.
      const int64_t part = p.M * p.N * (mode == RN_FP64 ? 16 : 8);
      int s = 1;
      while (s < 64 && 2 * s <= bk && p.K / (2 * s) >= 64 && 2 * s * part <= policy->footprint)
        s *= 2;
      p.splitk = s;
    } else {
      p.splitk = 1;
    }
  }
  if (p.splitk > 1) {
    p.off_part = off;
    off = align256(off + int64_t(p.splitk) * p.M * p.N * (mode == RN_FP64 ? 16 : 8));
  }
  p.ws_bytes = (size_t)off;
  p.flops = 8.0 * double(p.M) * double(p.N) * double(p.K);
  *P = p;
  return RN_OK;
}

rn_status check_c(const TdPlan& P, const rn_tensor* C) {
  if (!C) return fail(RN_ERR_INVALID, "C: null descriptor");
  if (C->rank != P.crank) return fail(RN_ERR_SHAPE, "C: rank differs from the derived rank");
  int want = (P.mode == RN_FP64) ? RN_C128 : RN_C64;
  if (C->dtype != want) return fail(RN_ERR_INVALID, "C: dtype does not match the mode");
  for (int j = 0; j < P.crank; ++j) {
    if (C->dims[j] != P.cdims[j]) return fail(RN_ERR_SHAPE, "C: dims differ from the derived dims");
    if (C->grid[j] != P.cgrid[j]) return fail(RN_ERR_GRID, "C: grid differs from the derived grid");
  }
  if (!C->data) return fail(RN_ERR_INVALID, "C: null data");
  return RN_OK;
}

}  // namespace rn
