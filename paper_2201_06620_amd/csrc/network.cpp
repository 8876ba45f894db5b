// Sliced tensor-network contraction on one GPU (Sections II.A and II.B).
//
// Every slice of a sliced network has the same shapes, so the slices run as
// one batch through every step of the path: each step is one batched
// block tensordot (permute A, permute B, batched complex GEMM).  A tensor
// carries a batch dimension only over the sliced labels it depends on, so a
// sub-network that touches no sliced bond is contracted once and broadcast
// (batch stride 0) into the steps that use it.  Slice projection is fused
// into the permute: a sliced axis of an input tensor becomes a batch bit.
// The per-slice scalars are summed in FP64 on the GPU at the end.
//
// Slice-sum mode views the slices as blocks of the unsliced network instead
// (Section II.B): the step where both dependents of a sliced bond meet is the
// step that contracts that bond, so there the slice index becomes a
// contracted bit rather than a batch bit, and later steps run once for it.
//
// To bound memory, only the last `batch_bits` sliced bonds run batched; the
// values of the others are fixed per pass (projection = a base offset on the
// inputs carrying that bond, its bit dropped from every map), and the passes
// run one after another in the same workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "rn_internal.hpp"

namespace rn {

namespace {

struct Arena {
  std::vector<std::pair<int64_t, int64_t>> free_list;  // (offset, size), sorted
  int64_t top = 0;
  int64_t peak = 0;
  int64_t alloc(int64_t size) {
    size = (size + 255) & ~int64_t(255);
    for (size_t i = 0; i < free_list.size(); ++i) {
      if (free_list[i].second >= size) {
        int64_t off = free_list[i].first;
        free_list[i].first += size;
        free_list[i].second -= size;
        if (free_list[i].second == 0) free_list.erase(free_list.begin() + i);
        return off;
      }
    }
    int64_t off = top;
    top += size;
    peak = std::max(peak, top);
    return off;
  }
  void release(int64_t off, int64_t size) {
    size = (size + 255) & ~int64_t(255);
    free_list.push_back({off, size});
    std::sort(free_list.begin(), free_list.end());
    std::vector<std::pair<int64_t, int64_t>> merged;
    for (auto& f : free_list) {
      if (!merged.empty() && merged.back().first + merged.back().second == f.first)
        merged.back().second += f.second;
      else
        merged.push_back(f);
    }
    if (!merged.empty() && merged.back().first + merged.back().second == top) {
      top = merged.back().first;
      merged.pop_back();
    }
    free_list = merged;
  }
};

struct NTensor {
  std::vector<int> labels;     // stored axis labels, outermost first (sliced excluded
                               // for intermediates; raw for inputs)
  uint32_t dmask = 0;          // slice indices this tensor depends on
  bool input = false;
  int input_idx = -1;
  int64_t off = -1;            // workspace offset (intermediates)
  int64_t bytes = 0;
  int64_t alloc = 0;           // arena bytes at off (bytes, or the unreduced partials)
  int nsum = 1;                // split-K partials it holds (summed by its reader's permute)
};

struct NStep {
  int a = 0, b = 0;
  int64_t M = 1, N = 1, K = 1;
  BitPerm permA, permB;
  bool permuteA = false, permuteB = false;
  int64_t offA = -1, offA2 = -1, offB = -1, offB2 = -1, offPart = -1;
  int nbb = 0;
  int64_t a_bs[RN_MAX_SLICED] = {0}, b_bs[RN_MAX_SLICED] = {0}, c_bs[RN_MAX_SLICED] = {0};
  int splitk = 1;
  int64_t abytes = 0, bbytes = 0, pbytes = 0;  // temporaries
  bool direct = false;  // small step: evaluated from the stored layouts
  DirectStep dstep;     // its bit maps (pointers filled at enqueue time)
  int level = 0;        // dependency level of its launch (1 = inputs only)
  int cluster = -1;     // subtree run by one workgroup (index), or -1
  bool fused = false;   // split-K partials left for the reader's permute to sum
  int height = 0;       // height inside that subtree
};

struct NetPlan {
  rn_mode mode;
  int es;
  int nsliced;
  int nout = 0;          // sliced bonds fixed per pass (slice indices 0..nout-1)
  bool slice_sum = false;
  // Per input: (outer slice index, stored bit) of each sliced axis it carries
  // whose value a pass fixes.
  std::vector<std::vector<std::pair<int, int>>> proj;
  int64_t sums_off = 0;  // per-pass FP64 sums when there is more than one pass
  std::vector<NTensor> T;
  std::vector<NStep> steps;
  int64_t ws_bytes = 0;
  double flops = 0;
  int max_rank = 0;
  std::vector<std::vector<int>> levels;  // step indices per dependency level
  std::vector<std::vector<int>> clusters;  // subtrees of tiny steps, by height
  int64_t table_off = 0;                 // grouped small-step tables in ws
};

int popc(uint32_t x) { return __builtin_popcount(x); }

// Sorted slice indices of a mask; the highest index is the batch LSB.
std::vector<int> mask_list(uint32_t m) {
  std::vector<int> v;
  for (int i = 0; i < 32; ++i)
    if ((m >> i) & 1) v.push_back(i);
  return v;
}

// Physical bit position of `label` (or of slice index `sidx`) in a stored
// tensor.  Inputs: raw labels, axis j at bit rank-1-j.  Intermediates:
// [batch bits | labels], label j at bit r-1-j, batch of slice index i at
// r + (number of indices in dmask greater than i).
int pos_of_label(const NTensor& t, int label) {
  int r = (int)t.labels.size();
  for (int j = 0; j < r; ++j)
    if (t.labels[j] == label) return r - 1 - j;
  return -1;
}

int pos_of_slice(const NTensor& t, int sidx, const std::vector<int>& sliced) {
  if (t.input) return pos_of_label(t, sliced[sidx]);
  int r = (int)t.labels.size();
  int above = 0;
  for (int i = sidx + 1; i < 32; ++i) above += (t.dmask >> i) & 1;
  return r + above;
}

// Launch levels of the path's steps, grouping tiny small steps into
// subtrees that one workgroup runs whole.
//
// The path is a tree (each intermediate feeds exactly one later step).  In
// path order, a tiny step (small, within kClusterStepRounds and
// kClusterStepWork) absorbs the subtrees
// rooted at its operands when they are tiny too and the union stays within
// the subtree limits (both operands if that fits, else the lighter one, else
// neither); its index maps are tabulated (tiny_map_words).  A subtree is one launch unit; its level is 1 + the highest
// level among the units that produce its outside operands, so a chain of
// dependent tiny steps costs workgroup barriers instead of one launch per
// dependency level.  Every other step is a unit of its own.
struct ClusterAcc {
  int steps = 0;
  int64_t work = 0, words = 0;  // multiply-adds, map words
  std::vector<int> cnt, ksum;  // steps and summed K per height (index h-1)
};

void form_clusters(NetPlan& P, int nt) {
  const int ns = (int)P.steps.size();
  auto tiny = [&](int s) {
    const NStep& st = P.steps[s];
    const int64_t out = (st.M * st.N) << st.nbb;
    return st.direct && ((out + 255) / 256) * ((st.K + 7) / 8) <= kClusterStepRounds &&
           out * st.K <= kClusterStepWork;
  };
  std::vector<int> root(ns);
  std::vector<int> height(ns, 1);
  std::vector<ClusterAcc> acc(ns);
  std::vector<std::vector<int>> members(ns);
  for (int s = 0; s < ns; ++s) {
    root[s] = s;
    members[s] = {s};
    NStep& st = P.steps[s];
    if (!tiny(s)) continue;
    const int64_t own = ((st.M * st.N) << st.nbb) * st.K;
    const int64_t own_words = tiny_map_words(st.M, st.N, st.K, st.nbb);
    std::vector<int> kids;
    for (int x : {st.a, st.b})
      if (x >= nt && tiny(x - nt)) kids.push_back(x - nt);  // root of its subtree
    // Try both operands' subtrees, then each alone (lighter first).
    std::sort(kids.begin(), kids.end(), [&](int u, int v) { return acc[u].work < acc[v].work; });
    std::vector<std::vector<int>> tries;
    if (kids.size() == 2) tries.push_back(kids);
    for (int k : kids) tries.push_back({k});
    ClusterAcc mine;
    mine.steps = 1;
    mine.work = own;
    mine.words = own_words;
    mine.cnt = {1};
    mine.ksum = {(int)st.K};
    std::vector<int> take;
    for (auto& t : tries) {
      ClusterAcc c;
      c.steps = 1;
      c.work = own;
      c.words = own_words;
      int h = 1;
      for (int k : t) {
        c.steps += acc[k].steps;
        c.work += acc[k].work;
        c.words += acc[k].words;
        h = std::max(h, height[k] + 1);
        if (c.cnt.size() < acc[k].cnt.size()) {
          c.cnt.resize(acc[k].cnt.size(), 0);
          c.ksum.resize(acc[k].ksum.size(), 0);
        }
        for (size_t i = 0; i < acc[k].cnt.size(); ++i) {
          c.cnt[i] += acc[k].cnt[i];
          c.ksum[i] += acc[k].ksum[i];
        }
      }
      if ((int)c.cnt.size() < h) {
        c.cnt.resize(h, 0);
        c.ksum.resize(h, 0);
      }
      c.cnt[h - 1] += 1;
      c.ksum[h - 1] += (int)st.K;
      bool ok = c.steps <= kClusterMaxSteps && c.work <= kClusterWork &&
                c.words <= kClusterMapWords;
      for (size_t i = 0; ok && i < c.cnt.size(); ++i)
        ok = c.cnt[i] <= kClusterMaxWidth && c.ksum[i] <= kDirectMaxK;
      if (ok) {
        mine = std::move(c);
        take = t;
        height[s] = h;
        break;
      }
    }
    for (int k : take) {
      for (int m : members[k]) root[m] = s;
      members[s].insert(members[s].end(), members[k].begin(), members[k].end());
      members[k].clear();
    }
    acc[s] = std::move(mine);
  }
  // Levels, unit by unit in path order (a subtree's root comes last in it,
  // and every outside operand's unit comes before).
  std::vector<int> tl(nt + ns, 0);
  P.levels.clear();
  P.clusters.clear();
  for (int s = 0; s < ns; ++s) {
    if (root[s] != s) continue;
    std::vector<int>& mem = members[s];
    std::sort(mem.begin(), mem.end(), [&](int u, int v) {
      return height[u] != height[v] ? height[u] < height[v] : u < v;
    });
    int L = 0;
    for (int m : mem)
      for (int x : {P.steps[m].a, P.steps[m].b})
        if (x < nt || root[x - nt] != s) L = std::max(L, tl[x]);
    ++L;
    if ((int)P.levels.size() < L) P.levels.resize(L);
    const int cid = mem.size() > 1 ? (int)P.clusters.size() : -1;
    if (cid >= 0) P.clusters.push_back(mem);
    for (int m : mem) {
      tl[nt + m] = L;
      P.steps[m].level = L;
      P.steps[m].cluster = cid;
      P.steps[m].height = cid >= 0 ? height[m] : 0;
      P.levels[L - 1].push_back(m);
    }
  }
}

rn_status plan_network(int32_t nt, const rn_tensor* T, const int32_t* const* labels,
                       int32_t nsteps, const int32_t* path, int32_t nsliced,
                       const int32_t* sliced, rn_mode mode, bool slice_sum, int batch_bits,
                       NetPlan* NP) {
  if (nt < 1 || !T || !labels) return fail(RN_ERR_INVALID, "empty network");
  if (nsteps != nt - 1 || (nsteps > 0 && !path))
    return fail(RN_ERR_INVALID, "path must have nt-1 steps");
  if (nsliced < 0 || nsliced > RN_MAX_SLICED || (nsliced > 0 && !sliced))
    return fail(RN_ERR_INVALID, "bad sliced labels");
  if (mode < RN_FP64 || mode > RN_BF16X3) return fail(RN_ERR_INVALID, "unknown mode");
  const int want = mode == RN_FP64 ? RN_C128 : RN_C64;
  NetPlan P;
  P.mode = mode;
  P.es = mode == RN_FP64 ? 16 : 8;
  P.nsliced = nsliced;
  P.slice_sum = slice_sum;
  P.nout = std::max(0, nsliced - std::max(0, batch_bits));
  P.proj.assign(nt, {});
  std::vector<int> sl(sliced, sliced + nsliced);
  std::map<int, int> count, slice_index;
  for (int i = 0; i < nsliced; ++i) {
    if (slice_index.count(sl[i])) return fail(RN_ERR_INVALID, "repeated sliced label");
    slice_index[sl[i]] = i;
  }
  for (int i = 0; i < nt; ++i) {
    const rn_tensor& t = T[i];
    if (t.rank < 0 || t.rank > 40) return fail(RN_ERR_INVALID, "tensor rank out of range");
    if (t.dtype != want) return fail(RN_ERR_INVALID, "tensor dtype does not match the mode");
    if (!t.data) return fail(RN_ERR_INVALID, "null tensor data");
    if (t.rank > 0 && !labels[i]) return fail(RN_ERR_INVALID, "null labels");
    NTensor nt_;
    nt_.input = true;
    nt_.input_idx = i;
    for (int j = 0; j < t.rank; ++j) {
      if (t.dims[j] != 2) return fail(RN_ERR_UNSUPPORTED, "network tensors need dims of 2");
      if (t.grid[j] != 1) return fail(RN_ERR_UNSUPPORTED, "network tensors must be unblocked");
      int l = labels[i][j];
      for (int q = 0; q < j; ++q)
        if (labels[i][q] == l) return fail(RN_ERR_INVALID, "label repeated within a tensor");
      nt_.labels.push_back(l);
      count[l]++;
      auto it = slice_index.find(l);
      if (it != slice_index.end()) {
        if (it->second >= P.nout)
          nt_.dmask |= 1u << it->second;
        else
          P.proj[i].push_back({it->second, t.rank - 1 - j});
      }
    }
    P.T.push_back(nt_);
  }
  for (auto& kv : count)
    if (kv.second != 2)
      return fail(RN_ERR_INVALID, "label " + std::to_string(kv.first) +
                                      " is not a bond between two tensors");
  for (int i = 0; i < nsliced; ++i)
    if (!count.count(sl[i])) return fail(RN_ERR_INVALID, "sliced label is not a bond");

  std::vector<bool> alive(nt + nsteps, false);
  for (int i = 0; i < nt; ++i) alive[i] = true;
  Arena arena;
  auto eff = [&](const NTensor& t) {
    std::vector<int> v;
    for (int l : t.labels)
      if (!slice_index.count(l)) v.push_back(l);
    return v;
  };
  for (int i = 0; i < nt; ++i) P.max_rank = std::max(P.max_rank, (int)eff(P.T[i]).size());
  const bool split_prec = (mode == RN_BF16X3);
  for (int s = 0; s < nsteps; ++s) {
    int a = path[2 * s], b = path[2 * s + 1];
    if (a < 0 || b < 0 || a >= nt + s || b >= nt + s || a == b || !alive[a] || !alive[b])
      return fail(RN_ERR_INVALID, "path step " + std::to_string(s) + " uses a dead tensor");
    alive[a] = alive[b] = false;
    const NTensor& ta = P.T[a];
    const NTensor& tb = P.T[b];
    std::vector<int> la = eff(ta), lb = eff(tb);
    // Contracted labels in the order of the larger operand.
    std::vector<int> shared;
    const std::vector<int>& ord = (lb.size() > la.size()) ? lb : la;
    const std::vector<int>& oth = (lb.size() > la.size()) ? la : lb;
    for (int l : ord)
      if (std::find(oth.begin(), oth.end(), l) != oth.end()) shared.push_back(l);
    std::vector<int> fa, fb;
    for (int l : la)
      if (std::find(shared.begin(), shared.end(), l) == shared.end()) fa.push_back(l);
    for (int l : lb)
      if (std::find(shared.begin(), shared.end(), l) == shared.end()) fb.push_back(l);
    NStep st;
    st.a = a;
    st.b = b;
    // Slice indices summed in this step (slice-sum mode): those both
    // operands depend on.  They are the outermost contracted bits.
    const uint32_t cmask = slice_sum ? (ta.dmask & tb.dmask) : 0u;
    const std::vector<int> csl = mask_list(cmask);
    const int ncs = (int)csl.size();
    int kb = (int)shared.size() + ncs, mb = (int)fa.size(), nbits = (int)fb.size();
    if (mb + nbits > 34) return fail(RN_ERR_UNSUPPORTED, "intermediate over 2^34 elements");
    st.M = int64_t(1) << mb;
    st.N = int64_t(1) << nbits;
    st.K = int64_t(1) << kb;
    uint32_t dc = (ta.dmask | tb.dmask) & ~cmask;
    std::vector<int> dcl = mask_list(dc);
    st.nbb = (int)dcl.size();
    // Stored bit of contracted bit q (0 = innermost) in an operand.
    auto kpos = [&](const NTensor& t, int q) {
      const int ns = (int)shared.size();
      return q < ns ? pos_of_label(t, shared[ns - 1 - q]) : pos_of_slice(t, csl[q - ns], sl);
    };
    // Operand permutations: [batch over own dmask | free | contracted].
    auto build = [&](const NTensor& t, const std::vector<int>& fr, BitPerm& bp) {
      bp.nbits = 0;
      for (int q = 0; q < kb; ++q) bp.src[bp.nbits++] = (int8_t)kpos(t, q);
      for (int q = (int)fr.size() - 1; q >= 0; --q)
        bp.src[bp.nbits++] = (int8_t)pos_of_label(t, fr[q]);
      std::vector<int> dl = mask_list(t.dmask & ~cmask);
      for (int q = (int)dl.size() - 1; q >= 0; --q)
        bp.src[bp.nbits++] = (int8_t)pos_of_slice(t, dl[q], sl);
    };
    build(ta, fa, st.permA);
    build(tb, fb, st.permB);
    st.permuteA = split_prec || !st.permA.identity();
    st.permuteB = split_prec || !st.permB.identity();
    // Batch strides.  Bit q of the GEMM batch index is slice index
    // dcl[nbb-1-q]; an operand not depending on it has stride 0.
    for (int q = 0; q < st.nbb; ++q) {
      int sidx = dcl[st.nbb - 1 - q];
      auto stride = [&](const NTensor& t, int64_t body) -> int64_t {
        const uint32_t bm = t.dmask & ~cmask;
        if (!((bm >> sidx) & 1)) return 0;
        int above = 0;
        for (int i = sidx + 1; i < 32; ++i) above += (bm >> i) & 1;
        return (int64_t(1) << above) * body;
      };
      st.a_bs[q] = stride(ta, st.M * st.K);
      st.b_bs[q] = stride(tb, st.N * st.K);
      st.c_bs[q] = (int64_t(1) << q) * st.M * st.N;
    }
    int64_t nbatch = int64_t(1) << st.nbb;
    auto stored_bits = [&](const NTensor& t) {
      return t.input ? (int)t.labels.size() : (int)t.labels.size() + popc(t.dmask);
    };
    st.direct = st.K <= kDirectMaxK && st.M * st.N * st.K * nbatch <= (int64_t(1) << 24) &&
                stored_bits(ta) < 31 && stored_bits(tb) < 31 && st.nbb <= 15;
    if (st.direct) {
      DirectStep& d = st.dstep;
      d.M = st.M;
      d.N = st.N;
      d.K = st.K;
      d.mbits = mb;
      d.nbits = nbits;
      d.kbits = kb;
      d.nbb = st.nbb;
      d.blocks_per_batch = (int)((st.M * st.N + 255) / 256);
      for (int i = 0; i < mb; ++i) d.am[i] = (int8_t)pos_of_label(ta, fa[mb - 1 - i]);
      for (int i = 0; i < nbits; ++i) d.bn[i] = (int8_t)pos_of_label(tb, fb[nbits - 1 - i]);
      for (int i = 0; i < kb; ++i) {
        d.ak[i] = (int8_t)kpos(ta, i);
        d.bk[i] = (int8_t)kpos(tb, i);
      }
      for (int q = 0; q < st.nbb; ++q) {
        int sidx = dcl[st.nbb - 1 - q];
        d.a_bs[q] = ((ta.dmask >> sidx) & 1) ? int64_t(1) << pos_of_slice(ta, sidx, sl) : 0;
        d.b_bs[q] = ((tb.dmask >> sidx) & 1) ? int64_t(1) << pos_of_slice(tb, sidx, sl) : 0;
      }
      for (int i = 0; i < P.nout; ++i) {
        auto pp = [&](const NTensor& t) -> int8_t {
          if (!t.input) return 0;
          for (auto& pr : P.proj[t.input_idx])
            if (pr.first == i) return (int8_t)(pr.second + 1);
          return 0;
        };
        d.a_pp[i] = pp(ta);
        d.b_pp[i] = pp(tb);
      }
      st.permuteA = st.permuteB = false;
    }
    st.abytes = (st.M * st.K << popc(ta.dmask & ~cmask)) * (split_prec ? 4 : P.es);
    st.bbytes = (st.N * st.K << popc(tb.dmask & ~cmask)) * (split_prec ? 4 : P.es);
    st.splitk = st.direct ? 1 : choose_splitk(mode, st.M, st.N, st.K, nbatch);
    st.pbytes = st.splitk > 1 ? int64_t(st.splitk) * nbatch * st.M * st.N * P.es : 0;
    NTensor tc;
    for (int l : fa) tc.labels.push_back(l);
    for (int l : fb) tc.labels.push_back(l);
    tc.dmask = dc;
    tc.bytes = nbatch * st.M * st.N * P.es;
    P.max_rank = std::max(P.max_rank, mb + nbits);
    P.flops += 8.0 * double(st.M) * double(st.N) * double(st.K) * double(nbatch);
    P.T.push_back(tc);
    P.steps.push_back(st);
    alive[nt + s] = true;
  }
  const NTensor& fin = P.T.back();
  if (!eff(fin).empty()) return fail(RN_ERR_INVALID, "network does not close to a scalar");
  form_clusters(P, nt);
  // Workspace in execution order: level by level; the small steps of a
  // level run together in one launch, so their results are all live at once
  // and their operands are released only after that launch; then one grouped
  // launch permutes the operands of all large steps of the level (their
  // permuted copies stay live until the level ends), and the large steps'
  // GEMMs run one after another.
  auto release_operand = [&](int id) {
    if (!P.T[id].input) arena.release(P.T[id].off, P.T[id].alloc);
  };
  // A large step with split K whose result is read by a large step that
  // permutes it leaves its partial sums unreduced: the reader's permute adds
  // them in ascending split order (the same sums as the reduction kernel) on
  // the way, which saves the reduction's launch and a write and read of C.
  // Only for two partials of at least 2^20 elements: the permute adds the
  // partials one after another per element, and with fewer elements it has
  // too few workgroups to hide that (measured: 16 partials of 2^16 elements
  // took a permute from 6 to 127 us).
  {
    std::vector<int> reader(P.T.size(), -1);
    for (int c = 0; c < (int)P.steps.size(); ++c) {
      reader[P.steps[c].a] = c;
      reader[P.steps[c].b] = c;
    }
    for (int si = 0; si < (int)P.steps.size(); ++si) {
      NStep& st = P.steps[si];
      const int c = reader[nt + si];
      if (st.direct || st.splitk != 2 || c < 0 || P.steps[c].direct) continue;
      if (P.T[nt + si].bytes / P.es < (int64_t(1) << 20)) continue;
      const NStep& rd = P.steps[c];
      if ((rd.a == nt + si && rd.permuteA) || (rd.b == nt + si && rd.permuteB)) {
        st.fused = true;
        P.T[nt + si].nsum = st.splitk;
      }
    }
  }
  for (auto& t : P.T) t.alloc = t.bytes;
  for (auto& lv : P.levels) {
    for (int si : lv)
      if (P.steps[si].direct) P.T[nt + si].off = arena.alloc(P.T[nt + si].bytes);
    for (int si : lv)
      if (P.steps[si].direct) {
        release_operand(P.steps[si].a);
        release_operand(P.steps[si].b);
      }
    for (int si : lv) {
      NStep& st = P.steps[si];
      if (st.direct) continue;
      if (st.permuteA) {
        st.offA = arena.alloc(st.abytes);
        if (split_prec) st.offA2 = arena.alloc(st.abytes);
      }
      if (st.permuteB) {
        st.offB = arena.alloc(st.bbytes);
        if (split_prec) st.offB2 = arena.alloc(st.bbytes);
      }
    }
    for (int si : lv) {
      NStep& st = P.steps[si];
      if (st.direct) continue;
      if (st.fused) {
        P.T[nt + si].alloc = st.pbytes;  // the partials are the tensor until it is read
        P.T[nt + si].off = arena.alloc(st.pbytes);
      } else {
        if (st.splitk > 1) st.offPart = arena.alloc(st.pbytes);
        P.T[nt + si].off = arena.alloc(P.T[nt + si].bytes);
        if (st.splitk > 1) arena.release(st.offPart, st.pbytes);
      }
      release_operand(st.a);
      release_operand(st.b);
    }
    for (int si : lv) {
      NStep& st = P.steps[si];
      if (st.direct) continue;
      if (st.permuteA) {
        arena.release(st.offA, st.abytes);
        if (split_prec) arena.release(st.offA2, st.abytes);
      }
      if (st.permuteB) {
        arena.release(st.offB, st.bbytes);
        if (split_prec) arena.release(st.offB2, st.bbytes);
      }
    }
  }
  P.sums_off = (arena.peak + 255) & ~int64_t(255);
  const int64_t npass = int64_t(1) << P.nout;
  P.table_off = P.sums_off + (npass > 1 ? ((16 * npass + 255) & ~int64_t(255)) : 0);
  int64_t tbytes = 0;
  for (auto& lv : P.levels) {
    int nd = 0, np = 0;
    int64_t words = 0;
    for (int si : lv) {
      const NStep& st = P.steps[si];
      nd += st.direct ? 1 : 0;
      np += st.direct ? 0 : (st.permuteA ? 1 : 0) + (st.permuteB ? 1 : 0);
      if (st.cluster >= 0) words += tiny_map_words(st.M, st.N, st.K, st.nbb);
    }
    if (nd) tbytes += (int64_t)grouped_direct_bound(nd, words);
    if (np && P.nout == 0) tbytes += (int64_t)grouped_perm_bound(np);
  }
  P.ws_bytes = P.table_off + tbytes;
  *NP = std::move(P);
  return RN_OK;
}

}  // namespace

// Address of tensor `id` in pass `pass`: an input carrying a sliced bond
// whose value the pass fixes starts at that value's half.
static const void* tensor_ptr(const NetPlan& P, const rn_tensor* T, char* w, int id, int64_t pass) {
  const NTensor& t = P.T[id];
  if (!t.input) return w + t.off;
  int64_t off = 0;
  for (auto& pr : P.proj[t.input_idx])
    if ((pass >> (P.nout - 1 - pr.first)) & 1) off += int64_t(1) << pr.second;
  return static_cast<const char*>(T[t.input_idx].data) + off * P.es;
}

// Parameter tables of the grouped launches of each level, with operand
// pointers resolved for this call: the small steps (pass 0; the kernel adds
// the projection offsets of later passes) and, when the network runs in one
// pass, the permutes of the large steps' operands.
struct LevelLaunches {
  std::vector<GroupedLaunch> direct, perm;
  std::vector<int> tile;  // per step: GEMM tile from the handle's tune table, or -1
};
static void build_net_tables(const NetPlan& P, const rn_tensor* T, void* ws,
                             std::vector<char>& blob, LevelLaunches& per_level) {
  char* w = static_cast<char*>(ws);
  const int nt = (int)P.T.size() - (int)P.steps.size();
  const bool split_prec = (P.mode == RN_BF16X3);
  blob.clear();
  per_level.direct.assign(P.levels.size(), GroupedLaunch{});
  per_level.perm.assign(P.levels.size(), GroupedLaunch{});
  std::vector<char> part;
  auto ptr = [&](int id) { return tensor_ptr(P, T, w, id, 0); };
  auto direct_of = [&](int si) {
    const NStep& st = P.steps[si];
    DirectStep d = st.dstep;
    d.A = ptr(st.a);
    d.B = ptr(st.b);
    d.C = w + P.T[nt + si].off;
    return d;
  };
  for (size_t L = 0; L < P.levels.size(); ++L) {
    std::vector<DirectStep> ds;
    std::vector<TinyStep> tiny;
    std::vector<int32_t> maps;
    std::vector<DirectJob> jobs;
    std::vector<PermLaunch> pj;
    // Subtrees first (one workgroup each, the longest-running jobs), their
    // steps by height, each with its height's run, its offset among that
    // height's outputs and its index maps.
    std::vector<int> seen;
    for (int si : P.levels[L]) {
      const int c = P.steps[si].cluster;
      if (c < 0 || std::find(seen.begin(), seen.end(), c) != seen.end()) continue;
      seen.push_back(c);
      const std::vector<int>& mem = P.clusters[c];
      DirectJob job{(int32_t)mem.size(), (int32_t)tiny.size(), (int32_t)maps.size(), 0};
      size_t run = tiny.size();
      int ooff = 0;
      std::vector<uint8_t> sel;  // the current height's byte table
      auto close_run = [&]() {
        tiny[run].run_end = (int32_t)(tiny.size() - job.first);
        tiny[run].run_total = ooff;
        tiny[run].sel = (int32_t)(maps.size() - job.map_first);
        sel.resize((sel.size() + 3) & ~size_t(3), 0);
        for (size_t i = 0; i < sel.size(); i += 4)
          maps.push_back((int32_t)(uint32_t(sel[i]) | uint32_t(sel[i + 1]) << 8 |
                                   uint32_t(sel[i + 2]) << 16 | uint32_t(sel[i + 3]) << 24));
        sel.clear();
      };
      for (size_t q = 0; q < mem.size(); ++q) {
        const int m = mem[q];
        const DirectStep d = direct_of(m);
        if (q > 0 && P.steps[m].height != P.steps[mem[q - 1]].height) {
          close_run();
          run = tiny.size();
          ooff = 0;
        }
        TinyStep t;
        t.A = d.A;
        t.B = d.B;
        t.C = d.C;
        t.mbits = d.mbits;
        t.nbits = d.nbits;
        t.K = (int32_t)d.K;
        t.nbb = d.nbb;
        t.ooff = ooff;
        t.map = (int32_t)(maps.size() - job.map_first);
        for (int i = 0; i < RN_MAX_SLICED; ++i) {
          t.a_pp[i] = d.a_pp[i];
          t.b_pp[i] = d.b_pp[i];
        }
        auto scatter = [](int64_t x, int bits, const int8_t* pos) {
          int64_t o = 0;
          for (int i = 0; i < bits; ++i)
            if ((x >> i) & 1) o += int64_t(1) << pos[i];
          return (int32_t)o;
        };
        for (int64_t x = 0; x < d.M; ++x) maps.push_back(scatter(x, d.mbits, d.am));
        for (int64_t x = 0; x < d.N; ++x) maps.push_back(scatter(x, d.nbits, d.bn));
        for (int64_t x = 0; x < d.K; ++x) maps.push_back(scatter(x, d.kbits, d.ak));
        for (int64_t x = 0; x < d.K; ++x) maps.push_back(scatter(x, d.kbits, d.bk));
        for (int side = 0; side < 2; ++side)
          for (int64_t x = 0; x < (int64_t(1) << d.nbb); ++x) {
            int64_t o = 0;
            for (int i = 0; i < d.nbb; ++i)
              if ((x >> i) & 1) o += side ? d.b_bs[i] : d.a_bs[i];
            maps.push_back((int32_t)o);
          }
        const int nout_step = (int)((d.M * d.N) << d.nbb);
        sel.insert(sel.end(), nout_step, (uint8_t)q);
        ooff += nout_step;
        tiny.push_back(t);
      }
      close_run();
      job.map_words = (int32_t)(maps.size() - job.map_first);
      jobs.push_back(job);
    }
    for (int si : P.levels[L]) {
      const NStep& st = P.steps[si];
      if (st.direct && st.cluster < 0) {
        jobs.push_back(DirectJob{1, (int32_t)ds.size(), 0, 0});
        ds.push_back(direct_of(si));
        continue;
      }
      if (!st.direct) {
        if (P.nout != 0) continue;
        for (int side = 0; side < 2; ++side) {
          if (!(side ? st.permuteB : st.permuteA)) continue;
          PermLaunch pl;
          pl.in = ptr(side ? st.b : st.a);
          pl.nsum = P.T[side ? st.b : st.a].nsum;
          pl.sstride = P.T[side ? st.b : st.a].bytes / P.es;
          pl.out = w + (side ? st.offB : st.offA);
          pl.out2 = split_prec ? w + (side ? st.offB2 : st.offA2) : nullptr;
          pl.perm = side ? st.permB : st.permA;
          pl.in_es = P.es;
          pl.kind = split_prec ? 1 : 0;
          pj.push_back(pl);
        }
        continue;
      }
    }
    if (!jobs.empty()) {
      GroupedLaunch G;
      size_t base = blob.size();
      grouped_direct_build(ds, tiny, maps, jobs, P.mode, part, G);
      G.params_off += base;
      G.tiny_off += base;
      G.maps_off += base;
      G.jobs_off += base;
      G.prefix_off += base;
      blob.insert(blob.end(), part.begin(), part.end());
      per_level.direct[L] = G;
    }
    if (!pj.empty()) {
      GroupedLaunch G;
      size_t base = blob.size();
      grouped_perm_build(pj, part, G);
      G.params_off += base;
      G.prefix_off += base;
      blob.insert(blob.end(), part.begin(), part.end());
      per_level.perm[L] = G;
    }
  }
}

// The GEMM tile of each large step from the handle's tune table (keyed by
// mode and log2 of M, N, K), -1 where there is no valid entry.
static void tuned_tiles(const rn_ctx* h, const NetPlan& P, LevelLaunches& L) {
  L.tile.assign(P.steps.size(), -1);
  for (size_t si = 0; si < P.steps.size(); ++si) {
    const NStep& st = P.steps[si];
    if (st.direct) continue;
    const int t = tuned_tile(h, P.mode, __builtin_ctzll((uint64_t)st.M),
                             __builtin_ctzll((uint64_t)st.N), __builtin_ctzll((uint64_t)st.K));
    if (gemm_tile_valid(P.mode, t, st.M, st.N)) L.tile[si] = t;
  }
}

// tab: device copy of the parameter table (in the workspace, or owned by a
// graph).
static rn_status enqueue_pass(const NetPlan& P, const rn_tensor* T, void* ws, hipStream_t s,
                              int64_t pass, double* sum_dev, double* slices_dev, Profiler* prof,
                              const LevelLaunches& per_level, const char* tab) {
  char* w = static_cast<char*>(ws);
  const bool split_prec = (P.mode == RN_BF16X3);
  auto ptr = [&](int id) { return tensor_ptr(P, T, w, id, pass); };
  hipError_t e;
  const int nt = (int)P.T.size() - (int)P.steps.size();
  for (size_t L = 0; L < P.levels.size(); ++L) {
    // All small steps of this level in one launch, then the permutes of the
    // large steps in one launch, then the large steps' GEMMs.
    if (per_level.direct[L].n > 0) {
      int ev = prof->begin(1, s);
      e = launch_direct_grouped(per_level.direct[L], tab, pass, P.nout, s);
      prof->end(ev, s);
      if (e != hipSuccess)
        return fail(RN_ERR_HIP, std::string("network small steps: ") + hipGetErrorString(e));
    }
    const bool grouped_perm = per_level.perm[L].n > 0;
    if (grouped_perm) {
      int ev = prof->begin(0, s);
      e = launch_permute_grouped(per_level.perm[L], tab, s);
      prof->end(ev, s);
      if (e != hipSuccess)
        return fail(RN_ERR_HIP, std::string("network permutes: ") + hipGetErrorString(e));
    }
    for (int si : P.levels[L]) {
      const NStep& st = P.steps[si];
      if (st.direct) continue;
      const void* am = ptr(st.a);
      const void* bm = ptr(st.b);
      const void* am2 = nullptr;
      const void* bm2 = nullptr;
      if (grouped_perm) {
        if (st.permuteA) {
          am = w + st.offA;
          am2 = split_prec ? w + st.offA2 : nullptr;
        }
        if (st.permuteB) {
          bm = w + st.offB;
          bm2 = split_prec ? w + st.offB2 : nullptr;
        }
      } else if (st.permuteA) {
        PermLaunch pl;
        pl.in = am;
        pl.nsum = P.T[st.a].nsum;
        pl.sstride = P.T[st.a].bytes / P.es;
        pl.out = w + st.offA;
        pl.out2 = split_prec ? w + st.offA2 : nullptr;
        pl.perm = st.permA;
        pl.in_es = P.es;
        pl.kind = split_prec ? 1 : 0;
        int ev = prof->begin(0, s);
        e = launch_permute(pl, s);
        prof->end(ev, s);
        if (e != hipSuccess)
          return fail(RN_ERR_HIP, std::string("network permute: ") + hipGetErrorString(e));
        am = pl.out;
        am2 = pl.out2;
      }
      if (!grouped_perm && st.permuteB) {
        PermLaunch pl;
        pl.in = bm;
        pl.nsum = P.T[st.b].nsum;
        pl.sstride = P.T[st.b].bytes / P.es;
        pl.out = w + st.offB;
        pl.out2 = split_prec ? w + st.offB2 : nullptr;
        pl.perm = st.permB;
        pl.in_es = P.es;
        pl.kind = split_prec ? 1 : 0;
        int ev = prof->begin(0, s);
        e = launch_permute(pl, s);
        prof->end(ev, s);
        if (e != hipSuccess)
          return fail(RN_ERR_HIP, std::string("network permute: ") + hipGetErrorString(e));
        bm = pl.out;
        bm2 = pl.out2;
      }
      GemmLaunch g;
      g.mode = P.mode;
      g.A = am;
      g.B = bm;
      g.A2 = am2;
      g.B2 = bm2;
      g.C = w + P.T[nt + si].off;
      g.M = st.M;
      g.N = st.N;
      g.K = st.K;
      g.lda = st.K;
      g.ldb = st.K;
      g.crow.shift = 62;
      g.crow.hi = 0;
      g.crow.lo = st.N;
      g.ccol.shift = 62;
      g.ccol.hi = 0;
      g.ccol.lo = 1;
      g.nbb = st.nbb;
      for (int q = 0; q < st.nbb; ++q) {
        g.a_bstride[q] = st.a_bs[q];
        g.b_bstride[q] = st.b_bs[q];
        g.c_bstride[q] = st.c_bs[q];
      }
      g.splitk = st.splitk;
      g.partial = st.splitk > 1 ? w + (st.fused ? P.T[nt + si].off : st.offPart) : nullptr;
      g.partial_only = st.fused;  // the reader's permute sums the partials
      if (si < (int)per_level.tile.size() && per_level.tile[si] >= 0 &&
          (!st.fused || gemm_tile_splits(P.mode, per_level.tile[si]))) {
        // A tuned tile; the planned split (and its partials) only if it splits.
        g.tile = per_level.tile[si];
        if (!gemm_tile_splits(P.mode, g.tile)) {
          g.splitk = 1;
          g.partial = nullptr;
        }
      }
      if ((e = launch_gemm(g, s, prof)) != hipSuccess)
        return fail(RN_ERR_HIP, std::string("network GEMM: ") + hipGetErrorString(e));
    }
  }
  const NTensor& fin = P.T.back();
  int64_t nvals = int64_t(1) << popc(fin.dmask);
  int ev = prof->begin(3, s);
  e = launch_sum_slices(ptr((int)P.T.size() - 1), P.es, nvals, sum_dev,
                        slices_dev ? slices_dev + 2 * pass * nvals : nullptr, s);
  prof->end(ev, s);
  if (e != hipSuccess) return fail(RN_ERR_HIP, std::string("slice sum: ") + hipGetErrorString(e));
  return RN_OK;
}

// Every pass in order; with several passes each writes its own FP64 sum and
// one more launch adds those in ascending pass order.
static rn_status enqueue_network(const NetPlan& P, const rn_tensor* T, void* ws, hipStream_t s,
                                 double* amp_dev, double* slices_dev, Profiler* prof,
                                 const LevelLaunches& launches, const char* tab) {
  const int64_t npass = int64_t(1) << P.nout;
  char* w = static_cast<char*>(ws);
  double* sums = reinterpret_cast<double*>(w + P.sums_off);
  rn_status st;
  for (int64_t pass = 0; pass < npass; ++pass) {
    double* out = npass > 1 ? sums + 2 * pass : amp_dev;
    if ((st = enqueue_pass(P, T, ws, s, pass, out, slices_dev, prof, launches, tab)) != RN_OK)
      return st;
  }
  if (npass > 1) {
    int ev = prof->begin(3, s);
    hipError_t e = launch_sum_c128(sums, npass, amp_dev, s);
    prof->end(ev, s);
    if (e != hipSuccess)
      return fail(RN_ERR_HIP, std::string("pass sum: ") + hipGetErrorString(e));
  }
  return RN_OK;
}

// Plan under the options: the largest batched-slice count whose workspace
// fits the cap.
static rn_status plan_fitting(int32_t nt, const rn_tensor* T, const int32_t* const* labels,
                              int32_t nsteps, const int32_t* path, int32_t nsliced,
                              const int32_t* sliced, rn_mode mode, const NetOpts& o,
                              NetPlan* P) {
  int bb = std::min(std::max(o.batch_bits, 0), std::max(nsliced, 0));
  for (;; --bb) {
    rn_status st = plan_network(nt, T, labels, nsteps, path, nsliced, sliced, mode, o.slice_sum,
                                bb, P);
    if (st != RN_OK) return st;
    if (o.footprint <= 0 || P->ws_bytes <= o.footprint) return RN_OK;
    if (bb == 0)
      return fail(RN_ERR_OOM, "network workspace " + std::to_string(P->ws_bytes) +
                                  " bytes exceeds the cap even with every slice in its own pass");
  }
}

// Exact structural signature of a network call: everything the plan
// depends on, nothing it does not (data pointers excluded).
static bool net_signature(int32_t nt, const rn_tensor* T, const int32_t* const* labels,
                          int32_t nsteps, const int32_t* path, int32_t nsliced,
                          const int32_t* sliced, rn_mode mode, const NetOpts& o,
                          std::vector<int64_t>& sig) {
  if (nt < 1 || !T || !labels || nsteps < 0 || nsliced < 0 || (nsteps > 0 && !path) ||
      (nsliced > 0 && !sliced))
    return false;
  sig.clear();
  size_t words = 7 + 2 * size_t(nt) + 2 * size_t(nsteps) + size_t(nsliced);
  for (int i = 0; i < nt; ++i) words += 3 * size_t(std::max(0, T[i].rank));
  sig.reserve(words);
  sig.push_back(mode);
  sig.push_back(o.slice_sum);
  sig.push_back(o.batch_bits);
  sig.push_back(o.footprint);
  sig.push_back(nt);
  sig.push_back(nsteps);
  sig.push_back(nsliced);
  for (int i = 0; i < nt; ++i) {
    const rn_tensor& t = T[i];
    if (t.rank < 0 || t.rank > RN_MAX_RANK || (t.rank > 0 && !labels[i])) return false;
    sig.push_back(t.rank);
    sig.push_back(t.dtype);
    for (int j = 0; j < t.rank; ++j) {
      sig.push_back(t.dims[j]);
      sig.push_back(t.grid[j]);
      sig.push_back(labels[i][j]);
    }
  }
  for (int i = 0; i < 2 * nsteps; ++i) sig.push_back(path[i]);
  for (int i = 0; i < nsliced; ++i) sig.push_back(sliced[i]);
  return true;
}

// Plan through the handle's cache (kept to 16 entries); with no handle, or
// arguments too malformed to sign, plan directly.
static rn_status cached_plan(rn_ctx* h, int32_t nt, const rn_tensor* T,
                             const int32_t* const* labels, int32_t nsteps, const int32_t* path,
                             int32_t nsliced, const int32_t* sliced, rn_mode mode,
                             const NetOpts& o, std::shared_ptr<NetPlan>* out) {
  std::vector<int64_t> sig;
  const bool signable = h && net_signature(nt, T, labels, nsteps, path, nsliced, sliced, mode, o, sig);
  if (signable) {
    auto& c = h->net_plans;
    for (size_t i = 0; i < c.size(); ++i) {
      if (c[i].first == sig) {
        for (int j = 0; j < nt; ++j)
          if (!T[j].data) return fail(RN_ERR_INVALID, "null tensor data");
        auto hit = c[i];
        c.erase(c.begin() + i);
        c.push_back(hit);
        *out = std::static_pointer_cast<NetPlan>(hit.second);
        return RN_OK;
      }
    }
  }
  auto P = std::make_shared<NetPlan>();
  rn_status st = plan_fitting(nt, T, labels, nsteps, path, nsliced, sliced, mode, o, P.get());
  if (st != RN_OK) return st;
  if (signable) {
    auto& c = h->net_plans;
    if (c.size() >= 16) c.erase(c.begin());
    c.push_back({std::move(sig), std::static_pointer_cast<void>(P)});
  }
  *out = P;
  return RN_OK;
}

rn_status network_plan(int32_t nt, const rn_tensor* T, const int32_t* const* labels,
                       int32_t nsteps, const int32_t* path, int32_t nsliced,
                       const int32_t* sliced, rn_mode mode, const NetOpts& o, size_t* ws_bytes,
                       double* flops, int32_t* max_rank, int* batch_bits) {
  return network_plan_h(nullptr, nt, T, labels, nsteps, path, nsliced, sliced, mode, o, ws_bytes,
                        flops, max_rank, batch_bits);
}

rn_status network_plan_h(rn_ctx* h, int32_t nt, const rn_tensor* T, const int32_t* const* labels,
                         int32_t nsteps, const int32_t* path, int32_t nsliced,
                         const int32_t* sliced, rn_mode mode, const NetOpts& o,
                         size_t* ws_bytes, double* flops, int32_t* max_rank, int* batch_bits) {
  std::shared_ptr<NetPlan> PP;
  rn_status st = cached_plan(h, nt, T, labels, nsteps, path, nsliced, sliced, mode, o, &PP);
  if (st != RN_OK) return st;
  const NetPlan& P = *PP;
  if (ws_bytes) *ws_bytes = (size_t)P.ws_bytes;
  if (flops) *flops = P.flops * double(int64_t(1) << P.nout);
  if (max_rank) *max_rank = P.max_rank;
  if (batch_bits) *batch_bits = P.nsliced - P.nout;
  return RN_OK;
}

static rn_status run_planned(rn_ctx* h, const NetPlan& P, int32_t nt, const rn_tensor* T,
                             const int32_t* const* labels, int32_t nsteps, const int32_t* path,
                             int32_t nsliced, const int32_t* sliced, rn_mode mode, void* ws,
                             size_t ws_bytes, hipStream_t s, double* amp_dev,
                             double* slices_dev, const uint64_t* base_key = nullptr);

rn_status network_run(rn_ctx* h, int32_t nt, const rn_tensor* T, const int32_t* const* labels,
                      int32_t nsteps, const int32_t* path, int32_t nsliced,
                      const int32_t* sliced, rn_mode mode, const NetOpts& o, void* ws,
                      size_t ws_bytes, hipStream_t s, double* amp_dev, double* slices_dev) {
  if (!amp_dev) return fail(RN_ERR_INVALID, "null amplitude buffer");
  std::shared_ptr<NetPlan> PP;
  rn_status st = cached_plan(h, nt, T, labels, nsteps, path, nsliced, sliced, mode, o, &PP);
  if (st != RN_OK) return st;
  return run_planned(h, *PP, nt, T, labels, nsteps, path, nsliced, sliced, mode, ws, ws_bytes, s,
                     amp_dev, slices_dev);
}

rn_status network_plan_keep(int32_t nt, const rn_tensor* T, const int32_t* const* labels,
                            int32_t nsteps, const int32_t* path, int32_t nsliced,
                            const int32_t* sliced, rn_mode mode, const NetOpts& o,
                            std::shared_ptr<void>* plan, size_t* ws_bytes, double* flops,
                            int* batch_bits) {
  auto P = std::make_shared<NetPlan>();
  rn_status st = plan_fitting(nt, T, labels, nsteps, path, nsliced, sliced, mode, o, P.get());
  if (st != RN_OK) return st;
  if (ws_bytes) *ws_bytes = (size_t)P->ws_bytes;
  if (flops) *flops = P->flops * double(int64_t(1) << P->nout);
  if (batch_bits) *batch_bits = P->nsliced - P->nout;
  *plan = std::static_pointer_cast<void>(P);
  return RN_OK;
}

rn_status network_run_planned(rn_ctx* h, const std::shared_ptr<void>& plan, int32_t nt,
                              const rn_tensor* T, const int32_t* const* labels, int32_t nsteps,
                              const int32_t* path, int32_t nsliced, const int32_t* sliced,
                              rn_mode mode, void* ws, size_t ws_bytes, hipStream_t s,
                              double* amp_dev, double* slices_dev) {
  if (!plan) return fail(RN_ERR_INVALID, "no plan");
  if (!amp_dev) return fail(RN_ERR_INVALID, "null amplitude buffer");
  for (int j = 0; j < nt; ++j)
    if (!T[j].data) return fail(RN_ERR_INVALID, "null tensor data");
  return run_planned(h, *std::static_pointer_cast<NetPlan>(plan), nt, T, labels, nsteps, path,
                     nsliced, sliced, mode, ws, ws_bytes, s, amp_dev, slices_dev);
}

// Graph keys of network calls: the part fixed by the call's descriptors
// (what a prepared call hashes once), then the per-call pointers, stream and
// tuning state.
static uint64_t net_key_base(const NetPlan& P, rn_mode mode, int32_t nt, const rn_tensor* T,
                             const int32_t* const* labels, int32_t nsteps, const int32_t* path,
                             int32_t nsliced, const int32_t* sliced) {
  uint64_t key = 1469598103934665603ull;
  key = hash_bytes(key, "network", 7);
  key = hash_bytes(key, &mode, sizeof(mode));
  key = hash_bytes(key, &P.slice_sum, sizeof(P.slice_sum));
  key = hash_bytes(key, &P.nout, sizeof(P.nout));
  key = hash_bytes(key, &nt, sizeof(nt));
  for (int i = 0; i < nt; ++i) {
    key = hash_tensor(key, T[i]);
    key = hash_bytes(key, labels[i], sizeof(int32_t) * (size_t)T[i].rank);
  }
  key = hash_bytes(key, path, sizeof(int32_t) * 2 * (size_t)nsteps);
  key = hash_bytes(key, &nsliced, sizeof(nsliced));
  key = hash_bytes(key, sliced, sizeof(int32_t) * (size_t)nsliced);
  return key;
}

static uint64_t net_key_call(uint64_t key, void* ws, double* amp_dev, double* slices_dev,
                             hipStream_t s) {
  key = hash_bytes(key, &ws, sizeof(ws));
  key = hash_bytes(key, &amp_dev, sizeof(amp_dev));
  key = hash_bytes(key, &slices_dev, sizeof(slices_dev));
  key = hash_bytes(key, &s, sizeof(s));
  const uint64_t tv = tune_version();
  return hash_bytes(key, &tv, sizeof(tv));
}

// Run a planned network (the plan matches these arguments).  base_key: the
// call's net_key_base when the caller has it.
static rn_status run_planned(rn_ctx* h, const NetPlan& P, int32_t nt, const rn_tensor* T,
                             const int32_t* const* labels, int32_t nsteps, const int32_t* path,
                             int32_t nsliced, const int32_t* sliced, rn_mode mode, void* ws,
                             size_t ws_bytes, hipStream_t s, double* amp_dev,
                             double* slices_dev, const uint64_t* base_key) {
  rn_status st;
  if (P.slice_sum && slices_dev && nsliced > 0)
    return fail(RN_ERR_INVALID, "per-slice values do not exist in slice-sum mode");
  if ((int64_t)ws_bytes < P.ws_bytes || (P.ws_bytes > 0 && !ws))
    return fail(RN_ERR_WORKSPACE, "workspace smaller than planned (" +
                                      std::to_string(P.ws_bytes) + " bytes needed)");
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return fail(RN_ERR_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
  if (use_graphs(h, s)) {
    const uint64_t base =
        base_key ? *base_key
                 : net_key_base(P, mode, nt, T, labels, nsteps, path, nsliced, sliced);
    const uint64_t key = net_key_call(base, ws, amp_dev, slices_dev, s);
    bool done = false;
    if ((st = replay_graph(h, key, s, &done)) != RN_OK || done) return st;
    if (seen_before(h, key)) {
      std::vector<char> blob;
      LevelLaunches launches;
      build_net_tables(P, T, ws, blob, launches);
      tuned_tiles(h, P, launches);
      if ((int64_t)blob.size() > P.ws_bytes - P.table_off)
        return fail(RN_ERR_WORKSPACE, "network parameter table exceeds its planned bound");
      return capture_and_launch(h, key, blob, s, [&](hipStream_t cs, char* tab) {
        return enqueue_network(P, T, ws, cs, amp_dev, slices_dev, &h->prof, launches, tab);
      });
    }
  }
  std::vector<char> blob;
  LevelLaunches launches;
  build_net_tables(P, T, ws, blob, launches);
  tuned_tiles(h, P, launches);
  if ((int64_t)blob.size() > P.ws_bytes - P.table_off)
    return fail(RN_ERR_WORKSPACE, "network parameter table exceeds its planned bound");
  char* tab = static_cast<char*>(ws) + P.table_off;
  if ((st = upload_table(h, blob, tab, s)) != RN_OK) return st;
  return enqueue_network(P, T, ws, s, amp_dev, slices_dev, &h->prof, launches, tab);
}

}  // namespace rn

using namespace rn;

extern "C" {

rn_status rn_contract_network_plan(rn_handle h, int32_t nt, const rn_tensor* T,
                                   const int32_t* const* labels, int32_t nsteps,
                                   const int32_t* path, int32_t nsliced, const int32_t* sliced,
                                   rn_mode mode, size_t* ws_bytes, double* flops,
                                   int32_t* max_rank) {
  const NetOpts o = h ? h->net : NetOpts{};
  return network_plan_h(h, nt, T, labels, nsteps, path, nsliced, sliced, mode, o, ws_bytes, flops,
                        max_rank, nullptr);
}

rn_status rn_contract_network(rn_handle h, int32_t nt, const rn_tensor* T,
                              const int32_t* const* labels, int32_t nsteps, const int32_t* path,
                              int32_t nsliced, const int32_t* sliced, rn_mode mode, void* ws,
                              size_t ws_bytes, void* stream, double* amp_dev,
                              double* slices_dev) {
  if (!h) return fail(RN_ERR_INVALID, "null handle");
  return network_run(h, nt, T, labels, nsteps, path, nsliced, sliced, mode, h->net, ws, ws_bytes,
                     static_cast<hipStream_t>(stream), amp_dev, slices_dev);
}

// A prepared network call: descriptors copied, planned and hashed once.
struct rn_prepared_net {
  rn_ctx* h = nullptr;
  rn_mode mode = RN_FP64;
  std::vector<rn_tensor> T;
  std::vector<std::vector<int32_t>> lab;
  std::vector<const int32_t*> labp;
  std::vector<int32_t> path, sliced;
  std::shared_ptr<NetPlan> plan;
  uint64_t base_key = 0;
};

rn_status rn_network_prepare(rn_handle h, int32_t nt, const rn_tensor* T,
                             const int32_t* const* labels, int32_t nsteps, const int32_t* path,
                             int32_t nsliced, const int32_t* sliced, rn_mode mode,
                             rn_prepared* out, size_t* ws_bytes) {
  if (!h || !out) return fail(RN_ERR_INVALID, "null handle or output");
  *out = nullptr;
  if (nt < 1 || !T || !labels || nsteps < 0 || (nsteps > 0 && !path) || nsliced < 0 ||
      nsliced > RN_MAX_SLICED || (nsliced > 0 && !sliced))
    return fail(RN_ERR_INVALID, "bad network arguments");
  for (int j = 0; j < nt; ++j) {
    if (T[j].rank < 0 || T[j].rank > RN_MAX_RANK || (T[j].rank > 0 && !labels[j]))
      return fail(RN_ERR_INVALID, "bad tensor " + std::to_string(j));
    if (!T[j].data) return fail(RN_ERR_INVALID, "null tensor data");
  }
  auto p = std::make_unique<rn_prepared_net>();
  p->h = h;
  p->mode = mode;
  p->T.assign(T, T + nt);
  p->lab.resize(nt);
  p->labp.resize(nt);
  for (int j = 0; j < nt; ++j) {
    p->lab[j].assign(labels[j], labels[j] + std::max(0, T[j].rank));
    p->labp[j] = p->lab[j].data();
  }
  p->path.assign(path, path + 2 * (size_t)nsteps);
  p->sliced.assign(sliced, sliced + nsliced);
  rn_status st = cached_plan(h, nt, p->T.data(), p->labp.data(), nsteps, p->path.data(),
                             nsliced, p->sliced.data(), mode, h->net, &p->plan);
  if (st != RN_OK) return st;
  p->base_key = net_key_base(*p->plan, mode, nt, p->T.data(), p->labp.data(), nsteps,
                             p->path.data(), nsliced, p->sliced.data());
  if (ws_bytes) *ws_bytes = (size_t)p->plan->ws_bytes;
  *out = p.release();
  return RN_OK;
}

rn_status rn_network_execute(rn_prepared p, void* ws, size_t ws_bytes, void* stream,
                             double* amp_dev, double* slices_dev) {
  if (!p) return fail(RN_ERR_INVALID, "null prepared call");
  if (!amp_dev) return fail(RN_ERR_INVALID, "null amplitude buffer");
  const int32_t nt = (int32_t)p->T.size();
  return run_planned(p->h, *p->plan, nt, p->T.data(), p->labp.data(),
                     (int32_t)(p->path.size() / 2), p->path.data(), (int32_t)p->sliced.size(),
                     p->sliced.data(), p->mode, ws, ws_bytes, static_cast<hipStream_t>(stream),
                     amp_dev, slices_dev, &p->base_key);
}

rn_status rn_network_release(rn_prepared p) {
  delete p;
  return RN_OK;
}

}  // extern "C"
