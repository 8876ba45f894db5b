// Host-side sanitizer run of the library's planner (test infrastructure):
// the plan entry points of the C ABI -- block tensordot plan, pair lists,
// footprints, streamed plan, batch plan and network plan -- on seeded random
// shapes and grids (dims 1, 2 and 4; mismatched contracted grids), ranks up
// to 64, and invalid arguments, with the host sources built with
// -fsanitize=address,undefined.  No device is touched: every call passes a
// null handle, and the network tensors a dummy data address no plan reads.
// Exits nonzero on an unexpected status; the sanitizers abort on any
// out-of-bounds access or undefined behaviour.
#include <cstdint>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/rn.h"

static uint64_t g_state = 777;
static uint64_t next_u64() {
  g_state += 0x9E3779B97F4A7C15ULL;
  uint64_t z = g_state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static int below(int n) { return (int)(next_u64() % (uint64_t)n); }

#define CHECK(c)                                                    \
  do {                                                              \
    if (!(c)) {                                                     \
      std::fprintf(stderr, "check failed line %d: %s (%s)\n", __LINE__, #c, \
                   rn_last_error());                                \
      return 1;                                                     \
    }                                                               \
  } while (0)

static void shuffle(std::vector<int32_t>& v) {
  for (int i = (int)v.size() - 1; i > 0; --i) std::swap(v[i], v[below(i + 1)]);
}

struct Case {
  rn_tensor A{}, B{};
  std::vector<int32_t> axA, axB;
};

static Case random_case(int max_rank) {
  Case c;
  int rA = below(max_rank + 1), rB = below(max_rank + 1);
  int k = below(std::min(rA, rB) + 1);
  std::vector<int32_t> pa(rA), pb(rB);
  for (int i = 0; i < rA; ++i) pa[i] = i;
  for (int i = 0; i < rB; ++i) pb[i] = i;
  shuffle(pa);
  shuffle(pb);
  c.A.rank = rA;
  c.B.rank = rB;
  c.A.dtype = c.B.dtype = RN_C64;
  const int64_t dimset[3] = {1, 2, 4};
  for (int i = 0; i < rA; ++i) c.A.dims[i] = dimset[below(3)];
  for (int i = 0; i < rB; ++i) c.B.dims[i] = dimset[below(3)];
  for (int i = 0; i < k; ++i) {
    c.axA.push_back(pa[i]);
    c.axB.push_back(pb[i]);
    c.B.dims[pb[i]] = c.A.dims[pa[i]];
  }
  for (int i = 0; i < rA; ++i) c.A.grid[i] = (int32_t)(c.A.dims[i] >> below(3 > c.A.dims[i] ? 1 : 3));
  for (int i = 0; i < rB; ++i) c.B.grid[i] = (int32_t)(c.B.dims[i] >> below(3 > c.B.dims[i] ? 1 : 3));
  for (int i = 0; i < rA; ++i) if (c.A.grid[i] < 1) c.A.grid[i] = 1;
  for (int i = 0; i < rB; ++i) if (c.B.grid[i] < 1) c.B.grid[i] = 1;
  return c;
}

static int tensordot_cases() {
  for (int t = 0; t < 3000; ++t) {
    Case c = random_case(t % 3 == 0 ? 64 : 12);
    int64_t abits = 0, bbits = 0, kbits = 0;  // index bits of A, B and the contraction
    for (int i = 0; i < c.A.rank; ++i) abits += __builtin_ctzll((uint64_t)c.A.dims[i]);
    for (int i = 0; i < c.B.rank; ++i) bbits += __builtin_ctzll((uint64_t)c.B.dims[i]);
    for (size_t i = 0; i < c.axA.size(); ++i) kbits += __builtin_ctzll((uint64_t)c.A.dims[c.axA[i]]);
    const int64_t bits = std::max(std::max(abits, bbits), abits + bbits - 2 * kbits);
    const int k = (int)c.axA.size();
    const rn_mode mode = (rn_mode)below(4);
    c.A.dtype = c.B.dtype = mode == RN_FP64 ? RN_C128 : RN_C64;
    rn_tensor C{};
    size_t ws = 0;
    double fl = 0;
    rn_status st = rn_block_tensordot_plan(nullptr, &c.A, &c.B, k, c.axA.data(), c.axB.data(),
                                           mode, &C, &ws, &fl);
    if (bits > 40) {
      CHECK(st == RN_ERR_UNSUPPORTED || st == RN_OK);
      continue;
    }
    CHECK(st == RN_OK);
    int64_t nblk = 1;
    for (int j = 0; j < C.rank; ++j) nblk *= C.grid[j];
    int64_t np = 0;
    for (int64_t b = 0; b < nblk && b < 4; ++b) {
      CHECK(rn_block_pairs(nullptr, &c.A, &c.B, k, c.axA.data(), c.axB.data(), b, nullptr, 0,
                           &np) == RN_OK);
      std::vector<int64_t> pairs(2 * (size_t)std::min<int64_t>(np, 1 << 12) + 2);
      CHECK(rn_block_pairs(nullptr, &c.A, &c.B, k, c.axA.data(), c.axB.data(), b, pairs.data(),
                           std::min<int64_t>(np, 1 << 12), &np) == RN_OK);
    }
    CHECK(rn_block_pairs(nullptr, &c.A, &c.B, k, c.axA.data(), c.axB.data(), nblk, nullptr, 0,
                         &np) == RN_ERR_INVALID);
    double e1 = 0, e2 = 0;
    CHECK(rn_block_footprint(&c.A, &c.B, k, c.axA.data(), c.axB.data(), &e1, &e2) == RN_OK);
    CHECK(e1 >= e2);
    double h2d = 0;
    st = rn_block_tensordot_streamed_plan(nullptr, &c.A, &c.B, k, c.axA.data(), c.axB.data(),
                                          mode, &C, &ws, &fl, &h2d);
    CHECK(st == RN_OK || st == RN_ERR_UNSUPPORTED);
    // Invalid variants: a repeated axis, an axis out of range, a grid that
    // does not divide its dim, a mode/dtype mismatch.
    if (k >= 2) {
      std::vector<int32_t> bad = c.axA;
      bad[1] = bad[0];
      CHECK(rn_block_tensordot_plan(nullptr, &c.A, &c.B, k, bad.data(), c.axB.data(), mode,
                                    &C, &ws, &fl) != RN_OK);
    }
    if (k >= 1) {
      std::vector<int32_t> bad = c.axA;
      bad[0] = c.A.rank;
      CHECK(rn_block_tensordot_plan(nullptr, &c.A, &c.B, k, bad.data(), c.axB.data(), mode,
                                    &C, &ws, &fl) == RN_ERR_INVALID);
    }
    if (c.A.rank >= 1) {
      rn_tensor A2 = c.A;
      A2.grid[0] = (int32_t)A2.dims[0] * 2;
      CHECK(rn_block_tensordot_plan(nullptr, &A2, &c.B, k, c.axA.data(), c.axB.data(), mode,
                                    &C, &ws, &fl) != RN_OK);
    }
    rn_tensor A3 = c.A;
    A3.dtype = mode == RN_FP64 ? RN_C64 : RN_C128;
    CHECK(rn_block_tensordot_plan(nullptr, &A3, &c.B, k, c.axA.data(), c.axB.data(), mode, &C,
                                  &ws, &fl) == RN_ERR_INVALID);
  }
  CHECK(rn_block_tensordot_plan(nullptr, nullptr, nullptr, 0, nullptr, nullptr, RN_FP64, nullptr,
                                nullptr, nullptr) == RN_ERR_INVALID);
  return 0;
}

static int batch_cases() {
  for (int t = 0; t < 60; ++t) {
    const int n = below(40);
    std::vector<Case> cs;
    while ((int)cs.size() < n) {
      Case c = random_case(10);
      int64_t bits = 0;
      for (int i = 0; i < c.A.rank; ++i) bits += __builtin_ctzll((uint64_t)c.A.dims[i]);
      for (int i = 0; i < c.B.rank; ++i) bits += __builtin_ctzll((uint64_t)c.B.dims[i]);
      if (bits > 30) continue;
      cs.push_back(c);
    }
    std::vector<rn_tensor> A(n + 1), B(n + 1), C(n + 1);
    std::vector<int32_t> ks(n + 1);
    std::vector<const int32_t*> pa(n + 1), pb(n + 1);
    for (int i = 0; i < n; ++i) {
      A[i] = cs[i].A;
      B[i] = cs[i].B;
      ks[i] = (int32_t)cs[i].axA.size();
      pa[i] = cs[i].axA.data();
      pb[i] = cs[i].axB.data();
    }
    size_t ws = 0;
    double fl = 0;
    const rn_mode mode = (rn_mode)(1 + below(3));
    CHECK(rn_block_tensordot_batch_plan(nullptr, n, A.data(), B.data(), ks.data(), pa.data(),
                                        pb.data(), mode, C.data(), &ws, &fl) == RN_OK);
    CHECK(n > 0 || ws == 0);
  }
  return 0;
}

static int network_cases() {
  // A random closed network: ring of nt rank-3 tensors plus chords; each
  // tensor's labels come from bonds it shares.  Path: contract in order.
  for (int t = 0; t < 200; ++t) {
    const int nt = 3 + below(12);
    std::vector<std::vector<int32_t>> labels(nt);
    int next_label = 0;
    for (int i = 0; i < nt; ++i) {  // ring bonds
      labels[i].push_back(next_label);
      labels[(i + 1) % nt].push_back(next_label);
      ++next_label;
    }
    for (int c = 0; c < nt; ++c) {  // chords
      int a = below(nt), b = below(nt);
      if (a == b || labels[a].size() > 5 || labels[b].size() > 5) continue;
      labels[a].push_back(next_label);
      labels[b].push_back(next_label);
      ++next_label;
    }
    std::vector<rn_tensor> T(nt);
    std::vector<const int32_t*> lp(nt);
    for (int i = 0; i < nt; ++i) {
      T[i] = rn_tensor{};
      T[i].rank = (int32_t)labels[i].size();
      T[i].dtype = RN_C64;
      T[i].data = reinterpret_cast<void*>(uintptr_t(0x1000));  // never dereferenced by a plan
      for (int j = 0; j < T[i].rank; ++j) {
        T[i].dims[j] = 2;
        T[i].grid[j] = 1;
      }
      lp[i] = labels[i].data();
    }
    std::vector<int32_t> path;
    int cur = 0;
    for (int s = 1; s < nt; ++s) {
      path.push_back(cur);
      path.push_back(s);
      cur = nt + s - 1;
    }
    std::vector<int32_t> sliced;
    for (int s = 0; s < below(4) && s < next_label; ++s) sliced.push_back(s);
    size_t ws = 0;
    double fl = 0;
    int32_t mr = 0;
    rn_status st = rn_contract_network_plan(nullptr, nt, T.data(), lp.data(), nt - 1, path.data(),
                                            (int32_t)sliced.size(), sliced.data(), RN_FP32_4M,
                                            &ws, &fl, &mr);
    CHECK(st == RN_OK || st == RN_ERR_UNSUPPORTED);
    // A path that uses an operand twice, and an unknown sliced label.
    std::vector<int32_t> bad = path;
    bad[2] = bad[0];
    CHECK(rn_contract_network_plan(nullptr, nt, T.data(), lp.data(), nt - 1, bad.data(), 0,
                                   nullptr, RN_FP32_4M, &ws, &fl, &mr) != RN_OK);
    int32_t unknown = next_label + 5;
    CHECK(rn_contract_network_plan(nullptr, nt, T.data(), lp.data(), nt - 1, path.data(), 1,
                                   &unknown, RN_FP32_4M, &ws, &fl, &mr) != RN_OK);
  }
  return 0;
}

int main() {
  if (tensordot_cases() || batch_cases() || network_cases()) return 1;
  std::printf("planner sanitizer run: ok\n");
  return 0;
}
