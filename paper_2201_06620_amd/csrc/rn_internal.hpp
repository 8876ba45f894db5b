// Internal declarations of the block tensordot library (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/rn.h"

namespace rn {

// Thread-local error message behind rn_last_error().
void set_error(const std::string& msg);
rn_status fail(rn_status s, const std::string& msg);

// ---------------------------------------------------------------------------
// Bit-level view of tensors.  Every dim is 2^a, every grid count 2^c, so a
// tensor of R = sum(a_j) index bits is a 2^R array and every relayout is a
// permutation of the R bits of the linear element index.  Logical bit
// (axis j, t) is bit t of coordinate x_j; its physical position in the
// block-major buffer is given by phys_pos().
// ---------------------------------------------------------------------------
struct Layout {
  int rank = 0;
  int abits[RN_MAX_RANK] = {0};  // log2 dims
  int cbits[RN_MAX_RANK] = {0};  // log2 grid
  int total = 0;                 // sum of abits
  int phys_pos(int axis, int t) const;
};

rn_status make_layout(const rn_tensor* T, const char* name, Layout* L);

// A bit permutation: output bit o (LSB = 0) reads input bit src[o].
// Input bits not listed are fixed by `in_base` (slice projections).
struct BitPerm {
  int nbits = 0;
  int8_t src[64] = {0};
  bool identity() const;
};

// Two-level index map for one GEMM dimension:
//   off(x) = (x >> shift) * hi + (x & ((1 << shift) - 1)) * lo   (elements).
struct Map2 {
  int shift = 62;
  int64_t hi = 0;
  int64_t lo = 1;
};

// Plan of one block tensordot (a GEMM C[M x N] = A[M x K] * B[N x K]^T).
struct TdPlan {
  rn_mode mode = RN_FP64;
  int es = 16;                      // bytes per complex element of A, B and C
  int mbits = 0, nbits = 0, kbits = 0;
  int64_t M = 1, N = 1, K = 1;
  int Mb = 0, Mi = 0, Nb = 0, Ni = 0;  // block / inner bit counts of C's layout
  int pairbits = 0;                     // contracted block bits on the refined grid
  BitPerm permA, permB;                 // storage -> GEMM layout
  bool permuteA = false, permuteB = false;
  Map2 crow, ccol;                      // GEMM (row, col) -> C offset
  // Derived C descriptor.
  int crank = 0;
  int64_t cdims[RN_MAX_RANK];
  int32_t cgrid[RN_MAX_RANK];
  // Refined-grid bookkeeping for pair lists.
  int k = 0;
  int32_t axA[RN_MAX_RANK], axB[RN_MAX_RANK];
  int pair_cbits[RN_MAX_RANK];  // refined contracted grid bits, pair order
  // Workspace sub-buffers (byte offsets; -1 when unused).
  int64_t off_a = -1, off_b = -1, off_a2 = -1, off_b2 = -1, off_part = -1;
  bool planar_ok = false;  // workspace holds planar or interleaved split-BF16 operands
  int splitk = 1;
  size_t ws_bytes = 0;
  double flops = 0;
};

// Network options of a handle (defaults when planning without one).
struct NetOpts {
  bool slice_sum = false;       // sum sliced bonds where they are contracted
  int batch_bits = 64;          // sliced bonds batched per pass (the rest loop)
  int64_t footprint = 0;        // workspace cap in bytes; 0: none
};

// Reduction-strategy options of a handle (defaults when planning without one).
struct SplitPolicy {
  int64_t pair_threshold = 0;                 // 0: heuristic
  int64_t footprint = int64_t(1) << 30;       // bytes of partial sums
};

// planar_ok: the call may stage split-BF16 operands in the planar Gauss form
// (six bf16 planes in one array, 12 bytes per complex instead of 8) or
// row-interleaved (hi and lo per 16 k of a row in one array): the single
// block tensordot entry points; their workspace is sized for it (the packed
// form's hi and lo arrays then sit inside that region).
rn_status plan_tensordot(const rn_tensor* A, const rn_tensor* B, int32_t k,
                         const int32_t* axesA, const int32_t* axesB, rn_mode mode,
                         TdPlan* P, bool allow_splitk = true,
                         const SplitPolicy* policy = nullptr, bool planar_ok = false);
rn_status check_c(const TdPlan& P, const rn_tensor* C);

// Optional per-launch event timing (rn_profile_enable).
struct Profiler {
  bool on = false;
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  // Record the start event of a launch of class `cls`; returns its index or -1.
  int begin(int cls, hipStream_t s);
  void end(int idx, hipStream_t s);
};

// ---------------------------------------------------------------------------
// Kernel launchers (kernels.hip).
// ---------------------------------------------------------------------------
struct PermLaunch {
  const void* in = nullptr;
  void* out = nullptr;
  void* out2 = nullptr;      // lo part for the bfloat16 split
  int64_t in_base = 0;       // element offset added to every input index
  BitPerm perm;              // output bit -> input bit
  int in_es = 8;             // input element bytes (8 or 16)
  int kind = 0;              // 0 copy, 1 split complex64 -> bf16 hi/lo (packed
                             // pairs), 2 planar-group split (Gauss form),
                             // 3 row-interleaved split (hi and lo per 16 k)
  int64_t gw = 0;            // kind 2: k per plane group, min(16, K)
  // The input holds nsum split-K partials sstride elements apart: each
  // element read is their sum in ascending order.
  int nsum = 1;
  int64_t sstride = 0;
};
hipError_t launch_permute(const PermLaunch& p, hipStream_t s);

// Batched GEMM over slices: batch index b has `nbb` bits; operand X is
// offset by sum over set bits i of b of X_bstride[i] elements.
struct GemmLaunch {
  rn_mode mode = RN_FP64;
  const void* A = nullptr;   // M x K, row stride lda (complex elements)
  const void* B = nullptr;   // N x K, row stride ldb
  const void* A2 = nullptr;  // bf16 lo parts (RN_BF16X3)
  const void* B2 = nullptr;
  void* C = nullptr;
  int64_t M = 0, N = 0, K = 0, lda = 0, ldb = 0;
  Map2 crow, ccol;
  int nbb = 0;
  int64_t a_bstride[RN_MAX_SLICED] = {0}, b_bstride[RN_MAX_SLICED] = {0},
          c_bstride[RN_MAX_SLICED] = {0};
  int splitk = 1;
  void* partial = nullptr;   // splitk > 1: [splitk][batch][M][N] complex, fp32/fp64
  int tile = -1;             // tile config index, -1 = choose
  bool planar = false;       // operands in planar Gauss form (permute kind 2;
                             // tile must be a planar one)
  bool interleaved = false;  // split-BF16 operands from permute kind 3: per row,
                             // per 16 k, 16 packed hi words then 16 lo words
                             // (A2 = A + 16 words, lda = 2K); the tile must be
                             // one of gemm_tile_interleaved, K a multiple of 16
  bool partial_only = false; // splitk > 1: leave the partials, launch no reduction
};
hipError_t launch_gemm(const GemmLaunch& g, hipStream_t s, Profiler* prof = nullptr);
int gemm_tile_count(rn_mode mode);
// Whether tile index `tile` may run a problem with an M x N output (the
// skinny kernel needs min(M, N) <= 8; launch_gemm falls back to the default).
bool gemm_tile_valid(rn_mode mode, int tile, int64_t M, int64_t N);
int gemm_default_tile(rn_mode mode, int64_t M, int64_t N, int64_t K);
// Whether tile index `tile` can split K across workgroups (the MFMA tiles;
// not the one-thread or skinny kernels).
bool gemm_tile_splits(rn_mode mode, int tile);
// Tiles that read planar operands (split-BF16 Gauss form: hi and lo planes
// re, im, re + im in groups of min(16, K) k, from permute kind 2, 12 bytes
// per complex in one array); only the single block tensordot stages
// operands that way.
bool gemm_tile_planar(rn_mode mode, int tile);
// Tiles that can also read row-interleaved split-BF16 operands (permute
// kind 3): per 16 k of a row one 128-byte line holds the hi and lo parts, so
// a K stage fetches whole lines instead of two half lines from two arrays.
// Only the single block tensordot stages operands that way.
bool gemm_tile_interleaved(rn_mode mode, int tile);
// The planar tile a single block tensordot uses by default for this shape,
// or -1.
int gemm_planar_default(rn_mode mode, int64_t M, int64_t N, int64_t K);

// Grouped launches: many problems (or permutations) in one kernel launch.
// The host builds a parameter table plus a prefix sum of workgroups per
// problem; the table is copied to device memory before the launch.
struct GroupedLaunch {
  int n = 0;
  int kind = 0, es = 8;       // permutes
  rn_mode mode = RN_FP64;     // GEMMs
  int tile = 0;
  int blocks = 0;
  size_t lds = 0;
  size_t params_off = 0, prefix_off = 0;
  size_t jobs_off = 0, tiny_off = 0, maps_off = 0;  // small steps
};
size_t grouped_perm_build(const std::vector<PermLaunch>& jobs, std::vector<char>& table,
                          GroupedLaunch& G);
hipError_t launch_permute_grouped(const GroupedLaunch& G, const void* table_dev, hipStream_t s);
size_t grouped_table_bound(rn_mode mode, int n);

// One small contraction step evaluated directly from the stored layouts
// (no relayout): C[b][m][n] = sum_k A[a_off(b) + amap(m, k)] * B[...], where
// amap scatters the bits of m and k to their physical positions in A.
struct DirectStep {
  const void* A = nullptr;
  const void* B = nullptr;
  void* C = nullptr;
  int64_t M = 1, N = 1, K = 1;
  int mbits = 0, nbits = 0, kbits = 0, nbb = 0;
  int blocks_per_batch = 1;
  int8_t am[40] = {0}, ak[40] = {0}, bn[40] = {0}, bk[40] = {0};
  int64_t a_bs[RN_MAX_SLICED] = {0}, b_bs[RN_MAX_SLICED] = {0};
  // Projection per pass: 1 + stored bit of the sliced bond the pass fixes
  // (slice index i of the fixed ones), 0 when the operand does not carry it.
  int8_t a_pp[RN_MAX_SLICED] = {0}, b_pp[RN_MAX_SLICED] = {0};
};
// A step of a subtree of tiny steps that one workgroup runs whole, height
// by height (height 1: every operand comes from outside the subtree).  Its
// index maps are tabulated on the host: in the job's map area from word
// `map` on, amap[M] (element offset in A of row m), bmap[N], koa[K], kob[K],
// abat[2^nbb], bbat[2^nbb] (offsets of slice batch b), all int32.  Each
// height also has a byte table in the map area, from word `sel` of its first
// step: entry t is the job index of the step that output t of the height
// belongs to.
struct TinyStep {
  const void* A = nullptr;
  const void* B = nullptr;
  void* C = nullptr;
  int32_t mbits = 0, nbits = 0, K = 1, nbb = 0;
  int32_t ooff = 0;       // first output of the step among its height's outputs
  int32_t run_end = 0;    // first step of a height: index past that height's steps
  int32_t run_total = 0;  // first step of a height: outputs of that height
  int32_t map = 0;        // word offset of its maps in the job's map area
  int32_t sel = 0;        // first step of a height: word offset of its byte table
  int32_t pad0 = 0;
  int8_t a_pp[RN_MAX_SLICED] = {0}, b_pp[RN_MAX_SLICED] = {0};
  int8_t pad[2] = {0, 0};
};
// Map words of a tiny step with these shapes, with its share of its
// height's byte table (rounded up by a word).
inline int64_t tiny_map_words(int64_t M, int64_t N, int64_t K, int nbb) {
  return 1 + M + N + 2 * K + 2 * (int64_t(1) << nbb) + ((M * N) << nbb) / 4;
}
// A job of a grouped small-step launch.  count == 1: entry `first` of the
// step list, one step whose outputs are spread over workgroups (256 per
// workgroup and slice batch).  count > 1: entries first .. first+count-1 of
// the tiny-step list, sorted by height, with their maps at words map_first
// .. map_first+map_words-1 of the map list: a subtree that one workgroup runs
// height by height with a workgroup barrier in between, so a chain of
// dependent tiny steps costs barriers instead of launches.
struct DirectJob {
  int32_t count, first, map_first, map_words;
};
constexpr int64_t kDirectMaxK = 4096;
// Subtrees: at most kClusterMaxSteps steps and kClusterMapWords map words
// (both held in LDS), at most kClusterMaxWidth steps per height; a step
// joins one only if its outputs (all slice batches) take at most
// kClusterStepRounds rounds of the workgroup's 256 lanes times groups of 8
// K terms (each round costs a memory round trip in one workgroup, while a
// step of its own spreads over many) and at most kClusterStepWork
// multiply-adds; a subtree holds at most kClusterWork multiply-adds.
constexpr int kClusterMaxSteps = 64;
constexpr int kClusterMaxWidth = 32;
constexpr int kClusterMapWords = 8192;
constexpr int64_t kClusterStepRounds = 4;
constexpr int64_t kClusterStepWork = int64_t(1) << 16;
constexpr int64_t kClusterWork = int64_t(1) << 18;
// Table bytes of a grouped small-step launch over n steps (any job split)
// whose subtrees hold map_words map words.
size_t grouped_direct_bound(int n, int64_t map_words);
// Bytes of the table of one grouped permute of n jobs.
size_t grouped_perm_bound(int n);
size_t grouped_direct_build(const std::vector<DirectStep>& steps,
                            const std::vector<TinyStep>& tiny, const std::vector<int32_t>& maps,
                            const std::vector<DirectJob>& jobs, rn_mode mode,
                            std::vector<char>& table, GroupedLaunch& G);
// pass / nout: the pass index and the number of sliced bonds a pass fixes
// (bit nout-1-i of pass is the value of fixed bond i).
hipError_t launch_direct_grouped(const GroupedLaunch& G, const void* table_dev, int64_t pass,
                                 int nout, hipStream_t s);
size_t grouped_gemm_build(const std::vector<GemmLaunch>& probs, int tile,
                          std::vector<char>& table, GroupedLaunch& G);
hipError_t launch_gemm_grouped(const GroupedLaunch& G, const void* table_dev, hipStream_t s);
size_t grouped_reduce_build(const std::vector<GemmLaunch>& probs, std::vector<char>& table,
                            GroupedLaunch& G);
hipError_t launch_reduce_grouped(const GroupedLaunch& G, const void* table_dev, hipStream_t s);
int choose_splitk(rn_mode mode, int64_t M, int64_t N, int64_t K, int64_t batch);

rn_status enqueue_tensordot(const TdPlan& P, const rn_tensor* A, const rn_tensor* B,
                            const rn_tensor* C, void* ws, hipStream_t s, Profiler* prof,
                            int tile = -1);

// Looks up the device address of the no-alloc scratch array on `device`
// (current) once per device; rn_create calls it.
rn_status noalloc_init(int device);

hipError_t launch_norm2(const void* x, int64_t n, int dtype, double* out, double* scratch,
                        hipStream_t s);
hipError_t launch_sum_c128(const double* vals, int64_t n, double* out, hipStream_t s);
hipError_t launch_add_into(void* c, const void* p, int64_t n, int es, hipStream_t s);
hipError_t launch_sum_slices(const void* vals, int es, int64_t n, double* out_sum,
                             double* out_each, hipStream_t s);

}  // namespace rn

// Captured launch sequences, replayed when a call repeats with identical
// arguments.  `pinned` holds the parameter tables the graph's copy node reads.
struct GraphEntry {
  uint64_t key = 0;
  hipGraphExec_t exec = nullptr;
  void* pinned = nullptr;  // staging of the parameter table
  void* table = nullptr;   // device copy of the table the graph's kernels read
  uint64_t last_use = 0;
};

// Opaque handle.
struct rn_ctx {
  int device = 0;
  void* red_scratch = nullptr;  // 4096 doubles of device memory for reductions
  rn::Profiler prof;
  // Tile choices from the autotuner: (mode, log2 M, log2 N, log2 K) -> tile.
  std::map<std::tuple<int, int, int, int>, int> tune;
  // Milliseconds per launch of every tile shape timed for that key.
  std::map<std::tuple<int, int, int, int>, std::vector<float>> tune_ms;
  // Batch tile groups timed by the autotuner (seconds, one serialized run of
  // the group's permute and GEMM), by group signature; the batch's stream
  // assignment uses them in place of its estimate.
  std::map<uint64_t, double> group_s;
  std::string tune_path;
  // Pinned staging for parameter tables of direct (not captured) launches.
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  hipEvent_t pinned_done = nullptr;
  bool graphs_enabled = true;
  rn::SplitPolicy split;
  rn::NetOpts net;
  // Batch: extra streams on which tile groups of one batch run side by side
  // (fork/join by events; default priority), created on first use.
  hipStream_t aux_streams[3] = {nullptr, nullptr, nullptr};
  hipEvent_t aux_fork = nullptr;
  hipEvent_t aux_join[3] = {nullptr, nullptr, nullptr};
  // Streamed contraction: host-to-device copy stream and its events.
  hipStream_t copy_stream = nullptr;
  hipEvent_t copy_ev[9] = {nullptr};
  std::vector<GraphEntry> graphs;
  std::vector<uint64_t> seen;  // keys run once directly; a repeat is captured
  // Network plans by exact structural signature (shapes, labels, path,
  // sliced labels, mode, options); most recently used last.
  std::vector<std::pair<std::vector<int64_t>, std::shared_ptr<void>>> net_plans;
  uint64_t use_clock = 0;
};

namespace rn {
int tuned_tile(const rn_ctx* h, rn_mode mode, int mbits, int nbits, int kbits);
// Bumped whenever a handle's tune table changes (graph keys include it).
uint64_t tune_version();
// Stage `bytes` of host table data and copy them to `dev` on stream s.
rn_status upload_table(rn_ctx* h, const std::vector<char>& table, void* dev, hipStream_t s);
uint64_t hash_bytes(uint64_t h, const void* p, size_t n);
uint64_t hash_tensor(uint64_t x, const rn_tensor& t);
// Graph cache: replay_graph launches the graph stored under `key` if any
// (*done = true); capture_and_launch copies `table` once into device memory
// the entry owns (on stream s, before the capture), records
// enqueue(stream, that copy), stores and launches it: replays read the same
// copy, so a replay is the kernels alone.  use_graphs: graphs are enabled, the stream is not the null
// stream, not already capturing, and kernel timing is off.
bool use_graphs(const rn_ctx* h, hipStream_t s);
// Network plan and run under explicit options (the C entry points pass the
// handle's).  *batch_bits receives the batched-slice count the plan chose.
rn_status network_plan(int32_t nt, const rn_tensor* T, const int32_t* const* labels,
                       int32_t nsteps, const int32_t* path, int32_t nsliced,
                       const int32_t* sliced, rn_mode mode, const NetOpts& o, size_t* ws_bytes,
                       double* flops, int32_t* max_rank, int* batch_bits);
// Plan once, run later (the server plans at submission and runs on its
// worker thread): the plan is opaque to the caller.
rn_status network_plan_keep(int32_t nt, const rn_tensor* T, const int32_t* const* labels,
                            int32_t nsteps, const int32_t* path, int32_t nsliced,
                            const int32_t* sliced, rn_mode mode, const NetOpts& o,
                            std::shared_ptr<void>* plan, size_t* ws_bytes, double* flops,
                            int* batch_bits);
rn_status network_run_planned(rn_ctx* h, const std::shared_ptr<void>& plan, int32_t nt,
                              const rn_tensor* T, const int32_t* const* labels, int32_t nsteps,
                              const int32_t* path, int32_t nsliced, const int32_t* sliced,
                              rn_mode mode, void* ws, size_t ws_bytes, hipStream_t s,
                              double* amp_dev, double* slices_dev);
// As network_plan, through the plan cache of handle h (may be null).
rn_status network_plan_h(rn_ctx* h, int32_t nt, const rn_tensor* T, const int32_t* const* labels,
                         int32_t nsteps, const int32_t* path, int32_t nsliced,
                         const int32_t* sliced, rn_mode mode, const NetOpts& o,
                         size_t* ws_bytes, double* flops, int32_t* max_rank, int* batch_bits);
rn_status network_run(rn_ctx* h, int32_t nt, const rn_tensor* T, const int32_t* const* labels,
                      int32_t nsteps, const int32_t* path, int32_t nsliced,
                      const int32_t* sliced, rn_mode mode, const NetOpts& o, void* ws,
                      size_t ws_bytes, hipStream_t s, double* amp_dev, double* slices_dev);
rn_status replay_graph(rn_ctx* h, uint64_t key, hipStream_t s, bool* done);
// True when `key` was run before (directly); otherwise remembers it.
bool seen_before(rn_ctx* h, uint64_t key);
rn_status capture_and_launch(rn_ctx* h, uint64_t key, const std::vector<char>& table,
                             hipStream_t s,
                             const std::function<rn_status(hipStream_t, char*)>& enqueue);
}  // namespace rn
