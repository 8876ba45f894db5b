/*
 * rn.h - C ABI of the MI355X (gfx950) block tensor contraction library.
 *
 * A block tensor is a dense complex tensor split into a uniform grid of
 * equal sub-tensors ("blocks") along each axis; the paper's block tensor
 * algebra (Section II.C) contracts two such tensors pair of blocks by pair of
 * blocks and sums the partial blocks into the output blocks.  This library
 * runs that contraction on one GPU: an index permutation of each operand
 * into a GEMM-ready layout, one complex GEMM whose K loop walks the coupled
 * block pairs, and the reduction of the partials into C, all in HIP kernels.
 *
 * Conventions shared by every entry point:
 *   - Every dim and every grid count is a power of two (tensors of quantum
 *     circuits have dim 2; a dim 2^a is handled as a axes of dim 2 fused);
 *     other values give RN_ERR_UNSUPPORTED.
 *   - Element layout: complex values interleaved (re, im), row-major.
 *     A tensor whose grid is not all ones is stored block-major: blocks in
 *     row-major order of their block coordinates, each block contiguous and
 *     row-major inside.  Grid all ones is the plain dense layout.
 *   - Pairing follows tensordot: axesA[i] is contracted with axesB[i], and
 *     the output lists A's free axes in A's order, then B's free axes in B's
 *     order (the pairwise contraction formula, Section II.A).
 *   - When the two operands split a contracted pair of axes into different
 *     numbers of blocks, both are viewed on the finer grid (the common
 *     refinement), which does not change the result.  C's grid is A's
 *     free-axis grid followed by B's free-axis grid.
 *   - Ownership: the caller allocates and owns every device buffer (tensor
 *     data, workspace, results) and keeps it alive until the stream has
 *     finished the enqueued work.  The library never frees caller memory.
 *   - Asynchrony: compute calls enqueue kernels on `stream` (a hipStream_t,
 *     NULL for the default stream) and return; they do not synchronise.
 *   - Errors: every call returns rn_status and never throws, and
 *     rn_last_error() gives a message for the calling thread.  Argument
 *     errors are found before any launch, so nothing has been enqueued.
 *     RN_ERR_HIP reports a HIP call that failed, e.g. a launch whose grid
 *     exceeds HIP's 2^32 work-items per dimension (the library refuses such
 *     a launch instead of wrapping its size); kernels of the same call
 *     enqueued before it may have run, and the output is then undefined.
 *   - Modes and dtypes: RN_FP64 computes in double with RN_C128 tensors;
 *     RN_FP32_4M, RN_FP32_3M and RN_BF16X3 take RN_C64 tensors and
 *     accumulate in float.
 */
#ifndef RN_H
#define RN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RN_MAX_RANK 64
#define RN_MAX_SLICED 15
/* Bytes of the fixed device scratch array of rn_block_tensordot_noalloc. */
#define RN_NOALLOC_SCRATCH_BYTES ((size_t)1 << 26)

typedef enum {
  RN_OK = 0,
  RN_ERR_INVALID = 1,     /* null pointer, bad rank/axis/label, mode-dtype mismatch */
  RN_ERR_SHAPE = 2,       /* paired dims differ, or C's dims are not the derived ones */
  RN_ERR_GRID = 3,        /* a grid count does not divide its dim, or C's grid differs */
  RN_ERR_WORKSPACE = 4,   /* workspace smaller than the plan requires */
  RN_ERR_OOM = 5,         /* a request can never fit the memory budget */
  RN_ERR_HIP = 6,         /* a HIP runtime call failed */
  RN_ERR_UNSUPPORTED = 7  /* dims or grids that are not powers of two, sizes over limits */
} rn_status;

typedef enum { RN_C64 = 1, RN_C128 = 2 } rn_dtype;

/* Arithmetic of the per-pair complex GEMM:
 *   RN_FP64    complex128, 4 real products per complex product, FP64 MFMA
 *              (a tune entry, from rn_autotune_batch or a tune file, may select
 *              the FP64 Gauss tile instead: 3 real products, same tolerance);
 *   RN_FP32_4M complex64, 4 real products, FP32 MFMA, FP32 accumulation;
 *   RN_FP32_3M complex64, 3 real products (Gauss), FP32 MFMA;
 *   RN_BF16X3  complex64 operands split as x = hi + lo (both bfloat16),
 *              products lo*hi + hi*lo + hi*hi on BF16 MFMA, FP32 accumulation. */
typedef enum { RN_FP64 = 0, RN_FP32_4M = 1, RN_FP32_3M = 2, RN_BF16X3 = 3 } rn_mode;

typedef struct rn_ctx* rn_handle;

/* Tensor descriptor.  data is a device pointer owned by the caller. */
typedef struct {
  int32_t rank;                /* 0 .. RN_MAX_RANK */
  int32_t dtype;               /* rn_dtype */
  int64_t dims[RN_MAX_RANK];   /* powers of two, >= 1 */
  int32_t grid[RN_MAX_RANK];   /* blocks per axis; power of two dividing dims[j] */
  void* data;
} rn_tensor;

/* Library context bound to one HIP device.  Holds plan caches only. */
rn_status rn_create(rn_handle* h, int device);
rn_status rn_destroy(rn_handle h);
const char* rn_status_str(rn_status s);
const char* rn_last_error(void);

/* ------------------------------------------------------------------------
 * Block tensordot (Section II.C, the four steps; tensordot semantics of the
 * commutative task in Section III).
 *
 * plan: validates A, B, k, axes and mode, and fills C's rank, dims, grid
 * and dtype (C->data is left untouched), the workspace the call needs, and
 * the useful flop count 8*M*N*K (M, N, K = products of A-free, B-free and
 * contracted dims).  Any output pointer may be NULL.
 *
 * rn_block_tensordot: C = sum over coupled block pairs of A_blk . B_blk,
 * written block-major into C->data (which must not alias A or B).  C must
 * carry exactly the rank, dims and grid the plan derives.  ws must be a
 * device buffer of at least the planned bytes (NULL allowed when 0).
 * ------------------------------------------------------------------------ */
rn_status rn_block_tensordot_plan(rn_handle h, const rn_tensor* A, const rn_tensor* B, int32_t k,
                                  const int32_t* axesA, const int32_t* axesB, rn_mode mode,
                                  rn_tensor* C, size_t* ws_bytes, double* flops);
rn_status rn_block_tensordot(rn_handle h, const rn_tensor* A, const rn_tensor* B, int32_t k,
                             const int32_t* axesA, const int32_t* axesB, rn_tensor* C,
                             rn_mode mode, void* ws, size_t ws_bytes, void* stream);

/* Block tensordot for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same contraction, plan, kernels and results as rn_block_tensordot, but
 * its workspace is a fixed device array compiled into the library
 * (RN_NOALLOC_SCRATCH_BYTES; each GPU the library runs on holds one until the
 * process ends), so the call takes no ws argument and allocates nothing
 * (no hipMalloc, hipFree, memset, event or stream creation; no kernel timing
 * either).  A plan that needs more workspace than the array holds fails with
 * RN_ERR_WORKSPACE before anything is enqueued.  Every call on one GPU shares
 * that GPU's array: calls whose kernels may overlap on one device (several
 * streams, or several threads without ordering) race and give undefined
 * results.  Nothing in the array needs to start at zero: each call writes
 * every workspace byte it reads.  The handle must have been created on that
 * device (rn_create looks up the array's device address). */
rn_status rn_block_tensordot_noalloc(rn_handle h, const rn_tensor* A, const rn_tensor* B,
                                     int32_t k, const int32_t* axesA, const int32_t* axesB,
                                     rn_tensor* C, rn_mode mode, void* stream);

/* Streamed block tensordot, for operands larger than device memory: the
 * commutative reduction of Section IV.A (pairs loaded as needed, each
 * product added into its output block), with A->data and B->data in HOST
 * memory (block-major, as for rn_block_tensordot; allocate with
 * hipHostMalloc so the copies overlap compute) and C->data in device memory.
 * Output block rows run outermost, then the coupled pairs in ascending
 * order, then the output block columns: each A block is copied once, each
 * B block once per output row.  Copies run on a copy stream the handle
 * owns, compute on `stream`; the call returns once everything is queued,
 * and the caller must keep A and B alive and unchanged until `stream` has
 * reached that point.  Device memory: C plus the planned workspace (two
 * staging slots per operand block, the permuted blocks and one partial
 * output block).  Paired axes must have equal grids on A and B
 * (RN_ERR_UNSUPPORTED otherwise).  The plan reports the workspace, useful
 * flops and the host-to-device bytes the call will copy.  Calls on one
 * handle share its copy stream and must not be issued from several threads
 * at once. */
rn_status rn_block_tensordot_streamed_plan(rn_handle h, const rn_tensor* A, const rn_tensor* B,
                                           int32_t k, const int32_t* axesA,
                                           const int32_t* axesB, rn_mode mode, rn_tensor* C,
                                           size_t* ws_bytes, double* flops, double* h2d_bytes);
rn_status rn_block_tensordot_streamed(rn_handle h, const rn_tensor* A, const rn_tensor* B,
                                      int32_t k, const int32_t* axesA, const int32_t* axesB,
                                      rn_tensor* C, rn_mode mode, void* ws, size_t ws_bytes,
                                      void* stream);

/* Pair list of one output block (step 2 of Section II.C): for C block
 * `cblock` (row-major linear block index) writes up to `cap` pairs
 * (A block index, B block index) into `pairs`, a host array of 2*cap
 * int64 values (NULL: count only), each a row-major linear index into the
 * operand's own stored grid, in the order the GEMM K loop visits them
 * (ascending contracted block coordinates on the refined grid).  When a
 * stored block is finer-split by the refinement, the same stored block index
 * appears for each of its refined pieces.  *npairs receives the count. */
rn_status rn_block_pairs(rn_handle h, const rn_tensor* A, const rn_tensor* B, int32_t k,
                         const int32_t* axesA, const int32_t* axesB, int64_t cblock,
                         int64_t* pairs, int64_t cap, int64_t* npairs);

/* Memory models of Section IV.A in elements: sequential reduction
 * B_k k_b (m_b + n_b) + m_b n_b (Eq. 1) and one pair plus accumulator
 * k_b (m_b + n_b) + m_b n_b (Eq. 2), for the blocks of this contraction on
 * the refined grid.  Host only; either output may be NULL. */
rn_status rn_block_footprint(const rn_tensor* A, const rn_tensor* B, int32_t k,
                             const int32_t* axesA, const int32_t* axesB, double* eq1_elems,
                             double* eq2_elems);

/* Many independent block tensordots in one call (same mode).  The paper runs
 * the block-pair contractions of a block tensordot (Section II.C) and the
 * copies of a sliced network (Section II.B) as independent tasks, and weighs
 * block size against per-task overhead (Section IV.B); here independent
 * problems share launches instead, so small ones do not each pay a launch.
 * Plans every
 * problem first (any invalid problem fails the whole call before anything is
 * enqueued).  The problems are grouped by GEMM tile shape; per group one
 * grouped launch relayouts the operands that need it and one grouped launch
 * contracts its problems (ordered by decreasing flops), the groups spread
 * over up to four streams joined back into `stream`.  Problems with few
 * output tiles and K >= 512 split K (partials in the workspace, summed in
 * ascending order by one grouped launch at the end), so results do not
 * depend on the other problems of the batch.  Per-problem parameters are
 * copied into the end of the workspace first.  ws_bytes from
 * rn_block_tensordot_batch_plan.  An empty batch (n = 0) is valid: it plans
 * to 0 bytes and 0 flops and enqueues nothing.  With graph replay on, a call identical to
 * an earlier captured one (descriptors, data pointers, axes, workspace
 * pointer and size, stream, tuning) replays its graph without planning
 * again; the earlier call was checked in full. */
rn_status rn_block_tensordot_batch_plan(rn_handle h, int32_t n, const rn_tensor* A,
                                        const rn_tensor* B, const int32_t* k,
                                        const int32_t* const* axesA,
                                        const int32_t* const* axesB, rn_mode mode, rn_tensor* C,
                                        size_t* ws_bytes, double* flops);
rn_status rn_block_tensordot_batch(rn_handle h, int32_t n, const rn_tensor* A,
                                   const rn_tensor* B, const int32_t* k,
                                   const int32_t* const* axesA, const int32_t* const* axesB,
                                   rn_tensor* C, rn_mode mode, void* ws, size_t ws_bytes,
                                   void* stream);

/* Tile-shape autotuner for batches.  Section IV.B's tuning system sizes each
 * task's resources from its footprint before it runs; on the GPU the
 * resource that decides speed is the GEMM tile shape, chosen here by
 * measurement.  For every problem shape (mode,
 * log2 M, log2 N, log2 K) of the batch that is not tuned yet, times each GEMM
 * tile configuration on that problem (one warm-up and three timed launches,
 * HIP events) and keeps the fastest.  Then, when the workspace is the size
 * rn_block_tensordot_batch_plan gives, times each tile group of the batch
 * once (its grouped relayout and GEMM, one after another); later batch calls
 * spread the groups over their streams by these times.  Runs synchronously
 * on `stream` and writes C (arguments as rn_block_tensordot_batch; C's
 * contents afterwards are unspecified).  The choices live in the handle and
 * are used by every later call on it; they never change during a call, and
 * neither tiles nor stream placement change any result bit.  When the
 * environment variable
 * RN_TUNE_CACHE names a file, rn_create loads it and every autotune run
 * rewrites it.  save/load/clear manage the table explicitly. */
rn_status rn_autotune_batch(rn_handle h, int32_t n, const rn_tensor* A, const rn_tensor* B,
                            const int32_t* k, const int32_t* const* axesA,
                            const int32_t* const* axesB, rn_tensor* C, rn_mode mode, void* ws,
                            size_t ws_bytes, void* stream);
/* Number of GEMM tile shapes of a mode (indices 0 .. n-1 in tune files;
 * index 0 is the one-thread-per-output kernel for tiny problems). */
int32_t rn_tile_count(rn_mode mode);
rn_status rn_tune_save(rn_handle h, const char* path);
rn_status rn_tune_load(rn_handle h, const char* path);
rn_status rn_tune_clear(rn_handle h);

/* Handle options.
 *   RN_OPT_GRAPHS: 1 (default) or 0; same as rn_set_graphs.
 *   RN_OPT_PAIR_SPLIT_THRESHOLD: number of coupled block pairs B_k at or above
 *     which a block tensordot splits its K loop at block-pair boundaries into
 *     separate partial sums, reduced afterwards in ascending order (the GPU form
 *     of the reduction strategy switch of Section IV.B: below the threshold the
 *     pairs stream through one accumulator, Eq. 2 memory; at or above it the
 *     pairs' partials exist side by side, as in the tree reduction).  0 (the
 *     default) leaves the choice to the built-in heuristic.
 *   RN_OPT_SPLIT_FOOTPRINT: bytes the partial sums of one split may occupy
 *     (default 1 GiB); the split count is lowered until it fits.
 *   RN_OPT_SLICE_SUM: 0 (default): sliced networks keep one result per slice
 *     to the end and sum them in FP64 (Section II.B); 1: a sliced bond is
 *     summed inside the step that contracts it (the slices viewed as blocks of
 *     one contraction), so later steps run once instead of once per value of
 *     that bond; the sum then happens in the mode's accumulation precision,
 *     and per-slice values do not exist (slices_dev must be NULL).
 *   RN_OPT_BATCHED_SLICE_BITS: at most this many sliced bonds (the last ones
 *     of `sliced`) run batched in one pass; the values of the others are fixed
 *     per pass (projection by a base offset) and the passes run one after
 *     another in the same workspace.  Default 64 (all batched).
 *   RN_OPT_NETWORK_FOOTPRINT: workspace cap in bytes for a network; the
 *     planner lowers the batched-slice count until the workspace fits, and
 *     fails with RN_ERR_OOM if it cannot.  0 (default): no cap.
 * Options affect plans and calls made on the handle afterwards. */
typedef enum {
  RN_OPT_GRAPHS = 0,
  RN_OPT_PAIR_SPLIT_THRESHOLD = 1,
  RN_OPT_SPLIT_FOOTPRINT = 2,
  RN_OPT_SLICE_SUM = 3,
  RN_OPT_BATCHED_SLICE_BITS = 4,
  RN_OPT_NETWORK_FOOTPRINT = 5
} rn_option;
rn_status rn_set_option(rn_handle h, rn_option opt, int64_t value);
rn_status rn_get_option(rn_handle h, rn_option opt, int64_t* value);

/* Graph replay.  When on (the default; RN_GRAPHS=0 in the environment turns
 * it off at rn_create), rn_block_tensordot_batch and rn_contract_network
 * record their launch sequence as a HIP graph the first time they run with a
 * given set of arguments on a non-default stream, and replay the graph when
 * the identical call repeats.  Never used on the NULL stream, inside a
 * caller's own stream capture, or while kernel timing is on. */
rn_status rn_set_graphs(rn_handle h, int on);

/* ------------------------------------------------------------------------
 * Sliced network contraction (Sections II.A and II.B).
 *
 * T[0..nt-1]: the network's tensors (every dim 2, grid all ones, dtype
 * matching the mode).  labels[i][j] is the integer bond label of axis j of
 * tensor i; a label carried by two tensors is a bond, and every label must
 * be a bond (the network closes to a scalar).  path: nt-1 pairs in
 * single-static-assignment form (ids >= nt name step results in order).  A
 * step sums over the labels its two operands share.  sliced: nsliced
 * (<= RN_MAX_SLICED) bond labels projected onto both basis values; slice s
 * fixes sliced[i] to bit (nsliced-1-i) of s.  All 2^nsliced slices run
 * batched through every step, and their scalar results are summed in FP64
 * in ascending s on the GPU.  amp_dev (device, 2 doubles) receives
 * (re, im) of the amplitude; slices_dev (device, 2*2^nsliced doubles, may be
 * NULL) receives each slice's value.
 * ------------------------------------------------------------------------ */
rn_status rn_contract_network_plan(rn_handle h, int32_t nt, const rn_tensor* T,
                                   const int32_t* const* labels, int32_t nsteps,
                                   const int32_t* path, int32_t nsliced, const int32_t* sliced,
                                   rn_mode mode, size_t* ws_bytes, double* flops,
                                   int32_t* max_rank);
rn_status rn_contract_network(rn_handle h, int32_t nt, const rn_tensor* T,
                              const int32_t* const* labels, int32_t nsteps, const int32_t* path,
                              int32_t nsliced, const int32_t* sliced, rn_mode mode, void* ws,
                              size_t ws_bytes, void* stream, double* amp_dev, double* slices_dev);

/* Prepared network call, for repeated amplitudes of one circuit (the
 * contraction of Sections II.A and II.B, as rn_contract_network).
 * rn_network_prepare copies the descriptors (tensors with their data
 * pointers, labels, path, sliced), plans under the handle's current options
 * and hashes the descriptors once; *ws_bytes receives the workspace size.
 * rn_network_execute runs it on `stream` with the given workspace and
 * outputs (same meaning and errors as rn_contract_network); the tensors'
 * contents may change between calls, their addresses may not.  A prepared
 * call belongs to its handle (one thread at a time, destroyed before it);
 * rn_network_release frees it (NULL is accepted). */
typedef struct rn_prepared_net* rn_prepared;
rn_status rn_network_prepare(rn_handle h, int32_t nt, const rn_tensor* T,
                             const int32_t* const* labels, int32_t nsteps, const int32_t* path,
                             int32_t nsliced, const int32_t* sliced, rn_mode mode,
                             rn_prepared* out, size_t* ws_bytes);
rn_status rn_network_execute(rn_prepared p, void* ws, size_t ws_bytes, void* stream,
                             double* amp_dev, double* slices_dev);
rn_status rn_network_release(rn_prepared p);

/* ------------------------------------------------------------------------
 * Amplitude server (continuous admission of sliced-network requests).
 * Each request is one amplitude of a sliced network (Sections II.A, II.B).
 * Admission follows the tuning rule of Section IV.B: work starts only when
 * its memory requirement fits what is free, so a device filled with
 * requests of similar size never runs out of memory.
 *
 * rn_server_create binds a server to a device with its own library handle,
 * a device arena of hbm_budget bytes (allocated once) and max_active slots
 * (HIP streams, 1..16).  rn_server_submit copies a request -- a network as
 * for rn_contract_network but with HOST tensor data -- into the server's
 * queue and returns a ticket; it never blocks on the GPU.  A worker thread
 * admits queued requests whenever a slot is free and the request's footprint
 * (its tensors + the planned workspace + 256 bytes) fits the free arena;
 * admitted requests run concurrently on their slots and keep their tensors
 * resident until they finish.  Admission order (rn_server_set_admission):
 * policy 0 admits in arrival order (the head waits for memory and blocks the
 * rest); policy 1, the default, admits the request with the fewest planned
 * flops first, except that a request overtaken max_overtakes times (default
 * 8) by later arrivals goes next, and while it does not fit the free memory
 * nothing else is admitted, so no request waits forever; while younger
 * requests wait, such aged requests occupy at most max_active - 1 slots (with
 * two or more), keeping one slot for the small work behind them.  A request whose
 * footprint exceeds the whole budget completes with status RN_ERR_OOM.
 * Results: amplitude, latency = completion - submit, and its split into
 * queueing and running time.  A request's amplitude does not depend on what
 * else runs (every kernel is deterministic and per-request).
 * rn_server_destroy waits for all submitted requests, then frees everything.
 * ------------------------------------------------------------------------ */
typedef struct rn_server* rn_server_t;
typedef struct {
  double amp[2];          /* (re, im) of the amplitude, FP64 slice sum */
  double latency_s;       /* completion - submit */
  double queue_s;         /* admission - submit */
  double run_s;           /* completion - admission */
  double footprint_bytes; /* arena bytes the request held */
  int32_t status;         /* RN_OK, RN_ERR_OOM, or the error of the enqueue */
  double start_s;         /* admission time, seconds since rn_server_create */
  double done_s;          /* completion time, seconds since rn_server_create */
} rn_result;
rn_status rn_server_create(int device, size_t hbm_budget, int32_t max_active, rn_server_t* srv);
rn_status rn_server_submit(rn_server_t srv, int32_t nt, const rn_tensor* T,
                           const int32_t* const* labels, int32_t nsteps, const int32_t* path,
                           int32_t nsliced, const int32_t* sliced, rn_mode mode,
                           uint64_t* ticket);
rn_status rn_server_set_admission(rn_server_t srv, int32_t policy, int32_t max_overtakes);
rn_status rn_server_poll(rn_server_t srv, uint64_t ticket, int32_t* done, rn_result* res);
rn_status rn_server_wait(rn_server_t srv, uint64_t ticket, rn_result* res);
rn_status rn_server_stats(rn_server_t srv, int64_t* queued, int64_t* active, int64_t* completed,
                          size_t* bytes_in_use);
rn_status rn_server_destroy(rn_server_t srv);

/* ------------------------------------------------------------------------
 * FP64 reductions on the GPU (slice sums and norms, Section II.B).
 * rn_norm2: out_dev[0] = sum |x|^2 over all elements of T, in FP64.
 * rn_sum_c128: out_dev[0..1] = sum of n complex128 values (device, n <= 2^20),
 * in a fixed order that does not depend on the launch.
 * ------------------------------------------------------------------------ */
rn_status rn_norm2(rn_handle h, const rn_tensor* T, double* out_dev, void* stream);
rn_status rn_sum_c128(rn_handle h, int64_t n, const double* vals_dev, double* out_dev,
                      void* stream);

/* ------------------------------------------------------------------------
 * Kernel timing (measurement support).  While enabled, every kernel this
 * handle enqueues is bracketed by two HIP events recorded on the stream it
 * runs on.  rn_profile_read waits for those events, returns the summed
 * milliseconds and launch counts per kernel class -- [0] permute, [1] complex
 * GEMM, [2] split-K reduction, [3] FP64 sums and norms -- and clears them.
 * Timing adds an event pair per launch; leave it off in production.
 * ------------------------------------------------------------------------ */
rn_status rn_profile_enable(rn_handle h, int on);
rn_status rn_profile_read(rn_handle h, double ms[4], int64_t count[4]);

#ifdef __cplusplus
}
#endif
#endif /* RN_H */
