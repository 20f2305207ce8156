/*
 * tgo -- task-group ordering on MI355X (gfx950).
 *
 * C ABI of the library libtgo.so.  It evaluates the temporal execution model of
 * Lazaro-Munoz et al., "Improving tasks throughput on accelerators using OpenCL
 * command concurrency" (Section 4), over launch orderings of a task group, and
 * runs the paper's ordering heuristic (Section 5.1, Algorithm 1).
 *
 * The model.  A task is an HtD transfer, a kernel K and a DtH transfer executed
 * in that order (Section 3; any stage may be empty, i.e. zero).  Commands are
 * issued in launch order through one FIFO queue per engine (Section 3.2, two-DMA
 * launch scheme; Section 4.1 FIFO simulator): the HtD engine runs the HtDs
 * back to back, K_j starts once HtD_j and K_{j-1} are done, DtH_j once K_j and
 * DtH_{j-1} are done.  Kernels never overlap each other and always take their
 * solo time (Section 4.1, last paragraph).  While an HtD and a DtH are both
 * moving data they are slowed down (Section 4.2.1); the paper gives no formula,
 * and this library's reading is that they then advance at p_htd/q and p_dth/q of
 * solo speed.  Time is integer nanoseconds: remaining transfer work is exact in
 * units of 1/q solo-ns and a completion estimate is rounded up to a whole ns.
 * T(ordering) is the completion time of the last DtH.
 *
 * Orderings are ranked lexicographically (rank 0 = identity 0,1,...,n-1).  Ties
 * for the best or worst ordering go to the lowest rank.
 *
 * Conventions for every call:
 *   - Pointers named d_* are device pointers (HBM); h_* are host pointers.  The
 *     caller owns every buffer.  Calls are asynchronous on `stream` (a
 *     hipStream_t; NULL = the default stream); buffers must stay alive until the
 *     stream is synchronized.
 *   - Return value: TGO_OK (0) or a negative TGO_E* code; nothing aborts and no
 *     exception crosses the ABI.  tgo_last_error() gives a thread-local detail
 *     string for the last failing call.  Argument errors the host can see are
 *     returned at once; errors in device-resident data (negative durations,
 *     overflow of the integer bounds, an index that is not a permutation) are
 *     reported through the status fields of the outputs.
 *   - Functions are reentrant; a handle (plan, surrogate, server) must not be
 *     used from two threads at once.
 *   - Scratch memory: tgo_exhaustive, tgo_exhaustive_mem, tgo_rounds,
 *     tgo_random_search and tgo_surrogate_pairs use device scratch owned by the
 *     library, one buffer per (device, stream), grown on demand (a growth
 *     waits for that stream's earlier work and allocates) and kept until the
 *     process ends.  Calls on different streams may therefore overlap; calls
 *     on one stream are ordered by the stream.  Destroy a stream only after
 *     its work has finished: a later stream with the same handle reuses its
 *     scratch.
 */
#ifndef TGO_H
#define TGO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TGO_MAX_N 16            /* largest group for evaluate / heuristic      */
#define TGO_MAX_EXHAUSTIVE_N 13 /* largest group enumerated in full (13! ranks) */
#define TGO_ROUNDS_MAX_PER_ORDER 479001600ull /* per-ordering output limit of tgo_rounds */
#define TGO_MAX_MEM_N 12        /* largest group of tgo_exhaustive_mem (12! ranks) */
#define TGO_MAX_CAPACITY (1ll << 62) /* largest device-memory capacity, bytes     */
#define TGO_MAX_CKE_N 12        /* largest group of tgo_exhaustive_cke (12! ranks) */

enum {
    TGO_OK = 0,
    TGO_EINVAL = -1,  /* bad argument: n out of range, NULL, bad model, not a permutation */
    TGO_ERANGE = -2,  /* a duration is negative or the integer bounds would overflow      */
    TGO_ENOMEM = -3,  /* allocation failed                                                 */
    TGO_EDEVICE = -4, /* a HIP runtime error; tgo_last_error() has the HIP message        */
};

typedef void *tgo_stream; /* hipStream_t */

/* Solo durations of one task, ns, each >= 0 (Section 3: HtD, K, DtH). */
typedef struct {
    int64_t htd_ns, kern_ns, dth_ns;
} tgo_task;

/* Device model.  dma_engines: 2 = separate HtD and DtH engines (the launch
 * scheme of Section 3.2 with three command queues); 1 = one engine for both
 * directions (the Section 3.2 scheme with two command queues: every HtD is
 * queued before every DtH, so transfers never overlap and run at solo speed;
 * the rates below are validated but have no effect).  Any other value is
 * TGO_EINVAL.  q = 1 << q_log2 (q_log2 in 0..10); overlapped transfers advance
 * at p_htd/q and p_dth/q of solo speed, 1 <= p <= q.  (q_log2 = 2, p = 3, 3)
 * is the benchmark default; (3, 3, 3) reproduces the worked timeline of
 * Section 4.1.  Every entry point below takes either scheme. */
typedef struct {
    int32_t dma_engines;
    int32_t q_log2;
    int32_t p_htd, p_dth;
} tgo_model;

/* Result of an enumeration over all n! orderings (the paper's best, worst and
 * average over every ordering: Section 6, speedups against the worst). */
typedef struct {
    int64_t min_ns, max_ns;
    uint64_t argmin_rank, argmax_rank; /* lowest rank among ties                  */
    uint64_t sum_lo, sum_hi;           /* exact 128-bit sum of T over the ranks   */
    uint64_t count;                    /* number of orderings (n!)                */
    uint64_t fingerprint;              /* sum over ranks r of (2r+1)*T_r mod 2^64 */
    double mean_ns;                    /* sum / count, rounded to nearest         */
    int32_t status;                    /* TGO_OK or the TGO_E* found on the device */
    int32_t n;
    uint8_t best[16], worst[16];       /* orderings at argmin / argmax            */
    uint8_t heur[16];                  /* Algorithm-1 ordering (tgo_batch only;    */
    int64_t heur_ns;                   /*  0xff / -1 when not computed)           */
} tgo_summary;

/* Error reporting for every call below (no passage of the paper: library
 * plumbing).  tgo_strerror: a static text for a TGO_E* code.  tgo_last_error:
 * the detail of the last failing call on this thread (valid until the next
 * call on the thread).  tgo_version: the ABI version, 1. */
const char *tgo_strerror(int code);
const char *tgo_last_error(void);
int tgo_version(void);

/* ---------------------------------------------------------------------------
 * tgo_evaluate -- predicted total time of given orderings (Section 4: the
 * model predicts a group's total time for a given launch ordering).
 *   d_tasks : n tasks (1 <= n <= TGO_MAX_N).
 *   d_orders: m orderings, row-major m x n bytes, each a permutation of 0..n-1.
 *   d_out   : m int64; T in ns, or a negative TGO_E* for a row that is not a
 *             permutation (TGO_EINVAL) or tasks out of range (TGO_ERANGE).
 * One GPU lane per ordering.
 */
int tgo_evaluate(const tgo_model *model, const tgo_task *d_tasks, int n, const uint8_t *d_orders,
                 int64_t m, int64_t *d_out, tgo_stream stream);

/* ---------------------------------------------------------------------------
 * tgo_predict -- one ordering from host buffers (Section 4's prediction for a
 * given ordering), computed on the current device: the call allocates a
 * small device buffer and a stream of its own, runs the evaluation kernel,
 * waits, and frees them.  *out_ns = T in ns.  Returns TGO_EINVAL for a bad
 * model, n outside 1..TGO_MAX_N or an h_order that is not a permutation,
 * TGO_ERANGE for durations outside [0, 2^40), TGO_EDEVICE on a HIP error.
 * Blocking; for many orderings use tgo_evaluate.
 */
int tgo_predict(const tgo_model *model, const tgo_task *h_tasks, int n, const uint8_t *h_order,
                int64_t *out_ns);

/* ---------------------------------------------------------------------------
 * tgo_exhaustive -- every ordering of one group (the brute force that Section 1
 * and Section 5.1 call infeasible at runtime), reduced to best / worst / mean.
 *   d_tasks     : n tasks, 1 <= n <= TGO_MAX_EXHAUSTIVE_N.
 *   d_per_order : NULL, or n! int64 receiving T at index = rank (n <= 12).
 *   d_summary   : one tgo_summary, written by the call (status set on error).
 */
int tgo_exhaustive(const tgo_model *model, const tgo_task *d_tasks, int n, int64_t *d_per_order,
                   tgo_summary *d_summary, tgo_stream stream);

/* ---------------------------------------------------------------------------
 * tgo_exhaustive_noalloc -- tgo_exhaustive for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, limits, errors and results as
 * tgo_exhaustive; the caller still passes the tasks, the optional
 * per-ordering buffer and the summary.  The call allocates nothing: its
 * scratch (block partials, accumulator, time-path word) is a fixed
 * per-device array of TGO_NOALLOC_SCRATCH_BYTES (2 MiB) that every device the
 * library runs on holds until the process ends, and the launch grid is bounded
 * so that the scratch always fits (the result does not depend on the grid).
 * The scratch is re-initialised by the call's own kernels (no memset), so a
 * call leaves nothing behind that the next one reads.  All calls on one device
 * share that array: calls that overlap on one device (different streams, or
 * threads) race and must be serialised by the caller.  The array's device
 * address is looked up once per device, on the first call with that device
 * current.
 */
#define TGO_NOALLOC_SCRATCH_BYTES (2u << 20)
int tgo_exhaustive_noalloc(const tgo_model *model, const tgo_task *d_tasks, int n, int64_t *d_per_order,
                           tgo_summary *d_summary, tgo_stream stream);

/* ---------------------------------------------------------------------------
 * tgo_heuristic -- Algorithm 1 (Section 5.1) for a batch of groups.
 *   d_tasks/d_offs: CSR batch, group g = d_tasks[d_offs[g] .. d_offs[g+1]),
 *                   sizes 1..TGO_MAX_N.
 *   d_orders      : n_groups x 16 bytes; the first n entries of row g are the
 *                   heuristic ordering of group g (task indices local to g).
 *   d_ns          : n_groups int64; T of that ordering, or a negative TGO_E*.
 * Readings of the selection functions (the paper describes them in words):
 *   first : largest K - HtD; ties to the longer DtH, then the lower index.
 *   next  : smallest |h_c - (t_K - t_HtD)| + |k_c - (t_DtH - max(t_HtD + h_c, t_K))|
 *           with t_* the completion times of the last HtD, K, DtH when the
 *           ordered set is simulated alone; ties to the lower index.
 *   last  : both orders (x, y) of the final two tasks scored
 *           fit(x | OT) + fit(y | OT + x) + d_y; ties to the shorter d_y, then
 *           to the order whose x has the lower index.
 */
int tgo_heuristic(const tgo_model *model, const tgo_task *d_tasks, const int32_t *d_offs,
                  int n_groups, uint8_t *d_orders, int64_t *d_ns, tgo_stream stream);

/* ---------------------------------------------------------------------------
 * Batched enumeration: many groups of uneven size in one persistent launch.
 * The paper's runtime reorders the task group that its proxy thread finds
 * waiting (Section 6.2); a batch holds many such groups.
 *
 * tgo_plan_create  -- device workspace for up to max_groups groups of at most
 *                     max_n (1..12) tasks (allocated here, freed by
 *                     tgo_plan_destroy) and a capture stream.  mem_budget (0:
 *                     the default of 64 MiB beyond the per-group records)
 *                     bounds the plan's device memory: it sets how many
 *                     tiles a group on the 64-bit time path is split into;
 *                     TGO_ENOMEM if even one per group does not fit.  Groups
 *                     larger than max_n get status TGO_EINVAL.
 * tgo_plan_autotune-- times candidate work decompositions (positions
 *                     enumerated per lane by group size, subtrees per lane per
 *                     tile, persistent grid size) on the given batch and keeps
 *                     the fastest.  Blocks until done; overwrites d_out.
 * tgo_plan_describe-- the chosen decomposition as a JSON object.
 * tgo_plan_set_decomposition -- sets the decomposition that describe reports
 *                     (m_by_n[n - 1]: positions enumerated per lane for group
 *                     size n = 1..12, each in 1..min(n, 5); lane_mult: subtrees
 *                     per lane in a tile, 1..64; blocks: persistent grid,
 *                     1..65536), e.g. one a tuning run saved, so that a later
 *                     process skips tgo_plan_autotune.  Results never depend
 *                     on it.  TGO_EINVAL for a value out of range (the plan is
 *                     then unchanged).
 * tgo_batch        -- for every group g of the CSR batch (tasks
 *                     d_tasks[d_offs[g] .. d_offs[g+1])), writes d_out[g]: the
 *                     full-enumeration summary plus the heuristic ordering
 *                     (heur, heur_ns).  Group sizes 1..12.  Groups whose
 *                     times could reach 2^31 ns are enumerated with 64-bit
 *                     time in the same launch sequence (a second persistent
 *                     kernel, per-tile partial summaries).  The launch
 *                     sequence is captured once into a HIP graph and replayed
 *                     while (d_tasks, d_offs, n_groups, d_out) stay the same.
 *                     Calls on one plan must not overlap on different streams.
 */
typedef struct tgo_plan tgo_plan;
int tgo_plan_create(const tgo_model *model, int max_groups, int max_n, size_t mem_budget, tgo_plan **out);
int tgo_plan_autotune(tgo_plan *plan, const tgo_task *d_tasks, const int32_t *d_offs, int n_groups,
                      tgo_summary *d_out, tgo_stream stream);
int tgo_plan_describe(const tgo_plan *plan, char *buf, size_t len);
int tgo_plan_set_decomposition(tgo_plan *plan, const int32_t *m_by_n, int lane_mult, int blocks);
int tgo_batch(tgo_plan *plan, const tgo_task *d_tasks, const int32_t *d_offs, int n_groups,
              tgo_summary *d_out, tgo_stream stream);
void tgo_plan_destroy(tgo_plan *plan);

/* ---------------------------------------------------------------------------
 * Learned proposal for groups too large to enumerate (n <= 16).  Not in the
 * paper, whose answer for large groups is the heuristic (Section 5.1); here
 * the heuristic stays a candidate and the exact model (Section 4) decides.
 *
 * Network: per-position features of the ordering (for each of 16 positions
 * the HtD, K, DtH of the task there as log1p(x / 1 us) / log1p(20 ms / 1 us),
 * zero past the group) -> 256 -> 256 -> 256 -> 1, ReLU between layers,
 * bfloat16 weights and activations with float32 accumulation on the matrix
 * cores.  Trained with mean squared error against y = T / LB - 1 (LB: the
 * largest machine lower bound of the group) and Adam on float32 masters.
 * Parameter order (float32, TGO_SURROGATE_PARAMS values): W1[256][48], b1[256],
 * W2[256][256], b2[256], W3[256][256], b3[256], W4[256], b4[1]; W[out][in].
 *
 * Sampled orderings: ordering s of group g under `seed` comes from one
 * Philox4x32-10 call (counter (s lo, s hi, g, 0), key (seed lo, seed hi)) and a
 * Fisher-Yates shuffle from the last position down, position i taking
 * hi32(x (i + 1)) and keeping x = lo32(x (i + 1)), x reloaded from the next
 * word every four draws.
 *
 * Search and pair generation evaluate orderings exactly with 32-bit time
 * where a group's times stay below 2^31 ns and with 64-bit time otherwise
 * (durations must lie in [0, 2^40): TGO_ERANGE outside).  All buffers below
 * are device memory; the surrogate owns max_rows rows of activations for
 * training and scoring, and the search's keys for max(max_rows, 2^20) rows
 * (8 bytes each: the search scores that many rows per launch).
 */
#define TGO_SURROGATE_PARAMS 144385

typedef struct {
    int64_t best_ns;       /* best exact T found: candidates and heuristic     */
    int64_t heur_ns;       /* T of the heuristic ordering                      */
    int64_t cand_best_ns;  /* best exact T among the sampled candidates (-1: none) */
    uint64_t best_sample;  /* sample index of that candidate                   */
    int32_t status, n;
    int32_t from_heuristic, pad;  /* 1 if the heuristic ordering is best_ns   */
    uint8_t best[16];      /* the best ordering                                */
} tgo_search_result;

typedef struct tgo_surrogate tgo_surrogate;
int tgo_surrogate_create(int64_t max_rows, int max_groups, tgo_surrogate **out);
void tgo_surrogate_destroy(tgo_surrogate *s);
int tgo_surrogate_param_count(void);
/* He-uniform weights from Philox(seed, parameter index), zero biases, Adam reset. */
int tgo_surrogate_init(tgo_surrogate *s, uint64_t seed, tgo_stream stream);
/* Host float32 parameters in (set; resets Adam) and out (get); both synchronize. */
int tgo_surrogate_set_params(tgo_surrogate *s, const float *h_params, tgo_stream stream);
int tgo_surrogate_get_params(tgo_surrogate *s, float *h_params, tgo_stream stream);
/* Parameters to / from a file: 8-byte magic "TGOSURR1", uint32 count
 * (TGO_SURROGATE_PARAMS), uint32 0, then the float32 masters little-endian.
 * Load rejects a wrong magic, count, length or a non-finite value
 * (TGO_EINVAL) and resets the optimizer state like set_params.  Blocking. */
int tgo_surrogate_save(tgo_surrogate *s, const char *path);
int tgo_surrogate_load(tgo_surrogate *s, const char *path);
/* Training pairs: per_group (multiple of 64) sampled orderings of every group,
 * d_orders [G*per_group][16] (0xff past n), d_gid, exact d_T (or the group's
 * negative status). d_status [G]. */
int tgo_surrogate_pairs(const tgo_model *model, const tgo_task *d_tasks, const int32_t *d_offs,
                        int n_groups, int64_t per_group, uint64_t seed, int32_t *d_status,
                        uint8_t *d_orders, int32_t *d_gid, int64_t *d_T, tgo_stream stream);
/* Scores of given orderings (rows <= max_rows): d_orders [rows][16], d_gid [rows]. */
int tgo_surrogate_score(tgo_surrogate *s, const tgo_task *d_tasks, const int32_t *d_offs, int n_groups,
                        const uint8_t *d_orders, const int32_t *d_gid, int64_t rows, float *d_scores,
                        tgo_stream stream);
/* Loss (mean squared error of the score against T / LB - 1) and its gradient
 * (d_grad: TGO_SURROGATE_PARAMS floats in the parameter layout, may be NULL)
 * on a batch of pairs: d_orders [rows][16], d_gid [rows], d_T [rows] (rows a
 * multiple of 64, <= max_rows).  Inputs, weights, hidden activations and the
 * back-propagated activation gradients are bf16, sums float32.  The batch's
 * intermediate values are kept for tgo_surrogate_get_batch. */
int tgo_surrogate_grad(tgo_surrogate *s, const tgo_task *d_tasks, const int32_t *d_offs, int n_groups,
                       const uint8_t *d_orders, const int32_t *d_gid, const int64_t *d_T, int rows,
                       float *d_grad, float *d_loss, tgo_stream stream);
/* One training step: the gradient of tgo_surrogate_grad on the batch, then
 * tgo_surrogate_adam_step with it (three kernel launches; d_loss receives the
 * batch loss before the update). */
int tgo_surrogate_train_step(tgo_surrogate *s, const tgo_task *d_tasks, const int32_t *d_offs,
                             int n_groups, const uint8_t *d_orders, const int32_t *d_gid,
                             const int64_t *d_T, int rows, float lr, float *d_loss, tgo_stream stream);
/* One Adam step (Kingma and Ba: beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected
 * moments, step count t starting at 1) of the float32 masters with a given
 * gradient d_grad (TGO_SURROGATE_PARAMS floats); refreshes the bf16 copies. */
int tgo_surrogate_adam_step(tgo_surrogate *s, const float *d_grad, float lr, tgo_stream stream);
/* Adam state to the host: first and second moments (float[TGO_SURROGATE_PARAMS]
 * each; either may be NULL) and the number of steps taken.  Synchronizes. */
int tgo_surrogate_get_moments(tgo_surrogate *s, float *h_m, float *h_v, int64_t *h_step, tgo_stream stream);
/* Values the last tgo_surrogate_grad computed for its first `rows` rows, to the
 * host, row-major: what = 0 features [rows][48] (bf16 bits), 1..3 hidden
 * activations h1..h3 [rows][256] (bf16 bits), 4 scores [rows] (float), 5..7
 * gradients of the loss with respect to the pre-activations of layers 3, 2, 1
 * [rows][256] (bf16 bits; zero where the ReLU is off).  Synchronizes. */
int tgo_surrogate_get_batch(tgo_surrogate *s, int what, int64_t rows, void *h_out, tgo_stream stream);
/* Surrogate-guided search: score `samples` sampled orderings per group, re-score
 * the `topk` (<= 64) best-scored exactly, return the best of those and the
 * heuristic ordering (ties to the heuristic).  d_keys (NULL: the group index)
 * names the sampling stream of each group, so a group gets the same result
 * whatever batch it is in. */
int tgo_surrogate_search(tgo_surrogate *s, const tgo_model *model, const tgo_task *d_tasks,
                         const int32_t *d_offs, const uint32_t *d_keys, int n_groups, int64_t samples,
                         int topk, uint64_t seed, tgo_search_result *d_out, tgo_stream stream);
/* The candidate stage of tgo_surrogate_search on its own (same arguments):
 * d_cand [n_groups][topk] receives, per group, the topk smallest keys in
 * ascending order, key = (score bits mapped to an unsigned integer of the same
 * order) << 32 | sample index, so ties in score go to the lower sample index;
 * ~0 where a group has fewer than topk samples or a size outside 1..16.  These
 * are exactly the orderings that the search re-scores with the exact model. */
int tgo_surrogate_candidates(tgo_surrogate *s, const tgo_model *model, const tgo_task *d_tasks,
                             const int32_t *d_offs, const uint32_t *d_keys, int n_groups, int64_t samples,
                             int topk, uint64_t seed, uint64_t *d_cand, tgo_stream stream);
/* Plain exact search: the heuristic plus `samples` sampled orderings per group
 * scored exactly (rounded up to a multiple of 64). */
int tgo_random_search(const tgo_model *model, const tgo_task *d_tasks, const int32_t *d_offs,
                      int n_groups, int64_t samples, uint64_t seed, tgo_search_result *d_out,
                      tgo_stream stream);

/* ---------------------------------------------------------------------------
 * Serving: a continuous-batching request loop.  The paper's proxy thread polls
 * a buffer of offloaded tasks, forms a task group, reorders and submits it
 * (Section 6.2); here requests (one task group each) arrive at any time.  The
 * task tables of admitted requests wait on the device, in one ring of task
 * rows per size class; a request is admitted when its rows fit in its ring,
 * and the rings get what the memory budget leaves after the server's own
 * device memory (plans, network workspaces, result buffers), so admission is
 * by memory and the device memory the server holds never exceeds
 * budget_bytes (tgo_server_create fails with TGO_ENOMEM if the budget cannot
 * hold one request per class).  A scheduler thread keeps up to `streams`
 * batches in flight on their own HIP streams: a free stream takes the oldest
 * admitted requests of one size class and launches them straight from the
 * ring; requests that arrive while others run are admitted as soon as rows
 * free up, and launched as soon as a stream does.
 * Groups with n <= small_max_n are enumerated in full (tgo_batch; answer =
 * the best ordering, with the heuristic's time beside it); larger groups use
 * the learned proposal (tgo_surrogate_search with the request's key as its
 * sampling key, so a request's answer is the same alone and in any mix).
 */
typedef struct {
    int64_t budget_bytes;   /* device memory the server may hold in all         */
    int32_t streams;        /* batches in flight (1..8)                        */
    int32_t max_batch;      /* groups per exhaustive batch (1..4096)           */
    int32_t max_batch_large;/* groups per surrogate batch (1..4096)            */
    int32_t small_max_n;    /* exhaustive up to this size (1..12)              */
    int32_t topk;           /* exact re-scores per large group (1..64)         */
    int32_t window_us;      /* while another batch is in flight, a free stream
                               waits up to this long (microseconds, measured
                               from the oldest waiting request's arrival) for
                               its batch to fill before launching it; 0 =
                               launch at once (0..100000)                       */
    int64_t samples;        /* scored samples per large group                  */
    uint64_t seed;          /* sampling seed                                   */
} tgo_server_config;

typedef struct {
    uint64_t id;
    int64_t t_arrive_ns, t_admit_ns, t_done_ns; /* steady clock of the host      */
    int32_t n, path;        /* path 0 = full enumeration, 1 = learned proposal   */
    int32_t status, pad;
    int64_t best_ns;        /* exact T of the returned ordering                */
    int64_t heur_ns;        /* exact T of the heuristic ordering               */
    uint8_t best[16];
} tgo_server_result;

typedef struct {
    uint64_t submitted, completed, batches, rejected;
    int64_t in_use_bytes, max_in_use_bytes;  /* device memory held: base + ring rows */
    int64_t queued, max_queued;              /* requests not yet launched            */
    int64_t base_bytes;                      /* the server's own buffers, plans,
                                                network workspaces                  */
    int64_t ring_rows[2];                    /* queue capacity (task rows) per class */
    int64_t budget_bytes;
} tgo_server_stats;

typedef struct tgo_server tgo_server;
void tgo_server_config_default(tgo_server_config *cfg);
/* sur may be NULL (then only groups with n <= small_max_n are accepted); its
 * parameters are copied. */
int tgo_server_create(const tgo_model *model, const tgo_server_config *cfg, tgo_surrogate *sur,
                      tgo_server **out);
/* Non-blocking, thread-safe; h_tasks is copied.  key names the sampling stream
 * of a large group (0: the request id). */
int tgo_server_submit(tgo_server *srv, const tgo_task *h_tasks, int n, uint32_t key, uint64_t *id);
/* Completed results, in completion order; *count <= max. */
int tgo_server_poll(tgo_server *srv, tgo_server_result *out, int max, int *count);
/* Block until every submitted request has completed (TGO_ERANGE on timeout). */
int tgo_server_drain(tgo_server *srv, int64_t timeout_ms);
int tgo_server_get_stats(tgo_server *srv, tgo_server_stats *out);
/* Replay an arrival trace in real time (request i submitted at
 * h_arrival_ns[i] - h_arrival_ns[0] after the call starts), wait for all, and
 * return the results in request order. */
int tgo_server_replay(tgo_server *srv, const tgo_task *h_tasks, const int32_t *h_offs,
                      const int64_t *h_arrival_ns, int n_requests, tgo_server_result *h_out,
                      int64_t timeout_ms);
void tgo_server_destroy(tgo_server *srv);

/* ---------------------------------------------------------------------------
 * tgo_rounds -- several workers offloading dependent tasks (Section 6.2: T
 * workers, each with a batch of dependent tasks; a worker hands over its next
 * task only when the previous one has completely finished).
 *   d_tasks : workers * rounds tasks; task (w, r) -- worker w's r-th task -- at
 *             index w * rounds + r.  1 <= workers, 1 <= rounds,
 *             workers * rounds <= 16, (workers!)^rounds < 2^32.
 *   NoReorder setup (Section 6.2): every task queued at t = 0, round by round,
 *     round r in a worker order pi_r; the HtD of (w, r) waits for the DtH of
 *     (w, r - 1) and the in-order queue waits behind it.  All
 *     (workers!)^rounds orderings are evaluated; rank = mixed radix workers!
 *     with pi_0 most significant, each pi_r ranked lexicographically.
 *     d_summary receives min / argmin / max / argmax / sum / mean /
 *     fingerprint over them (fingerprint = sum of (2 rank + 1) T mod 2^64);
 *     best[] and worst[] are launch sequences (task index per position,
 *     0xff-padded); n = workers * rounds; count = (workers!)^rounds.
 *   Heuristic setup (Section 6.2): a proxy takes every waiting task as a task
 *     group, orders it with Algorithm 1 and queues it, and looks for the next
 *     group when the HtD of the group's last task starts (or at the next
 *     arrival if none is waiting then).  d_summary->heur[] receives its launch
 *     sequence and heur_ns its total time (or a negative TGO_E*).
 *   d_per_order : NULL, or (workers!)^rounds int64 (at most
 *                 TGO_ROUNDS_MAX_PER_ORDER) receiving T at index = rank.
 *   d_groups    : NULL, or one uint16: bit j set if launch position j ends a
 *                 task group formed by the proxy.
 * Both launch schemes (model->dma_engines 1 or 2); the model has one kernel
 * queue (no concurrent kernels).  Durations must lie in [0, 2^40) ns, else
 * status = TGO_ERANGE.  Device buffers belong to the caller; the call
 * enqueues on `stream` and returns at once.
 */
int tgo_rounds(const tgo_model *model, const tgo_task *d_tasks, int workers, int rounds,
               int64_t *d_per_order, tgo_summary *d_summary, uint16_t *d_groups, tgo_stream stream);

/* ---------------------------------------------------------------------------
 * tgo_exhaustive_mem -- every ordering of a task group under a device-memory
 * limit.  Section 5 notes that tasks running concurrently hold their input
 * and output buffers at the same time, so the device memory can restrict
 * which tasks may form a group; the paper leaves it aside and assumes enough
 * memory.  Reading:
 *   task x holds d_mem[x] bytes of device memory from the start of its HtD
 *   to the end of its DtH, and at most `capacity` bytes are held at once.
 *   Two DMA engines: the HtD at the head of its queue starts only when its
 *   bytes fit beside those held (the HtDs behind it wait too).  One DMA
 *   engine: the ordering is cut greedily into consecutive sub-groups whose
 *   bytes fit together, each launched as its HtDs, then its DtHs (Section
 *   3.2 scheme), behind the previous sub-group.
 *   With capacity >= the sum of d_mem the results equal tgo_exhaustive's.
 *   d_tasks  : n tasks, 1 <= n <= TGO_MAX_MEM_N, durations in [0, 2^40) ns
 *              (else status = TGO_ERANGE).
 *   d_mem    : n int64 footprints in bytes, each in [0, capacity] (else
 *              status = TGO_EINVAL: a task that cannot fit alone never runs).
 *   capacity : bytes, 1..TGO_MAX_CAPACITY.
 *   d_per_order: NULL, or n! int64 receiving T at index = lexicographic rank.
 *   d_summary: min / argmin / max / argmax / sum / mean / fingerprint over the
 *              n! orderings as tgo_exhaustive (ties to the lowest rank);
 *              heur[] / heur_ns: Algorithm 1's ordering (same selection
 *              rules, its update step simulated under the limit) and its T.
 * Device buffers belong to the caller; the call enqueues on `stream` and
 * returns at once.
 */
int tgo_exhaustive_mem(const tgo_model *model, const tgo_task *d_tasks, const int64_t *d_mem, int n,
                       int64_t capacity, int64_t *d_per_order, tgo_summary *d_summary, tgo_stream stream);

/* tgo_evaluate_mem -- T of m given orderings (row-major m x n bytes, n <=
 * TGO_MAX_N, m <= 2^40) under the device-memory limit of tgo_exhaustive_mem.
 * d_out[i] = T in ns, or TGO_EINVAL for a row that is not a permutation or a
 * footprint outside [0, capacity], TGO_ERANGE for durations out of range. */
int tgo_evaluate_mem(const tgo_model *model, const tgo_task *d_tasks, const int64_t *d_mem, int n,
                     int64_t capacity, const uint8_t *d_orders, int64_t m, int64_t *d_out, tgo_stream stream);

/* ---------------------------------------------------------------------------
 * Concurrent kernels.  The paper's model runs one kernel at a time (Section
 * 4.1, last paragraph); its NoReorder experiments use one command queue per
 * kernel (Section 6.2), Section 3.2 says kernels from different queues overlap
 * only while the device's resources last, and the conclusion leaves
 * concurrent kernels to future work.  Reading: the device has `capacity`
 * units of computing resources (1..2^30, e.g. its compute units); the kernel
 * of task x holds d_units[x] of them (1..capacity) from its start to its end;
 * kernels are dispatched in launch order, each once its HtD has ended, the
 * kernel before it has started and its units fit beside the running kernels;
 * a kernel takes its solo time.  Transfers are unchanged (either DMA scheme,
 * overlap rates of the model).  Every kernel holding the whole capacity gives
 * the results of tgo_exhaustive / tgo_evaluate.  64-bit time throughout.
 *
 * tgo_exhaustive_cke -- every ordering of n <= TGO_MAX_CKE_N tasks, summary as
 *   tgo_exhaustive (optional per-ordering T by rank), plus Algorithm 1 with
 *   `update` under the same rule in heur / heur_ns.  Device-side errors in the
 *   summary status: TGO_ERANGE for a duration outside [0, 2^40), TGO_EINVAL
 *   for a unit count outside 1..capacity.
 * tgo_evaluate_cke -- T of m given orderings (rows of n bytes, n <= 16), or a
 *   negative TGO_E* per row (TGO_EINVAL: not a permutation or bad units).
 */
int tgo_exhaustive_cke(const tgo_model *model, const tgo_task *d_tasks, const int32_t *d_units, int n,
                       int32_t capacity, int64_t *d_per_order, tgo_summary *d_summary, tgo_stream stream);
int tgo_evaluate_cke(const tgo_model *model, const tgo_task *d_tasks, const int32_t *d_units, int n,
                     int32_t capacity, const uint8_t *d_orders, int64_t m, int64_t *d_out, tgo_stream stream);

/* ---------------------------------------------------------------------------
 * Real execution on the device, to validate the model (Sections 4.2, 4.3):
 * each task is an HtD copy from pinned host memory, a kernel, and a DtH copy,
 * launched with a scheme of Section 3.2 on HIP streams (one stream per command
 * queue, events for the dependencies inside a task) and timed with events.
 */
typedef struct tgo_hw tgo_hw;

/* Kernel kinds of a tgo_hw_task: HBM streams x = x * s + b through device
 * memory on every pass (bound by memory bandwidth); ALU loads each float once
 * and runs 64 dependent multiply-adds per pass in registers. */
#define TGO_HW_KERNEL_HBM 0
#define TGO_HW_KERNEL_ALU 1

typedef struct {
    int64_t htd_bytes;   /* bytes copied host -> device (0: no HtD)           */
    int64_t dth_bytes;   /* bytes copied device -> host (0: no DtH)           */
    int64_t kern_elems;  /* floats the kernel scales per pass                 */
    int32_t kern_iters;  /* passes (0: no kernel); the duration is linear in   */
                         /* kern_elems * kern_iters (Eq. 1)                   */
    int32_t kern_kind;   /* TGO_HW_KERNEL_HBM or TGO_HW_KERNEL_ALU (else       */
                         /* TGO_EINVAL)                                        */
} tgo_hw_task;

typedef struct {
    int64_t start_ns[3], end_ns[3]; /* HtD, K, DtH; ns after the group's start */
} tgo_hw_times;

/* Pinned host buffers, device buffers and three non-blocking streams for up
 * to max_tasks tasks of at most max_bytes per copy and max_kern_elems floats
 * per kernel, on the current device.  Owned by the handle. */
int tgo_hw_create(int max_tasks, int64_t max_bytes, int64_t max_kern_elems, tgo_hw **out);
void tgo_hw_destroy(tgo_hw *hw);
/* Run n tasks (h_tasks on the host) in h_order with the one- or two-DMA scheme
 * (dma_engines 1: one transfer stream holding every HtD then every DtH; 2: an
 * HtD stream, a kernel stream, a DtH stream), wait for them, and return the
 * makespan and, if h_cmds is not NULL, each task's command times (indexed by
 * task).  The streams are held for 2 ms first so that enqueueing on the host
 * does not delay the device.  Blocking. */
int tgo_hw_run(tgo_hw *hw, const tgo_hw_task *h_tasks, int n, const uint8_t *h_order, int dma_engines,
               int64_t *h_total_ns, tgo_hw_times *h_cmds);
/* Several workers with dependent tasks (Section 6.2, NoReorder setup) on the
 * device: task (w, r) at index w * rounds + r of h_tasks; h_seq lists the
 * workers * rounds task indices round by round (positions r * workers ..
 * hold round r's tasks).  The HtD of (w, r) waits for the DtH of (w, r - 1)
 * through an event on the in-order HtD stream; with one DMA engine each
 * round's HtDs then its DtHs go to the transfer stream.  Otherwise as
 * tgo_hw_run (h_cmds indexed by task).  Blocking. */
int tgo_hw_run_rounds(tgo_hw *hw, const tgo_hw_task *h_tasks, int workers, int rounds, const uint8_t *h_seq,
                      int dma_engines, int64_t *h_total_ns, tgo_hw_times *h_cmds);

/* Like tgo_hw_run, under a device-memory limit (the reading of
 * tgo_exhaustive_mem): h_mem[x] = task x's footprint in bytes (0..capacity),
 * capacity in 1..TGO_MAX_CAPACITY.  Two DMA engines: the HtD at position j is
 * made to wait (an event wait on the in-order HtD queue) for the DtH of the
 * last position whose buffers would not fit beside those of positions up to
 * j.  One DMA engine: the ordering is cut greedily into sub-groups whose
 * footprints fit together, each enqueued as its HtDs then its DtHs.  The
 * runner's buffers are allocated up front; the limit is enforced by these
 * waits, which is what a pool of `capacity` bytes would impose. */
int tgo_hw_run_mem(tgo_hw *hw, const tgo_hw_task *h_tasks, int n, const uint8_t *h_order, const int64_t *h_mem,
                   int64_t capacity, int dma_engines, int64_t *h_total_ns, tgo_hw_times *h_cmds);
/* The Heuristic setup of Section 6.2 on the device: a host proxy loop offers
 * task (w, r) once the DtH of (w, r - 1) has ended (polling its event), takes
 * every offered task as a group, orders it with Algorithm 1 (run on the
 * device, from the solo durations h_dur of the tasks, under `model`) and
 * enqueues it with the scheme of model->dma_engines; it looks again once the
 * HtD of the group's last task has started, or at the next arrival.
 * h_seq (16 bytes, optional) receives the submission order and h_groups
 * (optional) the group ends (bit j: position j ends a group); otherwise as
 * tgo_hw_run.  Blocking; TGO_ERANGE if the tasks do not finish within 120 s. */
int tgo_hw_run_proxy(tgo_hw *hw, const tgo_model *model, const tgo_hw_task *h_tasks, const tgo_task *h_dur,
                     int workers, int rounds, int64_t *h_total_ns, uint8_t *h_seq, uint16_t *h_groups,
                     tgo_hw_times *h_cmds);
/* An HtD of htd_bytes and, on another stream, a DtH of dth_bytes issued
 * dth_delay_ns after it (a device-side wait), as in the overlap experiment of
 * Section 4.2.1.  h_times[4] = HtD start, HtD end, DtH start, DtH end (ns).
 * Blocking. */
int tgo_hw_overlap(tgo_hw *hw, int64_t htd_bytes, int64_t dth_bytes, int64_t dth_delay_ns, int64_t *h_times);
/* Least-squares line y = slope * x + intercept over n >= 2 points (host); the
 * kernel model T = eta * m + gamma of Eq. 1, and transfer time against size. */
int tgo_fit_line(const double *h_x, const double *h_y, int n, double *slope, double *intercept);
/* Overlap rates from n overlap experiments (Section 4.2.1): h_times as
 * returned by tgo_hw_overlap (4 per experiment), h_solo the solo HtD and DtH
 * durations (2 per experiment).  With L the overlapped time of an experiment,
 * a transfer's solo work = its time outside the overlap + rho * L; rho is
 * fitted over all experiments as sum(solo - outside) / sum(L).  Experiments
 * without overlap are skipped (TGO_EINVAL if none overlaps). */
int tgo_fit_overlap(const int64_t *h_times, const int64_t *h_solo, int n, double *rho_htd, double *rho_dth);

/* Host helpers for the search space of Section 1 (the n! launch orderings of a
 * group, which every enumeration call ranks lexicographically, rank 0 = the
 * identity): tgo_rank gives the rank of a permutation h_order of 0..n-1
 * (TGO_EINVAL if it is not one, n outside 1..16), tgo_unrank the ordering of
 * a rank (TGO_ERANGE for rank >= n!).  Index arithmetic only, no device. */
int tgo_rank(int n, const uint8_t *h_order, uint64_t *rank);
int tgo_unrank(int n, uint64_t rank, uint8_t *h_order);

#ifdef __cplusplus
}
#endif
#endif /* TGO_H */
