/*
 * qap.h -- C ABI of libqap, the MI355X (gfx950) hot path of the pairwise-exchange
 * heuristics for the Quadratic Assignment Problem of Novoa & Qasem,
 * "GPU-accelerated Parallel Solutions to the Quadratic Assignment Problem"
 * (arXiv 2307.11248).
 *
 * Notation (Sec. 2.1 of the paper, restated 0-based):
 *   n        problem size: n units are assigned to n locations.
 *   F        flows between units,     row-major n x n int32: F[k*n + l].
 *   D        distances between locations, row-major n x n int32: D[i*n + j].
 *   perm     perm[i] is the unit stored in location i (a permutation of 0..n-1).
 *   cost     Eq. (1): z = sum_i sum_j F[perm[i]][perm[j]] * D[i][j], as int64.
 *   move     (r, s), r < s: exchange the contents of locations r and s (Sec. 4.1).
 *   packed   moves are numbered in packed upper-triangle order
 *              idx(r, s) = r*n - r*(r+1)/2 + (s - r - 1),
 *            which is lexicographic (r, s) order; ties between equal deltas always go
 *            to the lowest idx.
 *
 * Buffers: every pointer is owned by the caller.  "host" pointers are ordinary CPU
 * memory; "device" pointers are HIP device memory of the GPU the handle was created
 * on.  Host entry points block until their results are in host memory.  *_async entry
 * points enqueue work on the HIP stream `stream` (NULL = the default stream), return
 * without waiting, and neither read nor write their buffers from the host.
 *
 * Exactness: all flows and distances must lie in [0, 255].  Then every delta fits in
 * int32 with a wide margin (|delta| <= (2n-2) * 255 * 255 < 2^26 for n <= 512) and every
 * cost in int64, and all results are exact integers, identical to a plain CPU
 * evaluation of the paper's formulas.
 *
 * Errors are returned as negative codes (qap_strerror maps them to text).  A call that
 * fails leaves its output buffers in an unspecified state.  A handle may be used from
 * one host thread at a time.
 */
#ifndef QAP_H_
#define QAP_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QAP_NMAX 512
/* Largest n of the batched (qap_batch_*) and served (qap_server_*) searches: every n up
 * to QAP_NMAX. */
#define QAP_NMAX_BATCH 512

enum {
    QAP_OK = 0,
    QAP_E_INVALID = -1,   /* null pointer, n < 2, n > QAP_NMAX, k < 0, iters < 0, lo < 0, lo > hi,
                             iters + hi >= 2^31 - 1 (the tabu-until iteration must fit int32) */
    QAP_E_NOT_PERM = -2,  /* a row of perms is not a permutation of 0..n-1 */
    QAP_E_RANGE = -3,     /* a flow or distance lies outside [0, 255] */
    QAP_E_DEVICE = -4,    /* a HIP call failed */
    QAP_E_NOMEM = -5,     /* host or device allocation failed */
    QAP_E_BUSY = -6,      /* the server's queue is full (qap_server_submit*); nothing was queued */
    QAP_E_UNSUPPORTED = -7, /* valid request this build cannot serve (see the entry point) */
    QAP_E_SCRATCH = -8    /* qap_tabu_noalloc_async: the call needs more than its fixed scratch */
};

/* Bytes of the fixed device array that qap_tabu_noalloc_async takes its scratch from. */
#define QAP_NOALLOC_SCRATCH_BYTES (64u << 20)

typedef struct qap_ctx *qap_handle;

/* Text for an error code; never NULL. */
const char *qap_strerror(int code);

/*
 * Create a handle for one instance (F, D) of size n (Sec. 2.1) on the current HIP
 * device.  F and D are host pointers, read once and copied; the handle owns its device
 * copies until qap_destroy.  Returns QAP_E_RANGE if an entry lies outside [0, 255].
 * Every entry point serves every n <= QAP_NMAX: the searches hold the neighbourhood in
 * registers and F, F^T, D, D^T in LDS while that fits one workgroup (n <= 176 in the
 * batched kernels), and above that run the streamed kernel (neighbourhood in global
 * memory, only G = F[p][p] in LDS).  Above n = 256 they run its wide form, which keeps no
 * G (it reads F and F^T through the permutation), and the neighbourhood table is built by
 * a blocked matrix-core kernel.  QAP_E_UNSUPPORTED is left for a device whose LDS is
 * smaller than the streamed kernel needs.
 */
int qap_create(const int32_t *F, const int32_t *D, int32_t n, qap_handle *out);

/* Release a handle and its device memory.  NULL is accepted. */
int qap_destroy(qap_handle h);

/* n of a handle, or QAP_E_INVALID. */
int qap_size(qap_handle h);

/*
 * Eq. (1): costs[j] = z(perms[j]) for j < k.  perms: host int32[k][n]; costs: host
 * int64[k].  Every row is checked to be a permutation (QAP_E_NOT_PERM otherwise).
 */
int qap_cost(qap_handle h, const int32_t *perms, int32_t k, int64_t *costs);

/* Device/stream twin of qap_cost; rows are not checked, and a row that is not a
 * permutation yields costs[j] = INT64_MIN. */
int qap_cost_async(qap_handle h, const int32_t *d_perms, int32_t k, int64_t *d_costs,
                   void *stream);

/*
 * The whole pairwise-exchange neighbourhood (Sec. 4.1) of each start: for j < k and
 * every move (r, s), table[j * m + idx(r, s)] = z(perms[j] with r, s exchanged) -
 * z(perms[j]), m = n(n-1)/2, i.e. Eq. (2) with the diagonal term that the printed
 * equation omits (zero when D has a zero diagonal).  perms: host int32[k][n];
 * table: host int32[k][m].
 */
int qap_delta_table(qap_handle h, const int32_t *perms, int32_t k, int32_t *table);

/* Device/stream twin of qap_delta_table (rows are not checked). */
int qap_delta_table_async(qap_handle h, const int32_t *d_perms, int32_t k, int32_t *d_table,
                          void *stream);

/*
 * 2opt (Secs. 4.1-4.2), read as best improvement: from each start, repeatedly take the
 * move with the lowest delta (lowest idx among equal deltas) while that delta is
 * negative.  The search stops at a local optimum, or after max_iters moves when
 * max_iters > 0 (max_iters <= 0: no cap; the integer cost strictly decreases, so the
 * search always ends).
 *   perms     host int32[k][n]: the starts on entry, the final permutations on return.
 *   costs_out host int64[k]: their costs.
 *   steps_out host int32[k] or NULL: moves made by each start.
 */
int qap_2opt(qap_handle h, int32_t *perms, int32_t k, int32_t max_iters, int64_t *costs_out,
             int32_t *steps_out);

/* Device/stream twin of qap_2opt.  d_steps may be NULL.  Rows are checked on the device:
 * a row that is not a permutation is left as it is, with d_steps[j] = QAP_E_NOT_PERM and
 * d_costs[j] = INT64_MIN. */
int qap_2opt_async(qap_handle h, int32_t *d_perms, int32_t k, int32_t max_iters,
                   int64_t *d_costs, int32_t *d_steps, void *stream);

/*
 * Elementary tabu search with recency memory (Secs. 4.3-4.4), one independent search per
 * start, iterations it = 1 .. iters:
 *   - a move is tabu at iteration it iff its Tabuarr entry is > it (entries start at 0);
 *   - aspiration: a tabu move is allowed if it reaches a cost strictly below the best
 *     cost found so far;
 *   - the allowed move with the lowest delta is made, even if it worsens the cost (ties:
 *     lowest idx); the best permutation is replaced only on a strictly lower cost;
 *   - after the move (r, s) of iteration it, Tabuarr(r, s) = it + t, with the tenure t
 *     drawn from [lo, hi] as lo + ((x >> 32) * (hi - lo + 1) >> 32), where x is the first
 *     word of Philox4x64-10 (Salmon et al., SC'11) with key (seed, 0) and counter
 *     (it, start_id, 0, 0); start_id = j for the host entry point;
 *   - if no move is allowed the search stops early (Sec. 4.4).
 *   perms          host int32[k][n]: the starts on entry, the best permutations on return.
 *   best_costs_out host int64[k].
 *   iters_done_out host int32[k] or NULL: moves made (< iters only after an early stop).
 */
int qap_tabu(qap_handle h, int32_t *perms, int32_t k, int32_t iters, int32_t lo, int32_t hi,
             uint64_t seed, int64_t *best_costs_out, int32_t *iters_done_out);

/* Device/stream twin of qap_tabu; start j uses start_id = start_base + j.  d_done may be
 * NULL.  Rows are checked on the device as in qap_2opt_async. */
int qap_tabu_async(qap_handle h, int32_t *d_perms, int32_t k, int32_t iters, int32_t lo,
                   int32_t hi, uint64_t seed, int64_t start_base, int64_t *d_best,
                   int32_t *d_done, void *stream);

/*
 * qap_tabu_async that also keeps the frequency memory of Sec. 4.3: the number of times
 * each pair of locations was exchanged (the lower triangle of Tabuarr), and may use it
 * to diversify, which the paper leaves to future work (Sec. 7).
 *   div     0: the counts decide nothing, as in the paper (the searches and results are
 *           those of qap_tabu_async).  > 0: whenever the best cost has not improved for
 *           more than div iterations (counted from the last new best or the last such
 *           move), the next move is the non-tabu pair exchanged least often so far, ties
 *           to the lowest packed index, whatever its delta and without aspiration; if
 *           every move is tabu, the ordinary move is made.
 *   attr    what is tabu.  0: the pair of locations exchanged (Tabuarr, Sec. 4.3), as
 *           qap_tabu_async.  1: the units, after Zhu et al.'s marking of moved units
 *           (Sec. 3.1): the two units moved at iteration it are marked until it + t, and
 *           a move is tabu while either unit it would move is marked.  2: unit-location
 *           pairs, after Taillard's robust tabu search (cited in Sec. 4.3): after the move
 *           of iteration it neither of the two units may return to the location it left
 *           until it + t, and a move is tabu when both units it would move would return to
 *           such a location (needs k * n * n int32 of stream-ordered device scratch).
 *   d_freq  device int32[k][n(n-1)/2], overwritten: row j holds start j's counts at packed
 *           pair index r*n - r*(r+1)/2 + (s - r - 1) for r < s (the order of
 *           qap_delta_table); the counts sum to the moves made.
 * QAP_E_INVALID if d_freq is NULL with k > 0, div < 0 or attr not 0, 1 or 2; otherwise as
 * qap_tabu_async.  Every tile shape serves it, the streamed kernel included.
 */
int qap_tabu_freq_async(qap_handle h, int32_t *d_perms, int32_t k, int32_t iters, int32_t lo,
                        int32_t hi, uint64_t seed, int64_t start_base, int32_t div, int32_t attr,
                        int64_t *d_best, int32_t *d_done, int32_t *d_freq, void *stream);

/*
 * Debugging aid, to find the first step at which the device and a reference disagree:
 * qap_tabu_freq_async (same arguments and results) that also records the first
 * trace_cap moves of every start: d_trace is device int64[k][trace_cap][4], and move t
 * (made at iteration t + 1, t < trace_cap) of start j is written as (r, s, delta, cost
 * after the move) at d_trace[(j * trace_cap + t) * 4]; entries past the moves made are
 * left as they are.  It runs the frequency-memory kernels, so it is slower than
 * qap_tabu_async.  QAP_E_INVALID also for d_trace NULL with k > 0 or trace_cap < 0.
 */
int qap_tabu_trace_async(qap_handle h, int32_t *d_perms, int32_t k, int32_t iters, int32_t lo,
                         int32_t hi, uint64_t seed, int64_t start_base, int32_t div, int32_t attr,
                         int64_t *d_best, int32_t *d_done, int32_t *d_freq, int64_t *d_trace,
                         int32_t trace_cap, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): qap_tabu_async with the same
 * arguments, semantics and results, which calls no allocating routine.  Its scratch (the
 * neighbourhood tables, int32[k][n(n-1)/2] rounded up to 256 bytes, and for the streamed
 * kernels the tile state of every search) is carved
 * from one fixed array of QAP_NOALLOC_SCRATCH_BYTES per GPU, which the library holds
 * from the first qap_create on that GPU until the process ends.  A call that would need
 * more returns QAP_E_SCRATCH and enqueues nothing.  Every call on one GPU shares that
 * array: calls whose work overlaps on the device race and give undefined results, so
 * order them (one stream, or events).  Nothing in the array needs to start at zero.
 */
int qap_tabu_noalloc_async(qap_handle h, int32_t *d_perms, int32_t k, int32_t iters, int32_t lo,
                           int32_t hi, uint64_t seed, int64_t start_base, int64_t *d_best,
                           int32_t *d_done, void *stream);

/*
 * The plain delivery of qap_tabu_async: the same arithmetic and results, but one kernel
 * launch per start, issued back to back on `stream` (the launch shape the paper uses
 * for its per-search kernels, Sec. 4.4, one search at a time).  Kept as the baseline
 * the batched delivery is measured against.
 */
int qap_tabu_plain_async(qap_handle h, int32_t *d_perms, int32_t k, int32_t iters, int32_t lo,
                         int32_t hi, uint64_t seed, int64_t start_base, int64_t *d_best,
                         int32_t *d_done, void *stream);

/*
 * The search kernels alone: as qap_2opt_async / qap_tabu_async, but the neighbourhood
 * of each start is taken from d_table (device int32[k][m], m = n(n-1)/2, packed order)
 * instead of being computed first; it must be the neighbourhood of d_perms, e.g. from
 * qap_delta_table_async on the same stream.  d_table is only read.
 */
int qap_2opt_with_table_async(qap_handle h, int32_t *d_perms, const int32_t *d_table, int32_t k,
                              int32_t max_iters, int64_t *d_costs, int32_t *d_steps, void *stream);
int qap_tabu_with_table_async(qap_handle h, int32_t *d_perms, const int32_t *d_table, int32_t k,
                              int32_t iters, int32_t lo, int32_t hi, uint64_t seed,
                              int64_t start_base, int64_t *d_best, int32_t *d_done, void *stream);

/*
 * Batched tabu search over many instances of uneven n in one launch (the many starts
 * of Secs. 4.4 and 5.2, delivered for many instances at once).  Instance i (handle
 * hs[i], size n_i) runs k_per[i] starts with tenure range [lo_per[i], hi_per[i]] and
 * seed seed_per[i], all for `iters` iterations; its start j uses start_id = j, so every
 * result equals that of qap_tabu on the instance alone.  Starts and results are
 * concatenated in instance order: starts (and best permutations) int32[sum k_i n_i],
 * best costs int64[sum k_i], moves made int32[sum k_i].
 * qap_batch_create plans the batch (tile shape per instance: rows_per[i], or NULL / 0
 * for the library's choice; instances whose n no tile shape of the batched kernel
 * serves give QAP_E_UNSUPPORTED) and owns its device descriptors and neighbourhood
 * scratch until qap_batch_destroy.  qap_batch_run_async only enqueues kernels on
 * `stream` (it allocates nothing, so it may be captured in a HIP graph); the plan may
 * be run any number of times, one run at a time.  It is qap_batch_tables_async (every
 * start's neighbourhood table, Eq. (2), into the plan's scratch) followed by
 * qap_batch_search_async (every search, from those tables); the two halves may be
 * enqueued separately, in that order, on one stream.  The search half runs one kernel
 * per tile-shape variant in use; with more than one, they run on side streams of the
 * plan forked from and joined back to `stream` by events (one fewer side streams than
 * the hardware queues HIP gives the process, GPU_MAX_HW_QUEUES, unless the environment
 * variable QAP_BATCH_LANES, read by qap_batch_create, sets the count); results do not
 * depend on it.  qap_batch_size reports the number
 * of starts and of permutation entries.  A device-side row that is not a permutation is
 * left as it is, with best cost INT64_MIN and moves QAP_E_NOT_PERM.
 * Blocking host forms (rows of perms are checked; QAP_E_NOT_PERM otherwise):
 *   qap_tabu_batch         per-instance host arrays: perms[i] int32[k_per[i]][n_i] (the
 *                          starts on entry, the best permutations on return) and
 *                          best_out[i] int64[k_per[i]].
 *   qap_tabu_batch_concat  the concatenated layout above, with the moves made in
 *                          done_out (int32[sum k_i], may be NULL).
 */
typedef struct qap_batch *qap_batch_handle;
int qap_batch_create(const qap_handle *hs, int32_t m, const int32_t *k_per, int32_t iters,
                     const int32_t *lo_per, const int32_t *hi_per, const uint64_t *seed_per,
                     const int32_t *rows_per, qap_batch_handle *out);
/*
 * qap_batch_create for searches that keep the frequency memory of Sec. 4.3 and may use
 * the extensions of qap_tabu_freq_async: instance i's searches run with diversification
 * patience div_per[i] and tabu attribute attr_per[i] (as div and attr of
 * qap_tabu_freq_async; either array may be NULL for 0 everywhere).  Every result equals
 * qap_tabu_freq_async on the instance alone with start_base 0.  The plan owns the counts
 * of every search (int32 per packed pair) and, for attr 2, the unit x location table of
 * every such search (n_i * n_i int32).  All searches of such a plan run in one launch of
 * 512-lane workgroups with tiles of 2, 4 or 8 rows or the streamed form (rows_per as for
 * qap_batch_create; by default the library's shape, or the next larger tile that fits 512
 * lanes).  QAP_E_INVALID for div < 0 or attr outside 0..2; QAP_E_UNSUPPORTED also for
 * an instance whose shape leaves that kernel (which carries every shape and holds LDS
 * of its own) too little LDS (general instances of n above about 245); otherwise as
 * qap_batch_create.
 * qap_batch_run_async, qap_batch_tables_async and qap_batch_search_async run such plans
 * as any other; qap_batch_groups returns 1 and counts the searches per tile shape in the
 * slots of the 512-lane kernels and the streamed form.
 * qap_batch_freq_async enqueues on `stream` a copy of the counts of the plan's last run
 * into d_freq (device int32[sum_i k_i n_i (n_i - 1) / 2]: instance order, start order,
 * packed pair order); QAP_E_INVALID for a plan made by qap_batch_create.
 */
int qap_batch_create_freq(const qap_handle *hs, int32_t m, const int32_t *k_per, int32_t iters,
                          const int32_t *lo_per, const int32_t *hi_per, const uint64_t *seed_per,
                          const int32_t *rows_per, const int32_t *div_per, const int32_t *attr_per,
                          qap_batch_handle *out);
int qap_batch_freq_async(qap_batch_handle b, int32_t *d_freq, void *stream);
int qap_batch_size(qap_batch_handle b, int64_t *starts_out, int64_t *perm_ints_out);
/* Kernel dispatches of one qap_batch_search_async: returns the number of tile-shape
 * variants the plan uses (one dispatch each, forked onto side streams of `stream` and
 * joined back), and, when count_out (int32[9]) is not NULL, the searches per variant in
 * the order: tiles of 2, 4, 8 rows on 512 lanes, streamed, 2 rows on 128 and on 256
 * lanes, 4 rows on 256 and on 768 lanes, the wide streamed form (n above 256). */
int qap_batch_groups(qap_batch_handle b, int32_t *count_out);
int qap_batch_run_async(qap_batch_handle b, int32_t *d_perms, int64_t *d_best, int32_t *d_done,
                        void *stream);
int qap_batch_tables_async(qap_batch_handle b, const int32_t *d_perms, void *stream);
int qap_batch_search_async(qap_batch_handle b, int32_t *d_perms, int64_t *d_best, int32_t *d_done,
                           void *stream);
int qap_batch_destroy(qap_batch_handle b);
int qap_tabu_batch(const qap_handle *hs, int32_t m, int32_t *const *perms, const int32_t *k_per,
                   int32_t iters, const int32_t *lo_per, const int32_t *hi_per, const uint64_t *seed_per,
                   int64_t *const *best_out);
int qap_tabu_batch_concat(const qap_handle *hs, int32_t m, int32_t *perms, const int32_t *k_per,
                          int32_t iters, const int32_t *lo_per, const int32_t *hi_per,
                          const uint64_t *seed_per, int64_t *best_out, int32_t *done_out);

/*
 * Serving: tabu solves of uneven n submitted one at a time, run with continuous
 * batching over device-resident state (the many-search delivery of Secs. 4.4 and 5.2,
 * applied to a stream of requests).
 *
 * qap_server_create reserves a device memory pool of pool_bytes and slots for up to
 * max_active concurrent searches, on the current HIP device; chunk_ms is the device time
 * each search runs per step (0: every search runs to its end in one step).
 *
 * Submitting (never blocks; the request is queued and its ticket returned):
 *   qap_server_submit          a request on an existing handle h (its device copies of F
 *                              and D are used in place; the handle must stay alive until
 *                              the request has finished or been cancelled), one start
 *                              permutation (host int32[n], copied), iteration count,
 *                              tenure range [lo, hi] and Philox seed (start id 0).
 *   qap_server_submit_matrices the same with its own F and D (host int32[n][n], copied
 *                              into the pool on admission), which need no handle.
 * Both check as qap_create and qap_tabu do (QAP_E_INVALID, QAP_E_RANGE, QAP_E_NOT_PERM),
 * return QAP_E_NOMEM at once if the request's footprint (qap_server_footprint(s, n, sym)
 * bytes with its own matrices, sym = 1 when F and D are both symmetric, 4 n RS bytes
 * less on a handle) exceeds the whole pool, QAP_E_UNSUPPORTED if no kernel shape serves
 * n on this device, and QAP_E_BUSY if the queue already holds
 * qap_server_set_queue_limit requests (default 65536).
 *
 * Stepping: each step admits queued requests in arrival order while a slot is free and
 * their footprint fits the pool (a request that does not fit is passed over by later
 * ones that do, for at most 8 steps, after which nothing behind it is admitted first),
 * then runs one chunk of every admitted search in one launch (a second one for searches
 * above n = 256): each search runs until
 * about chunk_ms of device time has passed, stopping at an iteration boundary, with its
 * permutation, neighbourhood, tabu list and best solution kept in the pool in between.
 * Searches that finished are then collected and their slot and memory freed.  Every
 * result equals that of qap_tabu on the same instance, start, iterations, tenure range
 * and seed (start id 0), whatever else was admitted alongside and however it was
 * chunked.  Steps are driven by the caller, qap_server_step (blocks for one step and
 * returns how many searches finished, and the numbers still running and queued), or by
 * the server's own host thread between qap_server_start and qap_server_stop (while it
 * runs qap_server_step returns QAP_E_INVALID; qap_server_stop returns the error that
 * stopped the thread, if any, and is implied by qap_server_destroy).
 *
 * Collecting: qap_server_poll returns 1 and the best permutation (host int32[n], may be
 * NULL) and best cost (may be NULL) once the request has finished, after which its ticket
 * is forgotten; 0 while it is queued or running.  qap_server_result is the same with the
 * moves made and, in latency_ms_out[2] (may be NULL), the time from submission to the
 * step that finished it and the time spent queued, in ms.  A search that failed on the
 * device (its saved state found corrupt) returns QAP_E_DEVICE once, then is forgotten;
 * the other searches are unaffected.  An unknown ticket gives QAP_E_INVALID.
 *
 * qap_server_cancel drops a queued or running request (1; a running search leaves at
 * the next step boundary and its ticket is forgotten at once), or returns 0 if it has
 * already finished (its result stays to be collected).  qap_server_inject_failure is a
 * test hook: the running request's saved permutation is overwritten with an invalid one
 * before the next chunk, so that its search fails there as a corrupted search would
 * (QAP_E_INVALID unless the request is running).
 *
 * qap_server_stats fills int64[9]: running, queued, pool bytes in use, pool bytes,
 * steps, chunks run, searches finished, failed, cancelled.  Every server function may be
 * called from any host thread.
 */
typedef struct qap_server *qap_server_handle;
int qap_server_create(int64_t pool_bytes, int32_t max_active, double chunk_ms, qap_server_handle *out);
int64_t qap_server_footprint(qap_server_handle s, int32_t n, int32_t sym);
int qap_server_submit(qap_server_handle s, qap_handle h, const int32_t *start, int32_t iters, int32_t lo,
                      int32_t hi, uint64_t seed, int64_t *ticket_out);
int qap_server_submit_matrices(qap_server_handle s, const int32_t *F, const int32_t *D, int32_t n,
                               const int32_t *start, int32_t iters, int32_t lo, int32_t hi, uint64_t seed,
                               int64_t *ticket_out);
int qap_server_set_queue_limit(qap_server_handle s, int32_t max_queued);
/*
 * A served request with the extensions of qap_tabu_freq_async (div, attr as there): the
 * search keeps the frequency memory of Sec. 4.3 in the pool (with attr 2 its unit-location
 * table, with attr 1 its unit marks between chunks, n (n - 1) / 2 + n^2 or + n int32 more),
 * and its result equals qap_tabu_freq_async on the handle with start_base 0, however it
 * was chunked.  Such requests run in a launch of their own each step.  On a handle only;
 * QAP_E_UNSUPPORTED above n = 256, and where that launch's kernel, which carries every
 * tile shape, has too little LDS left for the request's (general, not symmetric,
 * instances of n above about 245); otherwise as qap_server_submit.
 * qap_server_poll_freq is qap_server_poll that also copies the counts into freq_out (host
 * int32[n (n - 1) / 2], packed pair order; may be NULL); QAP_E_INVALID, leaving the
 * request alone, if freq_out is not NULL and the request was not submitted this way.
 */
int qap_server_submit_freq(qap_server_handle s, qap_handle h, const int32_t *start, int32_t iters,
                           int32_t lo, int32_t hi, uint64_t seed, int32_t div, int32_t attr,
                           int64_t *ticket_out);
int qap_server_poll_freq(qap_server_handle s, int64_t ticket, int32_t *best_perm, int64_t *best_cost,
                         int32_t *freq_out);
int qap_server_step(qap_server_handle s, int32_t *active_out, int32_t *pending_out);
int qap_server_start(qap_server_handle s);
int qap_server_stop(qap_server_handle s);
int qap_server_poll(qap_server_handle s, int64_t ticket, int32_t *best_perm, int64_t *best_cost);
int qap_server_result(qap_server_handle s, int64_t ticket, int32_t *perm_out, int64_t *best_out,
                      int32_t *moves_out, double *latency_ms_out);
int qap_server_cancel(qap_server_handle s, int64_t ticket);
int qap_server_inject_failure(qap_server_handle s, int64_t ticket);
int qap_server_stats(qap_server_handle s, int64_t *out);
int qap_server_destroy(qap_server_handle s);

/*
 * Tile shape of the search kernels (the thread-configuration search of Sec. 5.2,
 * re-done for gfx950): each lane of a search's workgroup holds a block of `rows` x 4
 * neighbourhood entries in registers, rows in {1, 2, 4, 8, 16}; rows = -8 selects the
 * streamed kernel (tiles of 8 rows kept in global memory and updated in passes, D read
 * from global memory; 512 lanes; serves every n up to QAP_NMAX); 0 restores the
 * library's own choice, made per launch for tabu and 2opt: among the register tiles that
 * fit n, the one that needs the fewest rounds of workgroups over the compute units for
 * the launch's k starts (HIP's occupancy query), ties going to the smallest tile; else
 * the streamed kernel.  A shape set here (or by the autotuner) holds for every launch.
 * algo: 0 = tabu, 1 = 2opt, 2 = this instance inside a batch (qap_batch_create with
 * rows_per NULL or 0; rows 2, 4, 8 or -8; each search gets the smallest batched
 * workgroup with a lane per tile and per (index, family) task: 128, 256 or 512 lanes,
 * 768 for tiles of 4 rows beyond 512 tiles).  Returns QAP_E_UNSUPPORTED if the shape
 * does not fit this n (lanes or LDS).
 */
int qap_set_tile_rows(qap_handle h, int32_t algo, int32_t rows);

/* Tile rows currently used for algo, and the lanes per search in *lanes_out (may be
 * NULL); in the automatic mode, the shape of a launch of one start.  Same as
 * qap_launch_tile_rows(h, algo, 1, lanes_out). */
int qap_get_tile_rows(qap_handle h, int32_t algo, int32_t *lanes_out);

/* Tile rows (and lanes per search in *lanes_out, may be NULL) that a launch of k >= 1
 * starts of algo uses: the shape set for algo, or the automatic choice for k.
 * QAP_E_INVALID for bad arguments, QAP_E_UNSUPPORTED if no kernel serves n. */
int qap_launch_tile_rows(qap_handle h, int32_t algo, int32_t k, int32_t *lanes_out);

/*
 * Autotuner of the tile shape (replaces the paper's search over thread counts and block
 * sizes, Sec. 5.2 and Eq. (3), with measurement): for algo (as above) runs k searches of
 * `iters` iterations (2opt: at most `iters` moves) from fixed pseudo-random starts with
 * every shape that fits n, times the search kernel with HIP events (one warm-up run
 * first), stores the fastest as the handle's shape for algo and returns its rows.
 * ms_out (float[6] or NULL) receives the time per rows value 1, 2, 4, 8, 16, -8, or -1
 * where a shape does not fit.  Blocking; allocates its own device buffers; results do not
 * depend on the shape, only the time does.
 */
int qap_tune_tile_rows(qap_handle h, int32_t algo, int32_t k, int32_t iters, float *ms_out);

#ifdef __cplusplus
}
#endif

#endif /* QAP_H_ */
