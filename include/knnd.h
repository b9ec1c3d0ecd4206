/*
 * knnd.h -- C ABI of libknnd.so: comparator-based K-nearest-neighbor descent
 * with the Kullback-Leibler comparator, on an AMD Instinct MI355X (gfx950).
 *
 * Method: Baron & Darling, "Empirical complexity of comparator-based nearest
 * neighbor descent" (arXiv 2202.00517).
 *   - Problem statement (Abstract; Section 2.3): n points, each point x gets
 *     the K other points most similar to it in x's own order.
 *   - Comparator (Section 2.2; Section 4 scaling experiment): y ranks before z
 *     for x when D(x||y) < D(x||z), D(x||y) = sum_i x_i log(x_i / y_i),
 *     summed over all d+1 stored coordinates.  Asymmetric, not a metric.
 *     The descent needs only one total order per point (Section 2.1, a
 *     ranking system; Section 1.3 (a)): knnd_comparator lists the others
 *     this library offers.
 *   - Descent (Section 3.1): rounds of friend-of-a-friend candidate generation
 *     ("Meet": co-friends, friends of friends, friends of co-friends) and
 *     best-K selection ("Update"), each round computed from the round-start
 *     snapshot (Section 4.2).
 *   - Start (Section 3.2): a random K-out digraph without self-loops.
 *   - Stop (Section 3.3): after the first round whose sampled friend
 *     clustering rate does not increase.
 *
 * Exact conventions fixed by this library (the paper leaves them open):
 *   key(x,y)   : logs are the correctly rounded FP64 natural logs of the
 *                coordinates (FP32 inputs widened exactly); the key folds
 *                acc = fma(x_i, log x_i - log y_i, acc) for i = 0..d in
 *                ascending order, from acc = +0.0, all in FP64.
 *   order      : (key, index) lexicographic; ties go to the lower index.
 *   start      : draw a of point x is r = floor(H(seed,1,x,a) * (n-1) / 2^64),
 *                y = r + (r >= x); the first K distinct draws are the friends.
 *   FCR sample : s = 0..M-1 of round r: x = bnd(H(seed,2,r,s), n),
 *                a = bnd(H(seed,3,r,s), K), b' = bnd(H(seed,4,r,s), K-1),
 *                b = b' + (b' >= a); hit when F(x)[b] is a friend of
 *                F(x)[a] or F(x)[a] is a friend of F(x)[b].
 *   stop       : by default (KNND_STOP_FCR) after round r when
 *                hits_r <= hits_{r-1}, or no list changed (fixed point), or
 *                r == max_rounds; knnd_stop_rule lists the other rules.
 *   H          : SplitMix64-finalizer hash
 *                H(s,t,a,b) = mix64(mix64(mix64(s ^ t*0x9E3779B97F4A7C15) ^ a) ^ b).
 * Results depend only on (points, K, seed, fcr_samples, max_rounds, the stop
 * rule and its delta, the comparator): not on the precision mode, on tiling
 * or on scheduling.
 *
 * Threading: calls on distinct contexts/outputs may run concurrently.
 * Nothing is retained between calls except inside a knnd_ctx and the device
 * memory cache (knnd_release_cache).  No C++ exception crosses this ABI.  On
 * error, outputs are unspecified.
 */
#ifndef KNND_H
#define KNND_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KNND_ABI_VERSION 7

typedef enum {
    KNND_OK = 0,
    KNND_WARN_MAX_ROUNDS = 1,   /* stopped by the round cap, not by the stop test */
    KNND_ERR_ARG = -1,          /* null pointer, n < 2, d < 1, K < 2, K > n-1, K > 64,
                                   n >= 2^30, max_rounds < 1, unknown enum value */
    KNND_ERR_DOMAIN = -2,       /* a coordinate is NaN, infinite or <= 0 */
    KNND_ERR_NOMEM = -3,        /* device allocation failed */
    KNND_ERR_DEVICE = -4,       /* a HIP call failed, or no gfx950 device */
    KNND_ERR_UNSUPPORTED = -5   /* valid request the library does not implement */
} knnd_status;

typedef enum { KNND_F32 = 0, KNND_F64 = 1 } knnd_dtype;

/*
 * Precision of the key evaluation.  Every mode returns the same lists and
 * keys (the canonical FP64 ones); the mixed modes only change speed and the
 * `rescues` count.  In a mixed mode the cross term sum_i x_i log c_i is
 * formed on the matrix cores from 16-bit operands, each split into a high
 * and a low part (three products per pair, FP32 accumulation), and bounded
 * by a proven error bound; a candidate gets its canonical FP64 key when its
 * bound interval says it may enter the list.  The mixed modes apply when
 * d+1 <= 64, every coordinate is <= 1 (points of the simplex) and the logs
 * fit the 16-bit range; otherwise the exact hub form runs (same results).
 */
typedef enum {
    KNND_PREC_FP64 = 0,         /* every key computed in canonical FP64 */
    KNND_PREC_MIXED_BF16 = 1,   /* BF16 split operands, FP64 rescue */
    KNND_PREC_MIXED_FP16 = 2,   /* FP16 split operands, FP64 rescue */
    KNND_PREC_AUTO = 3          /* the exact FP64 form or the BF16 mixed form,
                                   whichever the library's autotuner measures
                                   faster on the first round's join (per group
                                   in batched calls, which tune in every
                                   mode; the second round's join then tries
                                   guarded 4096-slot receiver tables);
                                   choices are cached per
                                   workload shape in the process and, when the
                                   environment variable KNND_TUNE_CACHE names a
                                   file, in that file */
} knnd_precision;

/* flags */
#define KNND_FLAG_NO_SKIP 0x1   /* also evaluate candidates reached only through
                                   edges that were already present one round
                                   earlier (same result, more work) */
#define KNND_FLAG_PULL 0x2      /* join in pull form (each receiver gathers its
                                   candidates' log rows) instead of hub form
                                   (same result) */
#define KNND_FLAG_ATOMIC_CSR 0x4 /* build the reverse-neighbour lists with one
                                   device-wide atomic per edge (the form used
                                   above 2^25 points) instead of the bucketed
                                   counting sort (same result) */
#define KNND_FLAG_NO_GRAPH 0x10 /* batched calls: enqueue every round's kernels
                                   one by one instead of replaying the rounds
                                   after the third from captured graphs
                                   (same result) */
#define KNND_FLAG_NO_TUNE 0x20  /* no timing of candidate join schedules:
                                   k_hub_reg in the exact form, and
                                   KNND_PREC_AUTO runs the BF16 mixed form
                                   (same result) */
#define KNND_FLAG_NO_CARRY 0x8  /* evaluate every receiver in late rounds too,
                                   instead of carrying over the list and the
                                   evaluation count of a receiver whose
                                   neighbourhood did not change (same result,
                                   more work; see `carried` below) */

/*
 * Comparators (Section 2.1: any family of per-point total orders; Section 1.3
 * (a)).  Each ranks y before z for x by a key k(x, y), folded in FP64 over
 * the d+1 coordinates in ascending order from +0.0 with one fma per term, ties
 * to the lower index:
 *   KNND_CMP_KL          D(x||y): acc = fma(x_i, log x_i - log y_i, acc) (the
 *                        paper's; coordinates finite and > 0)
 *   KNND_CMP_KL_REVERSE  D(y||x): acc = fma(y_i, log y_i - log x_i, acc)
 *                        (coordinates finite and > 0)
 *   KNND_CMP_HELLINGER   t = sqrt(x_i) - sqrt(y_i), acc = fma(t, t, acc): twice
 *                        the squared Hellinger distance (coordinates finite
 *                        and >= 0; IEEE square roots)
 *   KNND_CMP_L2          t = x_i - y_i, acc = fma(t, t, acc): the squared
 *                        Euclidean distance (coordinates finite)
 * The logs are the correctly rounded FP64 logs of the coordinates, as above.
 * The mixed precision modes apply to KNND_CMP_KL only; with another
 * comparator every key is computed in FP64 (same results).
 */
typedef enum {
    KNND_CMP_KL = 0,
    KNND_CMP_KL_REVERSE = 1,
    KNND_CMP_HELLINGER = 2,
    KNND_CMP_L2 = 3
} knnd_comparator;

/*
 * Termination (Section 1.2, Table 1, and Section 1.3, item (b)).  Every
 * rule runs the same rounds and differs only in the round after which it
 * stops, so a run under one rule is a prefix of the run under any rule that
 * stops later.  Every
 * rule also stops at r == max_rounds (status KNND_WARN_MAX_ROUNDS when the
 * rule itself would not have stopped there).
 */
typedef enum {
    KNND_STOP_FCR = 0,          /* the paper's statistical criterion: stop after
                                   round r when hits_r <= hits_{r-1} (friend
                                   clustering rate no longer rising) or no list
                                   changed */
    KNND_STOP_FIXED_POINT = 1,  /* stop after the first round in which no list
                                   changed: no possible update remains */
    KNND_STOP_DELTA = 2         /* Dong et al.'s rule: stop after the first round
                                   whose update count u_r satisfies
                                   (double)u_r <= delta * (double)n * (double)K,
                                   evaluated in FP64 left to right */
} knnd_stop_rule;

typedef struct {
    int32_t precision;          /* knnd_precision */
    int32_t dtype;              /* knnd_dtype of `points` */
    int64_t fcr_samples;        /* M; <= 0 selects min(n, 10000) */
    int32_t max_rounds;         /* <= 0 selects 100 */
    int32_t flags;              /* KNND_FLAG_* */
    int32_t stop_rule;          /* knnd_stop_rule */
    int32_t comparator;         /* knnd_comparator */
    double delta;               /* KNND_STOP_DELTA only: finite, >= 0 */
} knnd_params;

/* Per-round record.  Entry 0 describes the initial graph (fcr_hits only). */
typedef struct {
    int64_t updates;            /* sum over x of |F_r(x) \ F_{r-1}(x)| */
    int64_t fcr_hits;           /* friend clustering hits out of M samples */
    int64_t evals_alg;          /* sum over x of |candidates of x|: one KL key per
                                   (x, distinct non-friend candidate) */
    int64_t evals_performed;    /* keys actually computed on the device */
    int64_t rescues;            /* FP64 rechecks (mixed precision only) */
    double ms;                  /* device time of the round (HIP events) */
    double ms_join;             /* device time of the join kernels (steps a2-a5) */
    double ms_hub;              /* part of ms_join: the hub kernel (keys or cross
                                   terms per snapshot edge; 0 in the pull form) */
    double ms_recv;             /* part of ms_join: the receiver kernels (dedup,
                                   rescue, merge, every size class) */
    int64_t carried;            /* receivers whose list and evaluation count were
                                   carried over from the last round: its list,
                                   its friends' and co-friends' lists were all
                                   unchanged and no list dropped it, so its
                                   candidate set is the same (Section 3.1) and
                                   every candidate lost again.  Single descents
                                   in the hub form, once a round changed at most
                                   0.1% of the entries; 0 otherwise */
    int64_t evals_carried;      /* the part of evals_alg those receivers add
                                   (counted, not evaluated again) */
} knnd_round_stats;

/* Fill *p with the defaults (FP64, F32 points, M = min(n,10000), 100 rounds,
   KNND_STOP_FCR, delta 0, KNND_CMP_KL, flags 0). */
void knnd_default_params(knnd_params* p);

/*
 * Device memory.  Scratch blocks a finished call or a destroyed context
 * gives back are kept in a per-process cache (per device, by rounded size,
 * at most half of the first device's memory or, if more, as much as the
 * library has had in use at once since the cache was last released; the
 * oldest are freed first) and reused by later calls, so
 * that repeated calls skip hipMalloc and hipFree.  knnd_release_cache()
 * returns every cached block to the device (blocks in use by live contexts
 * stay).  Thread-safe; returns KNND_OK.
 */
int knnd_release_cache(void);

/*
 * Bytes of device memory the library holds: *live in blocks that live
 * contexts and running calls use, *cached in the cache above (either pointer
 * may be NULL).  Every call and every destroyed context gives its blocks
 * back, so between calls *live is the memory of the live contexts (0 when
 * there are none).  Thread-safe; returns KNND_OK.
 */
int knnd_memory_stats(int64_t* live, int64_t* cached);

/*
 * Test support (failure injection): after knnd_test_fail_alloc(k) with
 * k >= 1, the k-th device allocation the library makes from then on fails as
 * if the device were out of memory (once); k <= 0 disarms.  Returns how many
 * allocations were still to go before the armed failure (0 when none was
 * armed or it has fired), so that a caller can tell whether a call reached
 * it.  A buffer the method needs turns such a failure into KNND_ERR_NOMEM
 * with every block given back; an optional one (the hub and mixed-precision
 * forms' buffers, the neighbourhood-tracking flags) makes the call run the
 * next form instead, with the same results.  Process-wide, not meant for
 * concurrent calls.
 */
int64_t knnd_test_fail_alloc(int64_t k);

/* Human-readable name of a knnd_status value (static storage). */
const char* knnd_status_string(int status);

int knnd_abi_version(void);

/*
 * The basic call (Abstract; Section 2.3 problem statement).
 *   points      host, [n][d+1] FP32 row-major, every coordinate finite and > 0
 *               (points of the open simplex; the library never clamps)
 *   out_idx     host, caller-allocated [n][K] int32: row x lists x's friends
 *               best first in (key, index) order
 *   out_updates host, caller-allocated [max_rounds] int64: entry r-1 is the
 *               number of list changes in round r
 *   max_rounds  round cap (>= 1)
 *   out_rounds  host, rounds executed
 * Uses the current HIP device and its null stream.  Returns a knnd_status.
 */
int knnd_build(const float* points, int64_t n, int32_t d, int32_t K, uint64_t seed,
               int32_t* out_idx, int64_t* out_updates, int32_t max_rounds,
               int32_t* out_rounds);

/*
 * Extended form.
 *   points      [n][d+1] in p->dtype; host memory when on_device == 0,
 *               device memory of the current HIP device when on_device != 0
 *   p           parameters (NULL = defaults)
 *   stream      hipStream_t as void* (NULL = null stream); all device work is
 *               enqueued on it; the host synchronises once per round (stop
 *               test) and fully before returning
 *   out_idx     [n][K] int32, same memory kind as points
 *   out_kl      optional [n][K] FP64 keys of out_idx, same memory kind
 *   stats       optional host array [max_rounds + 1]
 *   out_rounds  host
 */
int knnd_build_ex(const void* points, int64_t n, int32_t d, int32_t K, uint64_t seed,
                  const knnd_params* p, int32_t on_device, void* stream,
                  int32_t* out_idx, double* out_kl, knnd_round_stats* stats,
                  int32_t* out_rounds);

/*
 * For callers that cannot allocate device memory (serving loops and
 * harnesses that forbid hipMalloc / hipFree): the descent of knnd_build_ex
 * with device pointers (on_device = 1), with every device buffer carved from
 * a fixed scratch array of KNND_NOALLOC_MAX_BYTES that the library holds on
 * each device it runs on until the process ends.  The call allocates
 * nothing: no hipMalloc, hipFree, pinned host memory, events or memory-cache
 * blocks.  Same arguments, results and errors as knnd_build_ex, except:
 *   points, out_idx, out_kl   device memory of the current device (caller-owned)
 *   stats                     host array, as in knnd_build_ex; the ms fields are 0
 *   returns KNND_ERR_NOMEM, before any device work, when the buffers of the
 *   descent do not fit the scratch array.  The richest form that fits runs
 *   (mixed, else hub, else pull form; all give the same results): at K = 16
 *   and d = 10 about 6*10^4 points fit the mixed form, 3.5*10^4 the hub
 *   form and 2*10^5 the pull form.
 * Calls on one device share its scratch array, which keeps the last call's
 * contents: calls that overlap on one device race (run them in order on one
 * stream or serialise them).  The stream is synchronised once per round.
 */
#define KNND_NOALLOC_MAX_BYTES 268435456ull  /* 256 MiB per device */
int knnd_build_noalloc(const void* points, int64_t n, int32_t d, int32_t K, uint64_t seed,
                       const knnd_params* p, void* stream, int32_t* out_idx, double* out_kl,
                       knnd_round_stats* stats, int32_t* out_rounds);

/*
 * Batched form: B independent descents in one call (each instance exactly
 * what knnd_build_ex would return for it with the same params).
 *   inst        host array [B].  Per instance, inputs: points ([n][d+1] in
 *               p->dtype, host or device memory per on_device), n, d, K, seed;
 *               outputs: out_idx [n][K] int32 and optional out_kl [n][K] FP64
 *               (same memory kind as points), optional host stats
 *               [max_rounds + 1], host out_rounds, and status (KNND_OK or
 *               KNND_WARN_MAX_ROUNDS).
 *   p           shared parameters (NULL = defaults); fcr_samples <= 0 gives
 *               each instance min(n, 10000) samples.
 *   stream      as in knnd_build_ex; the host synchronises once per round for
 *               all instances together.
 * Instances are grouped by K and number of coordinates; a group runs as one
 * set of persistent kernel launches per round, and an instance leaves its
 * group's rounds after its own stop test.  Rounds after the third are one
 * launch of a captured graph holding every running group's kernels, each
 * group a branch of its own (two
 * graphs, one per parity of the double-buffered lists; captured again when
 * a whole group has stopped; KNND_FLAG_NO_GRAPH enqueues the kernels one by
 * one instead).  `ms` in an instance's stats is the device time of the
 * whole round of every running group; ms_join, ms_hub and ms_recv are 0.
 * Returns KNND_OK, KNND_WARN_MAX_ROUNDS when some instance hit
 * the round cap, or the first error (then every output is unspecified);
 * argument errors of any instance are reported before any device work.
 */
typedef struct {
    const void* points;
    int64_t n;
    int32_t d;
    int32_t K;
    uint64_t seed;
    int32_t* out_idx;
    double* out_kl;
    knnd_round_stats* stats;
    int32_t* out_rounds;
    int32_t status;
    int32_t reserved;
} knnd_instance;

int knnd_build_batched(knnd_instance* inst, int32_t B, const knnd_params* p, int32_t on_device,
                       void* stream);

/*
 * Exact K nearest neighbours of query points by exhaustive comparison (the
 * problem of Section 2.3 solved directly; the accuracy measure of Section 4.4
 * compares a descent's lists with these).  For query point q every other
 * point p is ranked by the same canonical key k(q, p) of the comparator
 * (knnd_comparator; KNND_CMP_KL: D(q||p)) and (key, index) order as the
 * descent.
 *   points   [n][d+1] of dtype (knnd_dtype), host or device memory per
 *            on_device; every coordinate in the comparator's domain;
 *            d+1 <= 256
 *   queries  [nq] int32 point indices (same memory kind), each in [0, n)
 *   tau      optional [nq] FP64 (same kind): an upper bound on each query's
 *            K-th smallest key, e.g. the K-th key of a descent's list for that
 *            point (saves one pass over the points); NULL: computed here
 *   out_idx  [nq][K] int32 (same kind): the K nearest in (key, index) order
 *   out_kl   optional [nq][K] FP64 keys (same kind)
 * Device scratch: about 49 KB per query.  Returns KNND_ERR_ARG for bad sizes,
 * a query index out of range or a tau below the K-th key,
 * an unknown comparator, KNND_ERR_UNSUPPORTED for d+1 > 256,
 * KNND_ERR_DOMAIN for bad coordinates.
 */
int knnd_exact_knn(const void* points, int64_t n, int32_t d, int32_t K, int32_t dtype,
                   int32_t comparator, const int32_t* queries, int64_t nq, const double* tau,
                   int32_t on_device, void* stream, int32_t* out_idx, double* out_kl);

/*
 * Step-by-step interface (the same path, one call per step).  A context owns
 * its device buffers until knnd_ctx_destroy.  Pointers marked "kind" are host
 * memory when on_device == 0 and device memory when on_device != 0.
 */
typedef struct knnd_ctx knnd_ctx;

/* Validate and upload points, build the comparator's feature table (the log
   table for the KL comparators).  points: [n][d+1] of kind. */
int knnd_ctx_create(const void* points, int64_t n, int32_t d, int32_t K, uint64_t seed,
                    const knnd_params* p, int32_t on_device, void* stream, knnd_ctx** out);

/* Random K-out start (Section 3.2), sorted lists, FCR of round 0 into st. */
int knnd_ctx_init_graph(knnd_ctx* c, knnd_round_stats* st);

/* Replace the current lists by idx [n][K] int32 and kl [n][K] FP64 (kind).
 * Rows must hold K distinct indices != x, sorted by (kl, index), with kl the
 * canonical keys.  Every edge counts as new at the next round.  The round
 * counter becomes `round`. */
int knnd_ctx_set_graph(knnd_ctx* c, const int32_t* idx, const double* kl, int32_t round,
                       int32_t on_device);

/* One synchronous round (Sections 3.1, 4.2) and its FCR sample (Section 3.3).
 * Fills st (host) and synchronises the context's stream. */
int knnd_ctx_round(knnd_ctx* c, knnd_round_stats* st);

/* One round for a share of the receivers.  Each vertex's new list is a task
 * of its own that reads only the round-start graph, which is what lets the
 * paper spread the vertices over processors (Section 4.2); a GPU's share of
 * a descent split over several GPUs is such a range.  The lists of points
 * first .. first+count-1 are recomputed exactly as knnd_ctx_round would;
 * every other list is carried over unchanged.  The next round skips no
 * candidate pair (an edge present a round earlier no longer means that the
 * pairs through it were evaluated then), so later rounds stay exact.  The hub
 * kernel computes only the keys those receivers read.  st counts the
 * share's evaluations, updates and rescues; fcr_hits is taken on the whole
 * graph after the round.  Returns KNND_ERR_ARG when the context has no graph
 * yet, first < 0, count < 1 or first + count > n.  Synchronises the
 * context's stream. */
int knnd_ctx_round_share(knnd_ctx* c, int64_t first, int64_t count, knnd_round_stats* st);

/* Copy the current lists out: idx [n][K] int32, kl optional [n][K] FP64 (kind). */
int knnd_ctx_get_graph(knnd_ctx* c, int32_t* idx, double* kl, int32_t on_device);

/* The co-friend lists (reverse neighbours, Section 3.1) of the current
   lists, as the next round builds them: the points x with y in F(x) are
   col[rowptr[y] .. rowptr[y+1]), each segment in increasing order.  rowptr
   [n+1] int64 and col [n*K] int32 are host memory (on_device must be 0, else
   KNND_ERR_UNSUPPORTED).  The join itself leaves the order inside a segment
   free (nothing it computes depends on it); the segments are sorted on the
   host here.  Synchronises the context's stream. */
int knnd_ctx_get_cofriends(knnd_ctx* c, int64_t* rowptr, int32_t* col, int32_t on_device);

/* Copy the feature table out: L [n][d+1] FP64 (kind): log x for the KL
   comparators, sqrt x for Hellinger, x for Euclidean. */
int knnd_ctx_get_log_table(knnd_ctx* c, double* L, int32_t on_device);

/* Rounds completed so far. */
int knnd_ctx_rounds(const knnd_ctx* c);

int knnd_ctx_destroy(knnd_ctx* c);

#ifdef __cplusplus
}
#endif

#endif /* KNND_H */
