/*
 * passjoin.h -- C ABI of libpassjoin, an MI355X (gfx950) implementation of the Pass-Join
 * edit-distance similarity join (G. Li, D. Deng, J. Wang, J. Feng, "Pass-Join: A
 * Partition-based Method for Similarity Joins").
 *
 * Problem (Sec. 2, Definition 1): given string sets R and S and a threshold tau, report every
 * pair <r, s> in R x S with ED(r, s) <= tau, where ED is the Levenshtein distance (unit-cost
 * insertions, deletions, substitutions).  The self-join (R = S, Sec. 2) reports each unordered
 * pair of distinct ids once.
 *
 * Method (run on the GPU, integers only, exact): even partition of every indexed string into
 * tau+1 segments (Sec. 3.1); an inverted index keyed by (length, slot, segment) (Sec. 3.2);
 * multi-match-aware substring selection (Sec. 4.2, Algorithm 2); extension-based verification
 * with tau_l = i-1, tau_r = tau+1-i (Sec. 5.2, Algorithm 3) using the length-aware band and the
 * expected-edit-distance early termination (Sec. 5.1, Lemma 4).  Strings shorter than tau+1 are
 * not partitionable (footnote to Sec. 3.1); pairs that involve one are verified directly.
 *
 * Conventions for every entry point:
 *  - Return value 0 (PJ_OK) on success, a negative PJ_E* code on failure.  On failure every
 *    output is zeroed, nothing is leaked, and pj_last_error() describes the cause.
 *  - Strings are raw bytes (no normalisation).  A string set is an arena: `bytes` holds all
 *    strings back to back, `offsets[k] .. offsets[k+1]` delimits string k (id k), offsets[0] must
 *    be 0 and offsets must be non-decreasing.  Lengths are limited to PJ_LEN_MAX, tau to
 *    [0, PJ_TAU_MAX].
 *  - Inputs are borrowed for the duration of the call; they are host pointers unless
 *    pj_options.inputs_on_device is set, in which case they are device pointers on the current
 *    HIP device.  Device inputs are checked before any kernel reads them: both pointers must
 *    be device (or managed) memory of the current device, the allocation holding `offsets`
 *    must hold n + 1 entries and the one holding `bytes` at least offsets[n] bytes (`bytes`
 *    may be NULL only when offsets[n] == 0); otherwise PJ_EINVAL.  The call returns when its
 *    results are complete.
 *  - Outputs are owned by the caller and released with pj_pairs_free / pj_index_free.
 *  - Results are sets with one canonical order, so a given input has exactly one correct output.
 *  - Calls are thread-safe with respect to each other; error text and statistics are kept per
 *    calling thread.
 */
#ifndef PASSJOIN_H
#define PASSJOIN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PJ_OK        0
#define PJ_EINVAL   -1   /* null pointer, n < 0, bad offsets, tau out of [0, PJ_TAU_MAX] */
#define PJ_ERANGE   -2   /* a string longer than PJ_LEN_MAX, a query tau outside the index */
#define PJ_ENOMEM   -3   /* host or device allocation failed, or the memory budget is exceeded */
#define PJ_EDEVICE  -4   /* a HIP runtime error */

#define PJ_TAU_MAX  63
#define PJ_LEN_MAX  2047

/* Execution modes (pj_options.mode). */
#define PJ_MODE_AUTO     0   /* the fastest available: currently PJ_MODE_BATCHED */
#define PJ_MODE_PLAIN    1   /* one kernel per phase, candidates materialised, host-sized */
#define PJ_MODE_BATCHED  2   /* length-bucketed persistent probe/verify, graph-captured phases */
#define PJ_MODE_SHARE_PREFIX 3 /* PJ_MODE_BATCHED with the big inverted lists verified by
                                  sharing computations on common prefixes (Sec. 5.3): list
                                  members in content order, each lane verifying a chain of
                                  consecutive members and resuming every DP after the rows the
                                  member shares with its predecessor (up to 16 stored rows).
                                  Same pairs and counters; pj_stats.shared_rows/shared_cells
                                  count the work taken over.  For tau <= 8 (larger tau: as
                                  PJ_MODE_BATCHED) */

/* A borrowed string set (see the conventions above). */
typedef struct {
    int64_t n;                 /* number of strings, >= 0 */
    const uint8_t* bytes;      /* concatenated string bytes (may be NULL when offsets[n] == 0) */
    const int32_t* offsets;    /* n + 1 offsets */
} pj_strings;

/* Result pairs, owned by the caller.  a[k], b[k] are ids; the list is sorted by (a, b) and has
 * no duplicates.  on_device tells where a and b live: 0 host memory (malloc), 1 device memory
 * (pj_options.outputs_on_device), 2 page-locked host memory (hipHostMalloc; host results of a
 * megabyte or more per array, which the device writes at the link's full rate).  Release with
 * pj_pairs_free whatever the kind. */
typedef struct {
    int64_t count;
    int32_t* a;
    int32_t* b;
    int32_t on_device;
} pj_pairs;

/* Substring selection (pj_options.selection): which substrings of a probe string are looked up
 * in the segment index.  All four find every similar pair (Sec. 4); they differ in how many
 * substrings and candidates they generate, multi-match the fewest (Lemma 3, Sec. 4.2).  Windows
 * of start positions, restricted to where the probe string has a substring of length l_i:
 *   multi-match  the intersection of [p_i - (i-1), p_i + (i-1)] and
 *                [p_i + Delta - (tau+1-i), p_i + Delta + (tau+1-i)]            (Sec. 4.2)
 *   position     [p_i - floor((tau-Delta)/2), p_i + floor((tau+Delta)/2)]    (Sec. 4.1)
 *   shift        [p_i - tau, p_i + tau]                                       (Sec. 4)
 *   length       every start position                                        (Sec. 4)
 * Delta = |probe string| - l.  Serving queries always use multi-match. */
#define PJ_SELECT_MULTIMATCH 0
#define PJ_SELECT_POSITION   1
#define PJ_SELECT_SHIFT      2
#define PJ_SELECT_LENGTH     3

/* Per-call options; a NULL pointer means all defaults (zero-initialised struct). */
typedef struct {
    void* hip_stream;          /* hipStream_t the work is ordered on; NULL = the null stream */
    int32_t inputs_on_device;  /* 1: pj_strings pointers are device pointers */
    int32_t outputs_on_device; /* 1: pj_pairs stay in device memory */
    int32_t mode;              /* PJ_MODE_* */
    int32_t selection;         /* PJ_SELECT_* (pj_self_join, pj_join, pj_tune); 0 = multi-match */
    int64_t mem_budget_bytes;  /* 0 = no limit; otherwise the device bytes a call may hold */
    const char* tune_cache;    /* autotune cache file (read, and written when tuning); NULL = none */
} pj_options;

/* Counters and phase times of the last call made on the calling thread. */
typedef struct {
    int64_t strings;       /* strings in the probe and indexed sets */
    int64_t index_entries; /* (string, slot) entries in the segment index */
    int64_t selected;      /* substrings selected by the multi-match windows and looked up */
    int64_t hits;          /* selected substrings that found a non-empty inverted list */
    int64_t candidates;    /* (y, x, i, p) candidates after the visiting-order filter: x[p, l_i]
                              equals segment i of y */
    int64_t cells;         /* DP cells evaluated by extension verification (Sec. 5.1 band) */
    int64_t accepted;      /* candidates that passed, before deduplication */
    int64_t side_pairs;    /* pairs examined directly because a string is shorter than tau+1 */
    int64_t pairs;         /* pairs reported */
    double ms_upload, ms_index, ms_probe, ms_verify, ms_output, ms_total;
    double ms_probe_kernel;    /* device time of the probe kernel launches (hipEvents) */
    double ms_verify_kernel;   /* device time of the verification kernel launches (hipEvents) */
    int64_t verify_launches;   /* verification kernel launches */
    double ms_list_kernel;     /* device time of the list-segment verification launches */
    int64_t list_cells;        /* cells evaluated by the list-segment verification */
    int64_t list_launches;     /* list-segment verification launches */
    int64_t key_collisions;    /* lookups whose hashed segment key matched a list of other
                                  bytes: rejected by the byte comparison before verification and
                                  not counted in candidates */
    int64_t shared_rows;       /* PJ_MODE_SHARE_PREFIX: DP rows taken from the previous member
                                  of a content-ordered list instead of being computed (Sec. 5.3) */
    int64_t shared_cells;      /* the cells of those rows (included in cells, which counts every
                                  cell of the method's band; cells - shared_cells were computed) */
    int64_t replayed;          /* pj_plan_run: 1 if the call replayed the plan's captured graph,
                                  0 if it ran the self-join anew (the strings had changed) */
} pj_stats;

/* Self-join (Sec. 2, Algorithm 1): every pair of distinct ids a < b of S with
 * ED(S[a], S[b]) <= tau, sorted by (a, b).  Pairs are found from the later string in
 * (length, id) order, which yields the same set as the paper's (length, bytes) order. */
int pj_self_join(const pj_strings* S, int32_t tau, const pj_options* opt, pj_pairs* out);

/* Self-join of a set that need not fit in device memory, in windows of lengths (the sliding
 * window of live inverted lists of Sec. 3.2 taken in blocks): a window [a, b] moves the strings
 * with lengths in [a - tau, b] to the device, lets the strings of length >= a probe, and keeps
 * the pairs whose longer string is at least a long, so every similar pair is reported by exactly
 * one window.  Windows are cut greedily so that their strings hold at most window_bytes bytes
 * (at least one length per window).  S and the result are in host memory
 * (opt->inputs_on_device and opt->outputs_on_device must be 0); the result equals
 * pj_self_join's.  The windows' pairs are kept on the device and sorted there once; pairs beyond
 * a 64th of the device memory free at the first window are sorted and moved to host memory in
 * batches, which the host merges (the device then holds the current window and one batch).
 * pj_last_stats sums the windows' counters.  Errors as pj_self_join, and PJ_EINVAL for
 * window_bytes <= 0. */
int pj_self_join_streamed(const pj_strings* S, int32_t tau, int64_t window_bytes,
                          const pj_options* opt, pj_pairs* out);

/* A prepared self-join of one device-resident string set, for callers that join the same data
 * repeatedly (the phases of Algorithm 1 as in pj_self_join): its launches are captured once in a
 * hipGraph and replayed.  pj_self_join_plan runs the self-join of S once (S in device memory:
 * opt->inputs_on_device = 1), recording the sizes each phase reads back, then captures the same
 * launches on a stream of the plan's own with device buffers of the plan's own, and records a
 * checksum of S.  The plan keeps S's pointers and the other options (mode, selection, tune
 * cache, the stream whose earlier work a run waits for): the caller keeps S's memory valid while
 * the plan exists.  Memory: the buffers of one self-join of S, held until pj_plan_free.  Errors
 * as pj_self_join, and PJ_EINVAL for host strings. */
typedef struct pj_plan pj_plan;
int pj_self_join_plan(const pj_strings* S, int32_t tau, const pj_options* opt, pj_plan** out);

/* Runs a plan: the result of pj_self_join on S as it is now, in new device arrays
 * (out->on_device = 1).  First checks on the device that S's offsets and bytes are those the
 * plan was made from (a checksum; the bytes read are bounded by the allocation measured at plan
 * time); if so, replays the graph (pj_last_stats() holds the plan's counters, replayed = 1);
 * otherwise runs the self-join of S anew (replayed = 0).  Two host synchronisations when
 * replaying.  Calls on one plan must not overlap. */
int pj_plan_run(pj_plan* plan, pj_pairs* out);
void pj_plan_free(pj_plan* plan);

/* Join of two sets (Definition 1, Sec. 3.2): every (r, s) with ED(R[r], S[s]) <= tau, sorted by
 * (r, s).  S is indexed and each r probes the lengths |r|-tau .. |r|+tau. */
int pj_join(const pj_strings* R, const pj_strings* S, int32_t tau, const pj_options* opt,
            pj_pairs* out);

/* Opaque device-resident index of one string set for every tau in [tau_min, tau_max]: the even
 * partition segments of Sec. 3.1 in inverted lists keyed by (length, slot, segment), Sec. 3.2.
 * Read-only after build; may be shared by concurrent pj_query calls. */
typedef struct pj_index pj_index;

/* Builds an index of S for every tau in [tau_min, tau_max] (0 <= tau_min <= tau_max <=
 * PJ_TAU_MAX).  S is copied to the device; the caller may release it after the call. */
int pj_build_index(const pj_strings* S, int32_t tau_min, int32_t tau_max, const pj_options* opt,
                   pj_index** out);

/* Number of strings and the tau range of an index (any pointer may be NULL). */
int pj_index_info(const pj_index* idx, int64_t* n, int32_t* tau_min, int32_t* tau_max,
                  int64_t* device_bytes);

/* Queries an index: query q (0 <= q < Q->n) with its own threshold taus[q] (a host array, each
 * in the index's range) is joined against the indexed set as in pj_join.  Pairs are
 * (q, s) sorted by (q, s). */
int pj_query(const pj_index* idx, const pj_strings* Q, const int32_t* taus, const pj_options* opt,
             pj_pairs* out);

/* For callers that cannot allocate memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): pj_query that makes no device allocation and, on success,
 * no host allocation.  Its device work buffers are one static device array per GPU (8 MiB,
 * held until the process ends) and its host staging is static; the results go to the caller's
 * host arrays out_q[k], out_s[k] (k < out_cap), sorted by (q, s), and *out_count receives the
 * number of pairs.  Q and taus are host memory (opt->inputs_on_device and
 * opt->outputs_on_device must be 0); the index must live on the current device.  Capacities:
 * at most 512 queries whose padded strings hold at most 256 KiB, at most 2^18 selected
 * substrings (the Lemma 2 bound, checked before any device work), at most 2^24 candidates and
 * 8,192 accepted candidates (checked on the device); beyond them, or when the pairs exceed
 * out_cap (then *out_count still holds their number), the call returns PJ_ERANGE.  Calls on
 * one process are serialised by the library; the static array keeps the last call's contents
 * and every call resets what must start at zero.  The pairs and all counters equal pj_query's.
 * Errors as pj_query, plus PJ_ERANGE for the capacities above. */
int pj_query_noalloc(const pj_index* idx, const pj_strings* Q, const int32_t* taus,
                     const pj_options* opt, int32_t* out_q, int32_t* out_s, int64_t out_cap,
                     int64_t* out_count);

/* ---- Serving: a request loop over a resident index ------------------------------------------
 *
 * A server owns worker slots, each with its own HIP stream (default priority) and device
 * scratch.  Submitted requests (a query set with per-query thresholds, joined against the index
 * as in pj_query) wait in a FIFO queue; a scheduler thread admits them continuously: whenever a
 * slot is free it merges queued requests into one device batch (up to max_batch_queries queries)
 * as long as the batch's estimated device footprint fits in what the in-flight batches leave of
 * mem_budget_bytes.  Batches on different slots run concurrently on the device.  A request's
 * result does not depend on what it was batched with.
 */
typedef struct pj_server pj_server;

typedef struct {
    int32_t slots;              /* device batches in flight at once, >= 1 */
    int32_t max_batch_queries;  /* queries merged into one device batch, >= 1 */
    int64_t mem_budget_bytes;   /* bound on the summed footprint estimates in flight plus the
                                   slots' fixed buffers (captured mode: about 33 MB per slot,
                                   taken off the budget at start; PJ_ENOMEM if they do not fit);
                                   0 = none.  The estimate leaves out each batch's accepted-
                                   candidate buffer (8 B per candidate, known only after the
                                   probe), so it bounds the other device memory only */
    const char* tune_cache;     /* autotune cache file read by the batches (see pj_tune); NULL =
                                   none.  The string is copied by pj_server_start. */
    int32_t eager;              /* 0: each slot replays one captured hipGraph of the device phases
                                   per batch (batches that exceed its fixed capacities run
                                   uncaptured); 1: every batch runs uncaptured */
} pj_server_config;

/* Timestamps (ms on the server's steady clock since pj_server_start) and admission data. */
typedef struct {
    double t_submit_ms;         /* pj_server_submit accepted the request */
    double t_admit_ms;          /* the scheduler placed it in a device batch */
    double t_done_ms;           /* its pairs were ready in host memory */
    int64_t footprint_bytes;    /* admission estimate: 48 B per selectable substring (hit
                                   record, its bucketed copy, prefix sum, count and scan
                                   scratch) + twice the query bytes */
    int32_t batch_requests;     /* requests in the same device batch */
    int32_t slot;               /* slot that ran it */
    int32_t deferrals;          /* 1 if it reached the head of the queue and could not start at
                                   once (no free slot, or the budget held no room), else 0 */
    int32_t deferred_by_memory; /* 1 if that wait was for memory while a slot was free */
} pj_request_info;

/* Starts a server over idx (which must outlive the server).  cfg NULL = {2, 256, 0, NULL, 0}. */
int pj_server_start(const pj_index* idx, const pj_server_config* cfg, pj_server** out);

/* Submits a request: Q (host memory, copied) with one threshold per query in the index's
 * range.  Returns a request id >= 0, or a negative PJ_E* code (PJ_ENOMEM when the request's own
 * footprint exceeds the budget left after the slots' fixed buffers).  Never blocks on device
 * work. */
int64_t pj_server_submit(pj_server* srv, const pj_strings* Q, const int32_t* taus);

/* Blocks until the request is done; its (q, s) pairs (sorted, q local to the request) go to
 * *out (host memory) and its timing to *info (may be NULL).  Each id can be collected once:
 * if several threads wait on one id, the first to return collects it and the others get
 * PJ_EINVAL. */
int pj_server_wait(pj_server* srv, int64_t request, pj_pairs* out, pj_request_info* info);

/* Stops admitting, finishes the work in flight and queued, then frees the server. */
int pj_server_stop(pj_server* srv);

/* Autotuning of the batched path's launch parameters.  None of them changes a result (the pairs
 * and all counters of pj_stats stay the same); they decide how the candidates of Algorithm 1 are
 * spread over the GPU: the persistent verification grid (waves per compute unit), the list
 * segments (64 candidates per lane slot) a wave takes at a time, the candidate count from which
 * an inverted list is verified a wave at a time instead of candidate by candidate, the probe
 * grid (blocks per compute unit) and its thread mapping, and how many members of one list each
 * lane verifies at once. */
typedef struct {
    int32_t verify_waves_per_cu;   /* 8, 16, 32, ..., 1024, powers of two (default 32) */
    int32_t seg_chunk;             /* 1, 2, 4, ..., 2048, powers of two (default 4) */
    int32_t big_list;              /* 16, 32, 64 or 128 (default 32) */
    int32_t probe_blocks_per_cu;   /* 4, 8 or 16 (default 8) */
    int32_t lane_cands;            /* list-segment candidates per lane: 1 or 2 (default 2) */
    int32_t probe_map;             /* probe threads: 0 a wave over consecutive (length, slot)
                                      pairs of a few probe strings, 1 a wave over 64 probe
                                      strings with one pair (default 0) */
    int32_t len_bucket;            /* key: bit length of the rounded mean string length */
    int32_t trials;                /* settings measured */
    double ms_default;             /* probe + verification kernel time, built-in defaults */
    double ms_best;                /* the same for the chosen setting */
} pj_tune_result;

/* Searches the launch parameters for the self-join of S (host memory) at tau by coordinate
 * descent (repeated until a pass changes nothing, at most 3 passes), timing the probe and
 * verification phases on the device (best of two runs per setting), and
 * records the best setting under (this GPU's architecture, tau, length bucket of S's mean
 * length).  The record is kept for the rest of the process; when opt->tune_cache names a file
 * it is also merged into that file (plain text, one setting per line), which later calls with
 * the same tune_cache read.  opt->inputs_on_device must be 0.  Each trial runs the full
 * self-join, so the cost is about 40-100 joins of S.  Returns PJ_OK or a PJ_E* code. */
int pj_tune(const pj_strings* S, int32_t tau, const pj_options* opt, pj_tune_result* out);

/* Releases pairs (host or device memory as recorded in on_device) and zeroes the struct. */
void pj_pairs_free(pj_pairs* pairs);

/* Releases an index; NULL is ignored. */
void pj_index_free(pj_index* idx);

/* Text describing the last failure on the calling thread ("" if none). */
const char* pj_last_error(void);

/* Copies the statistics of the last successful call on the calling thread. */
int pj_last_stats(pj_stats* out);

/* Library version string. */
const char* pj_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PASSJOIN_H */
