/*
 * pj_oracle.c -- CPU oracle for the Pass-Join edit-distance similarity join.
 *
 * TEST INFRASTRUCTURE.  This is the plain, slow reference that the GPU library is checked
 * against.  Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark load
 * it; the GPU library never does.  It shares no code, header, table or helper with the GPU
 * library: everything below is written out from the paper.
 *
 * Paper: G. Li, D. Deng, J. Wang, J. Feng, "Pass-Join: A Partition-based Method for Similarity
 * Joins".  Positions are 1-based, as in the paper.  Section numbers refer to that paper.
 *
 * Pins (checked by the CPU tests, not by this file): the worked examples of Sec. 2, 3.1, 4.1,
 * 4.2, 5.1 and 5.2, the Lemma 2 closed form, the Lemma 3 subset chain, brute-force edit distance
 * by breadth-first search over edit operations on tiny strings, metric invariants, and the
 * equality of the Pass-Join result with the brute-force join of Definition 1 (Theorem 6).
 */
#define _GNU_SOURCE
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define ORC_INF (1 << 29)

static int32_t imin(int32_t a, int32_t b) { return a < b ? a : b; }
static int32_t imax(int32_t a, int32_t b) { return a > b ? a : b; }
static int32_t iabs(int32_t a) { return a < 0 ? -a : a; }
/* floor(a / 2) for any sign of a */
static int32_t floor_half(int32_t a) { return a >= 0 ? a / 2 : -((-a + 1) / 2); }

/* ------------------------------------------------------------------------------------------ */
/* Edit distance                                                                               */
/* ------------------------------------------------------------------------------------------ */

/* Levenshtein distance by the textbook dynamic program (Sec. 2 definition; Sec. 5.1 recurrence:
 * M(i,j) = min(M(i-1,j)+1, M(i,j-1)+1, M(i-1,j-1)+delta), with M(0,j) = j and M(i,0) = i). */
int32_t orc_ed_full(const uint8_t* r, int32_t lr, const uint8_t* s, int32_t ls)
{
    int32_t* prev = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ls + 1));
    int32_t* cur = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ls + 1));
    for (int32_t j = 0; j <= ls; ++j) prev[j] = j;
    for (int32_t i = 1; i <= lr; ++i) {
        cur[0] = i;
        for (int32_t j = 1; j <= ls; ++j) {
            int32_t delta = (r[i - 1] == s[j - 1]) ? 0 : 1;
            cur[j] = imin(imin(prev[j] + 1, cur[j - 1] + 1), prev[j - 1] + delta);
        }
        int32_t* t = prev; prev = cur; cur = t;
    }
    int32_t d = prev[ls];
    free(prev);
    free(cur);
    return d;
}

/* min(ED(r, s), t + 1) by the 2t+1 diagonal band: only cells with |i - j| <= t are computed,
 * the others are taken as infinite, and the computation stops as soon as a whole row exceeds t
 * (the "length pruning" band and the prefix pruning that Sec. 5.1 attributes to earlier work).
 * Any alignment of cost <= t stays inside the band, so the result is exact whenever ED <= t. */
int32_t orc_ed_band_rows(const uint8_t* r, int32_t lr, const uint8_t* s, int32_t ls, int32_t t,
                         int32_t* rows_done)
{
    if (rows_done) *rows_done = 0;
    if (t < 0) return 0;
    if (iabs(lr - ls) > t) return t + 1;
    int32_t* prev = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ls + 1));
    int32_t* cur = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ls + 1));
    for (int32_t j = 0; j <= ls; ++j) prev[j] = (j <= t) ? j : ORC_INF;
    int32_t result = -1;
    for (int32_t i = 1; i <= lr && result < 0; ++i) {
        int32_t lo = imax(0, i - t), hi = imin(ls, i + t);
        int32_t row_min = ORC_INF;
        for (int32_t j = lo; j <= hi; ++j) {
            int32_t v;
            if (j == 0) {
                v = i;
            } else {
                int32_t up = (j >= imax(0, i - 1 - t) && j <= imin(ls, i - 1 + t)) ? prev[j] : ORC_INF;
                int32_t diag = (j - 1 >= imax(0, i - 1 - t) && j - 1 <= imin(ls, i - 1 + t))
                                   ? prev[j - 1] : ORC_INF;
                int32_t left = (j - 1 >= lo) ? cur[j - 1] : ORC_INF;
                int32_t delta = (r[i - 1] == s[j - 1]) ? 0 : 1;
                v = imin(imin(up + 1, left + 1), diag + delta);
            }
            cur[j] = v;
            row_min = imin(row_min, v);
        }
        if (row_min > t) result = t + 1;
        if (rows_done) *rows_done = i;
        int32_t* tmp = prev; prev = cur; cur = tmp;
    }
    if (result < 0) result = imin(prev[ls], t + 1);
    free(prev);
    free(cur);
    return result;
}

int32_t orc_ed_band(const uint8_t* r, int32_t lr, const uint8_t* s, int32_t ls, int32_t t)
{
    return orc_ed_band_rows(r, lr, s, ls, t, NULL);
}

/* ------------------------------------------------------------------------------------------ */
/* Even partition (Sec. 3.1)                                                                    */
/* ------------------------------------------------------------------------------------------ */

/* Splits a length-l string into tau+1 segments: with k = l - floor(l/(tau+1))*(tau+1), the first
 * tau+1-k segments have length floor(l/(tau+1)) and the last k have length ceil(l/(tau+1)).
 * start[i-1] = p_i (1-based start of segment i), len[i-1] = l_i; p_1 = 1, p_i = p_{i-1} + l_{i-1}
 * (Sec. 4, shift-based method, where p_i is defined). */
void orc_partition(int32_t l, int32_t tau, int32_t* start, int32_t* len)
{
    int32_t q = l / (tau + 1);
    int32_t k = l - q * (tau + 1);
    int32_t p = 1;
    for (int32_t i = 1; i <= tau + 1; ++i) {
        int32_t li = (i <= tau + 1 - k) ? q : q + 1;
        start[i - 1] = p;
        len[i - 1] = li;
        p += li;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Substring selection (Sec. 4)                                                                 */
/* ------------------------------------------------------------------------------------------ */

enum { ORC_SEL_LENGTH = 0, ORC_SEL_SHIFT = 1, ORC_SEL_POSITION = 2, ORC_SEL_MULTIMATCH = 3 };

/* Start-position window [*lo, *hi] (1-based, empty when *lo > *hi) of the substrings of a
 * length-n probe string that are selected for the inverted index of slot i over strings of
 * length l, Delta = n - l (signed: the join of two distinct sets probes lengths up to n + tau,
 * Sec. 3.2).  The four methods are written as the paper states them:
 *   length:      every start with a full substring of length l_i, [1, n - l_i + 1]   (Sec. 4)
 *   shift:       [p_i - tau, p_i + tau]  (no bounds applied, as the paper counts 2tau+1) (Sec. 4)
 *   position:    [max(1, p_i - floor((tau-Delta)/2)), min(n - l_i + 1, p_i + floor((tau+Delta)/2))]
 *                                                                                   (Sec. 4.1)
 *   multi-match: [max(bot_l, bot_r), min(top_l, top_r)] with
 *                bot_l = max(1, p_i - (i-1)),             top_l = min(n - l_i + 1, p_i + (i-1)),
 *                bot_r = max(1, p_i + Delta - (tau+1-i)), top_r = min(n - l_i + 1, p_i + Delta + (tau+1-i))
 *                                                                                   (Sec. 4.2)
 * Returns the number of start positions in the window (0 when empty). */
int32_t orc_window(int32_t method, int32_t n, int32_t l, int32_t tau, int32_t i,
                   int32_t* lo, int32_t* hi)
{
    int32_t start[128], len[128];
    orc_partition(l, tau, start, len);
    int32_t p = start[i - 1], li = len[i - 1];
    int32_t delta = n - l;
    int32_t last = n - li + 1;
    switch (method) {
    case ORC_SEL_LENGTH:
        *lo = 1; *hi = last;
        break;
    case ORC_SEL_SHIFT:
        *lo = p - tau; *hi = p + tau;
        break;
    case ORC_SEL_POSITION:
        *lo = imax(1, p - floor_half(tau - delta));
        *hi = imin(last, p + floor_half(tau + delta));
        break;
    default: {
        int32_t bot_l = imax(1, p - (i - 1));
        int32_t top_l = imin(last, p + (i - 1));
        int32_t bot_r = imax(1, p + delta - (tau + 1 - i));
        int32_t top_r = imin(last, p + delta + (tau + 1 - i));
        *lo = imax(bot_l, bot_r);
        *hi = imin(top_l, top_r);
        break;
    }
    }
    return (*hi >= *lo) ? (*hi - *lo + 1) : 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Verification (Sec. 5)                                                                        */
/* ------------------------------------------------------------------------------------------ */

/* VerifyStringPair (Sec. 5.1 and the function of Algorithm 3): returns min(t+1, ED(r, s)) using
 * the length-aware band and the expected-edit-distance early termination.
 *
 * r is the indexed string's part and s the probe string's part.  The matrix has the shorter part
 * as rows and the longer as columns ("let |s| >= |r|", Sec. 5.1); with equal lengths the rows are
 * r.  With Delta = columns - rows >= 0:
 *   - if Delta > t the distance exceeds t and nothing is computed;
 *   - row i computes only j in [i - floor((t-Delta)/2), i + floor((t+Delta)/2)] (and 0 <= j <= |cols|);
 *     cells outside that range are taken as infinite;
 *   - after each row i >= 1, E(i,j) = M(i,j) + |(|cols| - j) - (|rows| - i)| is formed for the
 *     row's cells; if every one exceeds t the computation stops and t+1 is returned (Lemma 4);
 *   - otherwise the result is min(t+1, M(|rows|, |cols|)).
 * *cells receives the number of recurrence cells evaluated (rows i >= 1, columns j >= 1, within
 * the band, up to and including the row that stopped the computation), *rows the last row
 * computed. */
int32_t orc_verify_pair(const uint8_t* r, int32_t lr, const uint8_t* s, int32_t ls, int32_t t,
                        int64_t* cells, int32_t* rows_done)
{
    const uint8_t *ra, *ca;
    int32_t nr, nc;
    if (lr <= ls) { ra = r; nr = lr; ca = s; nc = ls; }
    else          { ra = s; nr = ls; ca = r; nc = lr; }
    int32_t delta = nc - nr;
    if (cells) *cells = 0;
    if (rows_done) *rows_done = 0;
    if (delta > t) return t + 1;
    int32_t a = floor_half(t - delta);   /* cells left of the diagonal  */
    int32_t b = floor_half(t + delta);   /* cells right of the diagonal */

    int32_t* prev = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nc + 1));
    int32_t* cur = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nc + 1));
    /* row 0: M(0,j) = j inside the band */
    for (int32_t j = 0; j <= nc; ++j) prev[j] = (j <= b) ? j : ORC_INF;
    int64_t ncells = 0;
    int32_t result = -1;
    int32_t i;
    for (i = 1; i <= nr; ++i) {
        int32_t lo = imax(0, i - a), hi = imin(nc, i + b);
        int32_t plo = imax(0, i - 1 - a), phi = imin(nc, i - 1 + b);
        int32_t e_min = ORC_INF;
        for (int32_t j = lo; j <= hi; ++j) {
            int32_t v;
            if (j == 0) {
                v = i;
            } else {
                int32_t up = (j >= plo && j <= phi) ? prev[j] : ORC_INF;
                int32_t diag = (j - 1 >= plo && j - 1 <= phi) ? prev[j - 1] : ORC_INF;
                int32_t left = (j - 1 >= lo) ? cur[j - 1] : ORC_INF;
                int32_t d = (ra[i - 1] == ca[j - 1]) ? 0 : 1;
                v = imin(imin(up + 1, left + 1), diag + d);
                ncells += 1;
            }
            cur[j] = v;
            int32_t e = (v >= ORC_INF) ? ORC_INF : v + iabs((nc - j) - (nr - i));
            e_min = imin(e_min, e);
        }
        int32_t* tmp = prev; prev = cur; cur = tmp;
        if (e_min > t) { result = t + 1; break; }
    }
    if (rows_done) *rows_done = (result >= 0) ? i : nr;
    if (result < 0) result = imin(t + 1, prev[nc]);
    if (cells) *cells = ncells;
    free(prev);
    free(cur);
    return result;
}

/* Extension-based verification of one candidate (Sec. 5.2, Algorithm 3).  x (length n) is the
 * probe string, y (length l) the indexed string whose segment i (1-based) equals x[p .. p+l_i-1].
 * The strings are split around the shared segment: y_l = y[1, p_i-1], x_l = x[1, p-1],
 * y_r = y[p_i+l_i, l], x_r = x[p+l_i, n].  With tau_l = i-1 and tau_r = tau+1-i the candidate
 * passes iff VerifyStringPair(x_l, y_l, tau_l) <= tau_l and VerifyStringPair(x_r, y_r, tau_r) <=
 * tau_r; the right parts are only examined when the left parts pass.  Returns 1 on pass.
 * *cells receives the recurrence cells evaluated by both calls. */
int32_t orc_extension_verify(const uint8_t* x, int32_t n, const uint8_t* y, int32_t l,
                             int32_t tau, int32_t i, int32_t p, int64_t* cells)
{
    int32_t start[128], len[128];
    orc_partition(l, tau, start, len);
    int32_t pi = start[i - 1], li = len[i - 1];
    int32_t tau_l = i - 1, tau_r = tau + 1 - i;
    int64_t c_l = 0, c_r = 0;
    int32_t d_l = orc_verify_pair(y, pi - 1, x, p - 1, tau_l, &c_l, NULL);
    int32_t pass = 0;
    if (d_l <= tau_l) {
        int32_t d_r = orc_verify_pair(y + (pi - 1 + li), l - (pi - 1 + li),
                                      x + (p - 1 + li), n - (p - 1 + li), tau_r, &c_r, NULL);
        pass = (d_r <= tau_r);
    }
    if (cells) *cells = c_l + c_r;
    return pass;
}

/* ------------------------------------------------------------------------------------------ */
/* Results                                                                                     */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
    int64_t count;          /* number of pairs */
    int32_t* a;             /* pairs (a[k], b[k]) */
    int32_t* b;
    int64_t candidates;     /* (y, x, i, p) candidates generated by the index probe */
    int64_t cells;          /* recurrence cells evaluated by the extension verification */
    int64_t selected;       /* substrings selected and looked up */
    int64_t side_pairs;     /* pairs examined by the short-string side path */
    /* candidate list (only when requested): y, x, i, p, pass, cells */
    int64_t ncand;
    int32_t* cy; int32_t* cx; int32_t* ci; int32_t* cp; int32_t* cpass; int64_t* ccells;
    int64_t cap, ccap;
} orc_result;

static orc_result* res_new(void) { return (orc_result*)calloc(1, sizeof(orc_result)); }

static void res_push(orc_result* R, int32_t a, int32_t b)
{
    if (R->count == R->cap) {
        R->cap = R->cap ? R->cap * 2 : 1024;
        R->a = (int32_t*)realloc(R->a, sizeof(int32_t) * (size_t)R->cap);
        R->b = (int32_t*)realloc(R->b, sizeof(int32_t) * (size_t)R->cap);
    }
    R->a[R->count] = a;
    R->b[R->count] = b;
    R->count++;
}

static void res_push_cand(orc_result* R, int32_t y, int32_t x, int32_t i, int32_t p, int32_t pass,
                          int64_t cells)
{
    if (R->ncand == R->ccap) {
        R->ccap = R->ccap ? R->ccap * 2 : 1024;
        size_t c = (size_t)R->ccap;
        R->cy = (int32_t*)realloc(R->cy, sizeof(int32_t) * c);
        R->cx = (int32_t*)realloc(R->cx, sizeof(int32_t) * c);
        R->ci = (int32_t*)realloc(R->ci, sizeof(int32_t) * c);
        R->cp = (int32_t*)realloc(R->cp, sizeof(int32_t) * c);
        R->cpass = (int32_t*)realloc(R->cpass, sizeof(int32_t) * c);
        R->ccells = (int64_t*)realloc(R->ccells, sizeof(int64_t) * c);
    }
    int64_t k = R->ncand++;
    R->cy[k] = y; R->cx[k] = x; R->ci[k] = i; R->cp[k] = p; R->cpass[k] = pass;
    R->ccells[k] = cells;
}

static int cmp_pair(const void* u, const void* v)
{
    const int64_t a = *(const int64_t*)u, b = *(const int64_t*)v;
    return (a > b) - (a < b);
}

/* Sorts the pairs by (a, b) and removes duplicates: the join result is a set (Algorithm 1). */
static void res_sort_unique(orc_result* R)
{
    if (R->count == 0) return;
    int64_t* k = (int64_t*)malloc(sizeof(int64_t) * (size_t)R->count);
    for (int64_t t = 0; t < R->count; ++t)
        k[t] = ((int64_t)R->a[t] << 32) | (int64_t)(uint32_t)R->b[t];
    qsort(k, (size_t)R->count, sizeof(int64_t), cmp_pair);
    int64_t m = 0;
    for (int64_t t = 0; t < R->count; ++t)
        if (m == 0 || k[t] != k[m - 1]) k[m++] = k[t];
    for (int64_t t = 0; t < m; ++t) {
        R->a[t] = (int32_t)(k[t] >> 32);
        R->b[t] = (int32_t)(k[t] & 0xffffffff);
    }
    R->count = m;
    free(k);
}

void orc_result_free(orc_result* R)
{
    if (!R) return;
    free(R->a); free(R->b);
    free(R->cy); free(R->cx); free(R->ci); free(R->cp); free(R->cpass); free(R->ccells);
    free(R);
}

/* ------------------------------------------------------------------------------------------ */
/* Brute-force joins (Definition 1)                                                             */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
    const uint8_t* rc; const int32_t* ro; int64_t rn;   /* probe-side set */
    const uint8_t* sc; const int32_t* so; int64_t sn;   /* other set */
    int32_t tau;
    int32_t self;          /* 1: pairs a < b within one set */
    const int32_t* xs;     /* optional list of probe ids (NULL: all) */
    int64_t nx;
    int32_t tid, nthreads;
    orc_result* out;
} bf_job;

static void* bf_worker(void* arg)
{
    bf_job* J = (bf_job*)arg;
    int64_t nprobe = J->xs ? J->nx : J->rn;
    for (int64_t k = J->tid; k < nprobe; k += J->nthreads) {
        int32_t x = J->xs ? J->xs[k] : (int32_t)k;
        const uint8_t* xp = J->rc + J->ro[x];
        int32_t xl = J->ro[x + 1] - J->ro[x];
        int64_t y0 = (J->self && !J->xs) ? x + 1 : 0;
        for (int64_t y = y0; y < J->sn; ++y) {
            if (J->self && y == x) continue;
            int32_t yl = J->so[y + 1] - J->so[y];
            if (iabs(xl - yl) > J->tau) continue;   /* ED >= length difference */
            if (orc_ed_band(xp, xl, J->sc + J->so[y], yl, J->tau) <= J->tau) {
                if (J->self) res_push(J->out, imin(x, (int32_t)y), imax(x, (int32_t)y));
                else res_push(J->out, x, (int32_t)y);
            }
        }
    }
    return NULL;
}

static orc_result* bf_run(bf_job proto, int32_t nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    bf_job jobs[256];
    for (int32_t t = 0; t < nthreads; ++t) {
        jobs[t] = proto;
        jobs[t].tid = t;
        jobs[t].nthreads = nthreads;
        jobs[t].out = res_new();
        pthread_create(&th[t], NULL, bf_worker, &jobs[t]);
    }
    orc_result* R = res_new();
    for (int32_t t = 0; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
        for (int64_t k = 0; k < jobs[t].out->count; ++k)
            res_push(R, jobs[t].out->a[k], jobs[t].out->b[k]);
        orc_result_free(jobs[t].out);
    }
    res_sort_unique(R);
    return R;
}

/* All pairs (a, b), a < b, of one set with ED <= tau. */
orc_result* orc_self_join_bf(const uint8_t* chars, const int32_t* offs, int64_t n, int32_t tau,
                             int32_t nthreads)
{
    bf_job j = {chars, offs, n, chars, offs, n, tau, 1, NULL, 0, 0, 1, NULL};
    return bf_run(j, nthreads);
}

/* All pairs (r, s) in R x S with ED <= tau. */
orc_result* orc_join_bf(const uint8_t* rc, const int32_t* ro, int64_t rn, const uint8_t* sc,
                        const int32_t* so, int64_t sn, int32_t tau, int32_t nthreads)
{
    bf_job j = {rc, ro, rn, sc, so, sn, tau, 0, NULL, 0, 0, 1, NULL};
    return bf_run(j, nthreads);
}

/* For each listed string x of one set: every other string y of the set with ED(x, y) <= tau,
 * reported as (min(x,y), max(x,y)). */
orc_result* orc_partners_bf(const uint8_t* chars, const int32_t* offs, int64_t n,
                            const int32_t* xs, int64_t nx, int32_t tau, int32_t nthreads)
{
    bf_job j = {chars, offs, n, chars, offs, n, tau, 1, xs, nx, 0, 1, NULL};
    return bf_run(j, nthreads);
}

/* ------------------------------------------------------------------------------------------ */
/* Exact segment index: inverted lists L_l^i keyed by the segment's bytes (Sec. 3.2)            */
/* ------------------------------------------------------------------------------------------ */

typedef struct orc_node {
    int32_t l, i;               /* string length, segment slot (1-based) */
    const uint8_t* seg;         /* the segment's bytes, inside the arena */
    int32_t seglen;
    int32_t count, cap;
    int32_t* ids;               /* the inverted list, in insertion order */
    struct orc_node* next;
} orc_node;

typedef struct {
    orc_node** heads;
    uint64_t mask;
} orc_index;

static uint64_t seg_hash(int32_t l, int32_t i, const uint8_t* seg, int32_t len)
{
    uint64_t h = 1469598103934665603ull;     /* FNV-1a */
    h = (h ^ (uint64_t)(uint32_t)l) * 1099511628211ull;
    h = (h ^ (uint64_t)(uint32_t)i) * 1099511628211ull;
    for (int32_t k = 0; k < len; ++k) h = (h ^ seg[k]) * 1099511628211ull;
    return h;
}

static void index_init(orc_index* X, int64_t expected)
{
    uint64_t sz = 1024;
    while (sz < (uint64_t)(2 * expected)) sz <<= 1;
    X->heads = (orc_node**)calloc(sz, sizeof(orc_node*));
    X->mask = sz - 1;
}

static orc_node* index_find(const orc_index* X, int32_t l, int32_t i, const uint8_t* seg,
                            int32_t len)
{
    uint64_t h = seg_hash(l, i, seg, len) & X->mask;
    for (orc_node* e = X->heads[h]; e; e = e->next)
        if (e->l == l && e->i == i && e->seglen == len && memcmp(e->seg, seg, (size_t)len) == 0)
            return e;
    return NULL;
}

static void index_add(orc_index* X, int32_t l, int32_t i, const uint8_t* seg, int32_t len,
                      int32_t id)
{
    orc_node* e = index_find(X, l, i, seg, len);
    if (!e) {
        uint64_t h = seg_hash(l, i, seg, len) & X->mask;
        e = (orc_node*)calloc(1, sizeof(orc_node));
        e->l = l; e->i = i; e->seg = seg; e->seglen = len;
        e->next = X->heads[h];
        X->heads[h] = e;
    }
    if (e->count == e->cap) {
        e->cap = e->cap ? e->cap * 2 : 4;
        e->ids = (int32_t*)realloc(e->ids, sizeof(int32_t) * (size_t)e->cap);
    }
    e->ids[e->count++] = id;
}

static void index_free(orc_index* X)
{
    for (uint64_t h = 0; h <= X->mask; ++h) {
        orc_node* e = X->heads[h];
        while (e) {
            orc_node* nx = e->next;
            free(e->ids);
            free(e);
            e = nx;
        }
    }
    free(X->heads);
}

/* Inserts the tau+1 even-partition segments of string id into L_{|s|}^i (Algorithm 1, last
 * step).  Strings shorter than tau+1 cannot be partitioned (footnote to Sec. 3.1) and are not
 * indexed. */
static void index_string(orc_index* X, const uint8_t* s, int32_t len, int32_t tau, int32_t id)
{
    if (len < tau + 1) return;
    int32_t start[128], sl[128];
    orc_partition(len, tau, start, sl);
    for (int32_t i = 1; i <= tau + 1; ++i)
        index_add(X, len, i, s + start[i - 1] - 1, sl[i - 1], id);
}

/* Probes the index with string x (Algorithm 1 inner loops): for every length l in [lmin, lmax]
 * (l >= tau+1) and slot i, the window of the selection method (multi-match, Sec. 4.2, by
 * default; the length, shift and position methods of Sec. 4 and 4.1 select supersets of it)
 * selects start positions p (SubstringSelection, Algorithm 2), restricted to the positions
 * where x has a substring of length l_i; each selected substring x[p, l_i] found in L_l^i yields
 * the candidates (y, x, i, p) for y in L_l^i(x[p, l_i]), which are verified by extension
 * (Verification, Algorithm 3).  Accepted y are appended to R as (pair_a, pair_b) by the caller's
 * convention. */
static void probe_string(const orc_index* X, const uint8_t* chars, const int32_t* offs, int32_t x,
                         const uint8_t* xs, int32_t n, int32_t lmin, int32_t lmax, int32_t tau,
                         int32_t self, int32_t keep_cands, int32_t method, orc_result* R)
{
    for (int32_t l = imax(lmin, tau + 1); l <= lmax; ++l) {
        int32_t start[128], sl[128];
        orc_partition(l, tau, start, sl);
        for (int32_t i = 1; i <= tau + 1; ++i) {
            int32_t lo, hi;
            orc_window(method, n, l, tau, i, &lo, &hi);
            lo = imax(lo, 1);
            hi = imin(hi, n - sl[i - 1] + 1);
            for (int32_t p = lo; p <= hi; ++p) {
                R->selected++;
                const orc_node* e = index_find(X, l, i, xs + p - 1, sl[i - 1]);
                if (!e) continue;
                for (int32_t k = 0; k < e->count; ++k) {
                    int32_t y = e->ids[k];
                    int64_t cells = 0;
                    int32_t pass = orc_extension_verify(xs, n, chars + offs[y], l, tau, i, p,
                                                        &cells);
                    R->candidates++;
                    R->cells += cells;
                    if (keep_cands) res_push_cand(R, y, x, i, p, pass, cells);
                    if (pass) {
                        if (self) res_push(R, imin(x, y), imax(x, y));
                        else res_push(R, x, y);
                    }
                }
            }
        }
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Pass-Join self-join (Algorithm 1)                                                            */
/* ------------------------------------------------------------------------------------------ */

typedef struct { const uint8_t* c; const int32_t* o; int32_t tiebreak; } sort_ctx;

static int cmp_visit(const void* u, const void* v, void* arg)
{
    const sort_ctx* C = (const sort_ctx*)arg;
    int32_t a = *(const int32_t*)u, b = *(const int32_t*)v;
    int32_t la = C->o[a + 1] - C->o[a], lb = C->o[b + 1] - C->o[b];
    if (la != lb) return (la > lb) - (la < lb);
    if (C->tiebreak == 1) {
        int c = memcmp(C->c + C->o[a], C->c + C->o[b], (size_t)la);
        if (c != 0) return c;
    }
    return (a > b) - (a < b);
}

/* PASS-JOIN(S, tau): strings are visited by length and, within a length, by id
 * (tiebreak = 0) or by bytes then id (tiebreak = 1, the paper's alphabetical order).  Each
 * visited string x with |x| >= tau+1 probes L_l^i for |x|-tau <= l <= |x| over the strings
 * visited before it, and is then indexed.  Pairs with a string shorter than tau+1 are not
 * reachable through the index (footnote to Sec. 3.1); they are found by a direct distance
 * computation against the earlier-visited strings within the length filter.
 *
 * probe_stride > 1 restricts the probe step: only strings at visiting ranks r with
 * r % probe_stride == probe_offset probe (and take part in the direct path); every string is
 * still indexed in visiting order.  Each pair is reported by its later-visited string, so the
 * runs for offsets 0 .. probe_stride-1 are disjoint, their pairs together are the whole result
 * and their counters add up to the whole run's (this is how the work is split over processes).
 * keep_cands = 1 records every candidate (y, x, i, p) with its verdict and cells. */
orc_result* orc_self_join_pj(const uint8_t* chars, const int32_t* offs, int64_t n, int32_t tau,
                             int32_t tiebreak, int32_t probe_stride, int32_t probe_offset,
                             int32_t keep_cands, int32_t method)
{
    orc_result* R = res_new();
    if (probe_stride < 1) probe_stride = 1;
    if (probe_offset < 0 || probe_offset >= probe_stride) probe_offset = 0;
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t k = 0; k < n; ++k) order[k] = (int32_t)k;
    sort_ctx ctx = {chars, offs, tiebreak};
    qsort_r(order, (size_t)n, sizeof(int32_t), cmp_visit, &ctx);

    orc_index X;
    index_init(&X, n * (tau + 1));
    /* visited strings shorter than tau+1, in visiting order */
    int32_t* shorts = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t nshort = 0;

    for (int64_t rank = 0; rank < n; ++rank) {
        int32_t x = order[rank];
        const uint8_t* xs = chars + offs[x];
        int32_t xl = offs[x + 1] - offs[x];
        if (rank % probe_stride == probe_offset) {
            if (xl >= tau + 1)
                probe_string(&X, chars, offs, x, xs, xl, xl - tau, xl, tau, 1, keep_cands, method,
                             R);
            for (int64_t k = 0; k < nshort; ++k) {
                int32_t y = shorts[k];
                int32_t yl = offs[y + 1] - offs[y];
                if (xl - yl > tau) continue;
                R->side_pairs++;
                if (orc_ed_full(xs, xl, chars + offs[y], yl) <= tau)
                    res_push(R, imin(x, y), imax(x, y));
            }
        }
        if (xl >= tau + 1) index_string(&X, xs, xl, tau, x);
        else shorts[nshort++] = x;
    }
    index_free(&X);
    free(shorts);
    free(order);
    res_sort_unique(R);
    return R;
}

/* Join of two distinct sets (Sec. 3.2): the strings of S are indexed; each r of R probes the
 * indices of lengths |r|-tau .. |r|+tau, with the windows of Sec. 4.2 taken at the signed
 * Delta = |r| - l.  Strings of S shorter than tau+1 are compared with every r directly.
 * Pairs are (r, s).  Only the r with r % probe_stride == probe_offset probe (probe_stride = 1:
 * all of them); the runs for the offsets 0 .. probe_stride-1 split the result disjointly. */
orc_result* orc_join_pj(const uint8_t* rc, const int32_t* ro, int64_t rn, const uint8_t* sc,
                        const int32_t* so, int64_t sn, int32_t tau, int32_t keep_cands,
                        int32_t method, int32_t probe_stride, int32_t probe_offset)
{
    orc_result* R = res_new();
    if (probe_stride < 1) probe_stride = 1;
    if (probe_offset < 0 || probe_offset >= probe_stride) probe_offset = 0;
    orc_index X;
    index_init(&X, sn * (tau + 1));
    /* strings of S shorter than tau+1 */
    int32_t* shorts = (int32_t*)malloc(sizeof(int32_t) * (size_t)(sn > 0 ? sn : 1));
    int64_t nshort = 0;
    for (int64_t y = 0; y < sn; ++y) {
        int32_t yl = so[y + 1] - so[y];
        if (yl >= tau + 1) index_string(&X, sc + so[y], yl, tau, (int32_t)y);
        else shorts[nshort++] = (int32_t)y;
    }
    for (int64_t x = probe_offset; x < rn; x += probe_stride) {
        const uint8_t* xs = rc + ro[x];
        int32_t xl = ro[x + 1] - ro[x];
        probe_string(&X, sc, so, (int32_t)x, xs, xl, xl - tau, xl + tau, tau, 0, keep_cands,
                     method, R);
        for (int64_t k = 0; k < nshort; ++k) {
            int32_t y = shorts[k];
            int32_t yl = so[y + 1] - so[y];
            if (iabs(xl - yl) > tau) continue;
            R->side_pairs++;
            if (orc_ed_full(xs, xl, sc + so[y], yl) <= tau) res_push(R, (int32_t)x, y);
        }
    }
    free(shorts);
    index_free(&X);
    res_sort_unique(R);
    return R;
}
