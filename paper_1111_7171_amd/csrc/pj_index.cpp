// pj_index.cpp -- device-resident indices (one per tau of a range) and per-query-tau probing.
//
// pj_build_index keeps the length-sorted arena of S and, for each tau in [tau_min, tau_max], the
// sorted (key, g) entries and the bucket table of the even-partition segments (Sec. 3.1, 3.2).
// pj_query groups the queries by their threshold and runs the two-set join of Sec. 3.2 of each
// group against the index of that threshold.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "../../include/passjoin.h"
#include "pj_host_internal.h"
#include "pj_internal.h"

struct pj_index {
    int tau_min = 0, tau_max = -1;
    pj::Owned mem;
    pj::DevSet S;
    std::vector<pj::DevIndex> X;
    pj::IndexRef* refs = nullptr;    // device [kTauMax + 1], entries for tau_min .. tau_max
    bool has_entries = false;
    int device = 0;                  // the HIP device the index lives on
};

namespace pj {

void validate_host_strings(const pj_strings* S, const char* what);

const DevSet& index_set(const pj_index* idx) { return idx->S; }
const IndexRef* index_refs(const pj_index* idx) { return idx->refs; }
SymMap index_sym(const pj_index* idx) { return idx->X.front().sym; }
bool index_has_entries(const pj_index* idx) { return idx->has_entries; }
int index_device(const pj_index* idx) { return idx->device; }
const DevIndex& index_for(const pj_index* idx, int tau) { return idx->X[tau - idx->tau_min]; }
void index_taus(const pj_index* idx, int* lo, int* hi)
{
    *lo = idx->tau_min;
    *hi = idx->tau_max;
}

// Host copy of a string set whose pointers may be device pointers.
struct HostStrings {
    std::vector<uint8_t> bytes;
    std::vector<int32_t> offs;
    pj_strings view{};
};

static void to_host(const pj_strings* Q, bool on_device, HostStrings& H)
{
    if (!on_device) {
        H.view = *Q;
        return;
    }
    if (Q->n < 0 || !Q->offsets) throw Error(PJ_EINVAL, "Q: bad strings");
    H.offs.resize((size_t)Q->n + 1);
    hip_check(hipMemcpy(H.offs.data(), Q->offsets, sizeof(int32_t) * H.offs.size(),
                        hipMemcpyDeviceToHost), "download offsets");
    int64_t total = H.offs.back();
    if (total < 0) throw Error(PJ_EINVAL, "Q: bad offsets");
    H.bytes.resize((size_t)total + 1);
    if (total > 0)
        hip_check(hipMemcpy(H.bytes.data(), Q->bytes, (size_t)total, hipMemcpyDeviceToHost),
                  "download bytes");
    H.view.n = Q->n;
    H.view.bytes = H.bytes.data();
    H.view.offsets = H.offs.data();
}

int64_t query_selections(const pj_index* idx, int n, int tau);

// Joins the queries of Q (host memory, validated; taus[q] in the index's range) against the
// index in one device pass: probe, verify and the short-string path take each query's own
// threshold and per-tau index.  Appends (q << 32 | s) sorted by (q, s).
void run_query_batch(const pj_index* idx, const pj_strings* Q, const int32_t* taus,
                     std::vector<uint64_t>& pairs, pj_stats& stats, hipStream_t st,
                     const char* tune_cache)
{
    if (Q->n == 0) return;
    Workspace& W = thread_workspace();
    W.begin_call(0);
    DevSet P;
    build_set(Q, false, W, "Q", P, st);
    int tmax = 0;
    uint64_t bound = 0;
    for (int64_t q = 0; q < Q->n; ++q) {
        tmax = std::max(tmax, taus[q]);
        bound += (uint64_t)query_selections(idx, Q->offsets[q + 1] - Q->offsets[q], taus[q]);
    }
    int32_t* d_tau_id = (int32_t*)W.get("Q.tau_id", sizeof(int32_t) * (size_t)Q->n);
    int32_t* d_tau = (int32_t*)W.get("Q.tau", sizeof(int32_t) * (size_t)Q->n);
    hip_check(hipMemcpyAsync(d_tau_id, taus, sizeof(int32_t) * (size_t)Q->n, hipMemcpyHostToDevice,
                             st), "upload taus");
    hip_check(launch_gather_i32(d_tau_id, P.perm, Q->n, d_tau, st), "gather taus");
    ProbeSpec spec;
    spec.self = false;
    spec.tau = tmax;
    spec.q_tau = d_tau;
    spec.refs = idx->refs;
    spec.bound = bound;
    spec.has_entries = idx->has_entries;
    spec.sym = index_sym(idx);
    JoinScratch J;
    J.mode = PJ_MODE_BATCHED;
    J.tp = tune_lookup(tune_cache, tmax, Q->n ? (double)(Q->offsets[Q->n] - Q->offsets[0]) / (double)Q->n
                                             : 0.0);
    Timer tm(st);
    run_candidates(P, idx->S, spec, J, stats, tm, st);
    int32_t *da = nullptr, *db = nullptr;
    uint64_t M = finish_pairs(P, idx->S, false, J.out, J.naccepted, &da, &db, st);
    std::vector<int32_t> ha(M), hb(M);
    if (M) {
        hip_check(hipMemcpyAsync(ha.data(), da, sizeof(int32_t) * M, hipMemcpyDeviceToHost, st), "d2h");
        hip_check(hipMemcpyAsync(hb.data(), db, sizeof(int32_t) * M, hipMemcpyDeviceToHost, st), "d2h");
    }
    hip_check(hipStreamSynchronize(st), "sync");
    pairs.reserve(pairs.size() + M);
    for (uint64_t k = 0; k < M; ++k)
        pairs.push_back(((uint64_t)(uint32_t)ha[k] << 32) | (uint32_t)hb[k]);
}

// Substrings a length-n query with threshold tau selects against the lengths present in the
// index (Lemma 2 count per probed length): the bound on its hit records.
int64_t query_selections(const pj_index* idx, int n, int tau)
{
    const DevSet& S = idx->S;
    int64_t sel = 0;
    for (int l = std::max(n - tau, tau + 1); l <= n + tau && l <= kLenMax; ++l) {
        if (S.h_lenstart[l + 1] == S.h_lenstart[l]) continue;
        const int d = n - l;
        sel += (tau * tau - d * d) / 2 + tau + 1;
    }
    return sel;
}

// Admission estimate of one query: per substring it may select, a hit record (16 B), its
// bucketed copy (16 B), the candidate prefix sum (8 B), the per-hit count and scan scratch
// (8 B); plus its bytes twice (the uploaded and the length-sorted arena).  The accepted-
// candidate buffer (8 B per candidate found) is not known before the probe and is not counted.
int64_t query_footprint(const pj_index* idx, int n, int tau)
{
    return 48 * query_selections(idx, n, tau) + 2 * (int64_t)stride_of(n) + 64;
}

}  // namespace pj

using namespace pj;

extern "C" {

int pj_build_index(const pj_strings* S, int32_t tau_min, int32_t tau_max, const pj_options* opt,
                   pj_index** out)
{
    t_stats = pj_stats{};
    try {
        if (!out) throw Error(PJ_EINVAL, "null output");
        *out = nullptr;
        if (tau_min < 0 || tau_max > kTauMax || tau_min > tau_max)
            throw Error(PJ_EINVAL, "tau range [%d, %d] invalid", tau_min, tau_max);
        bool on_dev = opt && opt->inputs_on_device;
        if (!on_dev) validate_host_strings(S, "S");
        else if (!S) throw Error(PJ_EINVAL, "null pj_strings");
        hipStream_t st = opt ? (hipStream_t)opt->hip_stream : (hipStream_t)0;
        auto t0 = std::chrono::steady_clock::now();
        std::unique_ptr<pj_index> idx(new pj_index());
        idx->tau_min = tau_min;
        idx->tau_max = tau_max;
        idx->mem.budget = opt ? opt->mem_budget_bytes : 0;
        hip_check(hipGetDevice(&idx->device), "hipGetDevice");
        thread_workspace().begin_call(0);
        build_set(S, on_dev, idx->mem, "I", idx->S, st);
        idx->X.resize((size_t)(tau_max - tau_min + 1));
        int64_t entries = 0;
        std::vector<IndexRef> refs(kTauMax + 1);
        for (int t = tau_min; t <= tau_max; ++t) {
            DevIndex& X = idx->X[(size_t)(t - tau_min)];
            build_index(idx->S, t, idx->mem, "I.t" + std::to_string(t), X, st);
            entries += X.entries;
            refs[(size_t)t] = IndexRef{X.table, X.vals, X.mask,
                                       (uint32_t)(((1u << 21) + (uint32_t)t) / (uint32_t)(t + 1)), 1u,
                                       X.filter, X.filter_dir};
        }
        idx->has_entries = entries > 0;
        idx->refs = (IndexRef*)idx->mem.get("I.refs", sizeof(IndexRef) * (kTauMax + 1));
        hip_check(hipMemcpyAsync(idx->refs, refs.data(), sizeof(IndexRef) * (kTauMax + 1),
                                 hipMemcpyHostToDevice, st), "upload refs");
        hip_check(hipStreamSynchronize(st), "sync");
        t_stats.strings = idx->S.n;
        t_stats.index_entries = entries;
        t_stats.ms_index = std::chrono::duration<double, std::milli>(
                               std::chrono::steady_clock::now() - t0).count();
        t_stats.ms_total = t_stats.ms_index;
        *out = idx.release();
        t_last_ok_stats = t_stats;
        t_last_error.clear();
        return PJ_OK;
    } catch (const Error& e) {
        t_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        t_last_error = "host allocation failed";
        return PJ_ENOMEM;
    }
}

int pj_index_info(const pj_index* idx, int64_t* n, int32_t* tau_min, int32_t* tau_max,
                  int64_t* device_bytes)
{
    if (!idx) {
        t_last_error = "null index";
        return PJ_EINVAL;
    }
    if (n) *n = idx->S.n;
    if (tau_min) *tau_min = idx->tau_min;
    if (tau_max) *tau_max = idx->tau_max;
    if (device_bytes) *device_bytes = (int64_t)idx->mem.used;
    return PJ_OK;
}

void pj_index_free(pj_index* idx) { delete idx; }

int pj_query(const pj_index* idx, const pj_strings* Q, const int32_t* taus, const pj_options* opt,
             pj_pairs* out)
{
    t_stats = pj_stats{};
    if (out) {
        out->count = 0;
        out->a = out->b = nullptr;
        out->on_device = 0;
    }
    try {
        if (!out) throw Error(PJ_EINVAL, "null output");
        if (!idx) throw Error(PJ_EINVAL, "null index");
        if (!Q) throw Error(PJ_EINVAL, "null pj_strings");
        if (!taus && Q->n > 0) throw Error(PJ_EINVAL, "null taus");
        bool on_dev = opt && opt->inputs_on_device;
        if (!on_dev) validate_host_strings(Q, "Q");
        for (int64_t q = 0; q < Q->n; ++q)
            if (taus[q] < idx->tau_min || taus[q] > idx->tau_max)
                throw Error(PJ_ERANGE, "query %lld: tau %d outside the index range [%d, %d]",
                            (long long)q, taus[q], idx->tau_min, idx->tau_max);
        hipStream_t st = opt ? (hipStream_t)opt->hip_stream : (hipStream_t)0;
        auto t0 = std::chrono::steady_clock::now();
        HostStrings H;
        to_host(Q, on_dev, H);
        if (on_dev) validate_host_strings(&H.view, "Q");
        std::vector<uint64_t> pairs;
        run_query_batch(idx, &H.view, taus, pairs, t_stats, st, opt ? opt->tune_cache : nullptr);
        uint64_t M = pairs.size();
        std::vector<int32_t> a(M), b(M);
        for (uint64_t k = 0; k < M; ++k) {
            a[k] = (int32_t)(pairs[k] >> 32);
            b[k] = (int32_t)(pairs[k] & 0xffffffffu);
        }
        bool to_dev = opt && opt->outputs_on_device;
        size_t bytes = sizeof(int32_t) * (size_t)std::max<uint64_t>(M, 1);
        out->count = (int64_t)M;
        out->on_device = to_dev ? 1 : 0;
        if (to_dev) {
            void *pa = nullptr, *pb = nullptr;
            if (hipMalloc(&pa, bytes) != hipSuccess || hipMalloc(&pb, bytes) != hipSuccess) {
                (void)hipGetLastError();
                if (pa) (void)hipFree(pa);
                throw Error(PJ_ENOMEM, "output allocation failed");
            }
            out->a = (int32_t*)pa;
            out->b = (int32_t*)pb;
            if (M) {
                hip_check(hipMemcpy(pa, a.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice), "h2d");
                hip_check(hipMemcpy(pb, b.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice), "h2d");
            }
        } else {
            out->a = (int32_t*)malloc(bytes);
            out->b = (int32_t*)malloc(bytes);
            if (!out->a || !out->b) throw Error(PJ_ENOMEM, "host output allocation failed");
            if (M) {
                memcpy(out->a, a.data(), sizeof(int32_t) * M);
                memcpy(out->b, b.data(), sizeof(int32_t) * M);
            }
        }
        t_stats.strings = Q->n;
        t_stats.pairs = (int64_t)M;
        t_stats.ms_total = std::chrono::duration<double, std::milli>(
                               std::chrono::steady_clock::now() - t0).count();
        t_last_ok_stats = t_stats;
        t_last_error.clear();
        return PJ_OK;
    } catch (const Error& e) {
        t_last_error = e.msg;
        pj_pairs_free(out);
        return e.code;
    } catch (const std::bad_alloc&) {
        t_last_error = "host allocation failed";
        pj_pairs_free(out);
        return PJ_ENOMEM;
    }
}

}  // extern "C"
