// pj_noalloc.hip -- pj_query_noalloc: pj_query for callers that cannot allocate memory.
//
// The query batch runs the same device phases as a serving slot's captured pipeline
// (launch_graph_batch: counter reset by a fill kernel, multi-match probe, candidate prefix,
// extension verification, short-string side path, in-LDS sort and deduplication), but every
// device work buffer is carved out of one static device array, `scratch`, and the host staging
// lives in static host arrays: the call makes no device or host allocation.  Capacities are
// fixed (kNaQueries queries, kNaHits hit records, ...); a batch beyond them is refused with
// PJ_ERANGE before any device work, or after it when a device-side capacity overflowed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "../../include/passjoin.h"
#include "pj_host_internal.h"

namespace pj {

constexpr int kNaQueries = 512;                        // queries per call
constexpr uint64_t kNaHits = 1ull << 18;               // hit records (Lemma 2 bound of the batch)
constexpr uint64_t kNaChunks = (1ull << 24) / 1024;    // wave chunks: 2^24 candidates
constexpr uint64_t kNaAccepted = kGraphSortCap;        // accepted candidates (the sort's limit)
constexpr size_t kNaScratchBytes = 8ull << 20;         // device work buffers, one array per GPU
constexpr size_t kNaTablesMax = 32u << 10;             // host staging of the batch tables
constexpr size_t kNaArenaMax = (size_t)kNaQueries * 512 + 256;
constexpr size_t kNaResultMax = 72u << 10;
constexpr int kNaMaxDevices = 64;

}  // namespace pj

// The device work buffers of pj_query_noalloc on each GPU (one copy per device, held until the
// process ends).  Host code never uses this name as an address: kernels get the pointer that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint8_t scratch[pj::kNaScratchBytes];

namespace pj {

static std::mutex s_na_mu;                             // one call at a time per process
static void* s_na_scratch[kNaMaxDevices];              // hipGetSymbolAddress(scratch) per device
alignas(256) static uint8_t s_na_tables[kNaTablesMax];
alignas(256) static uint8_t s_na_arena[kNaArenaMax];
alignas(256) static uint8_t s_na_result[kNaResultMax];

// The current device's copy of `scratch`, resolved once per device with that device current.
static uint8_t* noalloc_scratch(int dev)
{
    if (dev < 0 || dev >= kNaMaxDevices) throw Error(PJ_EDEVICE, "device %d out of range", dev);
    if (!s_na_scratch[dev]) {
        void* p = nullptr;
        hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p) throw Error(PJ_EDEVICE, "no device address for the static scratch array");
        s_na_scratch[dev] = p;
    }
    return (uint8_t*)s_na_scratch[dev];
}

static void query_noalloc(const pj_index* idx, const pj_strings* Q, const int32_t* taus,
                          const pj_options* opt, int32_t* out_q, int32_t* out_s,
                          int64_t out_cap, int64_t* out_count)
{
    if (!idx || !Q || !out_count) throw Error(PJ_EINVAL, "null argument");
    *out_count = 0;
    if (out_cap < 0) throw Error(PJ_EINVAL, "negative output capacity");
    if (out_cap > 0 && (!out_q || !out_s)) throw Error(PJ_EINVAL, "null output arrays");
    if (opt && (opt->inputs_on_device || opt->outputs_on_device))
        throw Error(PJ_EINVAL, "pj_query_noalloc takes host queries and host output arrays");
    validate_host_strings(Q, "Q");
    if (Q->n > 0 && !taus) throw Error(PJ_EINVAL, "null taus");
    if (Q->n > kNaQueries)
        throw Error(PJ_ERANGE, "%lld queries exceed the %d a static-scratch call takes",
                    (long long)Q->n, kNaQueries);
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (dev != index_device(idx))
        throw Error(PJ_EINVAL, "the index lives on device %d, the current device is %d",
                    index_device(idx), dev);
    int tau_min = 0, tau_max = 0;
    index_taus(idx, &tau_min, &tau_max);
    for (int64_t q = 0; q < Q->n; ++q)
        if (taus[q] < tau_min || taus[q] > tau_max)
            throw Error(PJ_ERANGE, "query %lld: tau %d outside the index range [%d, %d]",
                        (long long)q, taus[q], tau_min, tau_max);
    t_stats.strings = Q->n;
    if (Q->n == 0) return;

    const BatchLayout L = batch_layout(kNaQueries, kNaHits, kNaChunks, kNaAccepted);
    if (batch_device_bytes(L) > kNaScratchBytes || L.tables_bytes > kNaTablesMax ||
        (size_t)L.bcap + 64 > kNaArenaMax || L.result_bytes > kNaResultMax)
        throw Error(PJ_EDEVICE, "static scratch layout does not fit its arrays");
    hipStream_t st = opt ? (hipStream_t)opt->hip_stream : (hipStream_t)0;

    std::lock_guard<std::mutex> lk(s_na_mu);
    int64_t bytes = 0;
    switch (pack_query_batch(idx, L, Q, taus, s_na_tables, s_na_arena, &bytes)) {
    case PackStatus::kOk: break;
    case PackStatus::kTooManySelections:
        throw Error(PJ_ERANGE, "the batch selects more than %llu substrings (Lemma 2 bound), "
                    "the static hit buffer's size", (unsigned long long)kNaHits);
    case PackStatus::kTooManyBytes:
        throw Error(PJ_ERANGE, "the batch's padded strings exceed %lld bytes",
                    (long long)L.bcap);
    default:
        throw Error(PJ_ERANGE, "the batch does not fit the static capacities");
    }
    uint8_t* base = noalloc_scratch(dev);
    const BatchBuffers B = carve_batch_buffers(L, base);
    GraphBatch G;
    setup_graph_batch(idx, L, B, TuneParams{}, G);
    hip_check(hipMemcpyAsync(B.tables, s_na_tables, L.tables_bytes, hipMemcpyHostToDevice, st),
              "upload batch tables");
    if (bytes > 0)
        hip_check(hipMemcpyAsync(B.arena, s_na_arena, (size_t)bytes, hipMemcpyHostToDevice, st),
                  "upload batch arena");
    hip_check(launch_graph_batch(G, st), "query batch");
    hip_check(hipMemcpyAsync(s_na_result, B.result, L.result_bytes, hipMemcpyDeviceToHost, st),
              "download result");
    hip_check(hipStreamSynchronize(st), "sync");
    const uint64_t* pairs = nullptr;
    unsigned long long flags = 0;
    const uint32_t m = batch_result(s_na_result, t_stats, &pairs, &flags);
    if (flags & 1) throw Error(PJ_ERANGE, "more hit records than the static buffer holds");
    if (flags & 2)
        throw Error(PJ_ERANGE, "more than %llu candidates", (unsigned long long)(kNaChunks * 1024));
    if (flags & 12)
        throw Error(PJ_ERANGE, "more than %d accepted candidates", (int)kNaAccepted);
    *out_count = (int64_t)m;
    t_stats.pairs = (int64_t)m;
    if ((int64_t)m > out_cap)
        throw Error(PJ_ERANGE, "%u pairs, the output arrays hold %lld", m, (long long)out_cap);
    for (uint32_t k = 0; k < m; ++k) {
        out_q[k] = (int32_t)(pairs[k] >> 32);
        out_s[k] = (int32_t)(pairs[k] & 0xffffffffu);
    }
}

}  // namespace pj

using namespace pj;

extern "C" int pj_query_noalloc(const pj_index* idx, const pj_strings* Q, const int32_t* taus,
                                const pj_options* opt, int32_t* out_q, int32_t* out_s,
                                int64_t out_cap, int64_t* out_count)
{
    t_stats = pj_stats{};
    try {
        query_noalloc(idx, Q, taus, opt, out_q, out_s, out_cap, out_count);
        t_last_ok_stats = t_stats;
        t_last_error.clear();
        return PJ_OK;
    } catch (const Error& e) {
        t_last_error = e.msg;
        return e.code;
    } catch (...) {
        t_last_error = "unexpected internal error";
        return PJ_EDEVICE;
    }
}
