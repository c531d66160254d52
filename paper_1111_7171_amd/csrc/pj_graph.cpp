// Captured query pipeline of a serving slot.
//
// A serving batch is small (tens to hundreds of queries), so its cost is launch and
// synchronisation overhead rather than device work.  Each slot therefore owns a plan: device
// buffers of fixed capacity at fixed addresses, a pinned host mirror of the batch's
// length-sorted arena and tables (packed on the host, which already holds the queries), and one
// instantiated hipGraph of every device phase -- counter reset, multi-match probe (Sec. 4.2),
// candidate prefix, extension verification (Sec. 5.2), the short-string side path,
// sort/deduplication of the accepted pairs, and the copy of the result to pinned memory.  The
// kernels read the batch's sizes from device memory, so the same graph serves every batch: a
// batch costs two host-to-device copies, one graph launch and one synchronisation.  A batch
// that does not fit the capacities, or overflows one on the device (flags in the result), is
// run by the caller through the uncaptured path instead.
#include <algorithm>
#include <cstring>
#include <memory>
#include <vector>

#include "pj_host_internal.h"

namespace pj {

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

BatchLayout batch_layout(int max_queries, uint64_t hcap, uint64_t chunk_cap, uint64_t acc_cap)
{
    BatchLayout L;
    L.qcap = std::max(1, max_queries);
    L.bcap = L.qcap * 512;
    L.hcap = hcap;
    L.chunk_cap = chunk_cap;
    L.acc_cap = acc_cap;
    size_t o = 8;
    L.off_lenstart = o; o += sizeof(int32_t) * (kLenTab + 1);
    o = align256(o);
    L.off_gbase = o; o += sizeof(int64_t) * kLenTab;
    L.off_perm = o; o += sizeof(int32_t) * (size_t)L.qcap;
    L.off_qtau = o; o += sizeof(int32_t) * (size_t)L.qcap;
    L.off_slen = o; o += sizeof(uint16_t) * (size_t)L.qcap;
    L.tables_bytes = align256(o);
    L.arena_bytes = align256((size_t)L.bcap + 64);
    L.result_bytes = sizeof(unsigned long long) * 12 + 8 + sizeof(uint64_t) * kGraphSortCap;
    return L;
}

size_t batch_device_bytes(const BatchLayout& L)
{
    return L.tables_bytes + L.arena_bytes + align256(sizeof(Hit) * L.hcap) +
           align256(sizeof(unsigned long long) * (L.hcap + 1)) +
           align256(sizeof(uint32_t) * L.chunk_cap) + align256(sizeof(uint64_t) * L.acc_cap) +
           align256(L.result_bytes);
}

BatchBuffers carve_batch_buffers(const BatchLayout& L, uint8_t* base)
{
    BatchBuffers B;
    size_t o = 0;
    B.tables = base + o; o += L.tables_bytes;
    B.arena = base + o; o += L.arena_bytes;
    B.hits = (Hit*)(base + o); o += align256(sizeof(Hit) * L.hcap);
    B.prefix = (unsigned long long*)(base + o); o += align256(sizeof(unsigned long long) * (L.hcap + 1));
    B.first = (uint32_t*)(base + o); o += align256(sizeof(uint32_t) * L.chunk_cap);
    B.acc = (uint64_t*)(base + o); o += align256(sizeof(uint64_t) * L.acc_cap);
    B.result = base + o;
    return B;
}

void setup_graph_batch(const pj_index* idx, const BatchLayout& L, const BatchBuffers& B,
                       const TuneParams& tp, GraphBatch& G)
{
    int tau_min = 0, tau_max = 0;
    index_taus(idx, &tau_min, &tau_max);
    auto* counters = (unsigned long long*)B.result;
    const DevSet& Y = index_set(idx);
    G = GraphBatch{};
    ProbeParams& pp = G.probe;
    pp.x_arena = B.arena;
    pp.x_slen = (const uint16_t*)(B.tables + L.off_slen);
    pp.x_lenstart = (const int32_t*)(B.tables + L.off_lenstart);
    pp.x_gbase = (const int64_t*)(B.tables + L.off_gbase);
    pp.g_begin = 0;
    pp.nl = 2 * tau_max + 1;
    pp.self = 0;
    pp.q_tau = (const int32_t*)(B.tables + L.off_qtau);
    pp.refs = index_refs(idx);
    pp.y_lenstart = Y.lenstart;
    pp.tau = tau_max;
    pp.ymin = Y.lmin;
    pp.ymax = Y.lmax;
    pp.hits = B.hits;
    pp.hit_cap = L.hcap;
    pp.counters = counters;
    pp.nx_dev = (const uint32_t*)B.tables;
    pp.sym = index_sym(idx);
    pp.selection = PJ_SELECT_MULTIMATCH;
    // grids sized for the batch capacity (a serving batch is small; idle blocks of a chip-wide
    // grid would still cost every batch their launch)
    const uint64_t probe_threads = (uint64_t)L.qcap * (uint64_t)pp.nl * (uint64_t)(tau_max + 1);
    G.probe_grid = (int)std::max<uint64_t>(1, std::min<uint64_t>(
        (uint64_t)device_cus() * tp.probe_blocks_per_cu, (probe_threads + 255) / 256));
    if (!index_has_entries(idx)) pp.ymax = -1;        // nothing indexed: the probe finds no list
    VerifyParams& vp = G.verify;
    vp.x_arena = pp.x_arena; vp.x_slen = pp.x_slen; vp.x_lenstart = pp.x_lenstart;
    vp.x_gbase = pp.x_gbase;
    vp.y_arena = Y.sarena; vp.y_lenstart = Y.lenstart; vp.y_gbase = Y.gbase;
    vp.wave_rounds = kBatchedRoundsMax;               // fixed chunk: the sizes are on device
    vp.y_inl = nullptr;                               // serving indices keep no inline copies
    vp.y_inl_base = nullptr;
    vp.hits = B.hits;
    vp.prefix = B.prefix;
    vp.tau = tau_max;
    vp.y_maxlen = Y.lmax;
    vp.exact_len = pp.sym.exact_len;
    vp.q_tau = pp.q_tau;
    vp.refs = pp.refs;
    vp.out = B.acc;
    vp.out_cap = L.acc_cap;
    vp.counters = counters;
    G.bcounts = counters + 8;
    vp.dev_counts = G.bcounts;
    G.verify_grid = std::max(1, std::min(device_cus() * tp.verify_waves_per_cu / 4, 256));
    G.first = B.first;
    G.chunk_cap = L.chunk_cap;
    // indexed strings shorter than tau_max + 1 go through the side path
    if (Y.n > 0 && Y.lmin <= tau_max) {
        const int top = std::min(tau_max, Y.lmax);
        G.y_first = (uint32_t)Y.h_lenstart[0];
        G.y_count = (uint32_t)(Y.h_lenstart[top + 1] - Y.h_lenstart[0]);
    }
    G.y_arena = Y.sarena; G.y_slen = Y.slen; G.y_lenstart = Y.lenstart; G.y_gbase = Y.gbase;
    G.xperm = (const int32_t*)(B.tables + L.off_perm);
    G.yperm = Y.perm;
    G.out_n = (uint32_t*)(counters + 12);
    G.out = (uint64_t*)(counters + 13);
}

PackStatus pack_query_batch(const pj_index* idx, const BatchLayout& L, const pj_strings* Q,
                            const int32_t* taus, uint8_t* h_tables, uint8_t* h_arena,
                            int64_t* arena_used)
{
    const int64_t n = Q->n;
    *arena_used = 0;
    if (n > L.qcap) return PackStatus::kTooManyQueries;
    int tau_min = 0, tau_max = 0;
    index_taus(idx, &tau_min, &tau_max);
    // the Lemma 2 bound on hit records decides whether the hit buffer can overflow at all
    uint64_t bound = 0;
    int32_t cnt[kLenTab + 1];
    std::fill(cnt, cnt + kLenTab + 1, 0);
    for (int64_t q = 0; q < n; ++q) {
        const int len = Q->offsets[q + 1] - Q->offsets[q];
        if (taus[q] < tau_min || taus[q] > tau_max) return PackStatus::kTauOutOfRange;
        bound += (uint64_t)query_selections(idx, len, taus[q]);
        cnt[len] += 1;
    }
    if (bound > L.hcap) return PackStatus::kTooManySelections;
    // length-sorted arena and tables (the build_set layout)
    auto* lenstart = (int32_t*)(h_tables + L.off_lenstart);
    auto* gbase = (int64_t*)(h_tables + L.off_gbase);
    auto* perm = (int32_t*)(h_tables + L.off_perm);
    auto* qtau = (int32_t*)(h_tables + L.off_qtau);
    auto* slen = (uint16_t*)(h_tables + L.off_slen);
    int64_t pos = 0, bytes = 0;
    for (int l = 0; l < kLenTab; ++l) {
        lenstart[l] = (int32_t)pos;
        gbase[l] = bytes;
        pos += cnt[l];
        bytes += (int64_t)cnt[l] * stride_of(l);
    }
    lenstart[kLenTab] = (int32_t)pos;
    if (bytes > L.bcap) return PackStatus::kTooManyBytes;
    int32_t* fill = cnt;                          // reused: next free position per length
    for (int l = 0; l < kLenTab; ++l) fill[l] = lenstart[l];
    for (int64_t q = 0; q < n; ++q) {             // stable: ids ascending within a length
        const int len = Q->offsets[q + 1] - Q->offsets[q];
        const int32_t gpos = fill[len]++;
        perm[gpos] = (int32_t)q;
        qtau[gpos] = taus[q];
        slen[gpos] = (uint16_t)len;
        uint8_t* dst = h_arena + gbase[len] + (int64_t)(gpos - lenstart[len]) * stride_of(len);
        if (len) memcpy(dst, Q->bytes + Q->offsets[q], (size_t)len);
        const int pad = (int)stride_of(len) - len;
        if (pad) memset(dst + len, 0, (size_t)pad);
    }
    *(uint32_t*)h_tables = (uint32_t)n;
    *arena_used = bytes;
    return PackStatus::kOk;
}

uint32_t batch_result(const uint8_t* h_result, pj_stats& stats, const uint64_t** pairs,
                      unsigned long long* flags)
{
    const auto* c = (const unsigned long long*)h_result;
    *flags = c[11];
    const uint32_t m = *(const uint32_t*)(c + 12);
    *pairs = (const uint64_t*)(c + 13);
    stats.hits += (int64_t)c[0];
    stats.candidates += (int64_t)(c[1] - c[5]);      // less the hashed-key collisions
    stats.key_collisions += (int64_t)c[5];
    stats.selected += (int64_t)c[2];
    stats.accepted += (int64_t)c[3];
    stats.cells += (int64_t)c[4];
    stats.side_pairs += (int64_t)c[6];
    return m;
}

struct GraphPlan {
    const pj_index* idx = nullptr;
    hipStream_t st = nullptr;
    BatchLayout L;
    Owned mem;
    BatchBuffers B;                 // device buffers of fixed capacity (owned by mem)
    uint8_t* h_tables = nullptr;    // pinned mirrors of the batch tables, arena and result
    uint8_t* h_arena = nullptr;
    uint8_t* h_result = nullptr;
    hipGraphExec_t exec = nullptr;

    ~GraphPlan()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (h_tables) (void)hipHostFree(h_tables);
        if (h_arena) (void)hipHostFree(h_arena);
        if (h_result) (void)hipHostFree(h_result);
    }
};

// Plan capacities: hit records, wave chunks of 1024 candidates, accepted candidates.
constexpr uint64_t kPlanHits = 1ull << 20;
constexpr uint64_t kPlanChunks = (1ull << 26) / 1024;
constexpr uint64_t kPlanAccepted = 1ull << 20;

// Device bytes a plan for max_queries queries allocates (its fixed-capacity buffers).
int64_t graph_plan_device_bytes(int max_queries)
{
    return (int64_t)batch_device_bytes(
        batch_layout(max_queries, kPlanHits, kPlanChunks, kPlanAccepted));
}

GraphPlan* graph_plan_create(const pj_index* idx, int max_queries, hipStream_t st,
                             const char* tune_cache)
{
    std::unique_ptr<GraphPlan> g(new GraphPlan());
    g->idx = idx;
    g->st = st;
    g->L = batch_layout(max_queries, kPlanHits, kPlanChunks, kPlanAccepted);
    const BatchLayout& L = g->L;
    uint8_t* base = (uint8_t*)g->mem.get("graph.buffers", batch_device_bytes(L));
    g->B = carve_batch_buffers(L, base);
    hip_check(hipHostMalloc((void**)&g->h_tables, L.tables_bytes, hipHostMallocDefault),
              "hipHostMalloc");
    hip_check(hipHostMalloc((void**)&g->h_arena, L.arena_bytes, hipHostMallocDefault),
              "hipHostMalloc");
    hip_check(hipHostMalloc((void**)&g->h_result, L.result_bytes, hipHostMallocDefault),
              "hipHostMalloc");
    memset(g->h_tables, 0, L.tables_bytes);

    const DevSet& Y = index_set(idx);
    double ymean = 0.0;
    for (int l = std::max(Y.lmin, 0); l <= Y.lmax; ++l)
        ymean += (double)l * (double)(Y.h_lenstart[l + 1] - Y.h_lenstart[l]);
    ymean = Y.n > 0 ? ymean / (double)Y.n : 0.0;
    int tau_min = 0, tau_max = 0;
    index_taus(idx, &tau_min, &tau_max);
    const TuneParams tp = tune_lookup(tune_cache, tau_max, ymean);
    GraphBatch G;
    setup_graph_batch(idx, L, g->B, tp, G);

    hipGraph_t graph = nullptr;
    hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "begin capture");
    hipError_t e1 = launch_graph_batch(G, st);
    hipError_t e2 = hipMemcpyAsync(g->h_result, g->B.result, L.result_bytes,
                                   hipMemcpyDeviceToHost, st);
    hipError_t e3 = hipStreamEndCapture(st, &graph);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        throw Error(PJ_EDEVICE, "query graph capture failed: %s",
                    hipGetErrorString(e1 != hipSuccess ? e1 : e2 != hipSuccess ? e2 : e3));
    }
    hipError_t e4 = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    hip_check(e4, "graph instantiate");
    return g.release();
}

void graph_plan_destroy(GraphPlan* g) { delete g; }

bool graph_plan_run(GraphPlan* g, const pj_strings* Q, const int32_t* taus,
                    std::vector<uint64_t>& pairs, pj_stats& stats)
{
    if (Q->n == 0) return true;
    int64_t bytes = 0;
    if (pack_query_batch(g->idx, g->L, Q, taus, g->h_tables, g->h_arena, &bytes) !=
        PackStatus::kOk)
        return false;
    hip_check(hipMemcpyAsync(g->B.tables, g->h_tables, g->L.tables_bytes, hipMemcpyHostToDevice,
                             g->st), "upload batch tables");
    if (bytes > 0)
        hip_check(hipMemcpyAsync(g->B.arena, g->h_arena, (size_t)bytes, hipMemcpyHostToDevice,
                                 g->st), "upload batch arena");
    hip_check(hipGraphLaunch(g->exec, g->st), "graph launch");
    hip_check(hipStreamSynchronize(g->st), "sync");
    pj_stats part{};
    const uint64_t* out = nullptr;
    unsigned long long flags = 0;
    const uint32_t m = batch_result(g->h_result, part, &out, &flags);
    if (flags != 0) return false;
    pairs.insert(pairs.end(), out, out + m);
    stats.hits += part.hits;
    stats.candidates += part.candidates;
    stats.key_collisions += part.key_collisions;
    stats.selected += part.selected;
    stats.accepted += part.accepted;
    stats.cells += part.cells;
    stats.side_pairs += part.side_pairs;
    stats.pairs += (int64_t)m;
    return true;
}

}  // namespace pj
