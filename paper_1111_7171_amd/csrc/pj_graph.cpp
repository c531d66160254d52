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

struct GraphPlan {
    const pj_index* idx = nullptr;
    hipStream_t st = nullptr;
    int tau_min = 0, tau_max = 0;
    int64_t qcap = 0, bcap = 0;
    uint64_t hcap = 1ull << 20;                 // hit records
    uint64_t chunk_cap = (1ull << 26) / 1024;   // wave chunks of 1024 candidates
    uint64_t acc_cap = 1ull << 20;              // accepted candidates before deduplication
    Owned mem;
    // device: tables = [nx (8 B) | lenstart | gbase | perm | q_tau | slen], mirrored in h_tables
    uint8_t* d_tables = nullptr;
    size_t off_lenstart = 0, off_gbase = 0, off_perm = 0, off_qtau = 0, off_slen = 0;
    size_t tables_bytes = 0;
    uint8_t* d_arena = nullptr;
    // device: result = [counters 8 x u64 | bcounts 4 x u64 | out_n (8 B) | out kGraphSortCap]
    uint8_t* d_result = nullptr;
    size_t result_bytes = 0;
    uint8_t* h_tables = nullptr;
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

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

GraphPlan* graph_plan_create(const pj_index* idx, int max_queries, hipStream_t st,
                             const char* tune_cache)
{
    std::unique_ptr<GraphPlan> g(new GraphPlan());
    g->idx = idx;
    g->st = st;
    index_taus(idx, &g->tau_min, &g->tau_max);
    g->qcap = std::max(1, max_queries);
    g->bcap = g->qcap * 512;
    const int64_t Q = g->qcap;

    size_t o = 8;
    g->off_lenstart = o; o += sizeof(int32_t) * (kLenTab + 1);
    o = align256(o);
    g->off_gbase = o; o += sizeof(int64_t) * kLenTab;
    g->off_perm = o; o += sizeof(int32_t) * (size_t)Q;
    g->off_qtau = o; o += sizeof(int32_t) * (size_t)Q;
    g->off_slen = o; o += sizeof(uint16_t) * (size_t)Q;
    g->tables_bytes = align256(o);
    g->result_bytes = sizeof(unsigned long long) * 12 + 8 + sizeof(uint64_t) * kGraphSortCap;

    g->d_tables = (uint8_t*)g->mem.get("graph.tables", g->tables_bytes);
    g->d_arena = (uint8_t*)g->mem.get("graph.arena", (size_t)g->bcap + 64);
    Hit* hits = (Hit*)g->mem.get("graph.hits", sizeof(Hit) * g->hcap);
    auto* prefix = (unsigned long long*)g->mem.get("graph.prefix",
                                                   sizeof(unsigned long long) * (g->hcap + 1));
    auto* first = (uint32_t*)g->mem.get("graph.first", sizeof(uint32_t) * g->chunk_cap);
    auto* acc = (uint64_t*)g->mem.get("graph.acc", sizeof(uint64_t) * g->acc_cap);
    g->d_result = (uint8_t*)g->mem.get("graph.result", g->result_bytes);
    hip_check(hipHostMalloc((void**)&g->h_tables, g->tables_bytes, hipHostMallocDefault),
              "hipHostMalloc");
    hip_check(hipHostMalloc((void**)&g->h_arena, (size_t)g->bcap + 64, hipHostMallocDefault),
              "hipHostMalloc");
    hip_check(hipHostMalloc((void**)&g->h_result, g->result_bytes, hipHostMallocDefault),
              "hipHostMalloc");
    memset(g->h_tables, 0, g->tables_bytes);

    auto* counters = (unsigned long long*)g->d_result;
    const DevSet& Y = index_set(idx);
    double ymean = 0.0;
    for (int l = std::max(Y.lmin, 0); l <= Y.lmax; ++l)
        ymean += (double)l * (double)(Y.h_lenstart[l + 1] - Y.h_lenstart[l]);
    ymean = Y.n > 0 ? ymean / (double)Y.n : 0.0;
    const TuneParams tp = tune_lookup(tune_cache, g->tau_max, ymean);
    GraphBatch G{};
    ProbeParams& pp = G.probe;
    pp.x_arena = g->d_arena;
    pp.x_slen = (const uint16_t*)(g->d_tables + g->off_slen);
    pp.x_lenstart = (const int32_t*)(g->d_tables + g->off_lenstart);
    pp.x_gbase = (const int64_t*)(g->d_tables + g->off_gbase);
    pp.g_begin = 0;
    pp.nl = 2 * g->tau_max + 1;
    pp.self = 0;
    pp.q_tau = (const int32_t*)(g->d_tables + g->off_qtau);
    pp.refs = index_refs(idx);
    pp.y_lenstart = Y.lenstart;
    pp.tau = g->tau_max;
    pp.ymin = Y.lmin;
    pp.ymax = Y.lmax;
    pp.hits = hits;
    pp.hit_cap = g->hcap;
    pp.counters = counters;
    pp.nx_dev = (const uint32_t*)g->d_tables;
    pp.sym = index_sym(idx);
    pp.selection = PJ_SELECT_MULTIMATCH;
    // grids sized for the plan's capacity (a serving batch is small; idle blocks of a
    // chip-wide grid would still cost every batch their launch)
    const uint64_t probe_threads = (uint64_t)Q * (uint64_t)pp.nl * (uint64_t)(g->tau_max + 1);
    G.probe_grid = (int)std::min<uint64_t>((uint64_t)device_cus() * tp.probe_blocks_per_cu,
                                           (probe_threads + 255) / 256);
    if (!index_has_entries(idx)) pp.ymax = -1;        // nothing indexed: the probe finds no list
    VerifyParams& vp = G.verify;
    vp.x_arena = pp.x_arena; vp.x_slen = pp.x_slen; vp.x_lenstart = pp.x_lenstart;
    vp.x_gbase = pp.x_gbase;
    vp.y_arena = Y.sarena; vp.y_lenstart = Y.lenstart; vp.y_gbase = Y.gbase;
    vp.wave_rounds = kBatchedRoundsMax;               // fixed chunk: the sizes are on device
    vp.y_inl = nullptr;                               // serving indices keep no inline copies
    vp.y_inl_base = nullptr;
    vp.hits = hits;
    vp.prefix = prefix;
    vp.tau = g->tau_max;
    vp.y_maxlen = Y.lmax;
    vp.exact_len = pp.sym.exact_len;
    vp.q_tau = pp.q_tau;
    vp.refs = pp.refs;
    vp.out = acc;
    vp.out_cap = g->acc_cap;
    vp.counters = counters;
    G.bcounts = counters + 8;
    vp.dev_counts = G.bcounts;
    G.verify_grid = std::max(1, std::min(device_cus() * tp.verify_waves_per_cu / 4, 256));
    G.first = first;
    G.chunk_cap = g->chunk_cap;
    // indexed strings shorter than tau_max + 1 go through the side path
    if (Y.n > 0 && Y.lmin <= g->tau_max) {
        const int top = std::min(g->tau_max, Y.lmax);
        G.y_first = (uint32_t)Y.h_lenstart[0];
        G.y_count = (uint32_t)(Y.h_lenstart[top + 1] - Y.h_lenstart[0]);
    }
    G.y_arena = Y.sarena; G.y_slen = Y.slen; G.y_lenstart = Y.lenstart; G.y_gbase = Y.gbase;
    G.xperm = (const int32_t*)(g->d_tables + g->off_perm);
    G.yperm = Y.perm;
    G.out_n = (uint32_t*)(counters + 12);
    G.out = (uint64_t*)(counters + 13);

    hipGraph_t graph = nullptr;
    hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "begin capture");
    hipError_t e1 = launch_graph_batch(G, st);
    hipError_t e2 = hipMemcpyAsync(g->h_result, g->d_result, g->result_bytes,
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
    const int64_t n = Q->n;
    if (n == 0) return true;
    if (n > g->qcap) return false;
    // the Lemma 2 bound on hit records decides whether the hit buffer can overflow at all
    uint64_t bound = 0;
    std::vector<int32_t> cnt(kLenTab + 1, 0);
    for (int64_t q = 0; q < n; ++q) {
        const int len = Q->offsets[q + 1] - Q->offsets[q];
        if (taus[q] < g->tau_min || taus[q] > g->tau_max) return false;
        bound += (uint64_t)query_selections(g->idx, len, taus[q]);
        cnt[len] += 1;
    }
    if (bound > g->hcap) return false;
    // length-sorted arena and tables, packed on the host (the build_set layout)
    auto* lenstart = (int32_t*)(g->h_tables + g->off_lenstart);
    auto* gbase = (int64_t*)(g->h_tables + g->off_gbase);
    auto* perm = (int32_t*)(g->h_tables + g->off_perm);
    auto* qtau = (int32_t*)(g->h_tables + g->off_qtau);
    auto* slen = (uint16_t*)(g->h_tables + g->off_slen);
    int64_t pos = 0, bytes = 0;
    for (int l = 0; l < kLenTab; ++l) {
        lenstart[l] = (int32_t)pos;
        gbase[l] = bytes;
        pos += cnt[l];
        bytes += (int64_t)cnt[l] * stride_of(l);
    }
    lenstart[kLenTab] = (int32_t)pos;
    if (bytes > g->bcap) return false;
    std::vector<int32_t> fill(lenstart, lenstart + kLenTab);
    for (int64_t q = 0; q < n; ++q) {           // stable: ids ascending within a length
        const int len = Q->offsets[q + 1] - Q->offsets[q];
        const int32_t gpos = fill[len]++;
        perm[gpos] = (int32_t)q;
        qtau[gpos] = taus[q];
        slen[gpos] = (uint16_t)len;
        uint8_t* dst = g->h_arena + gbase[len] + (int64_t)(gpos - lenstart[len]) * stride_of(len);
        if (len) memcpy(dst, Q->bytes + Q->offsets[q], (size_t)len);
        const int pad = stride_of(len) - len;
        if (pad) memset(dst + len, 0, (size_t)pad);
    }
    *(uint32_t*)g->h_tables = (uint32_t)n;
    hip_check(hipMemcpyAsync(g->d_tables, g->h_tables, g->tables_bytes, hipMemcpyHostToDevice,
                             g->st), "upload batch tables");
    if (bytes > 0)
        hip_check(hipMemcpyAsync(g->d_arena, g->h_arena, (size_t)bytes, hipMemcpyHostToDevice,
                                 g->st), "upload batch arena");
    hip_check(hipGraphLaunch(g->exec, g->st), "graph launch");
    hip_check(hipStreamSynchronize(g->st), "sync");
    const auto* c = (const unsigned long long*)g->h_result;
    const unsigned long long flags = c[11];
    if (flags != 0) return false;
    const uint32_t m = *(const uint32_t*)(c + 12);
    const auto* out = (const uint64_t*)(c + 13);
    pairs.insert(pairs.end(), out, out + m);
    stats.hits += (int64_t)c[0];
    stats.candidates += (int64_t)c[1];
    stats.selected += (int64_t)c[2];
    stats.accepted += (int64_t)c[3];
    stats.cells += (int64_t)c[4];
    stats.side_pairs += (int64_t)c[6];
    stats.pairs += (int64_t)m;
    return true;
}

}  // namespace pj
