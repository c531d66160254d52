// pj_host_internal.h -- host-side runtime pieces of libpassjoin shared by the join, index and
// serving translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <exception>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/passjoin.h"
#include "pj_internal.h"

namespace pj {

struct Error {
    int code;
    std::string msg;
    Error(int c, const char* fmt, ...);
};

void hip_check(hipError_t e, const char* what);

// Device allocator interface: named buffers, so a workspace can reuse them across calls.
struct Alloc {
    long long budget = 0;   // 0 = unlimited
    size_t used = 0;        // bytes requested in the current call
    virtual ~Alloc() = default;
    virtual void* get(const char* name, size_t bytes) = 0;
};

// Grow-only named buffers cached per thread (scratch of one call at a time).
struct Workspace : Alloc {
    struct Buf {
        void* p = nullptr;
        size_t cap = 0;
    };
    std::unordered_map<std::string, Buf> bufs;
    ~Workspace() override;
    void* get(const char* name, size_t bytes) override;
    void begin_call(long long b) { budget = b; used = 0; }
    void release_all();
};

// Allocations owned by a long-lived object (an index); freed with it.
struct Owned : Alloc {
    std::vector<void*> ptrs;
    ~Owned() override;
    void* get(const char* name, size_t bytes) override;
};

Workspace& thread_workspace();
int device_cus();

// Values the host reads back from the device to size the next phase.  A self-join plan
// (pj_plan.cpp) runs the join once recording them in order, then captures the same sequence of
// launches in a graph: while it captures, every read is served from the record, and nothing is
// read back, uploaded or synchronised (the plan's own buffers already hold the uploaded tables).
struct ReadTape {
    bool replay = false;
    std::vector<uint8_t> bytes;
    size_t pos = 0;
    std::vector<std::pair<void*, size_t>> pending;   // reads enqueued before the next sync
};
extern thread_local ReadTape* t_tape;
// device -> host read, complete after the next sync_readback on the stream
void readback(void* host, const void* dev, size_t bytes, hipStream_t st);
void sync_readback(hipStream_t st);
// forgets this thread's read-backs that no sync_readback completed (after waiting for their
// streams): their targets belong to a scope an exception is leaving
void drop_readbacks();
// declared in a function that issues read-backs into its own variables: when an exception
// leaves the function between a read-back and its sync, the read-back is dropped
struct ReadbackScope {
    int uncaught = std::uncaught_exceptions();
    ~ReadbackScope()
    {
        if (std::uncaught_exceptions() > uncaught) drop_readbacks();
    }
};
// host table -> device
void upload(void* dev, const void* host, size_t bytes, hipStream_t st);
// device memory = 0 with a kernel (bytes a multiple of 4)
void zero_words(void* dev, size_t bytes, hipStream_t st);

// hipEvent marks on one stream (none while a plan's graph is captured).
struct Timer {
    hipStream_t st;
    std::vector<hipEvent_t> evs;
    explicit Timer(hipStream_t s);
    ~Timer();
    int mark();
    double ms(int a, int b);
};

// Launch parameters of the batched path that do not change results (chosen by the autotuner,
// pj_tune.cpp; these are the built-in defaults).
struct TuneParams {
    int verify_waves_per_cu = 32;   // persistent grid of the verification kernels
    int seg_chunk = 4;              // list segments (64 members each) per wave chunk
    int big_list = 32;              // lists with at least this many candidates: list-segment kernel
    int probe_blocks_per_cu = 8;    // grid of the probe kernel
    int lane_cands = 2;             // list-segment candidates per lane (1 or 2)
    int probe_map = 0;              // probe threads: 0 string-major, 1 pair-major (64 strings)
};

bool tune_params_valid(const TuneParams& p);
// Parameters for a call: the autotune table entry for (this GPU, tau, length bucket of the
// probe set's mean length), read from the cache file when one is named, else the defaults.
TuneParams tune_lookup(const char* cache, int tau, double mean_len);

struct JoinScratch {
    int mode = PJ_MODE_AUTO;
    TuneParams tp;
    unsigned long long* counters = nullptr;
    Hit* hits = nullptr;
    unsigned long long* prefix = nullptr;
    uint64_t nhits = 0, ncand = 0;
    uint64_t* out = nullptr;
    uint64_t naccepted = 0;
    uint64_t guard_misses = 0;
    struct Mark { int a, b, kind; };     // event pairs around kernel launches (0 probe, 1 verify)
    std::vector<Mark> kernel_marks;
};

void build_set(const pj_strings* S, bool on_device, Alloc& A, const std::string& tag, DevSet& D,
               hipStream_t st);
void build_index(const DevSet& D, int tau, Alloc& A, const std::string& tag, DevIndex& X,
                 hipStream_t st, bool with_inline = false, bool with_share = false);
// What to probe: a uniform tau against one index, or per-probe thresholds (q_tau, by sorted
// position of the probe set) against the per-tau indices in refs.
struct ProbeSpec {
    bool self = false;
    int tau = 0;                       // uniform tau, or the largest tau of the batch
    const DevIndex* X = nullptr;       // uniform index
    const int32_t* q_tau = nullptr;    // device, per sorted position (mixed batch)
    const IndexRef* refs = nullptr;    // device, [kTauMax + 1] (mixed batch)
    uint64_t bound = 0;                // selection bound for a mixed batch (computed by the caller)
    SymMap sym;                        // the indexed set's symbol map (index keys)
    bool has_entries = true;           // some index has entries
    int selection = 0;                 // PJ_SELECT_*
    int probe_min_len = 0;             // self-join: only strings at least this long probe
};

void run_candidates(const DevSet& P, const DevSet& Y, const ProbeSpec& spec, JoinScratch& J,
                    pj_stats& stats, Timer& tm, hipStream_t st);
uint64_t finish_pairs(const DevSet& P, const DevSet& Y, bool self, const uint64_t* acc,
                      uint64_t m, int32_t** a_out, int32_t** b_out, hipStream_t st);
void emit_output(const int32_t* da, const int32_t* db, uint64_t M, bool to_device, pj_pairs* out,
                 hipStream_t st);

void validate_host_strings(const pj_strings* S, const char* what);
void run_query_batch(const pj_index* idx, const pj_strings* Q, const int32_t* taus,
                     std::vector<uint64_t>& pairs, pj_stats& stats, hipStream_t st,
                     const char* tune_cache);
int64_t query_footprint(const pj_index* idx, int n, int tau);
void index_taus(const pj_index* idx, int* lo, int* hi);
const DevSet& index_set(const pj_index* idx);
const IndexRef* index_refs(const pj_index* idx);
SymMap index_sym(const pj_index* idx);
bool index_has_entries(const pj_index* idx);
int index_device(const pj_index* idx);
int64_t query_selections(const pj_index* idx, int n, int tau);

// Fixed-capacity buffers of one mixed-tau query batch run by launch_graph_batch: the layout of
// the batch tables (nx | lenstart | gbase | perm | q_tau | slen, packed on the host), the arena
// and the device work buffers.  Used by the serving slots' captured pipelines (allocated) and
// by pj_query_noalloc (carved out of a static device array).
struct BatchLayout {
    int64_t qcap = 0, bcap = 0;             // queries, arena bytes
    uint64_t hcap = 0, chunk_cap = 0, acc_cap = 0;
    size_t off_lenstart = 0, off_gbase = 0, off_perm = 0, off_qtau = 0, off_slen = 0;
    size_t tables_bytes = 0, arena_bytes = 0;
    size_t result_bytes = 0;                // [counters 8 | bcounts 4 | out_n | out kGraphSortCap]
};
struct BatchBuffers {
    uint8_t* tables = nullptr;
    uint8_t* arena = nullptr;
    Hit* hits = nullptr;
    unsigned long long* prefix = nullptr;
    uint32_t* first = nullptr;
    uint64_t* acc = nullptr;
    uint8_t* result = nullptr;
};
enum class PackStatus { kOk, kTooManyQueries, kTauOutOfRange, kTooManySelections, kTooManyBytes };
BatchLayout batch_layout(int max_queries, uint64_t hcap, uint64_t chunk_cap, uint64_t acc_cap);
size_t batch_device_bytes(const BatchLayout& L);
BatchBuffers carve_batch_buffers(const BatchLayout& L, uint8_t* base);
void setup_graph_batch(const pj_index* idx, const BatchLayout& L, const BatchBuffers& B,
                       const TuneParams& tp, GraphBatch& G);
// Packs Q into the host mirrors of the tables and the arena; *arena_used = arena bytes to upload.
PackStatus pack_query_batch(const pj_index* idx, const BatchLayout& L, const pj_strings* Q,
                            const int32_t* taus, uint8_t* h_tables, uint8_t* h_arena,
                            int64_t* arena_used);
// Reads a batch result block: adds its counters to stats, returns the number of sorted
// (query << 32 | indexed id) pairs at *pairs; *flags != 0 means a capacity overflowed.
uint32_t batch_result(const uint8_t* h_result, pj_stats& stats, const uint64_t** pairs,
                      unsigned long long* flags);

// A serving slot's captured query pipeline (pj_graph.cpp): fixed-capacity device buffers, one
// instantiated hipGraph of the device phases, pinned staging for the batch and its result.
struct GraphPlan;
GraphPlan* graph_plan_create(const pj_index* idx, int max_queries, hipStream_t st,
                             const char* tune_cache);
void graph_plan_destroy(GraphPlan* g);
int64_t graph_plan_device_bytes(int max_queries);
// Runs one batch through the graph; false when the batch does not fit the plan's capacities or
// a device-side capacity overflowed (the caller then runs it with run_query_batch).  pairs get
// (query << 32 | indexed id), sorted.
bool graph_plan_run(GraphPlan* g, const pj_strings* Q, const int32_t* taus,
                    std::vector<uint64_t>& pairs, pj_stats& stats);
void release_thread_workspace();

// pj_self_join with the launch parameters given (the autotuner's trial runs)
int self_join_with(const pj_strings* S, int32_t tau, const pj_options* opt, pj_pairs* out,
                   const TuneParams* force);

extern thread_local std::string t_last_error;
extern thread_local pj_stats t_stats;
extern thread_local pj_stats t_last_ok_stats;

}  // namespace pj
