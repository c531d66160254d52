// pj_host.cpp -- host runtime and C ABI of libpassjoin.
//
// A call runs: validate -> upload -> length-sorted arena -> segment index -> probe -> verify
// (+ short-string path) -> deduplicate -> output.  Device scratch comes from a per-thread cache
// of grow-only buffers, so repeated calls on one thread do not reallocate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/passjoin.h"
#include "pj_internal.h"
#include "pj_host_internal.h"
#include "pj_validate.h"

namespace pj {

// Host results of at least this many bytes per array go to page-locked memory.
constexpr size_t kPinnedOutputMin = 1u << 20;

// Inverted lists with at least this many candidates are verified a 64-member segment per wave.
// Below this many candidates the batched path verifies the hits in probe order, in one launch.
constexpr uint64_t kBucketMinCandidates = 1ull << 20;

// ------------------------------------------------------------------------------------------
// Errors and per-thread state
// ------------------------------------------------------------------------------------------

thread_local std::string t_last_error;
thread_local pj_stats t_stats;
thread_local pj_stats t_last_ok_stats;

Error::Error(int c, const char* fmt, ...) : code(c)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    msg = buf;
}

void hip_check(hipError_t e, const char* what)
{
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (e == hipErrorOutOfMemory) throw Error(PJ_ENOMEM, "%s: %s", what, hipGetErrorString(e));
        throw Error(PJ_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    }
}

// ------------------------------------------------------------------------------------------
// Device memory
// ------------------------------------------------------------------------------------------

Workspace::~Workspace()
{
    for (auto& kv : bufs)
        if (kv.second.p) (void)hipFree(kv.second.p);
}

void* Workspace::get(const char* name, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    bytes = (bytes + 255) & ~(size_t)255;
    if (budget > 0 && used + bytes > (size_t)budget)
        throw Error(PJ_ENOMEM, "memory budget of %lld bytes exceeded (%s needs %zu more)",
                    (long long)budget, name, bytes);
    used += bytes;
    Buf& b = bufs[name];
    if (b.cap < bytes) {
        if (b.p) hip_check(hipFree(b.p), "hipFree");
        b.p = nullptr;
        b.cap = 0;
        size_t want = bytes + bytes / 8;
        hipError_t e = hipMalloc(&b.p, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            b.p = nullptr;
            throw Error(PJ_ENOMEM, "hipMalloc(%zu) for %s failed: %s", want, name,
                        hipGetErrorString(e));
        }
        b.cap = want;
    }
    return b.p;
}

void Workspace::release_all()
{
    for (auto& kv : bufs)
        if (kv.second.p) (void)hipFree(kv.second.p);
    bufs.clear();
}

Owned::~Owned()
{
    for (void* p : ptrs) (void)hipFree(p);
}

void* Owned::get(const char* name, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    bytes = (bytes + 255) & ~(size_t)255;
    if (budget > 0 && used + bytes > (size_t)budget)
        throw Error(PJ_ENOMEM, "memory budget of %lld bytes exceeded (%s)", (long long)budget,
                    name);
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(PJ_ENOMEM, "hipMalloc(%zu) for %s failed", bytes, name);
    }
    used += bytes;
    ptrs.push_back(p);
    return p;
}

static thread_local Workspace* t_ws = nullptr;

Workspace& thread_workspace()
{
    if (!t_ws) t_ws = new Workspace();
    return *t_ws;
}

void release_thread_workspace()
{
    delete t_ws;
    t_ws = nullptr;
}

int device_cus()
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        hip_check(hipGetDevice(&dev), "hipGetDevice");
        int v = 0;
        hip_check(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev),
                  "hipDeviceGetAttribute");
        cus = v > 0 ? v : 256;
    }
    return cus;
}

static int bitlen(uint64_t v)
{
    int b = 0;
    while (v) { ++b; v >>= 1; }
    return b;
}

// ------------------------------------------------------------------------------------------
// Read-backs (recorded by a plan's first run, served from the record while it captures)
// ------------------------------------------------------------------------------------------

thread_local ReadTape* t_tape = nullptr;

// Small read-backs land in a page-locked staging buffer of the calling thread, so that their
// copies are asynchronous: a copy into pageable memory makes the host wait for the stream, and
// the device then idles until the host launches the next kernel, once per read-back instead of
// once per sync_readback.  The values move to their destinations at the next sync_readback on
// the stream.  Buffers go back to a process-wide pool when their thread ends (no HIP call at
// thread exit).
namespace {

constexpr size_t kStageBytes = 64 << 10;     // per thread
constexpr size_t kStageMaxRead = 16 << 10;   // larger read-backs copy straight to their target

std::mutex g_stage_mu;
std::vector<uint8_t*> g_stage_pool;

struct ThreadStage {
    uint8_t* buf = nullptr;
    size_t used = 0;
    struct Pending {
        void* host;
        size_t off, bytes;
        hipStream_t st;
    };
    std::vector<Pending> pend;
    bool failed = false;                     // page-locked allocation refused: pageable copies

    uint8_t* get()
    {
        if (!buf && !failed) {
            {
                std::lock_guard<std::mutex> lk(g_stage_mu);
                if (!g_stage_pool.empty()) {
                    buf = g_stage_pool.back();
                    g_stage_pool.pop_back();
                }
            }
            if (!buf && hipHostMalloc((void**)&buf, kStageBytes, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                buf = nullptr;
                failed = true;
            }
        }
        return buf;
    }

    ~ThreadStage()
    {
        // a buffer with copies that no sync completed is not handed on (kept until exit)
        if (buf && pend.empty()) {
            std::lock_guard<std::mutex> lk(g_stage_mu);
            g_stage_pool.push_back(buf);
        }
    }
};

thread_local ThreadStage t_stage;

}  // namespace

void readback(void* host, const void* dev, size_t bytes, hipStream_t st)
{
    if (t_tape && t_tape->replay) {
        if (t_tape->pos + bytes > t_tape->bytes.size())
            throw Error(PJ_EDEVICE, "plan record exhausted (the join took another path)");
        memcpy(host, t_tape->bytes.data() + t_tape->pos, bytes);
        t_tape->pos += bytes;
        return;
    }
    ThreadStage& S = t_stage;
    const size_t need = (bytes + 15) & ~(size_t)15;
    uint8_t* buf = bytes <= kStageMaxRead ? S.get() : nullptr;
    if (buf && S.used + need <= kStageBytes) {
        hip_check(hipMemcpyAsync(buf + S.used, dev, bytes, hipMemcpyDeviceToHost, st),
                  "read back");
        S.pend.push_back({host, S.used, bytes, st});
        S.used += need;
    } else {
        hip_check(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, st), "read back");
    }
    if (t_tape) t_tape->pending.emplace_back(host, bytes);
}

void drop_readbacks()
{
    ThreadStage& S = t_stage;
    for (const auto& p : S.pend) (void)hipStreamSynchronize(p.st);
    (void)hipGetLastError();
    S.pend.clear();
    S.used = 0;
}

void sync_readback(hipStream_t st)
{
    if (t_tape && t_tape->replay) return;
    hip_check(hipStreamSynchronize(st), "sync");
    ThreadStage& S = t_stage;
    if (!S.pend.empty()) {
        size_t keep = 0;
        for (size_t k = 0; k < S.pend.size(); ++k) {
            const auto& p = S.pend[k];
            if (p.st == st) memcpy(p.host, S.buf + p.off, p.bytes);
            else S.pend[keep++] = p;        // another stream's read: still in flight
        }
        S.pend.resize(keep);
        if (keep == 0) S.used = 0;
    }
    if (t_tape) {
        for (const auto& p : t_tape->pending) {
            const uint8_t* b = (const uint8_t*)p.first;
            t_tape->bytes.insert(t_tape->bytes.end(), b, b + p.second);
        }
        t_tape->pending.clear();
    }
}

void upload(void* dev, const void* host, size_t bytes, hipStream_t st)
{
    if (t_tape && t_tape->replay) return;
    hip_check(hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, st), "upload");
}

void zero_words(void* dev, size_t bytes, hipStream_t st)
{
    hip_check(launch_fill_words((uint32_t*)dev, (uint64_t)(bytes / 4), 0u, st), "fill");
}

// ------------------------------------------------------------------------------------------
// Timing
// ------------------------------------------------------------------------------------------

Timer::Timer(hipStream_t s) : st(s) {}

Timer::~Timer()
{
    for (auto e : evs) (void)hipEventDestroy(e);
}

int Timer::mark()
{
    if (t_tape && t_tape->replay) return -1;
    hipEvent_t e;
    hip_check(hipEventCreate(&e), "hipEventCreate");
    hip_check(hipEventRecord(e, st), "hipEventRecord");
    evs.push_back(e);
    return (int)evs.size() - 1;
}

double Timer::ms(int a, int b)
{
    if (a < 0 || b < 0) return 0.0;
    float v = 0.f;
    hip_check(hipEventSynchronize(evs[b]), "hipEventSynchronize");
    hip_check(hipEventElapsedTime(&v, evs[a], evs[b]), "hipEventElapsedTime");
    return (double)v;
}

// ------------------------------------------------------------------------------------------
// Input validation and the length-sorted arena
// ------------------------------------------------------------------------------------------

void validate_host_strings(const pj_strings* S, const char* what)
{
    char msg[256];
    const int rc = check_host_strings(S, what, msg, sizeof msg);
    if (rc != PJ_OK) throw Error(rc, "%s", msg);
}

// Bytes of device memory readable from p: the rest of the allocation that holds p.  Throws
// PJ_EINVAL when p is not device (or managed) memory of the current device, so no kernel is
// ever handed a host, unregistered or foreign pointer.
static size_t device_extent(const void* p, const std::string& what)
{
    hipPointerAttribute_t attr{};
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(PJ_EINVAL, "%s: not a device pointer", what.c_str());
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        throw Error(PJ_EINVAL, "%s: not device memory (memory type %d)", what.c_str(),
                    (int)attr.type);
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (attr.type == hipMemoryTypeDevice && attr.device != dev)
        throw Error(PJ_EINVAL, "%s: memory of device %d, the current device is %d", what.c_str(),
                    attr.device, dev);
    void* base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, const_cast<void*>(p));
    if (e != hipSuccess || !base) {
        (void)hipGetLastError();
        throw Error(PJ_EINVAL, "%s: no device allocation holds this pointer", what.c_str());
    }
    return size - (size_t)((const uint8_t*)p - (const uint8_t*)base);
}

void build_set(const pj_strings* S, bool on_device, Alloc& A, const std::string& tag, DevSet& D,
               hipStream_t st)
{
    ReadbackScope rb_scope;
    if (!S) throw Error(PJ_EINVAL, "%s: null pj_strings", tag.c_str());
    size_t bytes_extent = 0;
    if (!on_device) validate_host_strings(S, tag.c_str());
    else {
        if (S->n < 0) throw Error(PJ_EINVAL, "%s: n < 0", tag.c_str());
        if (S->n >= (int64_t)INT32_MAX) throw Error(PJ_ERANGE, "%s: too many strings", tag.c_str());
        if (!S->offsets) throw Error(PJ_EINVAL, "%s: null offsets", tag.c_str());
        // every pointer a kernel will read is checked first: device memory, large enough
        if (device_extent(S->offsets, tag + ".offsets") < sizeof(int32_t) * (size_t)(S->n + 1))
            throw Error(PJ_EINVAL, "%s: offsets allocation holds fewer than n + 1 entries",
                        tag.c_str());
        if (S->bytes) bytes_extent = device_extent(S->bytes, tag + ".bytes");
    }
    const int64_t n = S->n;
    D.n = n;
    auto nm = [&](const char* s) { return tag + "." + s; };

    const int32_t* d_offs = nullptr;
    const uint8_t* d_bytes = nullptr;
    int64_t total = 0;
    if (on_device) {
        d_offs = S->offsets;
        d_bytes = S->bytes;
    } else {
        total = S->offsets[n];
        int32_t* o = (int32_t*)A.get(nm("offs").c_str(), sizeof(int32_t) * (size_t)(n + 1));
        hip_check(hipMemcpyAsync(o, S->offsets, sizeof(int32_t) * (size_t)(n + 1),
                                 hipMemcpyHostToDevice, st), "upload offsets");
        uint8_t* bb = (uint8_t*)A.get(nm("bytes").c_str(), (size_t)total + 16);
        if (total > 0)
            hip_check(hipMemcpyAsync(bb, S->bytes, (size_t)total, hipMemcpyHostToDevice, st),
                      "upload bytes");
        d_offs = o;
        d_bytes = bb;
    }

    // length histogram (+ validation of device inputs)
    int32_t* lcount = (int32_t*)A.get(nm("lcount").c_str(), sizeof(int32_t) * (kLenTab + 1));
    zero_words(lcount, sizeof(int32_t) * (kLenTab + 1), st);
    hip_check(launch_length_hist(d_offs, n, lcount, lcount + kLenTab, st), "length_hist");
    std::vector<int32_t> h(kLenTab + 1);
    int32_t dev_total = 0;
    readback(h.data(), lcount, sizeof(int32_t) * (kLenTab + 1), st);
    if (on_device && n > 0) readback(&dev_total, d_offs + n, sizeof(int32_t), st);
    sync_readback(st);
    int err = h[kLenTab];
    if (err & 1) throw Error(PJ_EINVAL, "%s: offsets[0] != 0", tag.c_str());
    if (err & 2) throw Error(PJ_EINVAL, "%s: offsets decrease", tag.c_str());
    if (err & 4) throw Error(PJ_ERANGE, "%s: a string is longer than %d", tag.c_str(), kLenMax);
    if (on_device && dev_total > 0) {
        // the bytes the arena kernel will read: offsets[n] of them from S->bytes
        if (!d_bytes) throw Error(PJ_EINVAL, "%s: null bytes with offsets[n] = %d", tag.c_str(),
                                  dev_total);
        if ((size_t)dev_total > bytes_extent)
            throw Error(PJ_EINVAL, "%s: offsets[n] = %d exceeds the %zu bytes of the bytes "
                        "allocation", tag.c_str(), dev_total, bytes_extent);
    }

    int64_t pos = 0, bytes = 0;
    D.lmin = kLenTab;
    D.lmax = -1;
    for (int l = 0; l < kLenTab; ++l) {
        D.h_lenstart[l] = (int32_t)pos;
        D.h_gbase[l] = bytes;
        if (h[l] > 0) {
            D.lmin = std::min(D.lmin, l);
            D.lmax = std::max(D.lmax, l);
        }
        pos += h[l];
        bytes += (int64_t)h[l] * stride_of(l);
    }
    D.h_lenstart[kLenTab] = (int32_t)pos;
    if (D.lmax < 0) D.lmin = 0;
    D.arena_bytes = bytes;

    D.lenstart = (int32_t*)A.get(nm("lenstart").c_str(), sizeof(int32_t) * (kLenTab + 1));
    D.gbase = (int64_t*)A.get(nm("gbase").c_str(), sizeof(int64_t) * kLenTab);
    upload(D.lenstart, D.h_lenstart, sizeof(int32_t) * (kLenTab + 1), st);
    upload(D.gbase, D.h_gbase, sizeof(int64_t) * kLenTab, st);

    D.perm = (int32_t*)A.get(nm("perm").c_str(), sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1));
    D.slen = (uint16_t*)A.get(nm("slen").c_str(), sizeof(uint16_t) * (size_t)std::max<int64_t>(n, 1));
    D.sarena = (uint8_t*)A.get(nm("sarena").c_str(), (size_t)bytes + 64);
    if (n == 0) return;

    // stable sort of ids by length -> perm
    Workspace& W = thread_workspace();
    uint32_t* k0 = (uint32_t*)W.get("lensort.k0", sizeof(uint32_t) * (size_t)n);
    uint32_t* k1 = (uint32_t*)W.get("lensort.k1", sizeof(uint32_t) * (size_t)n);
    uint32_t* v1 = (uint32_t*)W.get("lensort.v1", sizeof(uint32_t) * (size_t)n);
    size_t tb = radix_tmp_bytes((uint64_t)n);
    void* tmp = W.get("radix.tmp", tb);
    uint32_t* v0 = (uint32_t*)D.perm;
    hip_check(launch_iota_len_keys(d_offs, n, k0, v0, st), "len_keys");
    bool alt = false;
    hip_check(radix_sort_u32(k0, v0, k1, v1, (uint64_t)n, bitlen((uint64_t)std::max(D.lmax, 1)),
                             tmp, tb, &alt, st), "radix(len)");
    if (alt)
        hip_check(hipMemcpyAsync(D.perm, v1, sizeof(uint32_t) * (size_t)n,
                                 hipMemcpyDeviceToDevice, st), "perm copy");
    hip_check(launch_pack_arena(d_bytes, d_offs, D.perm, n, D.lenstart, D.gbase, D.sarena, D.slen,
                                D.lmax, st), "pack_arena");
}

// ------------------------------------------------------------------------------------------
// Segment index
// ------------------------------------------------------------------------------------------

void build_index(const DevSet& D, int tau, Alloc& A, const std::string& tag, DevIndex& X,
                 hipStream_t st, bool with_inline, bool with_share)
{
    ReadbackScope rb_scope;
    const int T1 = tau + 1;
    X.tau = tau;
    auto nm = [&](const char* s) { return tag + "." + s; };
    int64_t g_first = (T1 <= kLenMax + 1) ? D.h_lenstart[std::min(T1, kLenTab)] : D.n;
    int64_t g_count = D.n - g_first;
    int64_t E = g_count * T1;
    if (E >= (int64_t)UINT32_MAX) throw Error(PJ_ERANGE, "index too large (%lld entries)", (long long)E);
    X.entries = E;
    {
        // symbol map of the bytes the set contains: codes 1..sigma, 0 for absent bytes
        Workspace& WS = thread_workspace();
        uint32_t* bm = (uint32_t*)WS.get("index.bytemap", 8 * sizeof(uint32_t));
        zero_words(bm, 8 * sizeof(uint32_t), st);
        hip_check(launch_byte_presence(D, bm, st), "byte_presence");
        uint32_t hb[8];
        readback(hb, bm, sizeof hb, st);
        sync_readback(st);
        uint16_t code[256];
        int sigma = 0;
        for (int b = 0; b < 256; ++b)
            code[b] = (hb[b >> 5] >> (b & 31)) & 1u ? (uint16_t)(++sigma) : (uint16_t)0;
        const int sbits = std::max(1, bitlen((uint64_t)sigma));
        uint16_t* dcode = (uint16_t*)A.get(nm("sym").c_str(), sizeof code);
        upload(dcode, code, sizeof code, st);
        sync_readback(st);                  // code[] is on this stack frame
        X.sym = SymMap{dcode, sbits, kHashBits / sbits};
    }
    if (E == 0) {
        X.keys = (uint64_t*)A.get(nm("keys").c_str(), 16);
        X.vals = (uint32_t*)A.get(nm("vals").c_str(), 16);
        X.mask = 1023;
        X.table = (uint4*)A.get(nm("table").c_str(), sizeof(uint4) * 1024);
        hip_check(launch_clear_table(X.table, 1024, st), "clear_table");
        X.lists = 0;
        return;
    }
    std::vector<int64_t> ebase(kLenTab, 0);
    int64_t run = 0;
    for (int l = 0; l < kLenTab; ++l) {
        ebase[l] = run;
        if (l >= T1) run += (int64_t)(D.h_lenstart[l + 1] - D.h_lenstart[l]) * T1;
    }
    Workspace& W = thread_workspace();
    int64_t* d_ebase = (int64_t*)W.get("index.ebase", sizeof(int64_t) * kLenTab);
    upload(d_ebase, ebase.data(), sizeof(int64_t) * kLenTab, st);
    uint64_t* keys = (uint64_t*)A.get(nm("keys").c_str(), sizeof(uint64_t) * (size_t)E);
    uint32_t* vals = (uint32_t*)A.get(nm("vals").c_str(), sizeof(uint32_t) * (size_t)E);
    uint64_t* keys2 = (uint64_t*)W.get("index.keys2", sizeof(uint64_t) * (size_t)E);
    uint32_t* vals2 = (uint32_t*)W.get("index.vals2", sizeof(uint32_t) * (size_t)E);
    hip_check(launch_emit_segments(D, tau, d_ebase, g_first, g_count, X.sym, keys, vals, st),
              "emit");
    uint64_t grp_max = (uint64_t)(D.lmax - T1) * T1 + tau;
    int bits = kHashBits + std::max(1, bitlen(grp_max));
    size_t tb = radix_tmp_bytes((uint64_t)E);
    void* tmp = W.get("radix.tmp", tb);
    bool alt = false;
    hip_check(radix_sort_u64(keys, vals, keys2, vals2, (uint64_t)E, bits, tmp, tb, &alt, st),
              "radix(index)");
    if (alt) {
        hip_check(hipMemcpyAsync(keys, keys2, sizeof(uint64_t) * (size_t)E,
                                 hipMemcpyDeviceToDevice, st), "keys copy");
        hip_check(hipMemcpyAsync(vals, vals2, sizeof(uint32_t) * (size_t)E,
                                 hipMemcpyDeviceToDevice, st), "vals copy");
    }
    X.keys = keys;
    X.vals = vals;
    // inline copies of the members' strings (short strings only, and only within the budget):
    // the list-segment kernel then reads a list's strings contiguously
    std::vector<int64_t> inl_base(kLenTab, 0);
    if (with_inline && D.lmax <= kInlineMaxLen) {
        int64_t bytes = 0;
        for (int l = T1; l < kLenTab; ++l) {
            inl_base[l] = bytes - ebase[l] * stride_of(l);
            bytes += (int64_t)(D.h_lenstart[l + 1] - D.h_lenstart[l]) * T1 * stride_of(l);
        }
        const size_t need = (size_t)bytes + sizeof(int64_t) * kLenTab;
        if (A.budget == 0 || (long long)(A.used + need) <= A.budget) {
            X.inl = (uint8_t*)A.get(nm("inl").c_str(), (size_t)std::max<int64_t>(bytes, 16));
            X.inl_base = (int64_t*)A.get(nm("inl_base").c_str(), sizeof(int64_t) * kLenTab);
            upload(X.inl_base, inl_base.data(), sizeof(int64_t) * kLenTab, st);
            hip_check(launch_gather_inline(D, keys, vals, E, tau, X.inl_base, X.inl, st),
                      "gather_inline");
        }
    }
    // lists = runs of equal keys
    uint32_t* flags = (uint32_t*)W.get("index.flags", sizeof(uint32_t) * (size_t)E);
    uint32_t* runid = (uint32_t*)W.get("index.runid", sizeof(uint32_t) * (size_t)(E + 1));
    hip_check(launch_mark_heads(keys, E, flags, st), "mark_heads");
    size_t sb = scan_tmp_bytes((uint64_t)E);
    void* stmp = W.get("scan.tmp", sb);
    hip_check(scan_u32_to_u32(flags, runid, (uint64_t)E, stmp, sb, st), "scan(runs)");
    uint32_t nruns = 0;
    readback(&nruns, runid + E, sizeof(uint32_t), st);
    sync_readback(st);
    X.lists = nruns;
    uint32_t* runstart = (uint32_t*)W.get("index.runstart", sizeof(uint32_t) * (size_t)(nruns + 1));
    hip_check(launch_scatter_runstart(flags, runid, E, runstart, st), "runstart");
    uint64_t slots = 1024;
    while (slots < 2ull * nruns) slots <<= 1;
    X.mask = slots - 1;
    X.table = (uint4*)A.get(nm("table").c_str(), sizeof(uint4) * (size_t)slots);
    hip_check(launch_clear_table(X.table, slots, st), "clear_table");
    hip_check(launch_insert_runs(keys, runstart, nruns, (uint32_t)E, X.table, X.mask, st),
              "insert_runs");
    // the longest segment (even partition: lengths floor(l / (tau+1)) or one more)
    const int max_seg = (D.lmax + T1 - 1) / T1;
    if (max_seg > X.sym.exact_len || max_seg * X.sym.bits >= kFilterMinBits) {
        // key filter for hashed segments and long exact codes, blocked by (l, i) group (16 bits
        // per list)
        const uint32_t ngroups = (uint32_t)((D.lmax - T1 + 1) * T1);
        const uint64_t fwords = (uint64_t)nruns + 2ull * ngroups;
        X.filter = (uint32_t*)A.get(nm("filter").c_str(), sizeof(uint32_t) * (size_t)fwords);
        X.filter_dir = (uint32_t*)A.get(nm("filter_dir").c_str(),
                                        sizeof(uint32_t) * (size_t)(ngroups + 1));
        uint32_t* gfirst = (uint32_t*)W.get("index.gfirst", sizeof(uint32_t) * (size_t)ngroups);
        uint32_t* gend = (uint32_t*)W.get("index.gend", sizeof(uint32_t) * (size_t)ngroups);
        uint32_t* words = (uint32_t*)W.get("index.fwords", sizeof(uint32_t) * (size_t)ngroups);
        zero_words(gfirst, sizeof(uint32_t) * (size_t)ngroups, st);
        zero_words(gend, sizeof(uint32_t) * (size_t)ngroups, st);
        zero_words(X.filter, sizeof(uint32_t) * (size_t)fwords, st);
        const size_t fsb = scan_tmp_bytes(ngroups);
        void* fst = W.get("scan.tmp", std::max(fsb, sb));
        hip_check(launch_filter_build(keys, runstart, nruns, ngroups, gfirst, gend, words, fst, fsb,
                                      X.filter_dir, X.filter, st), "filter");
    }
    if (with_share) {
        // content order of every list (shared-prefix verification, Sec. 5.3): entries sorted by
        // (key, first 8 bytes of the string, g) -- by the bytes first, then stably by the key
        uint64_t* pk = (uint64_t*)W.get("share.pk", sizeof(uint64_t) * (size_t)E);
        uint32_t* pi = (uint32_t*)W.get("share.pi", sizeof(uint32_t) * (size_t)E);
        uint64_t* pk2 = (uint64_t*)W.get("index.keys2", sizeof(uint64_t) * (size_t)E);
        uint32_t* pi2 = (uint32_t*)W.get("index.vals2", sizeof(uint32_t) * (size_t)E);
        hip_check(launch_prefix8_keys(D, vals, E, pk, pi, st), "prefix8 keys");
        bool alt2 = false;
        hip_check(radix_sort_u64(pk, pi, pk2, pi2, (uint64_t)E, 64, tmp, tb, &alt2, st),
                  "radix(content)");
        uint32_t* order = alt2 ? pi2 : pi;
        uint32_t* order_alt = alt2 ? pi : pi2;
        uint64_t* k1 = alt2 ? pk : pk2;               // free key buffers
        uint64_t* k1_alt = alt2 ? pk2 : pk;
        hip_check(launch_gather_keys(keys, order, E, k1, st), "gather keys");
        bool alt3 = false;
        hip_check(radix_sort_u64(k1, order, k1_alt, order_alt, (uint64_t)E, bits, tmp, tb, &alt3,
                                 st), "radix(content key)");
        if (alt3) order = order_alt;
        X.svals = (uint32_t*)A.get(nm("svals").c_str(), sizeof(uint32_t) * (size_t)E);
        X.runlen = (uint32_t*)A.get(nm("runlen").c_str(), sizeof(uint32_t) * (size_t)E);
        hip_check(launch_gather_vals(vals, order, E, X.svals, st), "gather svals");
        hip_check(launch_run_lengths(runstart, nruns, (uint32_t)E, X.runlen, st), "run lengths");
    }
}

// ------------------------------------------------------------------------------------------
// Probe + verify + short-string path
// ------------------------------------------------------------------------------------------

// Upper bound on the selected substrings (Lemma 2 count per probed length), which bounds hits.
static uint64_t selection_bound(const DevSet& P, const DevSet& Y, int tau, bool self,
                                int64_t* probe_first, int min_len)
{
    const int T1 = tau + 1;
    uint64_t total = 0;
    for (int n = self ? std::max(min_len, 0) : 0; n < kLenTab; ++n) {
        int64_t cnt = P.h_lenstart[n + 1] - P.h_lenstart[n];
        if (cnt == 0) continue;
        int lo = self ? n - tau : n - tau, hi = self ? n : n + tau;
        uint64_t per = 0;
        for (int l = std::max(lo, T1); l <= hi && l <= kLenMax; ++l) {
            if (Y.h_lenstart[l + 1] == Y.h_lenstart[l]) continue;
            int d = n - l;
            per += (uint64_t)((tau * tau - d * d) / 2 + tau + 1);
        }
        total += per * (uint64_t)cnt;
    }
    const int first_len = std::max(T1, min_len);
    *probe_first = self ? (first_len <= kLenMax ? P.h_lenstart[first_len] : P.n) : 0;
    return total;
}

void run_candidates(const DevSet& P, const DevSet& Y, const ProbeSpec& spec, JoinScratch& J,
                    pj_stats& stats, Timer& tm, hipStream_t st)
{
    ReadbackScope rb_scope;
    Workspace& W = thread_workspace();
    const int tau = spec.tau;
    const bool self = spec.self;
    const int T1 = tau + 1;
    J.counters = (unsigned long long*)W.get("join.counters",
                                            kJoinCounters * sizeof(unsigned long long));
    zero_words(J.counters, kJoinCounters * sizeof(unsigned long long), st);
    int64_t probe_first = 0;
    uint64_t bound = spec.q_tau ? spec.bound
                                : selection_bound(P, Y, tau, self, &probe_first,
                                                  spec.probe_min_len);
    // the other selection methods select supersets of the multi-match windows: start the hit
    // buffer larger (an overflow re-runs the probe with the exact size anyway)
    if (spec.selection != PJ_SELECT_MULTIMATCH) bound *= (uint64_t)(2 * tau + 1);
    int64_t nprobe = P.n - probe_first;
    // hit records: the Lemma 2 bound can be far above the real count (long segments rarely
    // match), so start from a capped buffer and re-run the probe with the exact size if needed
    uint64_t hit_cap = std::min<uint64_t>(std::max<uint64_t>(bound, 1), 1ull << 26);
    const bool entries = spec.q_tau ? spec.has_entries : (spec.X && spec.X->entries > 0);
    int t_probe0 = tm.mark();
    unsigned long long c[kJoinCounters];
    for (int attempt = 0; attempt < 2; ++attempt) {
    J.hits = (Hit*)W.get("join.hits", sizeof(Hit) * (size_t)hit_cap);
    if (attempt > 0)
        zero_words(J.counters, kJoinCounters * sizeof(unsigned long long), st);
    if (nprobe > 0 && bound > 0 && entries) {
        ProbeParams pp{};
        pp.x_arena = P.sarena; pp.x_slen = P.slen; pp.x_lenstart = P.lenstart; pp.x_gbase = P.gbase;
        pp.g_begin = (uint32_t)probe_first;
        pp.nl = self ? T1 : 2 * tau + 1;
        pp.threads = (uint64_t)nprobe * (uint64_t)pp.nl * (uint64_t)T1;
        // the thread mapping the tuner chose (pair-major keeps a wave's lanes on windows of
        // one size when probe strings have few (length, slot) pairs); the plain path keeps the
        // string-major one
        if (!spec.q_tau && J.tp.probe_map == 1 && J.mode != PJ_MODE_PLAIN) {
            pp.xmajor = 1;
            pp.nx = (uint32_t)nprobe;
            pp.threads = ((uint64_t)nprobe + 63) / 64 * 64 * (uint64_t)pp.nl * (uint64_t)T1;
        }
        // tests force either thread mapping (it changes no result)
        if (const char* e = getenv("PJ_PROBE_XMAJOR")) {
            if (atoi(e) == 0 || spec.q_tau) {
                pp.xmajor = 0;
                pp.threads = (uint64_t)nprobe * (uint64_t)pp.nl * (uint64_t)T1;
            } else {
                pp.xmajor = 1;
                pp.nx = (uint32_t)nprobe;
                pp.threads = ((uint64_t)nprobe + 63) / 64 * 64 * (uint64_t)pp.nl * (uint64_t)T1;
            }
        }
        pp.self = self ? 1 : 0;
        pp.q_tau = spec.q_tau;
        pp.refs = spec.refs;
        pp.y_lenstart = Y.lenstart;
        if (spec.X) {
            pp.keys = spec.X->keys; pp.vals = spec.X->vals; pp.table = spec.X->table;
            pp.mask = spec.X->mask;
            pp.filter = spec.X->filter;
            pp.filter_dir = spec.X->filter_dir;
        }
        pp.tau = tau;
        pp.ymin = Y.lmin; pp.ymax = Y.lmax;
        pp.sym = spec.sym;
        pp.selection = spec.selection;
        if (!spec.q_tau && spec.selection == PJ_SELECT_MULTIMATCH && J.mode != PJ_MODE_PLAIN) {
            // the (length, slot) pairs grouped by window size, so a wave's lanes walk windows of
            // one size (the plain path keeps the natural order: it is the unscheduled baseline)
            uint16_t* order = (uint16_t*)W.get(
                "probe.order", sizeof(uint16_t) * (size_t)pp.nl * (size_t)T1);
            hip_check(launch_probe_order(tau, pp.nl, pp.self, order, st), "probe_order");
            pp.order = order;
        }
        pp.hits = J.hits; pp.hit_cap = hit_cap;
        pp.counters = J.counters;
        int k0 = tm.mark();
        hip_check(launch_probe(pp, device_cus() * J.tp.probe_blocks_per_cu, st), "probe");
        int k1 = tm.mark();
        J.kernel_marks.push_back({k0, k1, 0});
    }
    readback(c, J.counters, sizeof c, st);
    sync_readback(st);
    if (c[0] <= hit_cap) break;
    hit_cap = c[0];
    J.kernel_marks.clear();
    }
    int t_probe1 = tm.mark();
    J.nhits = c[0];
    J.ncand = c[1];
    stats.selected += (int64_t)c[2];
    stats.hits += (int64_t)c[0];
    stats.candidates += (int64_t)c[1];
    if (J.nhits > hit_cap) throw Error(PJ_EDEVICE, "hit buffer overflow (%llu > %llu)",
                                       (unsigned long long)J.nhits, (unsigned long long)hit_cap);

    const bool batched = J.mode != PJ_MODE_PLAIN;
    // batched: hits bucketed into [lists with < big_list candidates | the others], each part by
    // the length class of its lists' strings and then in slot order; small lists are verified
    // candidate by candidate, big ones a 64-member segment per wave, one launch per part and
    // length class (so that lists of short strings take the kernels that stage their strings
    // in LDS even when the set has long strings)
    uint64_t nsmall = J.nhits, nbig = 0;
    uint64_t sm_off[kLenClasses + 1] = {};     // small hits of class c: [sm_off[c], sm_off[c+1])
    uint64_t cls_off[kLenClasses + 1] = {};    // big hits of class c: [cls_off[c], cls_off[c+1])
    uint64_t sm_ncand[kLenClasses] = {};
    uint64_t cls_nseg[kLenClasses] = {};
    uint32_t* segp = nullptr;                  // class c's scan at segp + cls_off[c] + c
    // few candidates (a serving batch): the bucketing round trips would cost more than they save
    uint64_t bucket_min = kBucketMinCandidates;
    if (const char* e = getenv("PJ_BUCKET_MIN_CANDIDATES")) bucket_min = strtoull(e, nullptr, 10);
    if (batched && J.nhits > 0 && J.ncand >= bucket_min) {
        const unsigned g = slot_bucket_grid(J.nhits);
        const size_t nbb = (size_t)g * kHitBuckets;
        uint32_t* bb = (uint32_t*)W.get("join.bb", sizeof(uint32_t) * nbb);
        uint32_t* bb_off = (uint32_t*)W.get("join.bb_off", sizeof(uint32_t) * (nbb + 1));
        const size_t sb = scan_tmp_bytes(nbb);
        void* stmp = W.get("scan.tmp3", sb);
        Hit* sorted = (Hit*)W.get("join.hits2", sizeof(Hit) * (size_t)J.nhits);
        hip_check(launch_slot_bucket(J.hits, J.counters, J.nhits, (uint32_t)J.tp.big_list, bb,
                                     bb_off, stmp, sb, sorted, st), "slot_bucket");
        J.hits = sorted;
        // bucket 64 * c opens length class c of the small lists, 64 * (kLenClasses + c) that of
        // the big ones
        uint32_t start[2 * kLenClasses] = {};
        for (int c = 1; c < 2 * kLenClasses; ++c)
            readback(&start[c], bb_off + (size_t)g * 64 * c, sizeof(uint32_t), st);
        sync_readback(st);
        nsmall = start[kLenClasses];
        nbig = J.nhits - nsmall;
        for (int c = 0; c < kLenClasses; ++c) {
            sm_off[c] = start[c];
            cls_off[c] = start[kLenClasses + c] - nsmall;
        }
        sm_off[kLenClasses] = nsmall;
        cls_off[kLenClasses] = nbig;
    } else {
        // one range of small lists, of every length: the last class's bound is the set's
        for (int c = 0; c <= kLenClasses; ++c) sm_off[c] = (c == kLenClasses) ? nsmall : 0;
    }

    const Hit* bigp = J.hits + nsmall;

    // candidate prefix sums of the small lists, one scan per class (class c's at J.prefix +
    // sm_off[c] + c), list segments of the big ones
    J.prefix = (unsigned long long*)W.get(
        "join.prefix", sizeof(unsigned long long) * (size_t)(nsmall + kLenClasses));
    auto small_prefix = [&](int c) { return J.prefix + sm_off[c] + c; };
    // a class's candidate total: read back with the big lists' totals (nbig > 0), or alone
    // when several classes have small lists; with small lists of one class only and no big
    // lists, it is every candidate
    unsigned long long sm_total[kLenClasses] = {};
    int sm_classes = 0, sm_last = 0;
    for (int c = 0; c < kLenClasses; ++c)
        if (sm_off[c + 1] > sm_off[c]) {
            ++sm_classes;
            sm_last = c;
        }
    const bool read_totals = nbig > 0 || sm_classes > 1;
    if (nsmall > 0) {
        uint32_t* counts = (uint32_t*)W.get("join.counts", sizeof(uint32_t) * (size_t)nsmall);
        hip_check(launch_hit_counts(J.hits, nsmall, counts, st), "hit_counts");
        size_t sb = scan_tmp_bytes(nsmall);
        void* stmp = W.get("scan.tmp", sb);
        for (int c = 0; c < kLenClasses; ++c) {
            const uint64_t o = sm_off[c], nh = sm_off[c + 1] - o;
            if (nh == 0) continue;
            hip_check(scan_u32_to_u64(counts + o, small_prefix(c), nh, stmp, sb, st),
                      "scan(prefix)");
            if (read_totals)
                readback(&sm_total[c], small_prefix(c) + nh, sizeof(unsigned long long), st);
        }
        if (!read_totals) sm_total[sm_last] = J.ncand;
    }
    // shared-prefix verification of the big lists (Sec. 5.3): chains of list members
    const bool share = J.mode == PJ_MODE_SHARE_PREFIX && spec.X && spec.X->svals && nbig > 0;
    unsigned long long* cprefix = nullptr;
    uint64_t nchains = 0;
    if (share) {
        uint32_t* chains = (uint32_t*)W.get("join.chains", sizeof(uint32_t) * (size_t)nbig);
        cprefix = (unsigned long long*)W.get("join.cprefix",
                                             sizeof(unsigned long long) * (size_t)(nbig + 1));
        hip_check(launch_chain_counts(bigp, nbig, P.slen, spec.X->runlen, self ? 1 : 0, chains,
                                      st), "chain_counts");
        size_t sb = scan_tmp_bytes(nbig);
        void* stmp = W.get("scan.tmp2", sb);
        hip_check(scan_u32_to_u64(chains, cprefix, nbig, stmp, sb, st), "scan(chains)");
        unsigned long long nc = 0;
        readback(&nc, cprefix + nbig, sizeof nc, st);
        sync_readback(st);
        nchains = nc;
    } else if (nbig > 0) {
        uint32_t* segs = (uint32_t*)W.get("join.segs", sizeof(uint32_t) * (size_t)nbig);
        segp = (uint32_t*)W.get("join.segp", sizeof(uint32_t) * (size_t)(nbig + kLenClasses));
        size_t sb = scan_tmp_bytes(nbig);
        void* stmp = W.get("scan.tmp2", sb);
        uint32_t ns[kLenClasses] = {};
        for (int c = 0; c < kLenClasses; ++c) {
            const uint64_t o = cls_off[c], nb = cls_off[c + 1] - o;
            if (nb == 0) continue;
            hip_check(launch_seg_counts(bigp + o, nb,
                                        seg_members(class_maxlen(c, Y.lmax), tau,
                                                    J.tp.lane_cands),
                                        segs + o, st),
                      "seg_counts");
            hip_check(scan_u32_to_u32(segs + o, segp + o + c, nb, stmp, sb, st), "scan(segs)");
            readback(&ns[c], segp + o + c + nb, sizeof(uint32_t), st);
        }
        sync_readback(st);
        for (int c = 0; c < kLenClasses; ++c) cls_nseg[c] = ns[c];
    } else if (nsmall > 0 && read_totals) {
        sync_readback(st);
    }
    uint64_t ncand_small = 0;
    for (int c = 0; c < kLenClasses; ++c) {
        sm_ncand[c] = sm_total[c];
        ncand_small += sm_total[c];
    }

    // verify (+ short path); rerun once with an exact buffer when the first guess overflows
    uint64_t cap = std::min<uint64_t>(J.ncand + 4096, 1ull << 28);
    for (int attempt = 0; attempt < 2; ++attempt) {
        J.out = (uint64_t*)W.get("join.out", sizeof(uint64_t) * (size_t)cap);
        zero_words(J.counters + 3, (kJoinCounters - 3) * sizeof(unsigned long long), st);
        J.kernel_marks.erase(std::remove_if(J.kernel_marks.begin(), J.kernel_marks.end(),
                                            [](const JoinScratch::Mark& m) { return m.kind != 0; }),
                             J.kernel_marks.end());
        if (J.ncand > 0) {
            VerifyParams vp{};
            vp.x_arena = P.sarena; vp.x_slen = P.slen; vp.x_lenstart = P.lenstart;
            vp.x_gbase = P.gbase;
            vp.y_arena = Y.sarena; vp.y_lenstart = Y.lenstart; vp.y_gbase = Y.gbase;
            vp.vals = spec.X ? spec.X->vals : nullptr;
            vp.y_inl = spec.X ? spec.X->inl : nullptr;
            vp.y_inl_base = spec.X ? spec.X->inl_base : nullptr;
            vp.q_tau = spec.q_tau;
            vp.refs = spec.refs;
            vp.hits = J.hits; vp.prefix = small_prefix(kLenClasses - 1);
            vp.nhits = nsmall; vp.ncand = ncand_small;
            vp.tau = tau;
            vp.y_maxlen = Y.lmax;
            vp.exact_len = spec.sym.exact_len;
            vp.out = J.out; vp.out_cap = cap;
            vp.counters = J.counters;
            int k0 = tm.mark();
            if (batched) {
                // small lists, one launch per length class: long strings by row blocks with
                // compacted continuation queues, the others a candidate per lane
                bool long_c[kLenClasses] = {};
                int rounds_c[kLenClasses] = {};
                uint64_t max_chunks = 0, max_long = 0;
                for (int c = 0; c < kLenClasses; ++c) {
                    const uint64_t nc = sm_ncand[c];
                    if (nc == 0) continue;
                    long_c[c] = class_maxlen(c, Y.lmax) > kLongMinLen && tau + 1 <= kLongMaxW &&
                                !spec.q_tau && nc <= (1ull << 24);
                    // tests force either verification of long strings (it changes no result)
                    if (const char* e = getenv("PJ_LONG_VERIFY"))
                        long_c[c] = long_c[c] && atoi(e) != 0;
                    if (long_c[c]) {
                        max_long = std::max<uint64_t>(max_long, nc);
                        continue;
                    }
                    // at least ~32 wave chunks per CU before a wave takes more than one round
                    // of 64 candidates: a few long candidates (long strings, high tau) then
                    // still spread over the whole device
                    const uint64_t per = (uint64_t)device_cus() * 32ull * 64ull;
                    rounds_c[c] = (int)std::max<uint64_t>(
                        1, std::min<uint64_t>((uint64_t)kBatchedRoundsMax, nc / per));
                    // tests force the chunk size (it changes no result)
                    if (const char* e = getenv("PJ_BATCHED_ROUNDS"))
                        rounds_c[c] = std::max(1, std::min(kBatchedRoundsMax, atoi(e)));
                    max_chunks = std::max<uint64_t>(max_chunks, batched_chunks(nc, rounds_c[c]));
                }
                void* lsc = max_long ? W.get("join.long", long_scratch_bytes(max_long)) : nullptr;
                uint32_t* first = max_chunks
                    ? (uint32_t*)W.get("join.first", sizeof(uint32_t) * (size_t)max_chunks)
                    : nullptr;
                for (int c = 0; c < kLenClasses; ++c) {
                    const uint64_t nc = sm_ncand[c];
                    if (nc == 0) continue;
                    VerifyParams vs = vp;
                    vs.hits = J.hits + sm_off[c];
                    vs.prefix = small_prefix(c);
                    vs.nhits = sm_off[c + 1] - sm_off[c];
                    vs.ncand = nc;
                    vs.y_maxlen = class_maxlen(c, Y.lmax);
                    if (long_c[c]) {
                        hip_check(launch_verify_long(vs, nc, std::max(P.lmax, Y.lmax), lsc,
                                                     device_cus() * 8, st), "verify_long");
                    } else {
                        vs.wave_rounds = rounds_c[c];
                        const uint64_t nchunks = batched_chunks(nc, vs.wave_rounds);
                        // persistent: enough waves to fill the chip, each walking its chunks
                        const uint64_t waves = std::min<uint64_t>(
                            nchunks, (uint64_t)device_cus() * J.tp.verify_waves_per_cu);
                        hip_check(launch_verify_batched(vs, first, (int)((waves + 3) / 4), st),
                                  "verify_batched");
                    }
                    stats.verify_launches += 1;
                }
                if (share && nchains > 0) {
                    vp.svals = spec.X->svals;
                    vp.runlen = spec.X->runlen;
                    vp.self = self ? 1 : 0;
                    const uint64_t nchunks = (nchains + 63) / 64;
                    uint32_t* first = (uint32_t*)W.get("join.first2", sizeof(uint32_t) * (size_t)nchunks);
                    const uint64_t waves = std::min<uint64_t>(
                        nchunks, (uint64_t)device_cus() * J.tp.verify_waves_per_cu);
                    const int s0 = tm.mark();
                    hip_check(launch_verify_chains(vp, bigp, cprefix, nbig, nchains, first,
                                                   (int)((waves + 3) / 4), st),
                              "verify_chains");
                    const int s1 = tm.mark();
                    J.kernel_marks.push_back({s0, s1, 2});
                    stats.verify_launches += 1;
                    stats.list_launches += 1;
                }
                uint64_t max_seg_chunks = 0;
                for (int c = 0; c < kLenClasses; ++c)
                    max_seg_chunks = std::max<uint64_t>(max_seg_chunks,
                                                        seg_chunks(cls_nseg[c], J.tp.seg_chunk));
                uint32_t* first2 = max_seg_chunks
                    ? (uint32_t*)W.get("join.first2", sizeof(uint32_t) * (size_t)max_seg_chunks)
                    : nullptr;
                for (int c = 0; c < kLenClasses; ++c) {
                    const uint64_t nseg = cls_nseg[c];
                    if (nseg == 0) continue;
                    const uint64_t o = cls_off[c], nb = cls_off[c + 1] - o;
                    const uint64_t nchunks = seg_chunks(nseg, J.tp.seg_chunk);
                    const uint64_t waves = std::min<uint64_t>(
                        nchunks, (uint64_t)device_cus() * J.tp.verify_waves_per_cu);
                    VerifyParams vc = vp;
                    vc.y_maxlen = class_maxlen(c, Y.lmax);
                    const int s0 = tm.mark();
                    hip_check(launch_verify_segs(vc, bigp + o, segp + o + c, nb, nseg, first2,
                                                 J.tp.seg_chunk, J.tp.lane_cands,
                                                 (int)((waves + 3) / 4), st),
                              "verify_segs");
                    const int s1 = tm.mark();
                    J.kernel_marks.push_back({s0, s1, 2});
                    stats.verify_launches += 1;
                    stats.list_launches += 1;
                }
            } else {
                const uint64_t nchunks = (J.ncand + 1023) / 1024;
                const int grid = (int)std::min<uint64_t>(nchunks, (uint64_t)device_cus() * 16);
                hip_check(launch_verify(vp, grid, st), "verify");
                stats.verify_launches += 1;
            }
            int k1 = tm.mark();
            J.kernel_marks.push_back({k0, k1, 1});
        }
        hip_check(launch_short_path(P, Y, tau, self ? 1 : 0, spec.q_tau, J.out, cap, J.counters,
                                    st), "short_path");
        readback(c, J.counters, sizeof c, st);
        sync_readback(st);
        if (c[3] <= cap) break;
        cap = c[3];
    }
    int t_verify1 = tm.mark();
    J.naccepted = c[3];
    // a hashed key can match a list whose segment bytes differ (a 40-bit collision): the byte
    // guard rejects such a lookup before verification, and it is no candidate of the paper's
    // (x[p, l_i] equal to the member's segment i), so it leaves the candidate count
    stats.candidates -= (int64_t)c[5];
    stats.key_collisions += (int64_t)c[5];
    stats.accepted += (int64_t)c[3];
    stats.cells += (int64_t)(c[4] + c[7]);
    stats.shared_rows += (int64_t)c[8];
    stats.shared_cells += (int64_t)c[9];
    stats.list_cells += (int64_t)c[7];
    stats.side_pairs += (int64_t)c[6];
    J.guard_misses = c[5];
    stats.ms_probe += tm.ms(t_probe0, t_probe1);
    stats.ms_verify += tm.ms(t_probe1, t_verify1);
    for (const auto& km : J.kernel_marks) {
        double v = tm.ms(km.a, km.b);
        if (km.kind == 0) stats.ms_probe_kernel += v;
        else if (km.kind == 1) stats.ms_verify_kernel += v;
        else stats.ms_list_kernel += v;
    }
    J.kernel_marks.clear();
}

// Sorts and deduplicates accepted (gx, gy) into id pairs; returns device arrays (workspace).
uint64_t finish_pairs(const DevSet& P, const DevSet& Y, bool self, const uint64_t* acc,
                      uint64_t m, int32_t** a_out, int32_t** b_out, hipStream_t st)
{
    ReadbackScope rb_scope;
    Workspace& W = thread_workspace();
    if (m >= (uint64_t)UINT32_MAX) throw Error(PJ_ERANGE, "too many accepted candidates");
    int bbits = std::max(1, bitlen((uint64_t)std::max<int64_t>(std::max(P.n, Y.n) - 1, 1)));
    uint64_t* k0 = (uint64_t*)W.get("out.k0", sizeof(uint64_t) * (size_t)std::max<uint64_t>(m, 1));
    uint64_t* k1 = (uint64_t*)W.get("out.k1", sizeof(uint64_t) * (size_t)std::max<uint64_t>(m, 1));
    int32_t* a = (int32_t*)W.get("out.a", sizeof(int32_t) * (size_t)std::max<uint64_t>(m, 1));
    int32_t* b = (int32_t*)W.get("out.b", sizeof(int32_t) * (size_t)std::max<uint64_t>(m, 1));
    *a_out = a;
    *b_out = b;
    if (m == 0) return 0;
    hip_check(launch_pairs_to_keys(acc, m, P.perm, Y.perm, self ? 1 : 0, bbits, k0, st), "keys");
    size_t tb = radix_tmp_bytes(m);
    void* tmp = W.get("radix.tmp", tb);
    bool alt = false;
    hip_check(radix_sort_u64(k0, nullptr, k1, nullptr, m, 2 * bbits, tmp, tb, &alt, st),
              "radix(pairs)");
    uint64_t* ks = alt ? k1 : k0;
    uint32_t* flags = (uint32_t*)W.get("out.flags", sizeof(uint32_t) * (size_t)m);
    uint32_t* pos = (uint32_t*)W.get("out.pos", sizeof(uint32_t) * (size_t)(m + 1));
    hip_check(launch_unique_flags(ks, m, flags, st), "unique");
    size_t sb = scan_tmp_bytes(m);
    void* stmp = W.get("scan.tmp", sb);
    hip_check(scan_u32_to_u32(flags, pos, m, stmp, sb, st), "scan(unique)");
    hip_check(launch_compact_pairs(ks, flags, pos, m, bbits, a, b, st), "compact");
    uint32_t M = 0;
    readback(&M, pos + m, sizeof(uint32_t), st);
    sync_readback(st);
    return M;
}

void emit_output(const int32_t* da, const int32_t* db, uint64_t M, bool to_device, pj_pairs* out,
                 hipStream_t st)
{
    out->count = (int64_t)M;
    out->on_device = to_device ? 1 : 0;
    out->a = nullptr;
    out->b = nullptr;
    size_t bytes = sizeof(int32_t) * (size_t)std::max<uint64_t>(M, 1);
    if (to_device) {
        void *pa = nullptr, *pb = nullptr;
        if (hipMalloc(&pa, bytes) != hipSuccess || hipMalloc(&pb, bytes) != hipSuccess) {
            (void)hipGetLastError();
            if (pa) (void)hipFree(pa);
            throw Error(PJ_ENOMEM, "output allocation failed");
        }
        out->a = (int32_t*)pa;
        out->b = (int32_t*)pb;
        if (M) {
            hip_check(hipMemcpyAsync(pa, da, sizeof(int32_t) * M, hipMemcpyDeviceToDevice, st), "out");
            hip_check(hipMemcpyAsync(pb, db, sizeof(int32_t) * M, hipMemcpyDeviceToDevice, st), "out");
        }
    } else if (bytes >= kPinnedOutputMin) {
        // large results: page-locked host memory, allocated in place of pageable memory (fresh
        // pageable pages cost a fault on first touch, more than the copy itself) and filled at
        // the link's full rate
        void *pa = nullptr, *pb = nullptr;
        if (hipHostMalloc(&pa, bytes, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&pb, bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            if (pa) (void)hipHostFree(pa);
            throw Error(PJ_ENOMEM, "host output allocation failed");
        }
        out->on_device = 2;
        out->a = (int32_t*)pa;
        out->b = (int32_t*)pb;
        if (M) {
            hip_check(hipMemcpyAsync(pa, da, sizeof(int32_t) * M, hipMemcpyDeviceToHost, st), "out");
            hip_check(hipMemcpyAsync(pb, db, sizeof(int32_t) * M, hipMemcpyDeviceToHost, st), "out");
        }
    } else {
        out->a = (int32_t*)malloc(bytes);
        out->b = (int32_t*)malloc(bytes);
        if (!out->a || !out->b) {
            free(out->a);
            free(out->b);
            out->a = out->b = nullptr;
            throw Error(PJ_ENOMEM, "host output allocation failed");
        }
        if (M) {
            hip_check(hipMemcpyAsync(out->a, da, sizeof(int32_t) * M, hipMemcpyDeviceToHost, st), "out");
            hip_check(hipMemcpyAsync(out->b, db, sizeof(int32_t) * M, hipMemcpyDeviceToHost, st), "out");
        }
    }
    hip_check(hipStreamSynchronize(st), "sync");
}

// ------------------------------------------------------------------------------------------
// Entry points
// ------------------------------------------------------------------------------------------

static void check_tau(int32_t tau)
{
    if (tau < 0 || tau > kTauMax) throw Error(PJ_EINVAL, "tau %d out of [0, %d]", tau, kTauMax);
}

static hipStream_t stream_of(const pj_options* opt)
{
    return opt ? (hipStream_t)opt->hip_stream : (hipStream_t)0;
}

static void zero_pairs(pj_pairs* out)
{
    if (out) {
        out->count = 0;
        out->a = nullptr;
        out->b = nullptr;
        out->on_device = 0;
    }
}

template <typename F>
static int guarded(pj_pairs* out, F&& f)
{
    t_stats = pj_stats{};
    try {
        f();
        t_last_ok_stats = t_stats;
        t_last_error.clear();
        return PJ_OK;
    } catch (const Error& e) {
        t_last_error = e.msg;
        if (out) pj_pairs_free(out);
        zero_pairs(out);
        return e.code;
    } catch (const std::bad_alloc&) {
        t_last_error = "host allocation failed";
        if (out) pj_pairs_free(out);
        zero_pairs(out);
        return PJ_ENOMEM;
    } catch (...) {
        t_last_error = "unexpected internal error";
        if (out) pj_pairs_free(out);
        zero_pairs(out);
        return PJ_EDEVICE;
    }
}

static double mean_length(const DevSet& D)
{
    if (D.n == 0) return 0.0;
    double sum = 0.0;
    for (int l = std::max(D.lmin, 0); l <= D.lmax; ++l)
        sum += (double)l * (double)(D.h_lenstart[l + 1] - D.h_lenstart[l]);
    return sum / (double)D.n;
}

// A plan's run of the join stops before the result is copied out: the sorted pairs stay in the
// workspace (the plan's own) and their count is returned here.
struct PlanOut {
    int32_t* a = nullptr;
    int32_t* b = nullptr;
    uint64_t M = 0;
};

static void join_impl(const pj_strings* R, const pj_strings* S, int32_t tau, const pj_options* opt,
                      pj_pairs* out, bool self, const TuneParams* force = nullptr,
                      int probe_min_len = 0, PlanOut* po = nullptr)
{
    if (!out) throw Error(PJ_EINVAL, "null output");
    zero_pairs(out);
    check_tau(tau);
    if (opt && (opt->mode < PJ_MODE_AUTO || opt->mode > PJ_MODE_SHARE_PREFIX))
        throw Error(PJ_EINVAL, "unknown mode %d", opt->mode);
    if (opt && (opt->selection < PJ_SELECT_MULTIMATCH || opt->selection > PJ_SELECT_LENGTH))
        throw Error(PJ_EINVAL, "unknown selection method %d", opt->selection);
    hipStream_t st = stream_of(opt);
    bool on_dev = opt && opt->inputs_on_device;
    if (!on_dev) {
        // host inputs are fully validated before any device work
        validate_host_strings(self ? S : R, self ? "S" : "R");
        if (!self) validate_host_strings(S, "S");
    }
    Workspace& W = thread_workspace();
    W.begin_call(opt ? opt->mem_budget_bytes : 0);
    auto t0 = std::chrono::steady_clock::now();
    Timer tm(st);
    int e0 = tm.mark();
    DevSet P, Y;
    build_set(self ? S : R, on_dev, W, "P", P, st);
    if (!self) build_set(S, on_dev, W, "Y", Y, st);
    const DevSet& YY = self ? P : Y;
    int e1 = tm.mark();
    DevIndex X;
    const int mode = opt ? opt->mode : PJ_MODE_AUTO;
    build_index(YY, tau, W, "X", X, st, mode != PJ_MODE_PLAIN,
                mode == PJ_MODE_SHARE_PREFIX && tau + 1 <= kShareMaxW);
    int e2 = tm.mark();
    t_stats.strings = P.n + (self ? 0 : Y.n);
    t_stats.index_entries = X.entries;
    JoinScratch J;
    J.mode = opt ? opt->mode : PJ_MODE_AUTO;
    J.tp = force ? *force : tune_lookup(opt ? opt->tune_cache : nullptr, tau, mean_length(P));
    ProbeSpec spec;
    spec.self = self;
    spec.tau = tau;
    spec.X = &X;
    spec.sym = X.sym;
    spec.selection = opt ? opt->selection : PJ_SELECT_MULTIMATCH;
    spec.probe_min_len = probe_min_len;
    run_candidates(P, YY, spec, J, t_stats, tm, st);
    int e3 = tm.mark();
    int32_t *da = nullptr, *db = nullptr;
    uint64_t M = finish_pairs(P, YY, self, J.out, J.naccepted, &da, &db, st);
    if (po) {
        po->a = da;
        po->b = db;
        po->M = M;
    } else {
        emit_output(da, db, M, opt && opt->outputs_on_device, out, st);
    }
    int e4 = tm.mark();
    t_stats.pairs = (int64_t)M;
    t_stats.ms_upload = tm.ms(e0, e1);
    t_stats.ms_index = tm.ms(e1, e2);
    t_stats.ms_output = tm.ms(e3, e4);
    t_stats.ms_total = std::chrono::duration<double, std::milli>(
                           std::chrono::steady_clock::now() - t0).count();
}

// Self-join in length windows (for sets larger than device memory; the sliding window of live
// lists of Sec. 3.2 taken in blocks).  A similar pair is reported by the window holding the
// length of its longer string: window [a, b] joins the strings with lengths in [a - tau, b],
// where only strings of length >= a probe, and keeps the pairs whose longer string is at least
// a long.  Windows are chosen greedily so that the strings of [a - tau, b] hold at most
// window_bytes bytes (at least one length per window).  Host strings in, host pairs out.
static void join_streamed(const pj_strings* S, int32_t tau, int64_t window_bytes,
                          const pj_options* opt, pj_pairs* out)
{
    if (!out) throw Error(PJ_EINVAL, "null output");
    zero_pairs(out);
    check_tau(tau);
    if (window_bytes <= 0) throw Error(PJ_EINVAL, "window_bytes must be positive");
    if (opt && (opt->inputs_on_device || opt->outputs_on_device))
        throw Error(PJ_EINVAL, "streamed self-joins take host strings and return host pairs");
    validate_host_strings(S, "S");
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = S->n;
    std::vector<int64_t> cnt(kLenTab + 1, 0), bytes(kLenTab + 1, 0);
    for (int64_t k = 0; k < n; ++k) {
        const int l = S->offsets[k + 1] - S->offsets[k];
        ++cnt[l];
        bytes[l] += l;
    }
    auto span_bytes = [&](int lo, int hi) {
        int64_t t = 0;
        for (int l = std::max(lo, 0); l <= hi; ++l) t += bytes[l];
        return t;
    };
    // string lengths, scanned once per window (the windows' strings in ascending id order)
    std::vector<uint16_t> len((size_t)std::max<int64_t>(n, 1));
    for (int64_t k = 0; k < n; ++k) len[(size_t)k] = (uint16_t)(S->offsets[k + 1] - S->offsets[k]);
    pj_options o{};
    if (opt) o = *opt;
    o.outputs_on_device = 1;
    const hipStream_t st = stream_of(opt);
    pj_stats acc{};
    // Each pair comes from exactly one window.  The windows' pairs stay on the device as global
    // keys ga << bb | gb and are sorted there once; only when they would pass key_cap (a 64th of
    // the free device memory) is the batch held so far sorted and moved to the host as one run,
    // and the host then merges the runs.
    const int bb = std::max(1, bitlen((uint64_t)std::max<int64_t>(n - 1, 1)));
    uint64_t key_cap = 0;                                      // set with the first window's keys
    struct Batch {
        std::vector<std::pair<uint64_t*, uint64_t>> parts;    // device keys of each window
        uint64_t total = 0;
        unsigned long long* dropped = nullptr;                 // halo sentinels in the batch
        ~Batch()
        {
            for (auto& q : parts) (void)hipFree(q.first);
            if (dropped) (void)hipFree(dropped);
        }
    } batch;
    // device state, set up when the first window has pairs (an empty set touches no device)
    auto start_batches = [&]() {
        if (batch.dropped) return;
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            (void)hipGetLastError();
            free_b = 0;
        }
        key_cap = std::max<uint64_t>(1ull << 20, (uint64_t)(free_b / 64));
        // tests force small batches (it changes no result)
        if (const char* e = getenv("PJ_STREAM_KEY_CAP"))
            key_cap = (uint64_t)std::max(1LL, atoll(e));
        if (hipMalloc((void**)&batch.dropped, sizeof(unsigned long long)) != hipSuccess) {
            (void)hipGetLastError();
            batch.dropped = nullptr;
            throw Error(PJ_ENOMEM, "streamed join: counter allocation failed");
        }
        hip_check(hipMemsetAsync(batch.dropped, 0, sizeof(unsigned long long), st), "memset");
    };
    // sorts the batch on the device; returns the sorted keys (valid ones first) and their count.
    // Its buffers are reused by name from one batch to the next (no budget: the windows' own
    // scratch is the call's budgeted part)
    Workspace sorted_bufs;
    auto sort_batch = [&](uint64_t* valid_out) -> uint64_t* {
        const uint64_t m = batch.total;
        uint64_t* k0 = (uint64_t*)sorted_bufs.get("stream.k0", sizeof(uint64_t) * (size_t)m);
        uint64_t* k1 = (uint64_t*)sorted_bufs.get("stream.k1", sizeof(uint64_t) * (size_t)m);
        uint64_t off = 0;
        for (auto& q : batch.parts) {
            hip_check(hipMemcpyAsync(k0 + off, q.first, sizeof(uint64_t) * (size_t)q.second,
                                     hipMemcpyDeviceToDevice, st), "batch copy");
            off += q.second;
        }
        const size_t tb = radix_tmp_bytes(m);
        void* tmp = sorted_bufs.get("stream.tmp", tb);
        bool alt = false;
        hip_check(radix_sort_u64(k0, nullptr, k1, nullptr, m, 2 * bb, tmp, tb, &alt, st),
                  "radix(stream)");
        unsigned long long dropped = 0;
        hip_check(hipMemcpyAsync(&dropped, batch.dropped, sizeof dropped, hipMemcpyDeviceToHost,
                                 st), "dropped");
        hip_check(hipStreamSynchronize(st), "sync");
        *valid_out = m - (uint64_t)dropped;
        return alt ? k1 : k0;
    };
    auto clear_batch = [&]() {
        for (auto& q : batch.parts) (void)hipFree(q.first);
        batch.parts.clear();
        batch.total = 0;
        hip_check(hipMemsetAsync(batch.dropped, 0, sizeof(unsigned long long), st), "memset");
    };
    // host runs (only when the batch was moved off the device)
    std::vector<std::vector<uint64_t>> runs;
    auto spill = [&]() {
        if (batch.total == 0) return;
        uint64_t valid = 0;
        const uint64_t* ks = sort_batch(&valid);
        runs.emplace_back((size_t)valid);
        if (valid)
            hip_check(hipMemcpyAsync(runs.back().data(), ks, sizeof(uint64_t) * (size_t)valid,
                                     hipMemcpyDeviceToHost, st), "spill");
        hip_check(hipStreamSynchronize(st), "sync");
        clear_batch();
    };
    int lmax = -1;
    for (int l = 0; l <= kLenMax; ++l)
        if (cnt[l]) lmax = l;
    std::vector<int32_t> ids;
    std::vector<int32_t> offs;
    std::vector<uint8_t> buf;
    int a = 0;
    while (a <= lmax) {
        while (a <= lmax && cnt[a] == 0) ++a;
        if (a > lmax) break;
        int b = a;
        while (b + 1 <= lmax && span_bytes(a - tau, b + 1) <= window_bytes) ++b;
        // the window's strings in ascending id order (so local order is global order)
        const int lo = std::max(a - tau, 0);
        ids.clear();
        offs.assign(1, 0);
        buf.resize((size_t)std::max<int64_t>(span_bytes(lo, b), 1));
        for (int64_t k = 0; k < n; ++k) {
            const int l = len[(size_t)k];
            if (l < lo || l > b) continue;
            if (l) memcpy(buf.data() + offs.back(), S->bytes + S->offsets[k], (size_t)l);
            ids.push_back((int32_t)k);
            offs.push_back(offs.back() + l);
        }
        pj_strings sub{(int64_t)ids.size(), buf.data(), offs.data()};
        pj_pairs part{};
        t_stats = pj_stats{};
        join_impl(nullptr, &sub, tau, &o, &part, true, nullptr, a);
        // pairs with both strings in the halo [a - tau, a) come only from the short-string
        // path, so the length filter is needed only when the window holds strings <= tau long
        const bool filter = lo <= tau;
        if (part.count > 0) {
            const uint64_t m = (uint64_t)part.count;
            start_batches();
            if (batch.total > 0 && batch.total + m > key_cap) spill();
            Owned win;
            int32_t* d_ids = (int32_t*)win.get("win.ids", sizeof(int32_t) * ids.size());
            hip_check(hipMemcpyAsync(d_ids, ids.data(), sizeof(int32_t) * ids.size(),
                                     hipMemcpyHostToDevice, st), "ids");
            int32_t* d_offs = nullptr;
            if (filter) {
                d_offs = (int32_t*)win.get("win.offs", sizeof(int32_t) * offs.size());
                hip_check(hipMemcpyAsync(d_offs, offs.data(), sizeof(int32_t) * offs.size(),
                                         hipMemcpyHostToDevice, st), "offs");
            }
            uint64_t* kp = nullptr;
            if (hipMalloc((void**)&kp, sizeof(uint64_t) * (size_t)m) != hipSuccess) {
                (void)hipGetLastError();
                pj_pairs_free(&part);
                throw Error(PJ_ENOMEM, "streamed join: key buffer of %llu pairs",
                            (unsigned long long)m);
            }
            batch.parts.emplace_back(kp, m);
            batch.total += m;
            hip_check(launch_window_keys(part.a, part.b, m, d_ids, d_offs, filter ? a : 0, bb, kp,
                                         batch.dropped, st), "window keys");
            hip_check(hipStreamSynchronize(st), "sync");
        }
        pj_pairs_free(&part);
        acc.strings += t_stats.strings;
        acc.index_entries += t_stats.index_entries;
        acc.selected += t_stats.selected;
        acc.hits += t_stats.hits;
        acc.candidates += t_stats.candidates;
        acc.cells += t_stats.cells;
        acc.accepted += t_stats.accepted;
        acc.side_pairs += t_stats.side_pairs;
        acc.ms_upload += t_stats.ms_upload;
        acc.ms_index += t_stats.ms_index;
        acc.ms_probe += t_stats.ms_probe;
        acc.ms_verify += t_stats.ms_verify;
        acc.ms_output += t_stats.ms_output;
        acc.ms_probe_kernel += t_stats.ms_probe_kernel;
        acc.ms_verify_kernel += t_stats.ms_verify_kernel;
        acc.verify_launches += t_stats.verify_launches;
        acc.ms_list_kernel += t_stats.ms_list_kernel;
        acc.list_cells += t_stats.list_cells;
        acc.list_launches += t_stats.list_launches;
        acc.key_collisions += t_stats.key_collisions;
        acc.shared_rows += t_stats.shared_rows;
        acc.shared_cells += t_stats.shared_cells;
        a = b + 1;
    }
    if (runs.empty() && batch.total == 0) {
        // no pairs at all
        out->on_device = 0;
        out->count = 0;
        out->a = (int32_t*)malloc(sizeof(int32_t));
        out->b = (int32_t*)malloc(sizeof(int32_t));
        if (!out->a || !out->b) throw std::bad_alloc();
        acc.pairs = 0;
        acc.ms_total = std::chrono::duration<double, std::milli>(
                           std::chrono::steady_clock::now() - t0).count();
        t_stats = acc;
        return;
    }
    if (runs.empty()) {
        // every window's keys on the device: split the sorted keys into the output
        uint64_t valid = 0;
        const uint64_t* ks = sort_batch(&valid);
        int32_t* da = (int32_t*)sorted_bufs.get("stream.a", sizeof(int32_t) * (size_t)valid);
        int32_t* db = (int32_t*)sorted_bufs.get("stream.b", sizeof(int32_t) * (size_t)valid);
        hip_check(launch_split_keys(ks, valid, bb, da, db, st), "split");
        emit_output(da, db, valid, false, out, st);
        acc.pairs = (int64_t)valid;
        acc.ms_total = std::chrono::duration<double, std::milli>(
                           std::chrono::steady_clock::now() - t0).count();
        t_stats = acc;
        return;
    }
    spill();
    // k-way merge of the host runs straight into the output arrays
    size_t m = 0;
    for (const auto& r : runs) m += r.size();
    out->on_device = 0;
    out->a = (int32_t*)malloc(sizeof(int32_t) * std::max<size_t>(m, 1));
    out->b = (int32_t*)malloc(sizeof(int32_t) * std::max<size_t>(m, 1));
    if (!out->a || !out->b) throw std::bad_alloc();
    const uint64_t lo_mask = (1ull << bb) - 1;
    using Head = std::pair<uint64_t, size_t>;          // (key, run)
    std::vector<Head> heap;
    std::vector<size_t> pos(runs.size(), 0);
    for (size_t r = 0; r < runs.size(); ++r)
        if (!runs[r].empty()) heap.emplace_back(runs[r][0], r);
    auto greater = [](const Head& x, const Head& y) { return x.first > y.first; };
    std::make_heap(heap.begin(), heap.end(), greater);
    for (size_t k = 0; k < m; ++k) {
        std::pop_heap(heap.begin(), heap.end(), greater);
        const Head h = heap.back();
        heap.pop_back();
        out->a[k] = (int32_t)(h.first >> bb);
        out->b[k] = (int32_t)(h.first & lo_mask);
        const size_t r = h.second;
        if (++pos[r] < runs[r].size()) {
            heap.emplace_back(runs[r][pos[r]], r);
            std::push_heap(heap.begin(), heap.end(), greater);
        }
    }
    out->count = (int64_t)m;
    acc.pairs = (int64_t)m;
    acc.ms_total = std::chrono::duration<double, std::milli>(
                       std::chrono::steady_clock::now() - t0).count();
    t_stats = acc;
}

int self_join_with(const pj_strings* S, int32_t tau, const pj_options* opt, pj_pairs* out,
                   const TuneParams* force)
{
    return guarded(out, [&] { join_impl(nullptr, S, tau, opt, out, true, force); });
}

// ------------------------------------------------------------------------------------------
// Plans: a self-join's launches captured once in a hipGraph and replayed
// ------------------------------------------------------------------------------------------

// Makes w the calling thread's workspace for the scope (a plan's buffers are its own).
struct WorkspaceScope {
    Workspace* saved;
    explicit WorkspaceScope(Workspace* w) : saved(t_ws) { t_ws = w; }
    ~WorkspaceScope() { t_ws = saved; }
};

struct TapeScope {
    ReadTape* saved;
    explicit TapeScope(ReadTape* t) : saved(t_tape) { t_tape = t; }
    ~TapeScope() { t_tape = saved; }
};

}  // namespace pj

struct pj_plan {
    pj::Workspace ws;                   // destroyed last: the graph refers to its buffers
    hipStream_t st = nullptr;           // the plan's stream (captured, replayed)
    hipEvent_t ev = nullptr;            // orders the plan's stream after the caller's
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    unsigned long long* d_sum = nullptr;
    pj_strings S{};
    int32_t tau = 0;
    pj_options opt{};                   // the caller's options, outputs in device memory
    std::string tune_cache;             // the caller's tune cache path (opt points here)
    hipStream_t user_st = nullptr;
    int64_t bytes_cap = 0;              // the bytes allocation of S, measured at plan time
    unsigned long long sum = 0;         // checksum of S at plan time
    int32_t* da = nullptr;              // the captured join's sorted pairs (in ws)
    int32_t* db = nullptr;
    uint64_t M = 0;
    pj_stats stats{};                   // counters of the recorded run
    ~pj_plan()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (d_sum) (void)hipFree(d_sum);
        if (ev) (void)hipEventDestroy(ev);
        if (st) (void)hipStreamDestroy(st);
    }
};

namespace pj {

static unsigned long long plan_checksum(pj_plan* p)
{
    hip_check(launch_set_checksum(p->S.offsets, p->S.n, p->S.bytes, p->bytes_cap, p->d_sum, p->st),
              "checksum");
    unsigned long long v = 0;
    hip_check(hipMemcpyAsync(&v, p->d_sum, sizeof v, hipMemcpyDeviceToHost, p->st), "checksum");
    hip_check(hipStreamSynchronize(p->st), "sync");
    return v;
}

static void plan_make(const pj_strings* S, int32_t tau, const pj_options* opt, pj_plan* p)
{
    if (!S) throw Error(PJ_EINVAL, "null pj_strings");
    if (!opt || !opt->inputs_on_device)
        throw Error(PJ_EINVAL, "a plan takes device strings (opt->inputs_on_device = 1)");
    check_tau(tau);
    p->S = *S;
    p->tau = tau;
    p->opt = *opt;
    p->opt.outputs_on_device = 1;
    if (opt->tune_cache) {
        p->tune_cache = opt->tune_cache;
        p->opt.tune_cache = p->tune_cache.c_str();
    }
    p->user_st = stream_of(opt);
    hip_check(hipStreamCreateWithFlags(&p->st, hipStreamNonBlocking), "hipStreamCreate");
    hip_check(hipEventCreateWithFlags(&p->ev, hipEventDisableTiming), "hipEventCreate");
    if (hipMalloc((void**)&p->d_sum, sizeof(unsigned long long)) != hipSuccess) {
        (void)hipGetLastError();
        p->d_sum = nullptr;
        throw Error(PJ_ENOMEM, "plan: checksum buffer");
    }
    hip_check(hipEventRecord(p->ev, p->user_st), "hipEventRecord");
    hip_check(hipStreamWaitEvent(p->st, p->ev, 0), "hipStreamWaitEvent");
    pj_options o = p->opt;
    o.hip_stream = p->st;
    WorkspaceScope ws(&p->ws);
    ReadTape tape;
    TapeScope ts(&tape);
    // 1. the self-join, recording what each phase reads back (it validates S)
    pj_pairs unused{};
    PlanOut rec;
    join_impl(nullptr, S, tau, &o, &unused, true, nullptr, 0, &rec);
    p->stats = t_stats;
    p->da = rec.a;
    p->db = rec.b;
    p->M = rec.M;
    // 2. the same launches captured: every read-back is served from the record
    tape.replay = true;
    tape.pos = 0;
    hip_check(hipStreamBeginCapture(p->st, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
    PlanOut cap;
    try {
        join_impl(nullptr, S, tau, &o, &unused, true, nullptr, 0, &cap);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(p->st, &g);
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        throw;
    }
    hip_check(hipStreamEndCapture(p->st, &p->graph), "hipStreamEndCapture");
    t_stats = p->stats;                 // the captured run added its (equal) counts again
    if (cap.a != rec.a || cap.b != rec.b || cap.M != rec.M || tape.pos != tape.bytes.size())
        throw Error(PJ_EDEVICE, "plan: the captured join differs from the recorded one");
    hip_check(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    // 3. the checksum of S the runs compare with (its bytes bounded by their allocation)
    p->bytes_cap = 0;
    if (S->bytes) {
        hipPointerAttribute_t attr{};
        void* base = nullptr;
        size_t size = 0;
        if (hipPointerGetAttributes(&attr, S->bytes) == hipSuccess &&
            hipMemGetAddressRange(&base, &size, const_cast<uint8_t*>(S->bytes)) == hipSuccess &&
            base)
            p->bytes_cap = (int64_t)(size - (size_t)((const uint8_t*)S->bytes - (const uint8_t*)base));
        (void)hipGetLastError();
    }
    p->sum = plan_checksum(p);
}

static void plan_run(pj_plan* p, pj_pairs* out)
{
    if (!p) throw Error(PJ_EINVAL, "null plan");
    if (!out) throw Error(PJ_EINVAL, "null output");
    zero_pairs(out);
    const auto t0 = std::chrono::steady_clock::now();
    hip_check(hipEventRecord(p->ev, p->user_st), "hipEventRecord");
    hip_check(hipStreamWaitEvent(p->st, p->ev, 0), "hipStreamWaitEvent");
    if (plan_checksum(p) != p->sum) {
        // S changed since the plan was made: the self-join of S as it is now
        join_impl(nullptr, &p->S, p->tau, &p->opt, out, true);
        t_stats.replayed = 0;
        return;
    }
    hip_check(hipGraphLaunch(p->exec, p->st), "hipGraphLaunch");
    const size_t bytes = sizeof(int32_t) * (size_t)std::max<uint64_t>(p->M, 1);
    void *pa = nullptr, *pb = nullptr;
    if (hipMalloc(&pa, bytes) != hipSuccess || hipMalloc(&pb, bytes) != hipSuccess) {
        (void)hipGetLastError();
        if (pa) (void)hipFree(pa);
        (void)hipStreamSynchronize(p->st);
        throw Error(PJ_ENOMEM, "output allocation failed");
    }
    out->on_device = 1;
    out->a = (int32_t*)pa;
    out->b = (int32_t*)pb;
    out->count = (int64_t)p->M;
    if (p->M) {
        hip_check(hipMemcpyAsync(pa, p->da, sizeof(int32_t) * p->M, hipMemcpyDeviceToDevice, p->st),
                  "out");
        hip_check(hipMemcpyAsync(pb, p->db, sizeof(int32_t) * p->M, hipMemcpyDeviceToDevice, p->st),
                  "out");
    }
    hip_check(hipStreamSynchronize(p->st), "sync");
    t_stats = p->stats;
    t_stats.replayed = 1;
    t_stats.ms_total = std::chrono::duration<double, std::milli>(
                           std::chrono::steady_clock::now() - t0).count();
}

}  // namespace pj

using namespace pj;

extern "C" {

int pj_self_join(const pj_strings* S, int32_t tau, const pj_options* opt, pj_pairs* out)
{
    return guarded(out, [&] { join_impl(nullptr, S, tau, opt, out, true); });
}

int pj_self_join_streamed(const pj_strings* S, int32_t tau, int64_t window_bytes,
                          const pj_options* opt, pj_pairs* out)
{
    return guarded(out, [&] {
        if (!S) throw Error(PJ_EINVAL, "null pj_strings");
        join_streamed(S, tau, window_bytes, opt, out);
    });
}

int pj_join(const pj_strings* R, const pj_strings* S, int32_t tau, const pj_options* opt,
            pj_pairs* out)
{
    return guarded(out, [&] {
        if (!R || !S) throw Error(PJ_EINVAL, "null pj_strings");
        join_impl(R, S, tau, opt, out, false);
    });
}

int pj_self_join_plan(const pj_strings* S, int32_t tau, const pj_options* opt, pj_plan** out)
{
    if (!out) {
        t_last_error = "null plan output";
        return PJ_EINVAL;
    }
    *out = nullptr;
    auto* p = new (std::nothrow) pj_plan();
    if (!p) {
        t_last_error = "host allocation failed";
        return PJ_ENOMEM;
    }
    const int rc = guarded(nullptr, [&] { plan_make(S, tau, opt, p); });
    if (rc != PJ_OK) {
        delete p;
        return rc;
    }
    *out = p;
    return PJ_OK;
}

int pj_plan_run(pj_plan* plan, pj_pairs* out)
{
    return guarded(out, [&] { plan_run(plan, out); });
}

void pj_plan_free(pj_plan* plan)
{
    if (plan) (void)hipStreamSynchronize(plan->st);
    delete plan;
}

void pj_pairs_free(pj_pairs* p)
{
    if (!p) return;
    if (p->on_device == 2) {
        if (p->a) (void)hipHostFree(p->a);
        if (p->b) (void)hipHostFree(p->b);
    } else if (p->on_device) {
        if (p->a) (void)hipFree(p->a);
        if (p->b) (void)hipFree(p->b);
    } else {
        free(p->a);
        free(p->b);
    }
    p->a = p->b = nullptr;
    p->count = 0;
    p->on_device = 0;
}

const char* pj_last_error(void) { return t_last_error.c_str(); }

int pj_last_stats(pj_stats* out)
{
    if (!out) return PJ_EINVAL;
    *out = t_last_ok_stats;
    return PJ_OK;
}

const char* pj_version(void) { return "passjoin-gfx950 0.1"; }

}  // extern "C"
