// pj_internal.h -- types and kernel launchers shared by the device and host parts of libpassjoin.
//
// Device data layout (all in HBM, built once per string set):
//   * length-sorted arena: strings reordered by (length, id) and stored back to back, each at a
//     16-byte aligned slot of stride(l) = round_up(l, 16) bytes, so the byte offset of the string at
//     sorted position g of length l is gbase[l] + (g - lenstart[l]) * stride(l) -- computed from
//     two per-length tables, never gathered per string;
//   * perm[g] = original id of sorted position g, slen[g] = its length;
//   * segment index for one tau: (key, g) entries sorted by key, key = group(l, i) << 40 | code,
//     group(l, i) = (l - (tau+1)) * (tau+1) + (i-1), code = the segment's bytes when it has at
//     most 5 (exact) or the top 40 bits of a mixed polynomial hash otherwise; equal keys form one
//     inverted list L_l^i(w) whose members are in ascending g (Sec. 3.2);
//   * bucket table: open-addressing hash table key -> (start, count) of the list.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pj {

constexpr int kLenMax = 2047;          // PJ_LEN_MAX
constexpr int kLenTab = kLenMax + 2;   // per-length tables are indexed 0 .. kLenMax + 1
constexpr int kTauMax = 63;            // PJ_TAU_MAX
constexpr int kHashBits = 40;          // hash bits kept in an index key
constexpr uint64_t kEmptyKey = ~0ull;  // keys use at most 57 bits, so this never collides

__host__ __device__ inline int64_t stride_of(int l) { return (int64_t)((l + 15) & ~15); }
constexpr int kBatchedRoundsMax = 16;   // rounds of 64 candidates per batched-verify wave chunk
constexpr int kInlineMaxLen = 64;       // longest string the list-segment kernel keeps in registers

// Length classes of the big lists in the batched path (strings of at most kLenClass0 bytes, at
// most kLenClass1, longer): each class is verified by the list-segment kernel whose lane slots
// its strings fit (a class split at 48 bytes measured no faster).  The small lists are split
// the same way, for the batched kernel's LDS-staged form.  Hit buckets: small lists by class
// and slot, then big lists by class and slot.
constexpr int kLenClasses = 3;
constexpr int kLenClass0 = 40, kLenClass1 = 64;
constexpr int kHitBuckets = 128 * kLenClasses;
__host__ __device__ inline int len_class(int l)
{
    return (l > kLenClass0 ? 1 : 0) + (l > kLenClass1 ? 1 : 0);
}
// longest indexed string of length class c in a set whose longest string has ymax bytes
inline int class_maxlen(int c, int ymax)
{
    const int cap = c == 0 ? kLenClass0 : c == 1 ? kLenClass1 : ymax;
    return ymax < cap ? ymax : cap;
}

// Symbol map of an indexed set: code[b] = 1 + rank of byte b among the bytes the set contains
// (0: absent), bits = bit length of the largest code.  A segment of at most exact_len =
// floor(kHashBits / bits) bytes is keyed by its packed codes (exact: no byte guard); a longer
// one by a hash of its bytes.  A probe segment with an absent byte packs a 0 code, which no
// indexed key has.
// Exact keys of at least this many code bits are also tested against the key filter: their
// (l, i) groups hold few of the possible codes, so most lookups miss.
constexpr int kFilterMinBits = 24;

struct SymMap {
    const uint16_t* code = nullptr;   // device [256]
    int bits = 9;
    int exact_len = kHashBits / 9;
};

// Length-sorted device arena of one string set.
struct DevSet {
    int64_t n = 0;
    int lmin = 0, lmax = -1;            // smallest / largest length present (lmax < lmin: empty)
    int64_t arena_bytes = 0;
    uint8_t* sarena = nullptr;          // padded, length-sorted bytes
    int32_t* perm = nullptr;            // [n] sorted position -> id
    uint16_t* slen = nullptr;           // [n] sorted position -> length
    int32_t* lenstart = nullptr;        // [kLenTab + 1] first sorted position of each length
    int64_t* gbase = nullptr;           // [kLenTab] byte base of each length group
    // host copies of the per-length tables
    int32_t h_lenstart[kLenTab + 1];
    int64_t h_gbase[kLenTab];
};

// Segment index of one set for one tau.
struct DevIndex {
    int tau = 0;
    SymMap sym;
    int64_t entries = 0;                // (string, slot) entries
    int64_t lists = 0;                  // distinct keys (inverted lists)
    uint64_t* keys = nullptr;           // [entries] sorted
    uint32_t* vals = nullptr;           // [entries] sorted position g of the string
    uint4* table = nullptr;             // [mask + 1] {key lo, key hi, start, count}
    uint64_t mask = 0;
    // membership filter of the keys, blocked by (l, i) group: group g = key >> 40 owns the
    // words [filter_dir[g], filter_dir[g + 1]) (a power of two of them), in which each of its
    // keys sets two bits; a clear bit proves a key absent without reading the table (long,
    // hashed segments and long exact codes rarely match).  nullptr when every segment is
    // keyed exactly in fewer than kFilterMinBits bits.
    uint32_t* filter = nullptr;
    uint32_t* filter_dir = nullptr;     // [(lmax - tau) * (tau + 1) + 1]
    // inline copies of the members' strings in index order (strings of at most kInlineMaxLen
    // bytes; nullptr otherwise): entry j of length l at inl + inl_base[l] + j * stride_of(l)
    uint8_t* inl = nullptr;
    int64_t* inl_base = nullptr;        // [kLenTab] device
    // shared-prefix verification (Sec. 5.3): every list's members in content order (sorted by
    // the first 8 bytes of the string, then g), at the list's positions; and the full length of
    // each list at its first entry (other entries unused).  nullptr when not built.
    uint32_t* svals = nullptr;          // [entries]
    uint32_t* runlen = nullptr;         // [entries]
};

// Per-threshold view of a multi-tau index (serving): the bucket table and list entries of the
// index built for tau, and the divisor for tau+1.  Indexed by tau.
struct IndexRef {
    const uint4* table;
    const uint32_t* vals;
    uint64_t mask;
    uint32_t div_m;     // ceil(2^21 / (tau + 1)), see Div
    uint32_t present;   // 1 if an index for this tau exists
    const uint32_t* filter;       // DevIndex::filter / filter_dir
    const uint32_t* filter_dir;
};

// One selected substring that found a non-empty list: candidates (vals[start + m], x, i, p).
struct Hit {
    uint32_t gx;      // sorted position of the probe string in the probe set
    uint32_t start;   // first entry of the list in DevIndex::vals
    uint32_t count;   // list members that are candidates (after the visiting-order filter)
    uint32_t meta;    // (p - 1) | (i - 1) << 11 | l << 17
};

struct ProbeParams {
    // probe side
    const uint8_t* x_arena; const uint16_t* x_slen; const int32_t* x_lenstart;
    const int64_t* x_gbase;
    uint32_t g_begin;           // first probe position
    uint64_t threads;           // probe positions * nl * (tau+1)
    int nl;                     // lengths probed per string: tau+1 (self) or 2tau+1 (two sets)
    int self;                   // 1: self-join (l in [n-tau, n], y before x when l == n)
    const int32_t* q_tau;       // per-probe tau by sorted position (mixed-tau batch) or nullptr
    const IndexRef* refs;       // [kTauMax + 1] when q_tau is set
    // index side
    const int32_t* y_lenstart;  // to know which lengths are present
    const uint64_t* keys; const uint32_t* vals; const uint4* table; uint64_t mask;
    const uint32_t* filter; const uint32_t* filter_dir;   // key filter (nullptr: none)
    int tau;                    // uniform tau, or the largest tau of a mixed batch
    int ymin, ymax;             // indexed lengths present
    // output
    Hit* hits; uint64_t hit_cap;
    unsigned long long* counters;   // [0] hits, [1] candidates, [2] selected
    // device-resident probe count (captured batches): threads = *nx_dev * nl * (tau + 1)
    const uint32_t* nx_dev;
    SymMap sym;                 // the indexed set's symbol map (keys)
    int selection;              // PJ_SELECT_* window of start positions
    // the (length, slot) pairs of a probe string in the order the threads take them: a
    // permutation of 0 .. nl * (tau+1) - 1 grouped by window size, so that a wave's lanes walk
    // windows of one size (launch_probe_order); nullptr: natural order
    const uint16_t* order;
    // 1: threads pair-major over blocks of 64 probe strings (threads = nx rounded up to 64,
    // times nl * (tau+1)); not with q_tau or nx_dev
    int xmajor;
    uint32_t nx;                // probe strings (xmajor)
};

struct VerifyParams {
    const uint8_t* x_arena; const uint16_t* x_slen; const int32_t* x_lenstart;
    const int64_t* x_gbase;
    const uint8_t* y_arena; const int32_t* y_lenstart; const int64_t* y_gbase;
    const uint32_t* vals;
    // inline member strings of the index (DevIndex::inl / inl_base), or nullptr
    const uint8_t* y_inl; const int64_t* y_inl_base;
    const Hit* hits; const unsigned long long* prefix;   // [nhits + 1] exclusive prefix of counts
    uint64_t nhits; uint64_t ncand;
    int tau;                                              // uniform tau or the batch's largest
    int y_maxlen;                                         // longest indexed string
    const int32_t* q_tau;                                 // per-probe tau or nullptr
    const IndexRef* refs;                                 // [kTauMax + 1] when q_tau is set
    uint64_t* out; uint64_t out_cap;                      // accepted (gx << 32 | gy)
    unsigned long long* counters;    // [3] accepted, [4] cells, [5] guard misses, [7] list-segment cells
    // device-resident sizes (captured batches): [0] hits, [1] candidates, [2] wave chunks;
    // when set they replace nhits, ncand and the launch's chunk count
    const unsigned long long* dev_counts;
    int exact_len;              // segments up to this length have exact keys (no byte guard)
    int wave_rounds;            // batched verification: rounds of 64 candidates per wave chunk
    // shared-prefix verification: content-ordered lists and list lengths (DevIndex::svals,
    // runlen), and whether this is a self-join (lists of the probe's own length are then
    // filtered to the members visited before it, member by member)
    const uint32_t* svals;
    const uint32_t* runlen;
    int self;
};
// counters [8] rows and [9] cells that shared-prefix verification took from an earlier
// member's DP instead of computing them
constexpr int kJoinCounters = 12;

// ---- launchers (pj_device.hip) ----
hipError_t launch_length_hist(const int32_t* offs, int64_t n, int32_t* lcount, int32_t* err,
                              hipStream_t s);
hipError_t launch_iota_len_keys(const int32_t* offs, int64_t n, uint32_t* keys, uint32_t* vals,
                                hipStream_t s);
hipError_t launch_pack_arena(const uint8_t* bytes, const int32_t* offs, const int32_t* perm,
                             int64_t n, const int32_t* lenstart, const int64_t* gbase,
                             uint8_t* sarena, uint16_t* slen, int lmax, hipStream_t s);
// bytes present in a set's strings: bitmap (8 u32, zeroed by the caller)
hipError_t launch_byte_presence(const DevSet& S, uint32_t* bitmap, hipStream_t s);
hipError_t launch_emit_segments(const DevSet& S, int tau, const int64_t* ebase_dev,
                                int64_t g_first, int64_t g_count, const SymMap& sym,
                                uint64_t* keys, uint32_t* vals, hipStream_t s);
hipError_t launch_gather_inline(const DevSet& S, const uint64_t* keys, const uint32_t* vals,
                                int64_t E, int tau, const int64_t* inl_base, uint8_t* inl,
                                hipStream_t s);
hipError_t launch_mark_heads(const uint64_t* keys, int64_t E, uint32_t* flags, hipStream_t s);
hipError_t launch_scatter_runstart(const uint32_t* flags, const uint32_t* runid, int64_t E,
                                   uint32_t* runstart, hipStream_t s);
hipError_t launch_clear_table(uint4* table, uint64_t slots, hipStream_t s);
hipError_t launch_insert_runs(const uint64_t* keys, const uint32_t* runstart, uint32_t nruns,
                              uint32_t E, uint4* table, uint64_t mask, hipStream_t s);
// builds the (l, i)-blocked key filter of ngroups groups: filter_dir[0 .. ngroups] and the bits
// of every list's key in filter (at most nruns + 2 * ngroups words, zeroed by the caller);
// gfirst, gend, words: ngroups-entry scratch (gfirst and gend zeroed by the caller)
hipError_t launch_filter_build(const uint64_t* keys, const uint32_t* runstart, uint32_t nruns,
                               uint32_t ngroups, uint32_t* gfirst, uint32_t* gend, uint32_t* words,
                               void* scan_tmp, size_t scan_bytes, uint32_t* filter_dir,
                               uint32_t* filter, hipStream_t s);hipError_t launch_probe(const ProbeParams& P, int max_blocks, hipStream_t s);
// order[0 .. nl * (tau+1)): the (length, slot) pairs r = dl * (tau+1) + (i-1) of a probe string
// by decreasing multi-match window size (any order within a size)
hipError_t launch_probe_order(int tau, int nl, int self, uint16_t* order, hipStream_t s);
hipError_t launch_hit_counts(const Hit* hits, uint64_t nh, uint32_t* counts, hipStream_t s);
hipError_t launch_verify(const VerifyParams& V, int grid, hipStream_t s);
// batched path: bucket the hits (small lists, then big ones, each by length class and then
// slot) into out, bucket regions in order; bb: kHitBuckets * slot_bucket_grid(nh_cap) u32,
// bb_off: one more (bb_off[64 * c * grid] = first hit of the small lists of length class c,
// bb_off[64 * (kLenClasses + c) * grid] that of the big lists), scan_tmp:
// scan_tmp_bytes(kHitBuckets * grid).  Then verify with per-wave chunks
// (first: batched_chunks(ncand) u32 of scratch)
unsigned slot_bucket_grid(uint64_t nh_cap);
hipError_t launch_slot_bucket(const Hit* hits, const unsigned long long* nh_dev, uint64_t nh_cap,
                              uint32_t big, uint32_t* bb, uint32_t* bb_off, void* scan_tmp,
                              size_t scan_bytes, Hit* out, hipStream_t s);
// list-segment verification of the lists with >= big candidates (hits big[0 .. nbig), segp =
// exclusive scan of ceil(count / seg_members), nseg segments, `chunk` segments per wave chunk; first:
// seg_chunks(nseg, chunk) u32 of scratch)
// list segments of `members` candidates each (seg_members: what k_verify_segs expects)
int seg_members(int y_maxlen, int tau, int lane_cands);
hipError_t launch_seg_counts(const Hit* big, uint64_t nbig, int members, uint32_t* segs,
                             hipStream_t s);
hipError_t launch_verify_segs(const VerifyParams& V, const Hit* big, const uint32_t* segp,
                              uint64_t nbig, uint64_t nseg, uint32_t* first, int chunk,
                              int lane_cands, int grid, hipStream_t s);
uint64_t seg_chunks(uint64_t nseg, int chunk);
// shared-prefix verification (Sec. 5.3) of the big lists: a lane takes a chain of up to
// kChainMembers consecutive members of a content-ordered list.  chains: per big hit, its chain
// count (u32, launch_chain_counts); cprefix: exclusive u64 scan of it (nbig + 1); first:
// (nchains + 63) / 64 u32 of scratch.  Supports tau + 1 <= kShareMaxW (the caller checks).
constexpr int kChainMembers = 16;
constexpr int kShareMaxW = 9;
hipError_t launch_chain_counts(const Hit* big, uint64_t nbig, const uint16_t* x_slen,
                               const uint32_t* runlen, int self, uint32_t* chains, hipStream_t s);
hipError_t launch_verify_chains(const VerifyParams& V, const Hit* big,
                                const unsigned long long* cprefix, uint64_t nbig,
                                uint64_t nchains, uint32_t* first, int grid, hipStream_t s);
// content order of the entries: (key, first 8 bytes of the string, g) -> svals; list lengths at
// each list's first entry -> runlen
hipError_t launch_prefix8_keys(const DevSet& S, const uint32_t* vals, int64_t E, uint64_t* keys,
                               uint32_t* idx, hipStream_t s);
hipError_t launch_gather_keys(const uint64_t* keys, const uint32_t* idx, int64_t E,
                              uint64_t* out, hipStream_t s);
hipError_t launch_gather_vals(const uint32_t* vals, const uint32_t* idx, int64_t E, uint32_t* out,
                              hipStream_t s);
hipError_t launch_run_lengths(const uint32_t* runstart, uint32_t nruns, uint32_t E,
                              uint32_t* runlen, hipStream_t s);
hipError_t launch_verify_batched(const VerifyParams& V, uint32_t* first, int grid, hipStream_t s);
// long-string verification of the small-list hits (V.hits[0 .. V.nhits), ncand candidates,
// uniform tau + 1 <= kLongMaxW, no per-query tau) by row blocks: candidates in slot order, passes
// of at most 64 rows per task, unfinished tasks compacted into the next pass's queue, left parts
// before right parts.  max_rows bounds a part's rows (the longest string).  grid: blocks of one
// wave.  scratch: long_scratch_bytes(ncand) bytes.
constexpr int kLongMinLen = 128;
constexpr int kLongMaxW = 33;
size_t long_scratch_bytes(uint64_t ncand);
hipError_t launch_verify_long(const VerifyParams& V, uint64_t ncand, int max_rows, void* scratch,
                              int grid, hipStream_t s);
// wave chunks of 64 * rounds candidates (rounds in [1, kBatchedRoundsMax])
uint64_t batched_chunks(uint64_t ncand, int rounds);
// A captured query batch: every size is read from device memory, so one instantiated graph
// serves every batch.  counters: [0] hits [1] candidates [2] selected [3] accepted [4] cells
// [5] guard misses [6] side pairs [7] unused; bcounts: [0] hits [1] candidates [2] wave chunks
// [3] overflow flags (1 hits, 2 chunks, 4 accepted, 8 sort); out: the batch's sorted distinct
// (query id << 32 | indexed id) pairs, out_n their number.
struct GraphBatch {
    ProbeParams probe;          // nx_dev set; hits/hit_cap/counters set
    int probe_grid;
    VerifyParams verify;        // dev_counts = bcounts; prefix/out/out_cap/counters set
    int verify_grid;
    unsigned long long* bcounts;
    uint32_t* first; uint64_t chunk_cap;
    // short side path (indexed strings shorter than tau_max + 1), y_count == 0: none
    uint32_t y_first, y_count;
    const uint8_t* y_arena; const uint16_t* y_slen; const int32_t* y_lenstart;
    const int64_t* y_gbase;
    // output
    const int32_t* xperm; const int32_t* yperm;
    uint64_t* out; uint32_t* out_n;
};
constexpr int kGraphSortCap = 8192;     // accepted pairs a captured batch can sort
hipError_t launch_graph_batch(const GraphBatch& G, hipStream_t s);
hipError_t launch_short_path(const DevSet& P, const DevSet& Y, int tau, int self,
                             const int32_t* q_tau, uint64_t* out, uint64_t out_cap,
                             unsigned long long* counters, hipStream_t s);
hipError_t launch_pairs_to_keys(const uint64_t* acc, uint64_t m, const int32_t* xperm,
                                const int32_t* yperm, int self, int bbits, uint64_t* keys,
                                hipStream_t s);
hipError_t launch_unique_flags(const uint64_t* keys, uint64_t m, uint32_t* flags, hipStream_t s);
hipError_t launch_compact_pairs(const uint64_t* keys, const uint32_t* flags, const uint32_t* pos,
                                uint64_t m, int bbits, int32_t* a, int32_t* b, hipStream_t s);

// streamed self-joins: window pairs -> global keys (halo-only pairs as a counted sentinel that
// sorts last); sorted keys -> pair arrays
hipError_t launch_window_keys(const int32_t* a, const int32_t* b, uint64_t m, const int32_t* ids,
                              const int32_t* offs, int min_len, int bbits, uint64_t* keys,
                              unsigned long long* dropped, hipStream_t s);
hipError_t launch_split_keys(const uint64_t* keys, uint64_t m, int bbits, int32_t* a, int32_t* b,
                             hipStream_t s);
// p[0 .. n) = v (a kernel: capturable in a graph, unlike a memset node)
hipError_t launch_fill_words(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
// *sum = checksum of the device string set (offsets[0..n], bytes[0..min(offsets[n], cap)))
hipError_t launch_set_checksum(const int32_t* offs, int64_t n, const uint8_t* bytes, int64_t cap,
                               unsigned long long* sum, hipStream_t s);
hipError_t launch_gather_i32(const int32_t* in, const int32_t* perm, int64_t n, int32_t* out,
                             hipStream_t s);

// Exclusive scans; out has n + 1 entries (out[n] = total).
hipError_t scan_u32_to_u32(const uint32_t* in, uint32_t* out, uint64_t n, void* tmp,
                           size_t tmp_bytes, hipStream_t s);
hipError_t scan_u32_to_u64(const uint32_t* in, unsigned long long* out, uint64_t n, void* tmp,
                           size_t tmp_bytes, hipStream_t s);
size_t scan_tmp_bytes(uint64_t n);

// Stable LSD radix sort by the low `bits` bits of the keys, 8 bits per pass.  Buffers ping-pong;
// returns in *result_in_alt whether the sorted data ended in the alternate buffers.
hipError_t radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                          uint32_t* vals_alt, uint64_t n, int bits, void* tmp, size_t tmp_bytes,
                          bool* result_in_alt, hipStream_t s);
hipError_t radix_sort_u32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                          uint32_t* vals_alt, uint64_t n, int bits, void* tmp, size_t tmp_bytes,
                          bool* result_in_alt, hipStream_t s);
size_t radix_tmp_bytes(uint64_t n);

}  // namespace pj
