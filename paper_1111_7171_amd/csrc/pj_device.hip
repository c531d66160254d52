// pj_device.hip -- gfx950 kernels of libpassjoin (plain one-kernel-per-phase path).
//
// Everything here is integer work on wave64: no MFMA (nothing is a dense contraction).  The
// phases are HBM/L2-bound streaming (arena packing, index build, radix sort), random-access
// lookups (probe) and integer-VALU dynamic programming (verification).
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "pj_internal.h"
#include "pj_device_common.h"

namespace pj {

// ------------------------------------------------------------------------------------------
// Wave / block primitives (wave64, 256-thread blocks)
// ------------------------------------------------------------------------------------------

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

template <typename T>
__device__ inline T wave_incl_scan(T v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

template <typename T>
__device__ inline T wave_sum(T v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Exclusive scan over the 256 threads of a block; *total receives the block sum.
template <typename T>
__device__ inline T block_excl_scan(T v, T* s_wave, T* total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T inc = wave_incl_scan(v);
    if (lane == 63) s_wave[w] = inc;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
        T s = s_wave[k];
        if (k < w) off += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__device__ inline uint64_t lanemask_lt() { return (1ull << (threadIdx.x & 63)) - 1ull; }

// Wave-private append buffer in LDS: lanes push items without touching global atomics; the
// wave reserves space in the global output with one atomic per flush (a single-address device
// atomic is serialised across all XCDs, so one per item would throttle the kernel).  `buf`
// is this wave's region of CAP items; `fill` is wave-uniform.
template <typename T, int CAP>
struct WaveAppender {
    static_assert(CAP >= 64, "a push adds up to 64 items after at most one flush");
    T* buf;
    int fill;

    __device__ inline void flush(T* out, uint64_t cap, unsigned long long* counter)
    {
        if (fill == 0) return;
        const int lane = threadIdx.x & 63;
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(counter, (unsigned long long)fill);
        base = __shfl(base, 0, 64);
        for (int k = lane; k < fill; k += 64)
            if (base + (uint64_t)k < cap) out[base + k] = buf[k];
        fill = 0;
    }

    __device__ inline void push(bool flag, const T& item, T* out, uint64_t cap,
                                unsigned long long* counter)
    {
        const uint64_t m = __ballot(flag);
        if (m == 0) return;
        const int k = __popcll(m);
        if (fill + k > CAP) flush(out, cap, counter);
        if (flag) buf[fill + __popcll(m & lanemask_lt())] = item;
        fill += k;
    }
};

constexpr int kAppendCap = 256;

// ------------------------------------------------------------------------------------------
// Device-wide exclusive scan (reduce -> scan partials -> apply), 2048 elements per block
// ------------------------------------------------------------------------------------------

constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const TI* __restrict__ in, uint64_t n,
                                                        TO* __restrict__ partial)
{
    __shared__ TO s_wave[kWaves];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    TO sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) sum += (TO)in[base + k];
    TO tot;
    block_excl_scan<TO>(sum, s_wave, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

template <typename TO>
__global__ __launch_bounds__(kBlock) void k_scan_partials(TO* __restrict__ partial, uint64_t nb)
{
    __shared__ TO s_wave[kWaves];
    __shared__ TO s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (uint64_t c = 0; c < nb; c += kBlock) {
        uint64_t k = c + threadIdx.x;
        TO v = (k < nb) ? partial[k] : 0;
        TO tot;
        TO ex = block_excl_scan<TO>(v, s_wave, &tot);
        TO carry = s_carry;
        if (k < nb) partial[k] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = carry + tot;
        __syncthreads();
    }
}

template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void k_scan_apply(const TI* __restrict__ in, TO* __restrict__ out,
                                                       uint64_t n, const TO* __restrict__ partial)
{
    __shared__ TO s_wave[kWaves];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    TO v[kScanItems];
    TO sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? (TO)in[base + k] : 0;
        sum += v[k];
    }
    TO tot;
    TO run = block_excl_scan<TO>(sum, s_wave, &tot) + partial[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    // the thread holding the last element writes the total
    if (n > 0 && base <= n - 1 && n - 1 < base + kScanItems) out[n] = run;
}

size_t scan_tmp_bytes(uint64_t n)
{
    uint64_t nb = (n + kScanTile - 1) / kScanTile;
    return (size_t)(nb + 1) * sizeof(unsigned long long);
}

template <typename TO>
__global__ void k_zero_one(TO* __restrict__ out)
{
    if (threadIdx.x == 0) *out = 0;
}

template <typename TI, typename TO>
static hipError_t scan_impl(const TI* in, TO* out, uint64_t n, void* tmp, size_t tmp_bytes,
                            hipStream_t s)
{
    if (n == 0) {
        // a kernel, not a memset, so that the call can be captured in a graph
        hipLaunchKernelGGL((k_zero_one<TO>), dim3(1), dim3(64), 0, s, out);
        return hipGetLastError();
    }
    uint64_t nb = (n + kScanTile - 1) / kScanTile;
    if (tmp_bytes < (nb + 1) * sizeof(TO)) return hipErrorInvalidValue;
    TO* partial = (TO*)tmp;
    hipLaunchKernelGGL((k_scan_reduce<TI, TO>), dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, partial);
    hipLaunchKernelGGL((k_scan_partials<TO>), dim3(1), dim3(kBlock), 0, s, partial, nb);
    hipLaunchKernelGGL((k_scan_apply<TI, TO>), dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, n,
                       (const TO*)partial);
    return hipGetLastError();
}

hipError_t scan_u32_to_u32(const uint32_t* in, uint32_t* out, uint64_t n, void* tmp,
                           size_t tmp_bytes, hipStream_t s)
{
    return scan_impl<uint32_t, uint32_t>(in, out, n, tmp, tmp_bytes, s);
}

hipError_t scan_u32_to_u64(const uint32_t* in, unsigned long long* out, uint64_t n, void* tmp,
                           size_t tmp_bytes, hipStream_t s)
{
    return scan_impl<uint32_t, unsigned long long>(in, out, n, tmp, tmp_bytes, s);
}

// ------------------------------------------------------------------------------------------
// Stable LSD radix sort, 8-bit digits.  A block owns a tile of 16 rounds x 256 keys; within a
// round, keys with equal digits are ranked by wave ballots (8 ballots per key find its peers)
// and across waves/rounds by LDS counters, so every pass is stable.
// ------------------------------------------------------------------------------------------

constexpr int kRadixRounds = 16;
constexpr int kRadixTile = kBlock * kRadixRounds;

template <typename K>
__global__ __launch_bounds__(kBlock) void k_radix_hist(const K* __restrict__ keys, uint64_t n,
                                                       int shift, uint32_t* __restrict__ hist,
                                                       uint32_t nblocks)
{
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kRadixTile;
#pragma unroll 4
    for (int r = 0; r < kRadixRounds; ++r) {
        uint64_t idx = base + (uint64_t)r * kBlock + threadIdx.x;
        if (idx < n) atomicAdd(&cnt[(uint32_t)(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

template <typename K>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const K* __restrict__ keys,
                                                          const uint32_t* __restrict__ vals,
                                                          uint64_t n, int shift,
                                                          const uint32_t* __restrict__ offsets,
                                                          uint32_t nblocks,
                                                          K* __restrict__ keys_out,
                                                          uint32_t* __restrict__ vals_out)
{
    __shared__ uint32_t cnt[256];
    __shared__ uint32_t wcnt[kWaves][256];
    const int w = threadIdx.x >> 6;
    cnt[threadIdx.x] = offsets[(uint64_t)threadIdx.x * nblocks + blockIdx.x];
#pragma unroll
    for (int k = 0; k < kWaves; ++k) wcnt[k][threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kRadixTile;
    for (int r = 0; r < kRadixRounds; ++r) {
        uint64_t idx = base + (uint64_t)r * kBlock + threadIdx.x;
        bool valid = idx < n;
        K key = valid ? keys[idx] : (K)0;
        uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            uint64_t bb = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? bb : ~bb;
        }
        uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt());
        bool leader = valid && ((peers & lanemask_lt()) == 0);
        if (leader) wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = cnt[d] + rank;
            for (int k = 0; k < w; ++k) pos += wcnt[k][d];
            keys_out[pos] = key;
            if (vals) vals_out[pos] = vals[idx];
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int k = 0; k < kWaves; ++k) {
            add += wcnt[k][threadIdx.x];
            wcnt[k][threadIdx.x] = 0;
        }
        cnt[threadIdx.x] += add;
        __syncthreads();
    }
}

size_t radix_tmp_bytes(uint64_t n)
{
    uint64_t nb = (n + kRadixTile - 1) / kRadixTile;
    uint64_t h = 256 * nb;
    // histogram + its scan + scan partials
    return (size_t)(2 * (h + 1)) * sizeof(uint32_t) + scan_tmp_bytes(h) + 256;
}

template <typename K>
static hipError_t radix_impl(K* keys, uint32_t* vals, K* keys_alt, uint32_t* vals_alt,
                             uint64_t n, int bits, void* tmp, size_t tmp_bytes, bool* in_alt,
                             hipStream_t s)
{
    *in_alt = false;
    if (n <= 1 || bits <= 0) return hipSuccess;
    uint64_t nb = (n + kRadixTile - 1) / kRadixTile;
    uint64_t h = 256 * nb;
    if (tmp_bytes < radix_tmp_bytes(n)) return hipErrorInvalidValue;
    uint32_t* hist = (uint32_t*)tmp;
    uint32_t* offs = hist + (h + 1);
    void* stmp = (void*)(offs + (h + 1));
    size_t stmp_bytes = tmp_bytes - (size_t)(2 * (h + 1)) * sizeof(uint32_t);
    K* kin = keys; uint32_t* vin = vals;
    K* kout = keys_alt; uint32_t* vout = vals_alt;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL((k_radix_hist<K>), dim3((unsigned)nb), dim3(kBlock), 0, s, kin, n,
                           shift, hist, (uint32_t)nb);
        hipError_t e = scan_u32_to_u32(hist, offs, h, stmp, stmp_bytes, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_radix_scatter<K>), dim3((unsigned)nb), dim3(kBlock), 0, s, kin,
                           vin, n, shift, offs, (uint32_t)nb, kout, vout);
        K* tk = kin; kin = kout; kout = tk;
        uint32_t* tv = vin; vin = vout; vout = tv;
        *in_alt = !*in_alt;
    }
    return hipGetLastError();
}

hipError_t radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                          uint64_t n, int bits, void* tmp, size_t tmp_bytes, bool* in_alt,
                          hipStream_t s)
{
    return radix_impl<uint64_t>(keys, vals, keys_alt, vals_alt, n, bits, tmp, tmp_bytes, in_alt, s);
}

hipError_t radix_sort_u32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                          uint64_t n, int bits, void* tmp, size_t tmp_bytes, bool* in_alt,
                          hipStream_t s)
{
    return radix_impl<uint32_t>(keys, vals, keys_alt, vals_alt, n, bits, tmp, tmp_bytes, in_alt, s);
}

// ------------------------------------------------------------------------------------------
// String arena: length histogram + validation, (length, id) keys, packing
// ------------------------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_length_hist(const int32_t* __restrict__ offs,
                                                        int64_t n, int32_t* __restrict__ lcount,
                                                        int32_t* __restrict__ err)
{
    __shared__ int32_t h[kLenTab];
    for (int k = threadIdx.x; k < kLenTab; k += kBlock) h[k] = 0;
    __syncthreads();
    int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int32_t e = 0;
    if (id < n) {
        int32_t a = offs[id], b = offs[id + 1];
        int32_t l = b - a;
        if (id == 0 && a != 0) e |= 1;
        if (l < 0) e |= 2;
        else if (l > kLenMax) e |= 4;
        else atomicAdd(&h[l], 1);
    }
    if (e) atomicOr(err, e);
    __syncthreads();
    for (int k = threadIdx.x; k < kLenTab; k += kBlock)
        if (h[k]) atomicAdd(&lcount[k], h[k]);
}

__global__ __launch_bounds__(kBlock) void k_len_keys(const int32_t* __restrict__ offs, int64_t n,
                                                     uint32_t* __restrict__ keys,
                                                     uint32_t* __restrict__ vals)
{
    int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (id < n) {
        keys[id] = (uint32_t)(offs[id + 1] - offs[id]);
        vals[id] = (uint32_t)id;
    }
}

// One wave per sorted position: copies the string into its padded slot of the sorted arena.
// 2^lps_shift lanes per string, at least a quarter of the widest slot (16 when every slot is at
// most 64 bytes: a wave packs 4 strings at once, so their dependent loads of position, offsets
// and group base overlap; 32 up to 128 bytes; else 64)
__global__ __launch_bounds__(kBlock) void k_pack_arena(const uint8_t* __restrict__ bytes,
                                                       const int32_t* __restrict__ offs,
                                                       const int32_t* __restrict__ perm, int64_t n,
                                                       const int32_t* __restrict__ lenstart,
                                                       const int64_t* __restrict__ gbase,
                                                       uint8_t* __restrict__ sarena,
                                                       uint16_t* __restrict__ slen, int lps_shift)
{
    const int lps = 1 << lps_shift;
    const int sub = threadIdx.x & (lps - 1);
    int64_t g = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> lps_shift;
    const int64_t gstep = ((int64_t)gridDim.x * kBlock) >> lps_shift;
    for (; g < n; g += gstep) {
        int32_t id = perm[g];
        int32_t a = offs[id];
        int32_t l = offs[id + 1] - a;
        uint8_t* dst = sarena + gbase[l] + (g - lenstart[l]) * stride_of(l);
        int32_t st = (int32_t)stride_of(l);
        for (int32_t k = sub; k < st; k += lps) dst[k] = (k < l) ? bytes[a + k] : (uint8_t)0;
        if (sub == 0) slen[g] = (uint16_t)l;
    }
}

// ------------------------------------------------------------------------------------------
// Segment index
// ------------------------------------------------------------------------------------------

// One thread per (indexed string, slot): emits (key, g) at a position grouped by (l, i) and
// ordered by g inside the group, so a stable sort by key keeps lists in ascending g.
// bitmap of the bytes present in the strings of a set (one thread per string)
// Byte values present in the arena: one thread per 16-byte chunk of the length-sorted arena
// (coalesced wide loads); the chunk's length group l is found by binary search over the
// groups' byte ranges [gbase[l], gbase[l + 1]) (an empty group's range is empty), and only the
// bytes inside a string count, not the padding of its slot.
__global__ __launch_bounds__(kBlock) void k_byte_presence(const uint8_t* __restrict__ sarena,
                                                          const int64_t* __restrict__ gbase,
                                                          int64_t total,
                                                          uint32_t* __restrict__ bitmap)
{
    __shared__ uint32_t bm[8];
    if (threadIdx.x < 8) bm[threadIdx.x] = 0;
    __syncthreads();
    const int64_t nchunks = total >> 4;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nchunks;
         c += (int64_t)gridDim.x * kBlock) {
        const int64_t o = c << 4;
        int lo = 0, hi = kLenTab - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            const int64_t end = mid + 1 < kLenTab ? gbase[mid + 1] : total;
            if (end > o) hi = mid; else lo = mid + 1;
        }
        const int l = lo;
        const int within = (int)((o - gbase[l]) % stride_of(l));
        const int valid = l - within < 16 ? l - within : 16;
        const uint4 v = *reinterpret_cast<const uint4*>(sarena + o);
        const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (k < valid) {
                const uint32_t byte = (wd[k >> 2] >> ((k & 3) * 8)) & 255u;
                const uint32_t bit = 1u << (byte & 31u);
                if (!(bm[byte >> 5] & bit)) atomicOr(&bm[byte >> 5], bit);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < 8 && bm[threadIdx.x]) atomicOr(&bitmap[threadIdx.x], bm[threadIdx.x]);
}

__global__ __launch_bounds__(kBlock) void k_emit_segments(const uint8_t* __restrict__ sarena,
                                                          const uint16_t* __restrict__ slen,
                                                          const int32_t* __restrict__ lenstart,
                                                          const int64_t* __restrict__ gbase,
                                                          const int64_t* __restrict__ ebase,
                                                          int tau, int64_t g_first,
                                                          int64_t g_count, Div div, SymMap sym,
                                                          uint64_t* __restrict__ keys,
                                                          uint32_t* __restrict__ vals)
{
    __shared__ uint16_t s_sym[256];
    s_sym[threadIdx.x] = sym.code[threadIdx.x];
    __syncthreads();
    const int T1 = tau + 1;
    int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= g_count * T1) return;
    int64_t g = g_first + t / T1;
    int i = (int)(t % T1) + 1;
    int l = slen[g];
    Seg sg = partition_seg(l, i, tau, div);
    const uint8_t* s = sarena + gbase[l] + (g - lenstart[l]) * stride_of(l);
    uint64_t h = seg_code(s + sg.p - 1, sg.len, s_sym, sym.bits, sym.exact_len);
    int64_t nl = lenstart[l + 1] - lenstart[l];
    int64_t e = ebase[l] + (int64_t)(i - 1) * nl + (g - lenstart[l]);
    keys[e] = make_key(l, i, tau, sg.len, h, sym.exact_len);
    vals[e] = (uint32_t)g;
}

__global__ __launch_bounds__(kBlock) void k_mark_heads(const uint64_t* __restrict__ keys, int64_t E,
                                                       uint32_t* __restrict__ flags)
{
    int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < E) flags[e] = (e == 0 || keys[e] != keys[e - 1]) ? 1u : 0u;
}

// Inline copies of the list members' strings: entry j of the sorted index (length l, read from
// its key's group) gets the bytes of string vals[j], in a slot of stride_of(l) bytes at
// inl + inl_base[l] + j * stride_of(l).  Entries of one length are contiguous in the sorted
// index (the group is the key's top field), so the copies of one list are contiguous too.
__global__ __launch_bounds__(kBlock) void k_gather_inline(
    const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals, int64_t E, int tau,
    const uint8_t* __restrict__ sarena, const int32_t* __restrict__ lenstart,
    const int64_t* __restrict__ gbase, const int64_t* __restrict__ inl_base,
    uint8_t* __restrict__ inl)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= E) return;
    const int T1 = tau + 1;
    const int l = (int)((keys[j] >> kHashBits) / (uint64_t)T1) + T1;
    const uint32_t g = vals[j];
    const int64_t st = stride_of(l);
    const uint4* src = reinterpret_cast<const uint4*>(sarena + gbase[l] +
                                                      (int64_t)(g - (uint32_t)lenstart[l]) * st);
    uint4* dst = reinterpret_cast<uint4*>(inl + inl_base[l] + j * st);
    for (int q = 0; q < (int)(st >> 4); ++q) dst[q] = src[q];
}

__global__ __launch_bounds__(kBlock) void k_clear_table(uint4* __restrict__ table, uint64_t slots)
{
    uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < slots) table[k] = make_uint4(0xffffffffu, 0xffffffffu, 0u, 0u);
}

// runstart[r] = first entry of list r (runid[e] = number of list heads before e).
__global__ __launch_bounds__(kBlock) void k_scatter_runstart(const uint32_t* __restrict__ flags,
                                                             const uint32_t* __restrict__ runid,
                                                             int64_t E,
                                                             uint32_t* __restrict__ runstart)
{
    int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < E && flags[e]) runstart[runid[e]] = (uint32_t)e;
}

// One thread per list: inserts key -> (start, count) into the table by linear probing.
__global__ __launch_bounds__(kBlock) void k_insert_runs(const uint64_t* __restrict__ keys,
                                                        const uint32_t* __restrict__ runstart,
                                                        uint32_t nruns, uint32_t E,
                                                        uint4* __restrict__ table, uint64_t mask)
{
    uint32_t r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= nruns) return;
    uint32_t start = runstart[r];
    uint32_t end = (r + 1 < nruns) ? runstart[r + 1] : E;
    uint64_t key = keys[start];
    uint64_t slot = table_slot(key) & mask;
    while (true) {
        unsigned long long* kp = reinterpret_cast<unsigned long long*>(&table[slot]);
        unsigned long long prev = atomicCAS(kp, (unsigned long long)kEmptyKey,
                                            (unsigned long long)key);
        if (prev == (unsigned long long)kEmptyKey) {
            table[slot].z = start;
            table[slot].w = end - start;
            return;
        }
        slot = (slot + 1) & mask;
    }
}

// Key filter, blocked by (l, i) group.  First and one-past-last list of each (l, i) group (the arrays zeroed by the caller): lists are
// in key order and the group is the key's top bits, so a group's lists are consecutive
__global__ __launch_bounds__(kBlock) void k_filter_group_bounds(const uint64_t* __restrict__ keys,
                                                                const uint32_t* __restrict__ runstart,
                                                                uint32_t nruns,
                                                                uint32_t* __restrict__ gfirst,
                                                                uint32_t* __restrict__ gend)
{
    const uint32_t r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= nruns) return;
    const uint64_t g = keys[runstart[r]] >> kHashBits;
    if (r == 0 || (keys[runstart[r - 1]] >> kHashBits) != g) gfirst[g] = r;
    if (r + 1 == nruns || (keys[runstart[r + 1]] >> kHashBits) != g) gend[g] = r + 1;
}

// words of each group's block: a power of two >= lists / 2 (16 bits per list), at least one
__global__ __launch_bounds__(kBlock) void k_filter_block_words(const uint32_t* __restrict__ gfirst,
                                                               const uint32_t* __restrict__ gend,
                                                               uint32_t ngroups,
                                                               uint32_t* __restrict__ words)
{
    const uint32_t g = blockIdx.x * kBlock + threadIdx.x;
    if (g >= ngroups) return;
    const uint32_t need = (gend[g] - gfirst[g] + 1) >> 1;
    uint32_t w = 1;
    while (w < need) w <<= 1;
    words[g] = w;
}

// sets the filter bits of every list's key in its group's block (filter zeroed by the caller)
__global__ __launch_bounds__(kBlock) void k_filter_keys(const uint64_t* __restrict__ keys,
                                                        const uint32_t* __restrict__ runstart,
                                                        uint32_t nruns,
                                                        const uint32_t* __restrict__ dir,
                                                        uint32_t* __restrict__ filter)
{
    const uint32_t r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= nruns) return;
    const uint64_t key = keys[runstart[r]];
    const uint64_t h = table_slot(key);
    const uint64_t g = key >> kHashBits;
    const uint32_t base = dir[g];
    atomicOr(&filter[base + filter_word_in(h, dir[g + 1] - base - 1u)], filter_bits(h));
}

// ------------------------------------------------------------------------------------------
// Probe: multi-match substring selection + bucket lookup (Sec. 4.2, Algorithm 2)
// ------------------------------------------------------------------------------------------

// One thread per (probe string x, probed length l, slot i).  The thread walks the window
// [bot_i, top_i] with a rolling hash of x[p, l_i], looks each substring up, trims the list to
// the members visited before x (self-join, l == |x|), and appends non-empty lookups as hits.
// Threads map to triples string-major (a wave covers consecutive (l, i) pairs of one or a few
// probe strings) or, with XMAJ, pair-major over blocks of 64 probe strings (a wave's lanes are
// 64 consecutive probe strings with one (l, i) pair: windows of one size when the strings have
// a few pairs each).
constexpr int kProbeStep = 2;      // window positions a probe thread takes per step

template <bool XMAJ>
__global__ __launch_bounds__(kBlock) void k_probe(ProbeParams P, Div div)
{
    // bytes of probe strings a wave stages in LDS
    constexpr int kProbeStage = XMAJ ? 4096 : 2048;
    __shared__ Hit s_hits[kWaves][kAppendCap];
    __shared__ uint4 s_xs[kWaves][kProbeStage / 16];
    __shared__ uint16_t s_sym[256];
    s_sym[threadIdx.x] = P.sym.code[threadIdx.x];
    __syncthreads();
    const int sym_bits = P.sym.bits, exact_len = P.sym.exact_len;
    const int lane = threadIdx.x & 63;
    WaveAppender<Hit, kAppendCap> app{s_hits[threadIdx.x >> 6], 0};
    const int T1 = P.tau + 1;
    const uint64_t nthreads = P.nx_dev ? (uint64_t)*P.nx_dev * (uint64_t)P.nl * (uint64_t)T1
                                       : P.threads;
    uint64_t my_sel = 0, my_cand = 0;
    // grid-stride over (probe string, length, slot) triples; the loop bound is block-uniform so
    // every lane takes part in the wave-level appends
    using LdsU8 = const __attribute__((address_space(3))) uint8_t*;
    const LdsU8 stage = (LdsU8)(s_xs[threadIdx.x >> 6]);
    const uint64_t per = (uint64_t)P.nl * T1;
    for (uint64_t t0 = (uint64_t)blockIdx.x * kBlock; t0 < nthreads;
         t0 += (uint64_t)gridDim.x * kBlock) {
        const uint64_t t = t0 + threadIdx.x;
        bool valid = t < nthreads;
        // the wave's threads cover consecutive probe strings; when they are of one length and
        // their padded bytes fit the stage, the wave copies them to LDS with 16-byte loads and
        // every byte of the window walk below is read from there (wave-uniform decision)
        const uint64_t tw = t0 + (threadIdx.x & ~63u);
        uint32_t g_first = 0;
        bool staged = false;
        // XMAJ: threads t = block * 64 * per + pair * 64 + lane, string g_begin + block*64 + lane
        uint32_t gx_t = 0, r0 = 0;
        if constexpr (XMAJ) {
            const uint64_t b = t / (64 * per), q = t % (64 * per);
            gx_t = P.g_begin + (uint32_t)(b * 64 + q % 64);
            r0 = (uint32_t)(q / 64);
            valid = valid && gx_t < P.g_begin + P.nx;
        } else {
            gx_t = P.g_begin + (uint32_t)(t / per);
            r0 = (uint32_t)(t % per);
        }
        if (tw < nthreads) {
            uint32_t g_last;
            if constexpr (XMAJ) {
                g_first = P.g_begin + (uint32_t)(tw / (64 * per)) * 64u;
                g_last = min(g_first + 63u, P.g_begin + P.nx - 1u);
            } else {
                const uint64_t tl = min(tw + 63, nthreads - 1);
                g_first = P.g_begin + (uint32_t)(tw / per);
                g_last = P.g_begin + (uint32_t)(tl / per);
            }
            const int n0 = P.x_slen[g_first];
            const int64_t bytes = (int64_t)(g_last - g_first + 1) * stride_of(n0);
            if (P.x_slen[g_last] == n0 && bytes <= kProbeStage) {
                staged = true;
                const uint4* src = reinterpret_cast<const uint4*>(
                    P.x_arena + P.x_gbase[n0] + (int64_t)(g_first - P.x_lenstart[n0]) * stride_of(n0));
                // the previous iteration's reads of the stage were issued before these writes,
                // and a wave's LDS requests complete in order
                for (int q = lane; q < (int)(bytes >> 4); q += 64) s_xs[threadIdx.x >> 6][q] = src[q];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
        int n = 0, l = 0, i = 0, lo = 1, hi = 0, tau = P.tau;
        uint32_t gx = 0;
        Seg sg{1, 0};
        const uint8_t* x = nullptr;
        const uint4* table = P.table;
        const uint32_t* vals = P.vals;
        uint64_t mask = P.mask;
        const uint32_t* filter = P.filter;
        const uint32_t* fdir = P.filter_dir;
        if (valid) {
            gx = gx_t;
            const uint32_t rem = P.order ? (uint32_t)P.order[r0] : r0;
            i = (int)(rem % T1) + 1;
            const int dl = (int)(rem / T1);
            n = P.x_slen[gx];
            Div dv = div;
            if (P.q_tau) {                       // mixed-tau batch: this probe string's own tau
                tau = P.q_tau[gx];
                const IndexRef ref = P.refs[tau];
                table = ref.table;
                vals = ref.vals;
                mask = ref.mask;
                filter = ref.filter;
                fdir = ref.filter_dir;
                dv.d = (uint32_t)(tau + 1);
                dv.m = ref.div_m;
            }
            l = P.self ? n - dl : n - tau + dl;
            const bool in_window = i <= tau + 1 && dl <= (P.self ? tau : 2 * tau) && l >= tau + 1;
            // substrings selected for L_l^1 .. L_l^{tau+1}, whether or not strings of length l
            // exist (Algorithm 1 selects for every l in the length window): for multi-match
            // the Lemma 2 count, otherwise each slot's window size
            if (in_window && P.selection == 0 && i == 1) {
                const int d = n - l;
                my_sel += (uint64_t)((tau * tau - d * d) / 2 + tau + 1);
            }
            if (in_window) {
                sg = partition_seg(l, i, tau, dv);
                select_window(P.selection, n, l, tau, i, sg, &lo, &hi);
                if (P.selection != 0 && hi >= lo) my_sel += (uint64_t)(hi - lo + 1);
            }
            valid = in_window && (l >= P.ymin) && (l <= P.ymax) &&
                    (P.y_lenstart[l + 1] > P.y_lenstart[l]);
            if (valid)
                x = P.x_arena + P.x_gbase[n] + (int64_t)(gx - P.x_lenstart[n]) * stride_of(n);
        }
        const LdsU8 xs = stage + (int64_t)(gx - g_first) * stride_of(n);   // when staged
        auto rd = [&](int k) -> uint8_t { return staged ? xs[k] : x[k]; };
        uint64_t h = 0, top = 0;
        if (valid && lo <= hi) top = pow_hash(sg.len);   // HB^(len-1)
        // the (l, i) group's filter block
        const bool use_filter = valid && lo <= hi && filter &&
                                (sg.len > exact_len || sg.len * sym_bits >= kFilterMinBits);
        uint32_t fb = 0, fm = 0;
        if (use_filter) {
            const uint32_t g = (uint32_t)((l - (tau + 1)) * (tau + 1) + (i - 1));
            fb = fdir[g];
            fm = fdir[g + 1] - fb - 1u;
        }
        // the window has at most tau+1 positions for multi-match, more for the other methods;
        // the loop ends when no lane of the wave has a position left.  kProbeStep positions per
        // step: their bytes are read first, then their keys computed, then their filter words
        // (or, without a filter, their first table slots) read together, so a step waits on one
        // round trip per kind of read instead of one per position; hits are appended in position
        // order as before.
        for (int s0 = 0;; s0 += kProbeStep) {
            if (__ballot(valid && lo + s0 <= hi) == 0) break;
            bool act[kProbeStep];
            int outb[kProbeStep], inb[kProbeStep];
#pragma unroll
            for (int u = 0; u < kProbeStep; ++u) {
                const int p = lo + s0 + u;
                act[u] = valid && p <= hi;
                outb[u] = 0;
                inb[u] = 0;
                if (act[u] && s0 + u > 0) {              // the bytes leaving and entering x[p, l_i]
                    outb[u] = rd(p - 2);
                    inb[u] = rd(p - 2 + sg.len);
                }
            }
            uint64_t key[kProbeStep], hs[kProbeStep];
#pragma unroll
            for (int u = 0; u < kProbeStep; ++u) {
                key[u] = 0;
                hs[u] = 0;
                if (act[u]) {
                    if (s0 + u == 0) {
                        const int w0 = lo - 1;
                        h = 0;
                        if (sg.len <= exact_len)
                            for (int k = 0; k < sg.len; ++k) h = (h << sym_bits) | (uint64_t)s_sym[rd(w0 + k)];
                        else
                            for (int k = 0; k < sg.len; ++k) h = h * kHashBase + (uint64_t)rd(w0 + k) + 1ull;
                    } else {
                        h = roll_code(h, sg.len, (uint8_t)outb[u], (uint8_t)inb[u], top, s_sym,
                                      sym_bits, exact_len);
                    }
                    key[u] = make_key(l, i, tau, sg.len, h, exact_len);
                    hs[u] = table_slot(key[u]);
                }
            }
            // hashed segments and long exact codes rarely match: the group's filter block (one
            // cache line for a group of up to 64 lists, read again by the lane at every position
            // of its window) turns most of those lookups away before the table read
            uint32_t fw[kProbeStep];
#pragma unroll
            for (int u = 0; u < kProbeStep; ++u) {
                fw[u] = 0;
                if (act[u] && use_filter) fw[u] = filter[fb + filter_word_in(hs[u], fm)];
            }
            bool maybe[kProbeStep];
            uint4 tv[kProbeStep];
#pragma unroll
            for (int u = 0; u < kProbeStep; ++u) {
                const uint32_t fbits = filter_bits(hs[u]);
                maybe[u] = act[u] && (!use_filter || (fw[u] & fbits) == fbits);
                tv[u] = make_uint4(0u, 0u, 0u, 0u);
                if (maybe[u]) tv[u] = table[hs[u] & mask];
            }
#pragma unroll
            for (int u = 0; u < kProbeStep; ++u) {
                uint32_t start = 0, count = 0;
                if (maybe[u]) {
                    const uint64_t k = (uint64_t)tv[u].x | ((uint64_t)tv[u].y << 32);
                    bool hit = false;
                    if (k == key[u]) {
                        start = tv[u].z;
                        count = tv[u].w;
                        hit = true;
                    } else if (k != kEmptyKey) {
                        hit = table_lookup_from(table, mask, key[u], ((hs[u] & mask) + 1) & mask,
                                                &start, &count);
                    }
                    if (hit && P.self && l == n) {
                        // keep members with g < gx (lists are ascending in g)
                        uint32_t a = 0, b = count;
                        while (a < b) {
                            const uint32_t m = (a + b) >> 1;
                            if (vals[start + m] < gx) a = m + 1; else b = m;
                        }
                        count = a;
                    }
                    if (!hit) count = 0;
                }
                const int p = lo + s0 + u;
                const bool found = act[u] && count > 0;
                Hit hh;
                hh.gx = gx; hh.start = start; hh.count = count;
                hh.meta = (uint32_t)(p - 1) | ((uint32_t)(i - 1) << 11) | ((uint32_t)l << 17);
                app.push(found, hh, P.hits, P.hit_cap, &P.counters[0]);
                if (found) my_cand += count;
            }
        }
    }
    app.flush(P.hits, P.hit_cap, &P.counters[0]);
    my_cand = wave_sum(my_cand);
    my_sel = wave_sum(my_sel);
    if (lane == 0) {
        if (my_cand) atomicAdd(&P.counters[1], (unsigned long long)my_cand);
        if (my_sel) atomicAdd(&P.counters[2], (unsigned long long)my_sel);
    }
}

// ------------------------------------------------------------------------------------------
// Verify: extension-based verification (Sec. 5.2, Algorithm 3), lane per candidate, candidates
// distributed over lanes by a load-balanced search over the hits' prefix sums.
// ------------------------------------------------------------------------------------------

constexpr int kVerifyChunk = 1024;

template <int MAXW>
__global__ __launch_bounds__(kBlock) void k_verify(VerifyParams V, Div div)
{
    __shared__ unsigned long long sP[kVerifyChunk + 1];
    __shared__ uint64_t s_h0;
    const int lane = threadIdx.x & 63;
    uint64_t my_cells = 0, my_miss = 0;
    const uint64_t nchunks = (V.ncand + kVerifyChunk - 1) / kVerifyChunk;
    for (uint64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const uint64_t c0 = ch * kVerifyChunk;
        const uint64_t c1 = (c0 + kVerifyChunk < V.ncand) ? c0 + kVerifyChunk : V.ncand;
        if (threadIdx.x == 0) {
            uint64_t a = 0, b = V.nhits - 1;      // largest h with prefix[h] <= c0
            while (a < b) {
                uint64_t m = (a + b + 1) >> 1;
                if (V.prefix[m] <= c0) a = m; else b = m - 1;
            }
            s_h0 = a;
        }
        __syncthreads();
        const uint64_t h0 = s_h0;
        for (int k = threadIdx.x; k <= kVerifyChunk; k += kBlock)
            sP[k] = (h0 + k <= V.nhits) ? V.prefix[h0 + k] : ~0ull;
        __syncthreads();
        for (uint64_t c = c0 + threadIdx.x; c - c0 < (uint64_t)kVerifyChunk; c += kBlock) {
            bool pass = false;
            uint32_t gx = 0, gy = 0;
            if (c < c1) {
                int a = 0, b = kVerifyChunk;
                while (a < b) {
                    int m = (a + b + 1) >> 1;
                    if (sP[m] <= c) a = m; else b = m - 1;
                }
                const Hit hit = V.hits[h0 + a];
                const uint64_t mem = c - sP[a];
                gx = hit.gx;
                int tau = V.tau;
                const uint32_t* vals = V.vals;
                Div dv = div;
                if (V.q_tau) {
                    tau = V.q_tau[gx];
                    vals = V.refs[tau].vals;
                    dv.d = (uint32_t)(tau + 1);
                    dv.m = V.refs[tau].div_m;
                }
                gy = vals[hit.start + mem];
                const int p = (int)(hit.meta & 2047u) + 1;
                const int i = (int)((hit.meta >> 11) & 63u) + 1;
                const int l = (int)(hit.meta >> 17);
                const int n = V.x_slen[gx];
                const uint8_t* x = V.x_arena + V.x_gbase[n] +
                                   (int64_t)(gx - V.x_lenstart[n]) * stride_of(n);
                const uint8_t* y = V.y_arena + V.y_gbase[l] +
                                   (int64_t)(gy - V.y_lenstart[l]) * stride_of(l);
                const Seg sg = partition_seg(l, i, tau, dv);
                bool same = true;
                if (sg.len > V.exact_len)
                    for (int k = 0; k < sg.len; ++k) same &= (x[p - 1 + k] == y[sg.p - 1 + k]);
                if (!same) {
                    my_miss += 1;
                } else {
                    int cl = 0;
                    const int tl = i - 1, tr = tau + 1 - i;
                    int dl = vsp_global<MAXW>(y, sg.p - 1, x, p - 1, tl, &cl);
                    my_cells += cl;
                    if (dl <= tl) {
                        int cr = 0;
                        const int ry = sg.p - 1 + sg.len, rx = p - 1 + sg.len;
                        int dr = vsp_global<MAXW>(y + ry, l - ry, x + rx, n - rx, tr, &cr);
                        my_cells += cr;
                        pass = dr <= tr;
                    }
                }
            }
            uint64_t pm = __ballot(pass);
            if (pm) {
                int leader = __ffsll((unsigned long long)pm) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(&V.counters[3], (unsigned long long)__popcll(pm));
                base = __shfl(base, leader, 64);
                if (pass) {
                    uint64_t idx = base + (uint64_t)__popcll(pm & lanemask_lt());
                    if (idx < V.out_cap) V.out[idx] = ((uint64_t)gx << 32) | gy;
                }
            }
        }
        __syncthreads();
    }
    my_cells = wave_sum(my_cells);
    my_miss = wave_sum(my_miss);
    if (lane == 0) {
        if (my_cells) atomicAdd(&V.counters[4], (unsigned long long)my_cells);
        if (my_miss) atomicAdd(&V.counters[5], (unsigned long long)my_miss);
    }
}

// ------------------------------------------------------------------------------------------
// Batched verification.  Hits are bucketed by slot i, so the candidates of a wave almost always
// share (tau_l, tau_r) = (i - 1, tau + 1 - i) and run band DPs of exactly that width.  Each wave
// walks its own chunks of 64 x kWaveRounds consecutive candidates; the hit of each lane is found
// from the hits' end offsets with one OR-reduced boundary mask per 64 candidates.
// ------------------------------------------------------------------------------------------

constexpr int kWaveRounds = kBatchedRoundsMax;   // captured batches use the full chunk
constexpr uint64_t kWaveChunk = 64ull * kWaveRounds;

// Bucket of a hit: lists with at least `big` candidates after all smaller ones, each part in
// slot order.
// Bucket of a hit: small lists, then big ones (from 64 * kLenClasses on), each by the length
// class of the list's strings and then by slot
__device__ inline uint32_t hit_bucket(const Hit& v, uint32_t big)
{
    const uint32_t slot = (v.meta >> 11) & 63u;
    const uint32_t cls = (uint32_t)len_class((int)(v.meta >> 17));
    return (v.count < big ? 0u : 64u * (uint32_t)kLenClasses) + 64u * cls + slot;
}

// Bucketing of the hits in two passes without global atomics: bb[b * G + blk] = hits of
// bucket b that block blk meets in its grid-stride walk (G blocks, kBuckets buckets); after an
// exclusive scan of bb (bucket-major), the scatter pass walks the same hits in the same order
// and places each at its block's offset in its bucket plus a rank from LDS counters.  The
// regions come out in bucket order; order inside a region changes nothing downstream (the
// result is sorted).
__global__ __launch_bounds__(kBlock) void k_slot_hist(const Hit* __restrict__ hits,
                                                      const unsigned long long* __restrict__ nh_dev,
                                                      uint32_t big, uint32_t* __restrict__ bb)
{
    __shared__ uint32_t h[kHitBuckets];
    for (int b = threadIdx.x; b < kHitBuckets; b += kBlock) h[b] = 0;
    __syncthreads();
    const uint64_t nh = *nh_dev;
    for (uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x; k < nh;
         k += (uint64_t)gridDim.x * kBlock)
        atomicAdd(&h[hit_bucket(hits[k], big)], 1u);
    __syncthreads();
    for (int b = threadIdx.x; b < kHitBuckets; b += kBlock)
        bb[(uint64_t)b * gridDim.x + blockIdx.x] = h[b];
}

__global__ __launch_bounds__(kBlock) void k_slot_scatter(const Hit* __restrict__ hits,
                                                         const unsigned long long* __restrict__ nh_dev,
                                                         uint32_t big,
                                                         const uint32_t* __restrict__ bb_off,
                                                         Hit* __restrict__ out)
{
    __shared__ uint32_t run[kHitBuckets], cnt[kHitBuckets];
    for (int b = threadIdx.x; b < kHitBuckets; b += kBlock)
        run[b] = bb_off[(uint64_t)b * gridDim.x + blockIdx.x];
    const uint64_t nh = *nh_dev;
    for (uint64_t k0 = (uint64_t)blockIdx.x * kBlock; k0 < nh; k0 += (uint64_t)gridDim.x * kBlock) {
        for (int b = threadIdx.x; b < kHitBuckets; b += kBlock) cnt[b] = 0;
        __syncthreads();
        const uint64_t k = k0 + threadIdx.x;
        Hit v{};
        uint32_t sl = 0, rank = 0;
        if (k < nh) {
            v = hits[k];
            sl = hit_bucket(v, big);
            rank = atomicAdd(&cnt[sl], 1u);
        }
        __syncthreads();
        if (k < nh) out[run[sl] + rank] = v;
        __syncthreads();
        for (int b = threadIdx.x; b < kHitBuckets; b += kBlock) run[b] += cnt[b];
    }
}

// first[ch] = the hit containing candidate ch * chunk (largest h with prefix[h] <= it)
__global__ __launch_bounds__(kBlock) void k_chunk_starts(const unsigned long long* __restrict__ prefix,
                                                         uint64_t nhits, uint64_t nchunks,
                                                         uint64_t chunk,
                                                         uint32_t* __restrict__ first)
{
    const uint64_t ch = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (ch >= nchunks) return;
    const unsigned long long c0 = ch * chunk;
    uint64_t a = 0, b = nhits - 1;
    while (a < b) {
        const uint64_t m = (a + b + 1) >> 1;
        if (prefix[m] <= c0) a = m; else b = m - 1;
    }
    first[ch] = (uint32_t)a;
}

__device__ inline uint64_t wave_or64(uint64_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v |= __shfl_xor(v, d, 64);
    return v;
}

// VerifyStringPair with the band width fixed at compile time when the threshold is the same on
// every active lane of the wave (t <= 8), else the generic width class GMAXW.
template <int GMAXW, typename P>
__device__ inline int vsp_dispatch(P r, int lr, P s, int ls, int t, int* cells)
{
    const int t0 = __builtin_amdgcn_readfirstlane(t);
    if (t0 <= 8 && __ballot(t != t0) == 0) {
        switch (t0) {
        case 0: return vsp_fast<1>(r, lr, s, ls, t, cells);
        case 1: return vsp_fast<2>(r, lr, s, ls, t, cells);
        case 2: return vsp_fast<3>(r, lr, s, ls, t, cells);
        case 3: return vsp_fast<4>(r, lr, s, ls, t, cells);
        case 4: return vsp_fast<5>(r, lr, s, ls, t, cells);
        case 5: return vsp_fast<6>(r, lr, s, ls, t, cells);
        case 6: return vsp_fast<7>(r, lr, s, ls, t, cells);
        case 7: return vsp_fast<8>(r, lr, s, ls, t, cells);
        default: return vsp_fast<9>(r, lr, s, ls, t, cells);
        }
    }
    // wider uniform thresholds (long strings, tau up to 32): a class of at most 3 extra columns
    if constexpr (GMAXW > 9 && GMAXW <= 33) {
        if (__ballot(t != t0) == 0) {
            if (t0 + 1 <= 13) return vsp_fast<13>(r, lr, s, ls, t, cells);
            if constexpr (GMAXW > 17) {
                if (t0 + 1 <= 17) return vsp_fast<17>(r, lr, s, ls, t, cells);
                if (t0 + 1 <= 21) return vsp_fast<21>(r, lr, s, ls, t, cells);
                if (t0 + 1 <= 25) return vsp_fast<25>(r, lr, s, ls, t, cells);
                if (t0 + 1 <= 29) return vsp_fast<29>(r, lr, s, ls, t, cells);
            }
        }
    }
    return vsp_fast<GMAXW>(r, lr, s, ls, t, cells);
}

// STG: every lane copies its candidate's two strings into LDS slots of its own first (probe
// string x up to kStgX - 4 bytes, indexed string y up to kStgY - 4), so the band DP reads LDS
// instead of global memory byte by byte.  Launched for indexed strings of at most 48 bytes and
// tau <= 8: a hit pairs x with lists of lengths within tau of |x|, so |x| <= 56.  STG 2 is the
// form for indexed strings of at most 40 bytes (|x| <= 48) with 52- and 44-byte slots and a
// 128-pair buffer: 28 KB per block, 5 blocks per CU, registers held to 96 (a 104-byte spill);
// it is taken for tau 6..8, where the fifth wave paid (the self-join of 5x10^5 medium strings:
// 22.1 -> 21.5 ms at tau = 8), not below (2% slower at tau 2 and 4 on short strings).
constexpr int kStgX = 60, kStgY = 52;     // slot strides: odd word counts, conflict-free

// With STG the LDS slots allow 4 blocks per CU; the register budget is held to match
// (128 VGPRs, no spills), so 4 waves per SIMD hide the candidates' dependent loads.  The
// unstaged 9-wide form is held to 128 VGPRs too (it would take 135, 3 waves per SIMD; the
// budget costs an 8-byte spill and gains a wave: the self-join of 5x10^5 medium strings at
// tau 2..8 measured 37.5 -> 36.0 ms); the wider bands keep their registers.
template <int GMAXW, int STG>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(STG == 2 ? 5 : (STG || GMAXW <= 9) ? 4 : 1))) void k_verify_batched(VerifyParams V, Div div,
                                                           const uint32_t* __restrict__ first,
                                                           uint64_t nchunks)
{
    // slot strides and pair buffer: STG 2 the smaller ones (5 blocks per CU in LDS)
    constexpr int SX = STG == 2 ? 52 : kStgX, SY = STG == 2 ? 44 : kStgY;
    constexpr int ACAP = STG == 2 ? 128 : kAppendCap;
    __shared__ uint64_t s_acc[kWaves][ACAP];
    __shared__ uint32_t s_str[kWaves][STG ? 64 * (SX + SY) / 4 : 1];
    WaveAppender<uint64_t, ACAP> acc{s_acc[threadIdx.x >> 6], 0};
    const int lane = threadIdx.x & 63;
    using LdsBytes = const __attribute__((address_space(3))) uint8_t*;
    __attribute__((address_space(3))) uint32_t* xsw =
        (__attribute__((address_space(3))) uint32_t*)(s_str[threadIdx.x >> 6]) + lane * (SX / 4);
    __attribute__((address_space(3))) uint32_t* ysw =
        (__attribute__((address_space(3))) uint32_t*)(s_str[threadIdx.x >> 6]) + 64 * (SX / 4) +
        lane * (SY / 4);
    const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * kBlock) >> 6;
    uint64_t my_cells = 0, my_miss = 0;
    const uint64_t le_mask = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    const uint64_t nhits = V.dev_counts ? V.dev_counts[0] : V.nhits;
    const uint64_t ncand = V.dev_counts ? V.dev_counts[1] : V.ncand;
    const uint64_t nch = V.dev_counts ? V.dev_counts[2] : nchunks;
    const uint64_t chunk = 64ull * (uint64_t)V.wave_rounds;
    for (uint64_t ch = wave; ch < nch; ch += nwaves) {
        const uint64_t c0 = ch * chunk;
        const uint64_t cend = (c0 + chunk < ncand) ? c0 + chunk : ncand;
        uint64_t h = first[ch];
        unsigned long long hstart = V.prefix[h];
        for (uint64_t g0 = c0; g0 < cend; g0 += 64) {
            // end offsets of hits h .. h + 63; a boundary at relative position r means the
            // candidates from r on belong to later hits
            const uint64_t hk = h + (uint64_t)lane;
            const unsigned long long bk = (hk < nhits) ? V.prefix[hk + 1] : ~0ull;
            const uint64_t rel = bk - g0;                      // >= 1
            const uint64_t M = wave_or64(rel < 64 ? (1ull << rel) : 0ull);
            const int off = __popcll(M & le_mask);
            const unsigned long long bprev = __shfl(bk, off > 0 ? off - 1 : 0, 64);
            const unsigned long long hs = (off == 0) ? hstart : bprev;
            const uint64_t c = g0 + (uint64_t)lane;
            bool pass = false;
            uint32_t gx = 0, gy = 0;
            if (c < cend) {
                const Hit hit = V.hits[h + (uint64_t)off];
                const uint64_t mem = c - hs;
                gx = hit.gx;
                int tau = V.tau;
                const uint32_t* vals = V.vals;
                Div dv = div;
                if (V.q_tau) {
                    tau = V.q_tau[gx];
                    vals = V.refs[tau].vals;
                    dv.d = (uint32_t)(tau + 1);
                    dv.m = V.refs[tau].div_m;
                }
                gy = vals[hit.start + mem];
                const int p = (int)(hit.meta & 2047u) + 1;
                const int i = (int)((hit.meta >> 11) & 63u) + 1;
                const int l = (int)(hit.meta >> 17);
                const int n = V.x_slen[gx];
                const uint8_t* x = V.x_arena + V.x_gbase[n] +
                                   (int64_t)(gx - V.x_lenstart[n]) * stride_of(n);
                const uint8_t* y = V.y_arena + V.y_gbase[l] +
                                   (int64_t)(gy - V.y_lenstart[l]) * stride_of(l);
                const Seg sg = partition_seg(l, i, tau, dv);
                auto verify = [&](auto xp, auto yp) {
                    bool same = true;
                    if (sg.len > V.exact_len)
                        for (int k = 0; k < sg.len; ++k) same &= (xp[p - 1 + k] == yp[sg.p - 1 + k]);
                    if (!same) {
                        my_miss += 1;
                        return;
                    }
                    int cl = 0;
                    const int tl = i - 1, tr = tau + 1 - i;
                    const int dl = vsp_dispatch<GMAXW>(yp, sg.p - 1, xp, p - 1, tl, &cl);
                    my_cells += cl;
                    if (dl <= tl) {
                        int cr = 0;
                        const int ry = sg.p - 1 + sg.len, rx = p - 1 + sg.len;
                        const int dr =
                            vsp_dispatch<GMAXW>(yp + ry, l - ry, xp + rx, n - rx, tr, &cr);
                        my_cells += cr;
                        pass = dr <= tr;
                    }
                };
                if constexpr (STG > 0) {
                    const uint4* xq = reinterpret_cast<const uint4*>(x);
                    const uint4* yq = reinterpret_cast<const uint4*>(y);
#pragma unroll
                    for (int q = 0; q < (SX + 15) / 16; ++q) {
                        if (q * 16 < n) {
                            const uint4 v = xq[q];
                            if (4 * q < SX / 4) xsw[4 * q] = v.x;
                            if (4 * q + 1 < SX / 4) xsw[4 * q + 1] = v.y;
                            if (4 * q + 2 < SX / 4) xsw[4 * q + 2] = v.z;
                            if (4 * q + 3 < SX / 4) xsw[4 * q + 3] = v.w;
                        }
                    }
#pragma unroll
                    for (int q = 0; q < (SY + 15) / 16; ++q) {
                        if (q * 16 < l) {
                            const uint4 v = yq[q];
                            if (4 * q < SY / 4) ysw[4 * q] = v.x;
                            if (4 * q + 1 < SY / 4) ysw[4 * q + 1] = v.y;
                            if (4 * q + 2 < SY / 4) ysw[4 * q + 2] = v.z;
                            if (4 * q + 3 < SY / 4) ysw[4 * q + 3] = v.w;
                        }
                    }
                    verify((LdsBytes)(xsw), (LdsBytes)(ysw));
                } else {
                    verify(x, y);
                }
            }
            acc.push(pass, ((uint64_t)gx << 32) | gy, V.out, V.out_cap, &V.counters[3]);
            // the hit containing candidate g0 + 64 starts the next group
            const uint64_t nb = __ballot(rel <= 64);
            const int adv = __popcll(nb);
            if (adv > 0) {
                hstart = __shfl(bk, adv - 1, 64);
                h += (uint64_t)adv;
            }
        }
    }
    acc.flush(V.out, V.out_cap, &V.counters[3]);
    my_cells = wave_sum(my_cells);
    my_miss = wave_sum(my_miss);
    if (lane == 0) {
        if (my_cells) atomicAdd(&V.counters[4], (unsigned long long)my_cells);
        if (my_miss) atomicAdd(&V.counters[5], (unsigned long long)my_miss);
    }
}

// ------------------------------------------------------------------------------------------
// List-segment verification: a wave verifies up to 64 members of one inverted list against
// the same probe substring, so the probe string, the partition and both band geometries are
// wave-uniform and only the indexed string differs per lane.  Used for lists with at least
// kBigList candidates; smaller lists go through k_verify_batched.
// ------------------------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_seg_counts(const Hit* __restrict__ hits, uint64_t nbig,
                                                       uint32_t members, uint32_t* __restrict__ segs)
{
    const uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < nbig) segs[k] = (hits[k].count + members - 1u) / members;
}

// first[ch] = the list holding segment ch * chunk (largest h with segp[h] <= it)
__global__ __launch_bounds__(kBlock) void k_seg_chunk_starts(const uint32_t* __restrict__ segp,
                                                             uint64_t nbig, uint64_t nchunks,
                                                             uint32_t chunk,
                                                             uint32_t* __restrict__ first)
{
    const uint64_t ch = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (ch >= nchunks) return;
    const uint64_t s0 = ch * chunk;
    uint64_t a = 0, b = nbig - 1;
    while (a < b) {
        const uint64_t m = (a + b + 1) >> 1;
        if (segp[m] <= s0) a = m; else b = m - 1;
    }
    first[ch] = (uint32_t)a;
}

using LdsInts = const __attribute__((address_space(3))) int*;

template <int MAXW, int NC, int TS, typename LaneChars>
__device__ inline void vsp_seg_any(bool yrows, LdsChars U, int lu, const LaneChars (&V)[NC],
                                   int lv, int t, LdsInts tab, const bool (&act)[NC],
                                   int (&cells)[NC], int (&res)[NC])
{
    if constexpr (NC == 2) {
        // two candidates per lane: the packed 16-bit DP (register strings only)
        if (yrows) vsp_seg2<MAXW, true, TS>(U, lu, V, lv, t, tab, act, cells, res);
        else vsp_seg2<MAXW, false, TS>(U, lu, V, lv, t, tab, act, cells, res);
    } else {
        if (yrows) vsp_seg<MAXW, true, NC, TS>(U, lu, V, lv, t, tab, act, cells, res);
        else vsp_seg<MAXW, false, NC, TS>(U, lu, V, lv, t, tab, act, cells, res);
    }
}

// band width t + 1 for a uniform t <= 8 below the width class, else the class width GMAXW
template <int GMAXW, int NC, int TS, typename LaneChars>
__device__ inline void vsp_seg_dispatch(bool yrows, LdsChars U, int lu, const LaneChars (&V)[NC],
                                        int lv, int t, LdsInts tab, const bool (&act)[NC],
                                        int (&cells)[NC], int (&res)[NC])
{
    if (t + 1 >= GMAXW || t > 8) {
        vsp_seg_any<GMAXW, NC, TS>(yrows, U, lu, V, lv, t, tab, act, cells, res);
        return;
    }
#define PJ_SEG_CASE(T)                                                                      \
    case T:                                                                                 \
        if constexpr (T + 1 < GMAXW)                                                        \
            vsp_seg_any<T + 1, NC, TS>(yrows, U, lu, V, lv, t, tab, act, cells, res);       \
        break;
    switch (t) {
    PJ_SEG_CASE(0)
    PJ_SEG_CASE(1)
    PJ_SEG_CASE(2)
    PJ_SEG_CASE(3)
    PJ_SEG_CASE(4)
    PJ_SEG_CASE(5)
    PJ_SEG_CASE(6)
    PJ_SEG_CASE(7)
    PJ_SEG_CASE(8)
    default: break;
    }
#undef PJ_SEG_CASE
}

template <int MAXW, int KF, int TS>
__device__ inline void vsp_lane_or(bool yrows, LdsChars U, int lu, LdsLaneChars V, int lv, int t,
                                   LdsInts tab, bool act, int& cells, int& res)
{
    if (yrows) vsp_lane<MAXW, KF, true, TS>(U, lu, V, lv, t, tab, act, cells, res);
    else vsp_lane<MAXW, KF, false, TS>(U, lu, V, lv, t, tab, act, cells, res);
}

// vsp_lane at width t + 1 (the width class GMAXW when t + 1 reaches it); for t <= 4 the band
// index of the final cell, (t + |lu - lv|) / 2, is a compile-time constant too
template <int GMAXW, int TS>
__device__ inline void vsp_lane_dispatch(bool yrows, LdsChars U, int lu, LdsLaneChars V, int lv,
                                         int t, LdsInts tab, bool act, int& cells, int& res)
{
    static_assert(GMAXW >= 5 && GMAXW <= 9, "narrow width classes only");
    const int delta = lu > lv ? lu - lv : lv - lu;
    if (delta > t) {
        cells = 0;
        res = t + 1;
        return;
    }
    const int kf = (t + delta) >> 1;
    cells = 0;                                   // t < GMAXW always; kept defined regardless
    res = t + 1;
#define PJ_LANE(W, K) vsp_lane_or<W, K, TS>(yrows, U, lu, V, lv, t, tab, act, cells, res)
    switch (t) {
    case 0: PJ_LANE(1, 0); return;
    case 1: if (kf == 0) PJ_LANE(2, 0); else PJ_LANE(2, 1); return;
    case 2: if (kf == 1) PJ_LANE(3, 1); else PJ_LANE(3, 2); return;
    case 3: if (kf == 1) PJ_LANE(4, 1); else if (kf == 2) PJ_LANE(4, 2); else PJ_LANE(4, 3); return;
    case 4: if (kf == 2) PJ_LANE(5, 2); else if (kf == 3) PJ_LANE(5, 3); else PJ_LANE(5, 4); return;
    default: break;
    }
    if constexpr (GMAXW > 5) {
        if (t == 5 && GMAXW > 6) { PJ_LANE(6 < GMAXW ? 6 : GMAXW, -1); return; }
        if (t == 6 && GMAXW > 7) { PJ_LANE(7 < GMAXW ? 7 : GMAXW, -1); return; }
        if (t == 7 && GMAXW > 8) { PJ_LANE(8 < GMAXW ? 8 : GMAXW, -1); return; }
        PJ_LANE(GMAXW, -1);
    }
#undef PJ_LANE
}

// a wave-uniform load through the scalar cache (read-only data)
template <typename T>
__device__ inline T uniform_load(const T* p)
{
    return *(const __attribute__((address_space(4))) T*)p;
}

// The 40-byte class of the 5-wide band fits 8 blocks per CU in LDS; it is compiled for 8 waves
// per SIMD (at most 64 VGPRs) to match.
template <int GMAXW, int REGY, int NCT>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu((REGY == 40 && GMAXW <= 5) ? 8 : 1)))
void k_verify_segs(VerifyParams V, Div div,
                                                        const Hit* __restrict__ big,
                                                        const uint32_t* __restrict__ segp,
                                                        uint64_t /* hits (unused) */,
                                                        uint64_t nseg,
                                                        const uint32_t* __restrict__ first,
                                                        uint64_t nchunks, uint32_t seg_chunk)
{
    // NC candidates per lane: a list segment has 64 * NC members
    constexpr int NC = (REGY > 0 && GMAXW <= 9) ? NCT : 1;
    constexpr uint32_t SEG = 64u * NC;
    // one candidate per lane and indexed strings of at most REGY bytes: each lane copies its
    // string into an LDS slot of its own, from which the band DP reads it (vsp_lane)
    constexpr bool LANE = REGY > 0 && NC == 1 && GMAXW <= 9;
    // slot stride REGY + 4 bytes, an odd number of words, so a wave's reads at one offset hit
    // distinct banks; 16 bytes before the first slot and after the last absorb the reads of
    // columns outside the string (at most 4 bytes before a string, at most 12 after it: a DP
    // block reads up to 2 * MAXW - 2 - kfin past the part, with kfin >= t / 2)
    constexpr int SL = REGY + 4, YPAD = 16, YTAIL = 16;
    constexpr int kCap = 96;                               // pairs buffered per wave
    __shared__ uint64_t s_acc[kWaves][kCap];
    // the current probe string; the band DP reads at most 2 * MAXW bytes past a part's end
    // (vsp_seg and vsp_lane up to width 9; the wider classes keep 128).  An indexed string of
    // at most REGY bytes has probes of at most REGY + tau bytes.
    constexpr int XMAX = REGY > 0 ? REGY + (GMAXW <= 9 ? GMAXW - 1 : kTauMax) : kLenMax;
    constexpr int XPAD = GMAXW <= 9 ? 32 : 128;
    __shared__ uint32_t s_x[kWaves][(XMAX + 1 + XPAD + 3) / 4];
    __shared__ uint32_t s_q[kWaves][2 * SEG];             // left-part survivors
    // band tables of the current hit's two parts (row 0, distance offsets, first window, and
    // the rows of vsp_lane)
    constexpr int BTS = (GMAXW + 3) & ~3;
    constexpr int CT = LANE ? REGY + 4 : 0;               // cells table: rows 0 .. nr <= REGY
    __shared__ __attribute__((aligned(16))) int s_band[kWaves][2][6 * BTS + CT];
    constexpr int YW = LANE ? (YPAD + 64 * SL + YTAIL) / 4 : 1;
    __shared__ __attribute__((aligned(16))) uint32_t s_y[kWaves][YW];   // lane slots (LANE)
    WaveAppender<uint64_t, kCap> acc{s_acc[threadIdx.x >> 6], 0};
    const int lane = threadIdx.x & 63;
    uint32_t* sx = s_x[threadIdx.x >> 6];
    uint32_t* sq = s_q[threadIdx.x >> 6];
    const __attribute__((address_space(3))) uint8_t* xl8 =
        (const __attribute__((address_space(3))) uint8_t*)(sx);
    // this lane's slot (LANE)
    __attribute__((address_space(3))) uint32_t* ysw =
        (__attribute__((address_space(3))) uint32_t*)(s_y[threadIdx.x >> 6]) +
        (YPAD + lane * SL) / 4;
    const __attribute__((address_space(3))) uint8_t* ys8 =
        (const __attribute__((address_space(3))) uint8_t*)(ysw);
    // wave id as a scalar, so that everything derived from it is known to be wave-uniform
    const uint64_t wave = (uint64_t)blockIdx.x * kWaves +
                          (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * kWaves;
    uint64_t my_cells = 0, my_miss = 0;
    for (uint64_t ch = wave; ch < nchunks; ch += nwaves) {
        uint64_t sg_i = ch * seg_chunk;
        const uint64_t sg_end = (sg_i + seg_chunk < nseg) ? sg_i + seg_chunk : nseg;
        uint32_t h = uniform_load(first + ch);
        uint32_t sidx = (uint32_t)(sg_i - uniform_load(segp + h));
        while (sg_i < sg_end) {
            // everything about the hit is wave-uniform: probe string, slot, both parts
            const uint32_t* hw = reinterpret_cast<const uint32_t*>(big + h);
            const uint32_t gx = uniform_load(hw), start = uniform_load(hw + 1);
            const uint32_t count = uniform_load(hw + 2), meta = uniform_load(hw + 3);
            int tau = V.tau;
            const uint32_t* vals = V.vals;
            Div dv = div;
            if (V.q_tau) {
                tau = uniform_load(V.q_tau + gx);
                const IndexRef* rf = V.refs + tau;
                vals = uniform_load(&rf->vals);
                dv.d = (uint32_t)(tau + 1);
                dv.m = uniform_load(&rf->div_m);
            }
            const int p = (int)(meta & 2047u) + 1;
            const int i = (int)((meta >> 11) & 63u) + 1;
            const int l = (int)(meta >> 17);
            const int n = __builtin_amdgcn_readfirstlane((int)V.x_slen[gx]);
            const uint8_t* x = V.x_arena + uniform_load(V.x_gbase + n) +
                               (int64_t)(gx - (uint32_t)uniform_load(V.x_lenstart + n)) * stride_of(n);
            const int64_t ybase = uniform_load(V.y_gbase + l) -
                                  (int64_t)uniform_load(V.y_lenstart + l) * stride_of(l);
            const Seg sgm = partition_seg(l, i, tau, dv);
            // stage x in the wave's LDS buffer (its slot is 16-byte aligned); the previous
            // hit's reads were issued before these writes, and LDS requests of a wave complete
            // in order
            {
                const uint32_t* xw = reinterpret_cast<const uint32_t*>(x);
                for (int q = lane; q < ((n + 3) >> 2); q += 64) sx[q] = xw[q];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            // left parts: x[1, p-1] vs y[1, p_i-1] with t = i-1; right parts after the segment
            // with t = tau+1-i (Algorithm 3)
            const int tl = i - 1, tr = tau + 1 - i;
            const int ry = sgm.p - 1 + sgm.len, rx = p - 1 + sgm.len;
            // the previous hit's table reads were issued before these writes
            __attribute__((address_space(3))) int* tab_l =
                (__attribute__((address_space(3))) int*)s_band[threadIdx.x >> 6][0];
            __attribute__((address_space(3))) int* tab_r =
                (__attribute__((address_space(3))) int*)s_band[threadIdx.x >> 6][1];
            band_table(LdsChars{xl8}, p - 1, sgm.p - 1, tl, lane, BTS, NC == 2, tab_l, CT);
            band_table(LdsChars{xl8 + rx}, n - rx, l - ry, tr, lane, BTS, NC == 2, tab_r, CT);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const uint32_t hsegs = (count + SEG - 1) / SEG;
            const uint64_t left_in_chunk = sg_end - sg_i;
            const uint32_t s_stop = (uint64_t)(hsegs - sidx) < left_in_chunk
                                        ? hsegs : sidx + (uint32_t)left_in_chunk;
            // REGY > 0: the whole indexed string (at most REGY bytes, 16-byte aligned slot) goes
            // to registers with wide loads and is read at wave-uniform offsets
            // With the index's inline copies a list's strings are contiguous (entry e at
            // yinl + e * stride), so a segment's loads are coalesced and need no list entry first
            const uint8_t* yinl = nullptr;
            if (REGY > 0 && V.y_inl) yinl = V.y_inl + uniform_load(V.y_inl_base + l);
            // REGY > 0: the indexed string's words (at most REGY bytes) go to registers, or,
            // with LANE, straight into the lane's LDS slot (a wave's LDS requests complete in
            // order: the DP's reads see these words, the previous DP's reads did not); words
            // past the string are not loaded
            auto load_y = [&](uint32_t g, uint32_t e, uint32_t* yr) -> const uint8_t* {
                const uint8_t* y = yinl ? yinl + (int64_t)e * stride_of(l)
                                        : V.y_arena + ybase + (int64_t)g * stride_of(l);
                if constexpr (LANE) {
                    // every load first, then the writes: one wait for all of them.  A class
                    // of REGY = 40 loads 48 bytes (inside the 48-byte stride of its strings)
                    // and writes the slot's 10 words only
                    constexpr int NQ = (REGY + 15) / 16;
                    const uint4* yq = reinterpret_cast<const uint4*>(y);
                    uint4 v[NQ];
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
                        if (q * 16 < l) v[q] = yq[q];
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        if (q * 16 < l) {
                            ysw[4 * q] = v[q].x;
                            if (16 * q + 4 < REGY) ysw[4 * q + 1] = v[q].y;
                            if (16 * q + 8 < REGY) ysw[4 * q + 2] = v[q].z;
                            if (16 * q + 12 < REGY) ysw[4 * q + 3] = v[q].w;
                        }
                    }
                } else if (REGY > 0) {
                    const uint4* yq = reinterpret_cast<const uint4*>(y);
#pragma unroll
                    for (int q = 0; q < (REGY > 0 ? REGY / 16 : 0); ++q) {
                        const uint4 v = (q * 16 < l) ? yq[q] : make_uint4(0u, 0u, 0u, 0u);
                        yr[4 * q] = v.x; yr[4 * q + 1] = v.y;
                        yr[4 * q + 2] = v.z; yr[4 * q + 3] = v.w;
                    }
                }
                return y;
            };
            // Two phases per hit: the left parts of each segment, then the right parts of the
            // survivors, taken SEG at a time from a wave-private queue, so that a wave's
            // right-part rows are not spent on lanes whose left part already failed.  Each
            // iteration runs one band DP: a left step (next segment) or a right batch (SEG queued
            // survivors, or the rest once the segments are done).
            // A part whose two strings are both empty passes with no cells (ED 0 <= t): the
            // left parts of slot 1 (p = p_1 = 1) and the right parts of slot tau+1 (x and y both
            // end with the segment).  Then the other part runs directly on the segment members,
            // without the queue.
            const bool left_trivial = (p == 1) && (sgm.p == 1);
            const bool right_trivial = (rx == n) && (ry == l);
            uint32_t qn = 0;    // queued survivors (wave-uniform)
            for (;;) {
                const bool right = left_trivial ? sidx < s_stop
                                                : (qn >= SEG || (sidx >= s_stop && qn > 0));
                if (!right && sidx >= s_stop) break;
                const bool from_queue = right && !left_trivial;
                const uint32_t k = from_queue ? (qn < SEG ? qn : SEG) : 0;
                if (from_queue) {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                }
                uint32_t gy[NC], ent[NC];
                uint32_t yr[NC][(REGY > 0 && !LANE) ? REGY / 4 : 1];
                const uint8_t* y[NC];
                bool ok[NC];
                bool anyok = false;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const uint32_t slot = (uint32_t)c * 64u + (uint32_t)lane;
                    const uint32_t member = sidx * SEG + slot;
                    ok[c] = from_queue ? slot < k : member < count;
                    // every lane takes a valid candidate (an inactive one repeats the first
                    // queued candidate, k >= 1, or the hit's last member, count >= 1), so the
                    // loads below need no per-lane branch; only active lanes count.  The queue
                    // holds index entries (inline copies) or string positions.
                    uint32_t src;
                    if (from_queue) src = sq[ok[c] ? slot : 0u];     // slot < 2 * SEG
                    else src = start + (ok[c] ? member : count - 1u);
                    if (yinl) {
                        ent[c] = src;
                        // string positions are needed only to emit pairs
                        gy[c] = (right || right_trivial) ? vals[src] : 0u;
                    } else {
                        ent[c] = 0;
                        gy[c] = from_queue ? src : vals[src];
                    }
                    y[c] = load_y(gy[c], ent[c], yr[c]);
                    if (!from_queue && sgm.len > V.exact_len) {
                        // hashed key: compare the segment bytes before extension
                        // verification, which skips the segment
                        const LdsChars xs{xl8 + (p - 1)};
                        bool same = true;
                        if constexpr (LANE) {
                            const LdsLaneChars yc{ys8 + (sgm.p - 1)};
                            for (int q = 0; q < sgm.len; ++q) same &= (xs[q] == yc[q]);
                        } else if constexpr (REGY > 0) {
                            const RegChars yc{yr[c], sgm.p - 1};
                            for (int q = 0; q < sgm.len; ++q) same &= (xs[q] == yc[q]);
                        } else {
                            for (int q = 0; q < sgm.len; ++q)
                                same &= (xs[q] == (int)y[c][sgm.p - 1 + q]);
                        }
                        my_miss += (ok[c] && !same) ? 1 : 0;
                        ok[c] = ok[c] && same;
                    }
                    anyok = anyok || ok[c];
                }
                if (anyok) {
                    const int xo = right ? rx : 0, xl = right ? n - rx : p - 1;
                    const int yo = right ? ry : 0, yl = right ? l - ry : sgm.p - 1;
                    const int tt = right ? tr : tl;
                    int cl[NC], d[NC];
                    if constexpr (LANE) {
                        vsp_lane_dispatch<GMAXW, BTS>(yl <= xl, LdsChars{xl8 + xo}, xl,
                                                      LdsLaneChars{ys8 + yo}, yl, tt,
                                                      right ? tab_r : tab_l, ok[0], cl[0], d[0]);
                    } else if constexpr (REGY > 0) {
                        RegChars vc[NC];
#pragma unroll
                        for (int c = 0; c < NC; ++c) vc[c] = RegChars{yr[c], yo};
                        vsp_seg_dispatch<GMAXW, NC, BTS>(yl <= xl, LdsChars{xl8 + xo}, xl, vc,
                                                         yl, tt, right ? tab_r : tab_l, ok, cl,
                                                         d);
                    } else {
                        GlobalChars vc[NC];
#pragma unroll
                        for (int c = 0; c < NC; ++c) vc[c] = GlobalChars{y[c] + yo};
                        vsp_seg_dispatch<GMAXW, NC, BTS>(yl <= xl, LdsChars{xl8 + xo}, xl, vc,
                                                         yl, tt, right ? tab_r : tab_l, ok, cl,
                                                         d);
                    }
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        my_cells += (uint64_t)cl[c];
                        ok[c] = ok[c] && d[c] <= tt;
                    }
                }
                if (right || right_trivial) {
#pragma unroll
                    for (int c = 0; c < NC; ++c)
                        acc.push(ok[c], ((uint64_t)gx << 32) | gy[c], V.out, V.out_cap,
                                 &V.counters[3]);
                }
                if (!from_queue) {
                    ++sidx;
                    ++sg_i;
                }
                if (from_queue) {
                    // move the rest of the queue (entries SEG .. qn-1) to its front, all reads
                    // before the writes; every lane moves a word, those past the rest are free
                    const uint32_t rest = qn - k;
                    uint32_t mv[NC];
#pragma unroll
                    for (int c = 0; c < NC; ++c) mv[c] = sq[SEG + (uint32_t)(c * 64 + lane)];
#pragma unroll
                    for (int c = 0; c < NC; ++c) sq[(uint32_t)(c * 64 + lane)] = mv[c];
                    qn = rest;
                } else if (!right && !right_trivial) {
                    // survivors appended in lane order; a left step starts with qn < SEG, so
                    // the last word, 2 * SEG - 1, is never an entry and takes the other lanes'
                    // writes
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        const uint64_t surv = __builtin_amdgcn_ballot_w64(ok[c]);
                        const uint32_t at = qn + __builtin_amdgcn_mbcnt_hi(
                                                     (uint32_t)(surv >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)surv, 0u));
                        sq[ok[c] ? at : 2u * SEG - 1u] = yinl ? ent[c] : gy[c];
                        qn += (uint32_t)__builtin_popcountll(surv);
                    }
                }
            }
            ++h;
            sidx = 0;
        }
    }
    acc.flush(V.out, V.out_cap, &V.counters[3]);
    my_cells = wave_sum(my_cells);
    my_miss = wave_sum(my_miss);
    if (lane == 0) {
        if (my_cells) atomicAdd(&V.counters[7], (unsigned long long)my_cells);
        if (my_miss) atomicAdd(&V.counters[5], (unsigned long long)my_miss);
    }
}

// ------------------------------------------------------------------------------------------
// Short strings (length <= tau): not partitionable (footnote to Sec. 3.1).  One block per short
// string y of the indexed set; its partners are the probe-set strings in the length window
// [|y| - tau, |y| + tau] -- a contiguous range of sorted positions.  In a self-join a pair of
// two short strings is taken once (from the later one).
// ------------------------------------------------------------------------------------------

// ------------------------------------------------------------------------------------------
// Shared-prefix verification (Sec. 5.3).  The paper walks an inverted list in alphabetical
// order and lets each member's DP start from the rows its left (right) part shares with the
// previous member's.  In a wave the 64 lanes advance row by row together, so sharing rows
// between lanes saves nothing; here a lane walks a chain of kChainMembers consecutive members
// of a content-ordered list on its own, as the paper's loop does, keeping its previous
// member's first kShareRows rows per side in LDS.  Lanes of a wave take consecutive chains
// (the same list, or the next big lists).
// ------------------------------------------------------------------------------------------

// chains of one big hit: the whole list is walked in content order, so for a self-join's list
// of the probe string's own length the members visited after it are skipped one by one
__global__ __launch_bounds__(kBlock) void k_chain_counts(const Hit* __restrict__ big, uint64_t nbig,
                                                         const uint16_t* __restrict__ x_slen,
                                                         const uint32_t* __restrict__ runlen,
                                                         int self, uint32_t* __restrict__ chains)
{
    const uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= nbig) return;
    const Hit h = big[k];
    const int l = (int)(h.meta >> 17);
    const uint32_t full = (self && l == (int)x_slen[h.gx]) ? runlen[h.start] : h.count;
    chains[k] = (full + kChainMembers - 1u) / kChainMembers;
}

template <int MAXW>
__global__ __launch_bounds__(kBlock) void k_verify_chains(VerifyParams V, Div div,
                                                          const Hit* __restrict__ big,
                                                          const unsigned long long* __restrict__ cprefix,
                                                          uint64_t nbig, uint64_t nchains,
                                                          const uint32_t* __restrict__ first,
                                                          uint64_t nchunks)
{
    constexpr int NW = (MAXW + 7) / 8;
    __shared__ uint64_t s_acc[kWaves][kAppendCap];
    __shared__ uint32_t s_mat[kWaves][2][kShareRows * NW * 64];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    WaveAppender<uint64_t, kAppendCap> acc{s_acc[wv], 0};
    __attribute__((address_space(3))) uint32_t* matL =
        (__attribute__((address_space(3))) uint32_t*)(s_mat[wv][0]) + lane;
    __attribute__((address_space(3))) uint32_t* matR =
        (__attribute__((address_space(3))) uint32_t*)(s_mat[wv][1]) + lane;
    const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * kBlock) >> 6;
    uint64_t my_cells = 0, my_miss = 0, my_srows = 0, my_scells = 0;
    const uint64_t le_mask = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    for (uint64_t ch = wave; ch < nchunks; ch += nwaves) {
        const uint64_t c0 = ch * 64ull;
        const uint64_t h = first[ch];
        // the chain of each lane: boundaries of hits h .. h + 63 inside [c0, c0 + 64)
        const uint64_t hk = h + (uint64_t)lane;
        const unsigned long long bk = (hk < nbig) ? cprefix[hk + 1] : ~0ull;
        const uint64_t rel = bk - c0;
        const uint64_t M = wave_or64(rel < 64 ? (1ull << rel) : 0ull);
        const int off = __popcll(M & le_mask);
        const unsigned long long bprev = __shfl(bk, off > 0 ? off - 1 : 0, 64);
        const unsigned long long hs = (off == 0) ? cprefix[h] : bprev;
        const uint64_t c = c0 + (uint64_t)lane;
        const bool valid = c < nchains;
        Hit hit{0, 0, 0, 0};
        int n = 0, l = 0, p = 1, i = 1;
        uint32_t m0 = 0, m1 = 0;
        const uint8_t* x = nullptr;
        Seg sg{1, 0};
        if (valid) {
            hit = big[h + (uint64_t)off];
            p = (int)(hit.meta & 2047u) + 1;
            i = (int)((hit.meta >> 11) & 63u) + 1;
            l = (int)(hit.meta >> 17);
            n = V.x_slen[hit.gx];
            x = V.x_arena + V.x_gbase[n] + (int64_t)(hit.gx - V.x_lenstart[n]) * stride_of(n);
            const uint32_t full = (V.self && l == n) ? V.runlen[hit.start] : hit.count;
            m0 = (uint32_t)(c - hs) * (uint32_t)kChainMembers;
            m1 = min(m0 + (uint32_t)kChainMembers, full);
            sg = partition_seg(l, i, V.tau, div);
        }
        const int tl = i - 1, tr = V.tau + 1 - i;
        const int ry = sg.p - 1 + sg.len, rx = p - 1 + sg.len;
        SharePrev pl{nullptr, 0, 0, 0, 0}, pr{nullptr, 0, 0, 0, 0};
        for (int it = 0; it < kChainMembers; ++it) {
            const uint32_t m = m0 + (uint32_t)it;
            bool cand = valid && m < m1;
            uint32_t gy = 0;
            if (cand) {
                gy = V.svals[hit.start + m];
                if (V.self && l == n && gy >= hit.gx) cand = false;    // visited after x
            }
            bool pass = false;
            if (cand) {
                const uint8_t* y = V.y_arena + V.y_gbase[l] +
                                   (int64_t)(gy - V.y_lenstart[l]) * stride_of(l);
                bool same = true;
                if (sg.len > V.exact_len)
                    for (int k = 0; k < sg.len; ++k) same &= (x[p - 1 + k] == y[sg.p - 1 + k]);
                if (!same) {
                    my_miss += 1;
                } else {
                    const int dl = share_part<MAXW>(y, sg.p - 1, x, p - 1, tl, pl, matL, my_cells,
                                                    my_srows, my_scells);
                    if (dl <= tl) {
                        const int dr = share_part<MAXW>(y + ry, l - ry, x + rx, n - rx, tr, pr,
                                                        matR, my_cells, my_srows, my_scells);
                        pass = dr <= tr;
                    }
                }
            }
            acc.push(pass, ((uint64_t)hit.gx << 32) | gy, V.out, V.out_cap, &V.counters[3]);
        }
    }
    acc.flush(V.out, V.out_cap, &V.counters[3]);
    my_cells = wave_sum(my_cells);
    my_miss = wave_sum(my_miss);
    my_srows = wave_sum(my_srows);
    my_scells = wave_sum(my_scells);
    if (lane == 0) {
        if (my_cells) atomicAdd(&V.counters[4], (unsigned long long)my_cells);
        if (my_miss) atomicAdd(&V.counters[5], (unsigned long long)my_miss);
        if (my_srows) atomicAdd(&V.counters[8], (unsigned long long)my_srows);
        if (my_scells) atomicAdd(&V.counters[9], (unsigned long long)my_scells);
    }
}

// Content order of the index entries: the first 8 bytes of each entry's string, big-endian,
// so that comparing keys compares the strings' first 8 bytes; idx = entry number.
__global__ __launch_bounds__(kBlock) void k_prefix8_keys(const uint32_t* __restrict__ vals, int64_t E,
                                                         const uint8_t* __restrict__ sarena,
                                                         const uint16_t* __restrict__ slen,
                                                         const int32_t* __restrict__ lenstart,
                                                         const int64_t* __restrict__ gbase,
                                                         uint64_t* __restrict__ keys,
                                                         uint32_t* __restrict__ idx)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= E) return;
    const uint32_t g = vals[e];
    const int l = slen[g];
    const uint8_t* w = sarena + gbase[l] + (int64_t)(g - lenstart[l]) * stride_of(l);
    uint64_t k = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b) k = (k << 8) | (uint64_t)(b < l ? w[b] : 0);
    keys[e] = k;
    idx[e] = (uint32_t)e;
}

__global__ __launch_bounds__(kBlock) void k_gather_keys(const uint64_t* __restrict__ keys,
                                                        const uint32_t* __restrict__ idx, int64_t E,
                                                        uint64_t* __restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < E) out[e] = keys[idx[e]];
}

__global__ __launch_bounds__(kBlock) void k_gather_vals(const uint32_t* __restrict__ vals,
                                                        const uint32_t* __restrict__ idx, int64_t E,
                                                        uint32_t* __restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < E) out[e] = vals[idx[e]];
}

__global__ __launch_bounds__(kBlock) void k_run_lengths(const uint32_t* __restrict__ runstart,
                                                        uint32_t nruns, uint32_t E,
                                                        uint32_t* __restrict__ runlen)
{
    const uint32_t r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= nruns) return;
    const uint32_t st = runstart[r];
    runlen[st] = ((r + 1 < nruns) ? runstart[r + 1] : E) - st;
}

// ------------------------------------------------------------------------------------------
// Long-string verification by row blocks.  A candidate's part DP runs for hundreds of rows
// when it passes and stops after a few when it does not, so 64 candidates in lockstep leave
// most lanes idle.  Here the candidates of the small lists are materialised in slot order (one
// (tau_l, tau_r) per slot, so a wave's 64 tasks share the band width class), and the DPs run in
// passes: a pass takes up to K rows of every live task, and the tasks still running after them
// go, with their band row (values min(M, t+1) in bytes: min(., t+1) commutes with the
// recurrence and every decision compares with t), to a compacted queue for the next pass.
// Left parts run first; candidates whose left part passes become right-part tasks (Algorithm
// 3 examines right parts only after the left parts pass).  A pass stages its rows' characters
// in LDS first, so the row loop reads no global memory.
// ------------------------------------------------------------------------------------------

constexpr int kContMaxRows = 64;     // rows of one pass (at most)
constexpr int kContW = 33;           // widest band class
// 16-byte blocks staged per lane and pass: A needs K + 15 bytes, B up to kContW + K + 15 + 15
constexpr int kStageA = (kContMaxRows + 15 + 15) / 16;
constexpr int kStageB = (kContW + kContMaxRows + 15 + 15) / 16;

// A task: {gx, gy, meta, n} and the byte offsets of x and y in their arenas.
struct LongRec {
    uint4 a;        // gx, gy, meta (p, i, l), n = |x|
    uint4 b;        // x offset (lo, hi), y offset (lo, hi)
};
// A task that continues: the task, the rows done, its band row as bytes.
struct ContRec {
    LongRec rec;
    uint4 st[3];    // st[0].x = rows done; bytes 4 .. 4 + kContW - 1 = min(M[k], t + 1)
};

// per slot (i - 1): number of candidates of the small-list hits
__global__ __launch_bounds__(kBlock) void k_long_slot_counts(const Hit* __restrict__ hits, uint64_t nh,
                                                             uint32_t* __restrict__ slot_cnt)
{
    __shared__ uint32_t s_cnt[64];
    if (threadIdx.x < 64) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    for (uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x; k < nh;
         k += (uint64_t)gridDim.x * kBlock)
        atomicAdd(&s_cnt[(hits[k].meta >> 11) & 63u], hits[k].count);
    __syncthreads();
    if (threadIdx.x < 64 && s_cnt[threadIdx.x]) atomicAdd(&slot_cnt[threadIdx.x], s_cnt[threadIdx.x]);
}

// one wave: exclusive scan of the 64 slot counts into off[0..64], cursor = off
__global__ void k_long_slot_offsets(const uint32_t* __restrict__ slot_cnt, uint32_t* __restrict__ off,
                                    uint32_t* __restrict__ cursor)
{
    const int lane = threadIdx.x;
    const uint32_t c = slot_cnt[lane];
    const uint32_t incl = wave_incl_scan(c);
    off[lane] = incl - c;
    cursor[lane] = incl - c;
    if (lane == 63) off[64] = incl;
}

// Candidates of the small-list hits to their slots' regions.  A block walks a contiguous range
// of hits twice: first counting its candidates per slot in LDS, then, after reserving each
// slot's share with one global atomic, writing them (a global atomic per hit on the 64 slot
// cursors would serialise).
__global__ __launch_bounds__(kBlock) void k_long_scatter(const Hit* __restrict__ hits, uint64_t nh,
                                                         const uint32_t* __restrict__ vals,
                                                         const uint16_t* __restrict__ x_slen,
                                                         const int32_t* __restrict__ x_lenstart,
                                                         const int64_t* __restrict__ x_gbase,
                                                         const int32_t* __restrict__ y_lenstart,
                                                         const int64_t* __restrict__ y_gbase,
                                                         uint32_t* __restrict__ cursor,
                                                         LongRec* __restrict__ cands)
{
    __shared__ uint32_t s_cnt[64];
    __shared__ uint32_t s_pos[64];
    const uint64_t per = (nh + gridDim.x - 1) / gridDim.x;
    const uint64_t h0 = (uint64_t)blockIdx.x * per;
    const uint64_t h1 = min(h0 + per, nh);
    if (threadIdx.x < 64) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    for (uint64_t k = h0 + threadIdx.x; k < h1; k += kBlock) {
        const Hit h = hits[k];
        atomicAdd(&s_cnt[(h.meta >> 11) & 63u], h.count);
    }
    __syncthreads();
    if (threadIdx.x < 64)
        s_pos[threadIdx.x] = s_cnt[threadIdx.x] ? atomicAdd(&cursor[threadIdx.x], s_cnt[threadIdx.x]) : 0u;
    __syncthreads();
    for (uint64_t k = h0 + threadIdx.x; k < h1; k += kBlock) {
        const Hit h = hits[k];
        const int n = x_slen[h.gx];
        const int l = (int)(h.meta >> 17);
        const uint64_t xo = (uint64_t)(x_gbase[n] + (int64_t)(h.gx - x_lenstart[n]) * stride_of(n));
        const uint32_t base = atomicAdd(&s_pos[(h.meta >> 11) & 63u], h.count);
        for (uint32_t m = 0; m < h.count; ++m) {
            const uint32_t gy = vals[h.start + m];
            const uint64_t yo = (uint64_t)(y_gbase[l] + (int64_t)(gy - y_lenstart[l]) * stride_of(l));
            LongRec r;
            r.a = make_uint4(h.gx, gy, h.meta, (uint32_t)n);
            r.b = make_uint4((uint32_t)xo, (uint32_t)(xo >> 32), (uint32_t)yo, (uint32_t)(yo >> 32));
            cands[base + m] = r;
        }
    }
}

// The tasks [b0, b1) of one slot for one wave (one task per lane): up to K rows of each task's
// part DP on M values in diagonal coordinates (band index k holds column j = i - a + k of row i;
// up = index k + 1, left = k - 1 of this row, diagonal = k; cells outside the band or left of
// column 0 start large and only see large inputs, so column 0 follows from the recurrence;
// indices right of column nc never feed a cell inside the matrix).  The expected distance of
// index k is M + |b - k| (b = a + Delta, the final cell's index); a row whose smallest one
// exceeds t stops the DP (Lemma 4).  The characters come from the lane's LDS stage (element q at
// stage[q * 64]): A[row + q] for q < kContMaxRows, then B[row - a + q] (256 outside B).
template <int MAXW>
__device__ inline void cont_chunk(const VerifyParams& V, const Div& div, int side, int slot,
                                  bool fresh, const LongRec* __restrict__ fin,
                                  const ContRec* __restrict__ cin, uint32_t b0, uint32_t b1, int K,
                                  ContRec* __restrict__ cout, uint32_t* __restrict__ cout_cnt,
                                  LongRec* __restrict__ rout, uint32_t* __restrict__ rout_cnt,
                                  uint32_t qbase,
                                  __attribute__((address_space(3))) uint32_t* stage32,
                                  WaveAppender<uint64_t, kAppendCap>& acc, uint64_t& my_cells,
                                  uint64_t& my_miss)
{
    constexpr int BIG = 1 << 20;
    const int lane = threadIdx.x & 63;
    // the lane's 16-byte blocks: block q at byte (q * 64 + lane) * 16 of the wave's stage
    const __attribute__((address_space(3))) uint8_t* stage8 =
        (const __attribute__((address_space(3))) uint8_t*)stage32;
    const int i = slot + 1;
    const int t = side == 0 ? i - 1 : V.tau + 1 - i;
    const uint32_t k = b0 + (uint32_t)lane;
    bool act = k < b1;
    LongRec rec;
    rec.a = make_uint4(0u, 0u, 0u, 0u);
    rec.b = rec.a;
    int M[MAXW];                                          // every lane runs the row loop
#pragma unroll
    for (int q = 0; q < MAXW; ++q) M[q] = BIG;
    int row = 0, nr = 0, nc = 0, a = 0, b = 0, st = 0;    // st: 0 running, 1 pass, 2 fail, 3 none
    const uint8_t* A = nullptr;
    const uint8_t* B = nullptr;
    const uint8_t* A_end = nullptr;     // end of the padded slot of A's / B's string
    const uint8_t* B_end = nullptr;
    if (act) {
        ContRec cr;
        if (fresh) rec = fin[k];
        else { cr = cin[k]; rec = cr.rec; }
        const uint32_t meta = rec.a.z;
        const int p = (int)(meta & 2047u) + 1;
        const int l = (int)(meta >> 17);
        const int n = (int)rec.a.w;
        const uint8_t* x = V.x_arena + ((uint64_t)rec.b.y << 32 | rec.b.x);
        const uint8_t* y = V.y_arena + ((uint64_t)rec.b.w << 32 | rec.b.z);
        const Seg sg = partition_seg(l, i, V.tau, div);
        const uint8_t* r = side == 0 ? y : y + sg.p - 1 + sg.len;
        const uint8_t* s = side == 0 ? x : x + p - 1 + sg.len;
        const int lr = side == 0 ? sg.p - 1 : l - (sg.p - 1 + sg.len);
        const int ls = side == 0 ? p - 1 : n - (p - 1 + sg.len);
        const uint8_t* yend = y + stride_of(l);
        const uint8_t* xend = x + stride_of(n);
        if (lr <= ls) { A = r; nr = lr; B = s; nc = ls; A_end = yend; B_end = xend; }
        else          { A = s; nr = ls; B = r; nc = lr; A_end = xend; B_end = yend; }
        const int delta = nc - nr;
        a = (t - delta) >> 1;
        b = (t + delta) >> 1;
        if (fresh) {
            bool ok = true;
            if (side == 0 && sg.len > V.exact_len) {
                for (int q = 0; q < sg.len; ++q) ok &= (x[p - 1 + q] == y[sg.p - 1 + q]);
                if (!ok) my_miss += 1;
            }
            if (!ok) st = 3;                               // not a candidate
            else if (delta > t) st = 2;                    // no row
            else if (nr == 0) st = (nc <= t) ? 1 : 2;
#pragma unroll
            for (int q = 0; q < MAXW; ++q) {
                const int j = q - a;
                M[q] = (j >= 0 && j <= min(nc, b)) ? j : BIG;
            }
        } else {
            row = (int)cr.st[0].x;
            const uint32_t wv[12] = {cr.st[0].x, cr.st[0].y, cr.st[0].z, cr.st[0].w,
                                     cr.st[1].x, cr.st[1].y, cr.st[1].z, cr.st[1].w,
                                     cr.st[2].x, cr.st[2].y, cr.st[2].z, cr.st[2].w};
#pragma unroll
            for (int q = 0; q < MAXW; ++q) M[q] = (int)((wv[1 + q / 4] >> (8 * (q % 4))) & 255u);
        }
    }
    // the pass's rows in sub-blocks of kContMaxRows: each stages its characters (the 16-byte
    // blocks holding A[row .. row + 64) and B[max(row - a, 0) .. row - a + MAXW + 64), each block
    // only if it starts inside its string's padded slot, 16-byte aligned; all loads are issued
    // before the first LDS write) and runs its rows
    const bool run = act && st == 0;
    bool running = run;
    for (int sub = 0; sub < K; sub += kContMaxRows) {
        if (__ballot(running) == 0) break;
        const int Ks = min(kContMaxRows, K - sub);
        int oA = 0, oB = 0, ib0 = 0;
        // the previous sub-block's LDS reads were issued before these writes (in order)
        if (running) {
            const uint8_t* pa = A + row;
            const uint8_t* pa0 = (const uint8_t*)((uintptr_t)pa & ~(uintptr_t)15);
            oA = (int)(pa - pa0);
            ib0 = max(row - a, 0);
            const uint8_t* pb = B + ib0;
            const uint8_t* pb0 = (const uint8_t*)((uintptr_t)pb & ~(uintptr_t)15);
            oB = (int)(pb - pb0);
            uint4 va[kStageA], vb[kStageB];
#pragma unroll
            for (int q = 0; q < kStageA; ++q)
                va[q] = (pa0 + 16 * q < A_end) ? reinterpret_cast<const uint4*>(pa0)[q] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
            for (int q = 0; q < kStageB; ++q)
                vb[q] = (pb0 + 16 * q < B_end) ? reinterpret_cast<const uint4*>(pb0)[q] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
            for (int q = 0; q < kStageA; ++q) {
                stage32[q * 256 + 0] = va[q].x; stage32[q * 256 + 1] = va[q].y;
                stage32[q * 256 + 2] = va[q].z; stage32[q * 256 + 3] = va[q].w;
            }
#pragma unroll
            for (int q = 0; q < kStageB; ++q) {
                const int o = (kStageA + q) * 256;
                stage32[o + 0] = vb[q].x; stage32[o + 1] = vb[q].y;
                stage32[o + 2] = vb[q].z; stage32[o + 3] = vb[q].w;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        {
            // every lane runs the rows of the sub-block, so the loop's control flow stays
            // wave-uniform (a lane's own exit would make the compiler copy the band and the
            // window at every row); a lane that is not running, or stops, computes rows whose
            // values are never used, and its reads stay inside its stage (ncs = 0: no column
            // byte is read)
            const int ncs = running ? nc : 0;
            // byte q of the lane's A blocks / B blocks (lane-interleaved 16-byte blocks)
            auto sa = [&](int q) -> int { return (int)stage8[((q >> 4) * 64) * 16 + (q & 15)]; };
            auto sb = [&](int ib) -> int {             // B[ib], 256 outside B
                const int q = oB + ib - ib0;
                return ((unsigned)ib < (unsigned)ncs)
                           ? (int)stage8[((kStageA + (q >> 4)) * 64) * 16 + (q & 15)] : 256;
            };
            // the window of rows r and r + 1: w[q] = B[rowstart + r - a + q], q <= MAXW (rows
            // taken in pairs, so the window shifts by two every second row)
            int w[MAXW + 1];
#pragma unroll
            for (int q = 0; q <= MAXW; ++q) w[q] = sb(row - a + q);
            const int rowstart = row;
            bool live = running;                       // the lane's rows still count
            // row r of the sub-block on the window w[O .. O + MAXW); false once no lane counts
            auto step = [&](int r, auto o) -> bool {
                constexpr int O = decltype(o)::value;
                const int ai = sa(oA + r);
                int left = BIG, emin = BIG;
#pragma unroll
                for (int q = 0; q < MAXW; ++q) {
                    const int up = (q + 1 < MAXW) ? M[(q + 1) < MAXW ? q + 1 : q] : BIG;
                    // min(up + 1, left + 1, diagonal + [mismatch]) as one three-way min of
                    // up, left and diagonal - [match], plus one
                    const int dm = M[q] - ((ai == w[q + O]) ? 1 : 0);
                    const int v = min(min(up, left), dm) + 1;
                    M[q] = v;
                    left = v;
                    const uint32_t ub = (uint32_t)b, uq = (uint32_t)q;
                    emin = min(emin, (int)(max(ub, uq) - min(ub, uq) + (uint32_t)v));
                }
                const int nrow = rowstart + r + 1;
                const bool fail = emin > t;            // Lemma 4: stop, return t + 1
                const bool last = nrow == nr;
                row = live ? nrow : row;
                // the final cell (band index b) only on a row where some lane ends
                int out = BIG;
                if (__ballot(live && !fail && last)) {
#pragma unroll
                    for (int q = 0; q < MAXW; ++q) out = (q == b) ? M[q] : out;
                }
                const int nst = fail ? 2 : last ? (out <= t ? 1 : 2) : 0;
                st = live ? nst : st;
                live = live && nst == 0;
                return __ballot(live) != 0;
            };
            for (int r = 0; r < Ks; r += 2) {
                if (!step(r, std::integral_constant<int, 0>{})) break;
                if (r + 1 >= Ks || !step(r + 1, std::integral_constant<int, 1>{})) break;
                if (r + 2 >= Ks) break;
#pragma unroll
                for (int q = 0; q + 1 < MAXW; ++q) w[q] = w[q + 2];
                w[MAXW - 1] = sb(rowstart - a + MAXW + r + 1);
                w[MAXW] = sb(rowstart - a + MAXW + r + 2);
            }
            running = st == 0;
        }
    }
    if (run && (st == 1 || st == 2)) my_cells += (uint64_t)band_cells(row, nc, a, b);
    // outcomes
    const bool cont = run && st == 0;
    {
        const uint64_t m = __ballot(cont);
        if (m) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(&cout_cnt[slot], (uint32_t)__popcll(m));
            base = __shfl(base, 0, 64);
            if (cont) {
                ContRec c;
                c.rec = rec;
                uint32_t wds[12];
                wds[0] = (uint32_t)row;
#pragma unroll
                for (int q = 1; q < 12; ++q) wds[q] = 0;
#pragma unroll
                for (int q = 0; q < MAXW; ++q) {
                    const uint32_t v = (uint32_t)min(M[q], t + 1);
                    wds[1 + q / 4] |= v << (8 * (q % 4));
                }
                c.st[0] = make_uint4(wds[0], wds[1], wds[2], wds[3]);
                c.st[1] = make_uint4(wds[4], wds[5], wds[6], wds[7]);
                c.st[2] = make_uint4(wds[8], wds[9], wds[10], wds[11]);
                cout[qbase + base + (uint32_t)__popcll(m & lanemask_lt())] = c;
            }
        }
    }
    if (side == 0) {
        const bool pass = act && st == 1;
        const uint64_t m = __ballot(pass);
        if (m) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(&rout_cnt[slot], (uint32_t)__popcll(m));
            base = __shfl(base, 0, 64);
            if (pass) rout[qbase + base + (uint32_t)__popcll(m & lanemask_lt())] = rec;
        }
    } else {
        acc.push(act && st == 1, ((uint64_t)rec.a.x << 32) | rec.a.y, V.out, V.out_cap,
                 &V.counters[3]);
    }
}

// One pass over the tasks of both sides, so that a candidate's right part starts in the pass
// after its left part passes and runs beside the other candidates' left parts.  Three groups of
// tasks, each in per-slot regions that start at off[slot]:
//  0: left parts (side 0), fresh from fin_l (counts cnt_l; the first pass) or continuing from
//     cin_l (counts cnt_l); cnt_l null when no left part is left;
//  1: right parts new in this pass: fin_r[lo_r[slot], hi_r[slot]) (lo_r null: none);
//  2: right parts continuing from cin_r (counts cnt_r; null: none).
// Continuing tasks go to cout_l / cout_r (counts cout_l_cnt / cout_r_cnt); left parts that pass
// are appended to rout (counts rout_cnt), right parts that pass to the pair buffer.
struct ContPass {
    const LongRec* fin_l;
    const ContRec* cin_l;
    const uint32_t* cnt_l;
    const LongRec* fin_r;
    const uint32_t* lo_r;
    const uint32_t* hi_r;
    const ContRec* cin_r;
    const uint32_t* cnt_r;
    const uint32_t* off;
    ContRec* cout_l;
    uint32_t* cout_l_cnt;
    ContRec* cout_r;
    uint32_t* cout_r_cnt;
    LongRec* rout;
    uint32_t* rout_cnt;
    uint32_t* zero_l;        // count buffers the next pass writes (read by the previous pass
    uint32_t* zero_r;        // only): cleared here
    int K;
};

__global__ __launch_bounds__(64) void k_verify_cont(VerifyParams V, Div div, ContPass P)
{
    if (blockIdx.x == 0) {
        if (P.zero_l) P.zero_l[threadIdx.x] = 0u;
        if (P.zero_r) P.zero_r[threadIdx.x] = 0u;
    }
    __shared__ uint64_t s_acc[kAppendCap];
    __shared__ uint4 s_stage[(kStageA + kStageB) * 64];
    WaveAppender<uint64_t, kAppendCap> acc{s_acc, 0};
    const int lane = threadIdx.x & 63;
    __attribute__((address_space(3))) uint32_t* stage =
        (__attribute__((address_space(3))) uint32_t*)s_stage + 4 * lane;
    uint64_t my_cells = 0, my_miss = 0;
    // chunks of 64 tasks: group 0's slots, then group 1's, then group 2's (lane = slot)
    const bool sl = lane <= V.tau;
    const uint32_t c0 = (sl && P.cnt_l) ? P.cnt_l[lane] : 0u;
    const uint32_t c1 = (sl && P.lo_r) ? P.hi_r[lane] - P.lo_r[lane] : 0u;
    const uint32_t c2 = (sl && P.cnt_r) ? P.cnt_r[lane] : 0u;
    const uint32_t n0 = (c0 + 63u) / 64u, n1 = (c1 + 63u) / 64u, n2 = (c2 + 63u) / 64u;
    const uint32_t i0 = wave_incl_scan(n0), i1 = wave_incl_scan(n1), i2 = wave_incl_scan(n2);
    const uint32_t T0 = __shfl(i0, 63, 64), T1 = __shfl(i1, 63, 64), T2 = __shfl(i2, 63, 64);
    const uint32_t total = T0 + T1 + T2;
    for (uint32_t ch = blockIdx.x; ch < total; ch += gridDim.x) {
        const int g = ch < T0 ? 0 : (ch < T0 + T1 ? 1 : 2);
        const uint32_t loc = g == 0 ? ch : (g == 1 ? ch - T0 : ch - T0 - T1);
        const uint32_t incl = g == 0 ? i0 : (g == 1 ? i1 : i2);
        const uint32_t nch = g == 0 ? n0 : (g == 1 ? n1 : n2);
        const uint32_t cc = g == 0 ? c0 : (g == 1 ? c1 : c2);
        const int slot = __popcll(__ballot(incl <= loc));
        const uint32_t first = __shfl(incl - nch, slot, 64);
        const uint32_t cs = __shfl(cc, slot, 64);
        const uint32_t base = P.off[slot];
        const uint32_t b0 = (loc - first) * 64u;
        const uint32_t b1 = min(b0 + 64u, cs);
        const int side = g == 0 ? 0 : 1;
        const bool fresh = g == 0 ? P.cin_l == nullptr : g == 1;
        const LongRec* fi = g == 0 ? (fresh ? P.fin_l + base : nullptr)
                                   : (g == 1 ? P.fin_r + base + P.lo_r[slot] : nullptr);
        const ContRec* ci = g == 0 ? (fresh ? nullptr : P.cin_l + base)
                                   : (g == 2 ? P.cin_r + base : nullptr);
        ContRec* cout = side == 0 ? P.cout_l : P.cout_r;
        uint32_t* cout_cnt = side == 0 ? P.cout_l_cnt : P.cout_r_cnt;
        const int t = side == 0 ? slot : V.tau - slot;
#define PJ_CONT(W) cont_chunk<W>(V, div, side, slot, fresh, fi, ci, b0, b1, P.K, cout, cout_cnt,  \
                                 P.rout, P.rout_cnt, base, stage, acc, my_cells, my_miss)
        if (t + 1 <= 5) PJ_CONT(5);
        else if (t + 1 <= 9) PJ_CONT(9);
        else if (t + 1 <= 13) PJ_CONT(13);
        else if (t + 1 <= 17) PJ_CONT(17);
        else if (t + 1 <= 21) PJ_CONT(21);
        else if (t + 1 <= 25) PJ_CONT(25);
        else if (t + 1 <= 29) PJ_CONT(29);
        else PJ_CONT(33);
#undef PJ_CONT
    }
    acc.flush(V.out, V.out_cap, &V.counters[3]);
    my_cells = wave_sum(my_cells);
    my_miss = wave_sum(my_miss);
    if (lane == 0) {
        if (my_cells) atomicAdd(&V.counters[4], (unsigned long long)my_cells);
        if (my_miss) atomicAdd(&V.counters[5], (unsigned long long)my_miss);
    }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, int n, uint32_t v)
{
    for (int k = threadIdx.x; k < n; k += blockDim.x) p[k] = v;
}

template <int MAXW>
__global__ __launch_bounds__(kBlock) void k_short(const uint8_t* __restrict__ x_arena,
                                                  const uint16_t* __restrict__ x_slen,
                                                  const int32_t* __restrict__ x_lenstart,
                                                  const int64_t* __restrict__ x_gbase,
                                                  int x_lmax,
                                                  const uint8_t* __restrict__ y_arena,
                                                  const uint16_t* __restrict__ y_slen,
                                                  const int32_t* __restrict__ y_lenstart,
                                                  const int64_t* __restrict__ y_gbase,
                                                  uint32_t y_first, uint32_t y_count, int tau,
                                                  int self, const int32_t* __restrict__ q_tau,
                                                  uint64_t* __restrict__ out,
                                                  uint64_t out_cap,
                                                  unsigned long long* __restrict__ counters)
{
    const int lane = threadIdx.x & 63;
    for (uint32_t yi = blockIdx.x; yi < y_count; yi += gridDim.x) {
        const uint32_t gy = y_first + yi;
        const int ly = y_slen[gy];
        const uint8_t* y = y_arena + y_gbase[ly] + (int64_t)(gy - y_lenstart[ly]) * stride_of(ly);
        const int lo_len = ly - tau < 0 ? 0 : ly - tau;
        int hi_len = ly + tau;
        if (hi_len > x_lmax) hi_len = x_lmax;
        if (hi_len < lo_len) continue;
        const uint32_t g0 = (uint32_t)x_lenstart[lo_len], g1 = (uint32_t)x_lenstart[hi_len + 1];
        uint64_t examined = 0;
        for (uint32_t base = g0; base < g1; base += kBlock) {
            uint32_t gx = base + threadIdx.x;
            bool pass = false;
            if (gx < g1) {
                const int lx = x_slen[gx];
                const int tx = q_tau ? q_tau[gx] : tau;      // the pair's threshold
                const int dlen = lx > ly ? lx - ly : ly - lx;
                bool take = ly <= tx && dlen <= tx && !(self && lx <= tau && gx >= gy);
                if (take) {
                    const uint8_t* x = x_arena + x_gbase[lx] +
                                       (int64_t)(gx - x_lenstart[lx]) * stride_of(lx);
                    int c = 0;
                    pass = vsp_global<MAXW>(y, ly, x, lx, tx, &c) <= tx;
                    examined += 1;
                }
            }
            uint64_t pm = __ballot(pass);
            if (pm) {
                int leader = __ffsll((unsigned long long)pm) - 1;
                unsigned long long b = 0;
                if (lane == leader) b = atomicAdd(&counters[3], (unsigned long long)__popcll(pm));
                b = __shfl(b, leader, 64);
                if (pass) {
                    uint64_t idx = b + (uint64_t)__popcll(pm & lanemask_lt());
                    if (idx < out_cap) out[idx] = ((uint64_t)gx << 32) | gy;
                }
            }
        }
        examined = wave_sum(examined);
        if (lane == 0 && examined) atomicAdd(&counters[6], (unsigned long long)examined);
    }
}

// ------------------------------------------------------------------------------------------
// Output: map accepted (gx, gy) to ids, sort, deduplicate (the result is a set, Algorithm 1)
// ------------------------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_pairs_to_keys(const uint64_t* __restrict__ acc,
                                                          uint64_t m,
                                                          const int32_t* __restrict__ xperm,
                                                          const int32_t* __restrict__ yperm,
                                                          int self, int bbits,
                                                          uint64_t* __restrict__ keys)
{
    uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= m) return;
    uint64_t v = acc[k];
    uint32_t a = (uint32_t)xperm[v >> 32];
    uint32_t b = (uint32_t)yperm[v & 0xffffffffu];
    if (self && b < a) { uint32_t t = a; a = b; b = t; }
    keys[k] = ((uint64_t)a << bbits) | b;
}

__global__ __launch_bounds__(kBlock) void k_unique_flags(const uint64_t* __restrict__ keys,
                                                         uint64_t m, uint32_t* __restrict__ flags)
{
    uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < m) flags[k] = (k == 0 || keys[k] != keys[k - 1]) ? 1u : 0u;
}

__global__ __launch_bounds__(kBlock) void k_compact_pairs(const uint64_t* __restrict__ keys,
                                                          const uint32_t* __restrict__ flags,
                                                          const uint32_t* __restrict__ pos,
                                                          uint64_t m, int bbits,
                                                          int32_t* __restrict__ a,
                                                          int32_t* __restrict__ b)
{
    uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < m && flags[k]) {
        uint64_t v = keys[k];
        a[pos[k]] = (int32_t)(v >> bbits);
        b[pos[k]] = (int32_t)(v & ((1ull << bbits) - 1));
    }
}

// out[g] = in[perm[g]]: per-id values (a query's tau) moved to sorted positions.
__global__ __launch_bounds__(kBlock) void k_gather_i32(const int32_t* __restrict__ in,
                                                       const int32_t* __restrict__ perm, int64_t n,
                                                       int32_t* __restrict__ out)
{
    int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g < n) out[g] = in[perm[g]];
}

// ------------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------------

static inline unsigned blocks_for(uint64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

hipError_t launch_length_hist(const int32_t* offs, int64_t n, int32_t* lcount, int32_t* err,
                              hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_length_hist, dim3(blocks_for(n)), dim3(kBlock), 0, s, offs, n, lcount, err);
    return hipGetLastError();
}

hipError_t launch_iota_len_keys(const int32_t* offs, int64_t n, uint32_t* keys, uint32_t* vals,
                                hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_len_keys, dim3(blocks_for(n)), dim3(kBlock), 0, s, offs, n, keys, vals);
    return hipGetLastError();
}

hipError_t launch_pack_arena(const uint8_t* bytes, const int32_t* offs, const int32_t* perm,
                             int64_t n, const int32_t* lenstart, const int64_t* gbase,
                             uint8_t* sarena, uint16_t* slen, int lmax, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t widest = stride_of(std::max(lmax, 0));
    const int lps_shift = widest <= 64 ? 4 : widest <= 128 ? 5 : 6;
    const uint64_t threads = (uint64_t)n << lps_shift;
    uint64_t blocks = (threads + kBlock - 1) / kBlock;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_pack_arena, dim3((unsigned)blocks), dim3(kBlock), 0, s, bytes, offs, perm,
                       n, lenstart, gbase, sarena, slen, lps_shift);
    return hipGetLastError();
}

hipError_t launch_byte_presence(const DevSet& S, uint32_t* bitmap, hipStream_t s)
{
    if (S.n == 0) return hipSuccess;
    const uint64_t nchunks = (uint64_t)S.arena_bytes >> 4;
    if (nchunks == 0) return hipSuccess;
    const unsigned grid = (unsigned)std::min<uint64_t>(blocks_for(nchunks), 2048);
    hipLaunchKernelGGL(k_byte_presence, dim3(grid), dim3(kBlock), 0, s, S.sarena, S.gbase,
                       (int64_t)S.arena_bytes, bitmap);
    return hipGetLastError();
}

hipError_t launch_emit_segments(const DevSet& S, int tau, const int64_t* ebase_dev,
                                int64_t g_first, int64_t g_count, const SymMap& sym,
                                uint64_t* keys, uint32_t* vals, hipStream_t s)
{
    if (g_count <= 0) return hipSuccess;
    if (!sym.code || sym.bits < 1 || sym.bits > 9 || sym.exact_len * sym.bits > kHashBits)
        return hipErrorInvalidValue;
    uint64_t threads = (uint64_t)g_count * (tau + 1);
    hipLaunchKernelGGL(k_emit_segments, dim3(blocks_for(threads)), dim3(kBlock), 0, s, S.sarena,
                       S.slen, S.lenstart, S.gbase, ebase_dev, tau, g_first, g_count,
                       make_div(tau + 1), sym, keys, vals);
    return hipGetLastError();
}

hipError_t launch_mark_heads(const uint64_t* keys, int64_t E, uint32_t* flags, hipStream_t s)
{
    if (E <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mark_heads, dim3(blocks_for(E)), dim3(kBlock), 0, s, keys, E, flags);
    return hipGetLastError();
}

hipError_t launch_gather_inline(const DevSet& S, const uint64_t* keys, const uint32_t* vals,
                                int64_t E, int tau, const int64_t* inl_base, uint8_t* inl,
                                hipStream_t s)
{
    if (E <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_inline, dim3(blocks_for(E)), dim3(kBlock), 0, s, keys, vals, E,
                       tau, S.sarena, S.lenstart, S.gbase, inl_base, inl);
    return hipGetLastError();
}

hipError_t launch_clear_table(uint4* table, uint64_t slots, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_table, dim3(blocks_for(slots)), dim3(kBlock), 0, s, table, slots);
    return hipGetLastError();
}

hipError_t launch_scatter_runstart(const uint32_t* flags, const uint32_t* runid, int64_t E,
                                   uint32_t* runstart, hipStream_t s)
{
    if (E <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_runstart, dim3(blocks_for(E)), dim3(kBlock), 0, s, flags, runid, E,
                       runstart);
    return hipGetLastError();
}

hipError_t launch_filter_build(const uint64_t* keys, const uint32_t* runstart, uint32_t nruns,
                               uint32_t ngroups, uint32_t* gfirst, uint32_t* gend, uint32_t* words,
                               void* scan_tmp, size_t scan_bytes, uint32_t* filter_dir,
                               uint32_t* filter, hipStream_t s)
{
    if (ngroups == 0) return hipSuccess;
    if (nruns > 0)
        hipLaunchKernelGGL(k_filter_group_bounds, dim3(blocks_for(nruns)), dim3(kBlock), 0, s, keys,
                           runstart, nruns, gfirst, gend);
    hipLaunchKernelGGL(k_filter_block_words, dim3(blocks_for(ngroups)), dim3(kBlock), 0, s, gfirst,
                       gend, ngroups, words);
    hipError_t e = scan_u32_to_u32(words, filter_dir, ngroups, scan_tmp, scan_bytes, s);
    if (e != hipSuccess) return e;
    if (nruns > 0)
        hipLaunchKernelGGL(k_filter_keys, dim3(blocks_for(nruns)), dim3(kBlock), 0, s, keys,
                           runstart, nruns, filter_dir, filter);
    return hipGetLastError();
}

hipError_t launch_insert_runs(const uint64_t* keys, const uint32_t* runstart, uint32_t nruns,
                              uint32_t E, uint4* table, uint64_t mask, hipStream_t s)
{
    if (nruns == 0) return hipSuccess;
    hipLaunchKernelGGL(k_insert_runs, dim3(blocks_for(nruns)), dim3(kBlock), 0, s, keys, runstart,
                       nruns, E, table, mask);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_hit_counts(const Hit* __restrict__ hits, uint64_t nh,
                                                       uint32_t* __restrict__ counts)
{
    uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < nh) counts[k] = hits[k].count;
}

hipError_t launch_hit_counts(const Hit* hits, uint64_t nh, uint32_t* counts, hipStream_t s)
{
    if (nh == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hit_counts, dim3(blocks_for(nh)), dim3(kBlock), 0, s, hits, nh, counts);
    return hipGetLastError();
}

// Multi-match window size of slot i for a length difference delta = n - l (Sec. 4.2: the
// start positions p_i - (i-1) .. p_i + (i-1) intersected with p_i + delta - (tau+1-i) ..
// p_i + delta + (tau+1-i)), 0 when empty
__device__ inline int mm_window_size(int tau, int i, int delta)
{
    const int r = tau + 1 - i;
    const int a = (i - 1) < delta + r ? (i - 1) : delta + r;
    const int b = (i - 1) < r - delta ? (i - 1) : r - delta;
    const int sz = a + b + 1;
    return sz > 0 ? sz : 0;
}

// One block: the (length, slot) pairs of a probe string grouped by decreasing window size
// (a counting sort on the size; the order within a size is whatever the atomics give).  Pairs
// of one size take equally many steps of the probe's window walk, so a wave whose lanes hold
// them keeps all its lanes busy.
__global__ __launch_bounds__(kBlock) void k_probe_order(int tau, int nl, int self,
                                                        uint16_t* __restrict__ order)
{
    constexpr int kSizes = 2 * kTauMax + 2;      // window sizes 0 .. 2 tau + 1
    __shared__ uint32_t cnt[kSizes];
    const int T1 = tau + 1, per = nl * T1;
    auto size_of = [&](int r) {
        const int dl = r / T1, i = r % T1 + 1;
        return mm_window_size(tau, i, self ? dl : tau - dl);
    };
    for (int k = threadIdx.x; k < kSizes; k += kBlock) cnt[k] = 0;
    __syncthreads();
    for (int r = threadIdx.x; r < per; r += kBlock) atomicAdd(&cnt[size_of(r)], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int k = kSizes - 1; k >= 0; --k) {
            const uint32_t c = cnt[k];
            cnt[k] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int r = threadIdx.x; r < per; r += kBlock)
        order[atomicAdd(&cnt[size_of(r)], 1u)] = (uint16_t)r;
}

hipError_t launch_probe_order(int tau, int nl, int self, uint16_t* order, hipStream_t s)
{
    if (tau < 0 || tau > kTauMax || nl < 1 || nl > 2 * kTauMax + 1 || !order)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_probe_order, dim3(1), dim3(kBlock), 0, s, tau, nl, self, order);
    return hipGetLastError();
}

hipError_t launch_probe(const ProbeParams& P, int max_blocks, hipStream_t s)
{
    if (P.threads == 0) return hipSuccess;
    if (!P.sym.code) return hipErrorInvalidValue;
    const uint64_t blocks = std::min<uint64_t>(blocks_for(P.threads), (uint64_t)max_blocks);
    if (P.xmajor) {
        if (P.q_tau || P.nx_dev || P.nx == 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_probe<true>, dim3((unsigned)blocks), dim3(kBlock), 0, s, P,
                           make_div(P.tau + 1));
    } else {
        hipLaunchKernelGGL(k_probe<false>, dim3((unsigned)blocks), dim3(kBlock), 0, s, P,
                           make_div(P.tau + 1));
    }
    return hipGetLastError();
}

template <int W>
static void verify_w(const VerifyParams& V, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((k_verify<W>), dim3(grid), dim3(kBlock), 0, s, V, make_div(V.tau + 1));
}

template <int W>
static void verify_batched_w(const VerifyParams& V, const uint32_t* first, uint64_t nchunks,
                             int grid, hipStream_t s)
{
    if (W == 9 && V.tau >= 6 && V.tau <= 8 && V.y_maxlen <= 40)
        hipLaunchKernelGGL((k_verify_batched<W, (W == 9 ? 2 : 0)>), dim3(grid), dim3(kBlock), 0,
                           s, V, make_div(V.tau + 1), first, nchunks);
    else if (W == 9 && V.tau <= 8 && V.y_maxlen <= kStgY - 4)
        hipLaunchKernelGGL((k_verify_batched<W, (W == 9 ? 1 : 0)>), dim3(grid), dim3(kBlock), 0,
                           s, V, make_div(V.tau + 1), first, nchunks);
    else
        hipLaunchKernelGGL((k_verify_batched<W, 0>), dim3(grid), dim3(kBlock), 0, s, V,
                           make_div(V.tau + 1), first, nchunks);
}

uint64_t batched_chunks(uint64_t ncand, int rounds)
{
    const uint64_t chunk = 64ull * (uint64_t)rounds;
    return (ncand + chunk - 1) / chunk;
}

unsigned slot_bucket_grid(uint64_t nh_cap)
{
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((nh_cap + kBlock - 1) / kBlock, 2048));
}

hipError_t launch_slot_bucket(const Hit* hits, const unsigned long long* nh_dev, uint64_t nh_cap,
                              uint32_t big, uint32_t* bb, uint32_t* bb_off, void* scan_tmp,
                              size_t scan_bytes, Hit* out, hipStream_t s)
{
    if (nh_cap == 0) return hipSuccess;
    const unsigned grid = slot_bucket_grid(nh_cap);
    hipLaunchKernelGGL(k_slot_hist, dim3(grid), dim3(kBlock), 0, s, hits, nh_dev, big, bb);
    hipError_t e = scan_u32_to_u32(bb, bb_off, (uint64_t)grid * kHitBuckets, scan_tmp, scan_bytes,
                                   s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_slot_scatter, dim3(grid), dim3(kBlock), 0, s, hits, nh_dev, big, bb_off,
                       out);
    return hipGetLastError();
}

template <int W, int NC>
static void verify_segs_wn(const VerifyParams& V, const Hit* big, const uint32_t* segp,
                           uint64_t nbig, uint64_t nseg, const uint32_t* first, uint64_t nchunks,
                           uint32_t chunk, int grid, hipStream_t s)
{
    // one candidate per lane with strings of at most 40 bytes: 44-byte lane slots, so that 8
    // blocks fit a CU's LDS
    if (NC == 1 && W <= 9 && V.y_maxlen <= 40)
        hipLaunchKernelGGL((k_verify_segs<W, (NC == 1 && W <= 9) ? 40 : 48, NC>), dim3(grid),
                           dim3(kBlock), 0, s, V, make_div(V.tau + 1), big, segp, nbig, nseg,
                           first, nchunks, chunk);
    else if (V.y_maxlen <= 48)
        hipLaunchKernelGGL((k_verify_segs<W, 48, NC>), dim3(grid), dim3(kBlock), 0, s, V,
                           make_div(V.tau + 1), big, segp, nbig, nseg, first, nchunks, chunk);
    else if (V.y_maxlen <= 64)
        hipLaunchKernelGGL((k_verify_segs<W, 64, NC>), dim3(grid), dim3(kBlock), 0, s, V,
                           make_div(V.tau + 1), big, segp, nbig, nseg, first, nchunks, chunk);
    else
        hipLaunchKernelGGL((k_verify_segs<W, 0, 1>), dim3(grid), dim3(kBlock), 0, s, V,
                           make_div(V.tau + 1), big, segp, nbig, nseg, first, nchunks, chunk);
}

template <int W>
static void verify_segs_w(const VerifyParams& V, const Hit* big, const uint32_t* segp,
                          uint64_t nbig, uint64_t nseg, const uint32_t* first, uint64_t nchunks,
                          uint32_t chunk, int lane_cands, int grid, hipStream_t s)
{
    if constexpr (W <= 9) {
        if (lane_cands == 2) {
            verify_segs_wn<W, 2>(V, big, segp, nbig, nseg, first, nchunks, chunk, grid, s);
            return;
        }
    }
    verify_segs_wn<W, 1>(V, big, segp, nbig, nseg, first, nchunks, chunk, grid, s);
}

uint64_t seg_chunks(uint64_t nseg, int chunk) { return (nseg + (uint64_t)chunk - 1) / (uint64_t)chunk; }

// members per list segment: 64 per candidate a lane takes (two per lane only when the indexed
// strings fit in registers and the band is at most 9 wide)
int seg_members(int y_maxlen, int tau, int lane_cands)
{
    return (lane_cands == 2 && y_maxlen <= 64 && tau + 1 <= 9) ? 128 : 64;
}

hipError_t launch_seg_counts(const Hit* big, uint64_t nbig, int members, uint32_t* segs,
                             hipStream_t s)
{
    if (nbig == 0) return hipSuccess;
    hipLaunchKernelGGL(k_seg_counts, dim3(blocks_for(nbig)), dim3(kBlock), 0, s, big, nbig,
                       (uint32_t)members, segs);
    return hipGetLastError();
}

hipError_t launch_verify_segs(const VerifyParams& V, const Hit* big, const uint32_t* segp,
                              uint64_t nbig, uint64_t nseg, uint32_t* first, int chunk,
                              int lane_cands, int grid, hipStream_t s)
{
    if (nbig == 0 || nseg == 0) return hipSuccess;
    if (chunk < 1 || grid < 1 || lane_cands < 1 || lane_cands > 2) return hipErrorInvalidValue;
    const uint64_t nchunks = seg_chunks(nseg, chunk);
    const uint32_t c = (uint32_t)chunk;
    hipLaunchKernelGGL(k_seg_chunk_starts, dim3(blocks_for(nchunks)), dim3(kBlock), 0, s, segp,
                       nbig, nchunks, c, first);
    const int w = V.tau + 1;
    const int lc = lane_cands;
    if (w <= 5) verify_segs_w<5>(V, big, segp, nbig, nseg, first, nchunks, c, lc, grid, s);
    else if (w <= 9) verify_segs_w<9>(V, big, segp, nbig, nseg, first, nchunks, c, lc, grid, s);
    else if (w <= 17) verify_segs_w<17>(V, big, segp, nbig, nseg, first, nchunks, c, lc, grid, s);
    else if (w <= 33) verify_segs_w<33>(V, big, segp, nbig, nseg, first, nchunks, c, lc, grid, s);
    else verify_segs_w<64>(V, big, segp, nbig, nseg, first, nchunks, c, lc, grid, s);
    return hipGetLastError();
}

hipError_t launch_chain_counts(const Hit* big, uint64_t nbig, const uint16_t* x_slen,
                               const uint32_t* runlen, int self, uint32_t* chains, hipStream_t s)
{
    if (nbig == 0) return hipSuccess;
    hipLaunchKernelGGL(k_chain_counts, dim3(blocks_for(nbig)), dim3(kBlock), 0, s, big, nbig,
                       x_slen, runlen, self, chains);
    return hipGetLastError();
}

hipError_t launch_verify_chains(const VerifyParams& V, const Hit* big,
                                const unsigned long long* cprefix, uint64_t nbig,
                                uint64_t nchains, uint32_t* first, int grid, hipStream_t s)
{
    if (nbig == 0 || nchains == 0) return hipSuccess;
    if (grid < 1 || V.tau + 1 > kShareMaxW || !V.svals || !V.runlen) return hipErrorInvalidValue;
    const uint64_t nchunks = (nchains + 63) / 64;
    hipLaunchKernelGGL(k_chunk_starts, dim3(blocks_for(nchunks)), dim3(kBlock), 0, s, cprefix,
                       nbig, nchunks, 64ull, first);
    const Div div = make_div(V.tau + 1);
    if (V.tau + 1 <= 5)
        hipLaunchKernelGGL((k_verify_chains<5>), dim3(grid), dim3(kBlock), 0, s, V, div, big,
                           cprefix, nbig, nchains, first, nchunks);
    else
        hipLaunchKernelGGL((k_verify_chains<9>), dim3(grid), dim3(kBlock), 0, s, V, div, big,
                           cprefix, nbig, nchains, first, nchunks);
    return hipGetLastError();
}

hipError_t launch_prefix8_keys(const DevSet& S, const uint32_t* vals, int64_t E, uint64_t* keys,
                               uint32_t* idx, hipStream_t s)
{
    if (E == 0) return hipSuccess;
    hipLaunchKernelGGL(k_prefix8_keys, dim3(blocks_for((uint64_t)E)), dim3(kBlock), 0, s, vals,
                       E, S.sarena, S.slen, S.lenstart, S.gbase, keys, idx);
    return hipGetLastError();
}

hipError_t launch_gather_keys(const uint64_t* keys, const uint32_t* idx, int64_t E,
                              uint64_t* out, hipStream_t s)
{
    if (E == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_keys, dim3(blocks_for((uint64_t)E)), dim3(kBlock), 0, s, keys,
                       idx, E, out);
    return hipGetLastError();
}

hipError_t launch_gather_vals(const uint32_t* vals, const uint32_t* idx, int64_t E, uint32_t* out,
                              hipStream_t s)
{
    if (E == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_vals, dim3(blocks_for((uint64_t)E)), dim3(kBlock), 0, s, vals,
                       idx, E, out);
    return hipGetLastError();
}

hipError_t launch_run_lengths(const uint32_t* runstart, uint32_t nruns, uint32_t E,
                              uint32_t* runlen, hipStream_t s)
{
    if (nruns == 0) return hipSuccess;
    hipLaunchKernelGGL(k_run_lengths, dim3(blocks_for(nruns)), dim3(kBlock), 0, s, runstart,
                       nruns, E, runlen);
    return hipGetLastError();
}

// count arrays of 256 u32: slot counts, offsets, cursors, right tasks, three left and three right
// continuation counts, two snapshots of the right-task counts
constexpr int kLongCounts = 12;

size_t long_scratch_bytes(uint64_t ncand)
{
    const uint64_t rc = (ncand * sizeof(LongRec) + 255) & ~(uint64_t)255;
    const uint64_t cc = (ncand * sizeof(ContRec) + 255) & ~(uint64_t)255;
    // candidates, right tasks, two left and two right continuation queues
    return kLongCounts * 256 * sizeof(uint32_t) + 2 * rc + 4 * cc;
}

__global__ void k_copy_u32(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src, int n)
{
    for (int k = threadIdx.x; k < n; k += blockDim.x) dst[k] = src[k];
}

hipError_t launch_verify_long(const VerifyParams& V, uint64_t ncand, int max_rows, void* scratch,
                              int grid, hipStream_t s)
{
    if (V.nhits == 0 || ncand == 0) return hipSuccess;
    if (V.tau + 1 > kContW || grid < 1 || V.q_tau || max_rows < 0) return hipErrorInvalidValue;
    uint8_t* p = (uint8_t*)scratch;
    uint32_t* slot_cnt = (uint32_t*)p;
    uint32_t* off = slot_cnt + 256;
    uint32_t* cursor = off + 256;
    uint32_t* right_cnt = cursor + 256;
    uint32_t* cl[3] = {right_cnt + 256, right_cnt + 512, right_cnt + 768};
    uint32_t* cr[3] = {right_cnt + 1024, right_cnt + 1280, right_cnt + 1536};
    uint32_t* snap[2] = {right_cnt + 1792, right_cnt + 2048};
    const uint64_t rc = (ncand * sizeof(LongRec) + 255) & ~(uint64_t)255;
    const uint64_t cc = (ncand * sizeof(ContRec) + 255) & ~(uint64_t)255;
    uint8_t* q = p + kLongCounts * 256 * sizeof(uint32_t);
    LongRec* cands = (LongRec*)q;
    LongRec* right = (LongRec*)(q + rc);
    ContRec* cont_l[2] = {(ContRec*)(q + 2 * rc), (ContRec*)(q + 2 * rc + cc)};
    ContRec* cont_r[2] = {(ContRec*)(q + 2 * rc + 2 * cc), (ContRec*)(q + 2 * rc + 3 * cc)};
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, s, slot_cnt, kLongCounts * 256, 0u);
    const unsigned hb = (unsigned)std::min<uint64_t>(blocks_for(V.nhits), 4096);
    hipLaunchKernelGGL(k_long_slot_counts, dim3(hb), dim3(kBlock), 0, s, V.hits, V.nhits, slot_cnt);
    hipLaunchKernelGGL(k_long_slot_offsets, dim3(1), dim3(64), 0, s, slot_cnt, off, cursor);
    hipLaunchKernelGGL(k_long_scatter, dim3(hb), dim3(kBlock), 0, s, V.hits,
                       V.nhits, V.vals, V.x_slen, V.x_lenstart, V.x_gbase, V.y_lenstart,
                       V.y_gbase, cursor, cands);
    const Div div = make_div(V.tau + 1);
    // pass lengths: 16, 16, 32, 64, ..., 512 rows; PJ_LONG_PASSES (a comma list, the last entry
    // repeated) sets them (tests and tuning; it changes no result)
    int sched[16], nsched = 0;
    if (const char* e = getenv("PJ_LONG_PASSES")) {
        for (const char* c = e; *c && nsched < 16;) {
            const int v = atoi(c);
            if (v < 1 || v > 4096) return hipErrorInvalidValue;
            sched[nsched++] = v;
            while (*c && *c != ',') ++c;
            if (*c == ',') ++c;
        }
    }
    // Pass j runs the left parts (until every left part has had max_rows rows), the right parts
    // appended by passes before j (the range between the snapshots of the right-task counts taken
    // before passes j - 1 and j) and the right parts continuing from pass j - 1; it ends when the
    // right parts appended by the last left pass have had max_rows rows.  Continuation counts
    // rotate over three buffers per side: pass j reads c[j % 3], writes c[(j + 1) % 3] (cleared
    // by pass j - 1, or at the start) and clears c[(j + 2) % 3] (read by pass j - 1).
    bool left = true;
    int done_l = 0, done_r = 0;
    for (int pass = 0;; ++pass) {
        const int K = nsched ? sched[pass < nsched ? pass : nsched - 1]
                             : (pass == 0 ? 16 : std::min(512, 16 << (pass - 1)));
        if (pass > 0)
            hipLaunchKernelGGL(k_copy_u32, dim3(1), dim3(256), 0, s, snap[pass % 2], right_cnt, 256);
        ContPass P{};
        if (left) {
            P.fin_l = pass == 0 ? cands : nullptr;
            P.cin_l = pass == 0 ? nullptr : cont_l[pass % 2];
            P.cnt_l = pass == 0 ? slot_cnt : cl[pass % 3];
            P.cout_l = cont_l[(pass + 1) % 2];
            P.cout_l_cnt = cl[(pass + 1) % 3];
            P.zero_l = cl[(pass + 2) % 3];
            P.rout = right;
            P.rout_cnt = right_cnt;
        }
        if (pass > 0) {
            P.fin_r = right;
            P.lo_r = snap[(pass + 1) % 2];      // snap[0] is zero before pass 2
            P.hi_r = snap[pass % 2];
            P.cin_r = cont_r[pass % 2];
            P.cnt_r = cr[pass % 3];
        }
        P.cout_r = cont_r[(pass + 1) % 2];
        P.cout_r_cnt = cr[(pass + 1) % 3];
        P.zero_r = cr[(pass + 2) % 3];
        P.off = off;
        P.K = K;
        hipLaunchKernelGGL(k_verify_cont, dim3(grid), dim3(64), 0, s, V, div, P);
        if (left) {
            done_l += K;
            if (done_l >= max_rows) left = false;
        } else {
            done_r += K;
            if (done_r >= max_rows) break;
        }
    }
    return hipGetLastError();
}

hipError_t launch_verify_batched(const VerifyParams& V, uint32_t* first, int grid, hipStream_t s)
{
    if (V.ncand == 0) return hipSuccess;
    if (V.wave_rounds < 1 || V.wave_rounds > kWaveRounds) return hipErrorInvalidValue;
    const uint64_t nchunks = batched_chunks(V.ncand, V.wave_rounds);
    hipLaunchKernelGGL(k_chunk_starts, dim3(blocks_for(nchunks)), dim3(kBlock), 0, s, V.prefix,
                       V.nhits, nchunks, 64ull * (uint64_t)V.wave_rounds, first);
    const int w = V.tau + 1;
    if (w <= 9) verify_batched_w<9>(V, first, nchunks, grid, s);
    else if (w <= 17) verify_batched_w<17>(V, first, nchunks, grid, s);
    else if (w <= 33) verify_batched_w<33>(V, first, nchunks, grid, s);
    else verify_batched_w<64>(V, first, nchunks, grid, s);
    return hipGetLastError();
}

hipError_t launch_verify(const VerifyParams& V, int grid, hipStream_t s)
{
    if (V.ncand == 0) return hipSuccess;
    const int w = V.tau + 1;
    if (w <= 2) verify_w<2>(V, grid, s);
    else if (w <= 3) verify_w<3>(V, grid, s);
    else if (w <= 5) verify_w<5>(V, grid, s);
    else if (w <= 9) verify_w<9>(V, grid, s);
    else if (w <= 17) verify_w<17>(V, grid, s);
    else if (w <= 33) verify_w<33>(V, grid, s);
    else verify_w<64>(V, grid, s);
    return hipGetLastError();
}

template <int W>
static void short_w(const DevSet& P, const DevSet& Y, int tau, int self, const int32_t* q_tau,
                    uint32_t y_first, uint32_t y_count, uint64_t* out, uint64_t cap,
                    unsigned long long* ctr, hipStream_t s)
{
    unsigned grid = y_count < 65536 ? y_count : 65536;
    hipLaunchKernelGGL((k_short<W>), dim3(grid), dim3(kBlock), 0, s, P.sarena, P.slen, P.lenstart,
                       P.gbase, P.lmax, Y.sarena, Y.slen, Y.lenstart, Y.gbase, y_first, y_count,
                       tau, self, q_tau, out, cap, ctr);
}

hipError_t launch_short_path(const DevSet& P, const DevSet& Y, int tau, int self,
                             const int32_t* q_tau, uint64_t* out, uint64_t out_cap,
                             unsigned long long* counters, hipStream_t s)
{
    if (Y.n == 0 || P.n == 0 || Y.lmin > tau) return hipSuccess;
    const int top = tau < Y.lmax ? tau : Y.lmax;
    uint32_t y_first = (uint32_t)Y.h_lenstart[0];
    uint32_t y_end = (uint32_t)Y.h_lenstart[top + 1];
    if (y_end <= y_first) return hipSuccess;
    uint32_t cnt = y_end - y_first;
    const int w = tau + 1;
    if (w <= 2) short_w<2>(P, Y, tau, self, q_tau, y_first, cnt, out, out_cap, counters, s);
    else if (w <= 5) short_w<5>(P, Y, tau, self, q_tau, y_first, cnt, out, out_cap, counters, s);
    else if (w <= 9) short_w<9>(P, Y, tau, self, q_tau, y_first, cnt, out, out_cap, counters, s);
    else if (w <= 17) short_w<17>(P, Y, tau, self, q_tau, y_first, cnt, out, out_cap, counters, s);
    else if (w <= 33) short_w<33>(P, Y, tau, self, q_tau, y_first, cnt, out, out_cap, counters, s);
    else short_w<64>(P, Y, tau, self, q_tau, y_first, cnt, out, out_cap, counters, s);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Captured query batches: the sizes of a batch live in device memory, so one instantiated graph
// of these launches serves every batch of a serving slot.
// ------------------------------------------------------------------------------------------

__global__ void k_fill_u64(unsigned long long* __restrict__ p, int n, unsigned long long v)
{
    for (int k = threadIdx.x; k < n; k += blockDim.x) p[k] = v;
}

// One block: exclusive prefix of the hits' candidate counts, then the batch's sizes.  An
// overflow (more hits than the buffer holds, or more wave chunks than the chunk table holds)
// sets a flag and leaves nothing to verify; the host then runs the batch without the graph.
__global__ __launch_bounds__(kBlock) void k_batch_prefix(const Hit* __restrict__ hits,
                                                         const unsigned long long* __restrict__ counters,
                                                         uint64_t hit_cap,
                                                         unsigned long long* __restrict__ prefix,
                                                         unsigned long long* __restrict__ bc,
                                                         uint64_t chunk_cap)
{
    __shared__ unsigned long long s_w[kWaves];
    uint64_t nh = counters[0];
    unsigned long long flags = 0;
    if (nh > hit_cap) {
        flags |= 1;
        nh = 0;
    }
    unsigned long long carry = 0;
    for (uint64_t b = 0; b < nh; b += kBlock) {
        const uint64_t k = b + threadIdx.x;
        const unsigned long long v = k < nh ? (unsigned long long)hits[k].count : 0ull;
        unsigned long long tot;
        const unsigned long long ex = block_excl_scan(v, s_w, &tot);
        if (k < nh) prefix[k] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        prefix[nh] = carry;
        uint64_t nch = (carry + kWaveChunk - 1) / kWaveChunk;
        if (nch > chunk_cap) {
            flags |= 2;
            nch = 0;
        }
        bc[0] = nh;
        bc[1] = (flags & 2) ? 0ull : carry;
        bc[2] = nch;
        bc[3] = flags;
    }
}

// first[ch] for a captured batch (grid-stride; sizes from bc)
__global__ __launch_bounds__(kBlock) void k_chunk_starts_dev(const unsigned long long* __restrict__ prefix,
                                                             const unsigned long long* __restrict__ bc,
                                                             uint32_t* __restrict__ first)
{
    const uint64_t nh = bc[0], nch = bc[2];
    for (uint64_t ch = (uint64_t)blockIdx.x * kBlock + threadIdx.x; ch < nch;
         ch += (uint64_t)gridDim.x * kBlock) {
        const unsigned long long c0 = ch * kWaveChunk;
        uint64_t a = 0, b = nh - 1;
        while (a < b) {
            const uint64_t m = (a + b + 1) >> 1;
            if (prefix[m] <= c0) a = m; else b = m - 1;
        }
        first[ch] = (uint32_t)a;
    }
}

// One block: the batch's accepted (gx, gy) become (query id << 32 | indexed id) keys, sorted in
// LDS (bitonic), deduplicated and compacted in order.  More than kGraphSortCap accepted pairs,
// or more than the accepted buffer held, sets a flag and outputs nothing.
__global__ __launch_bounds__(kBlock) void k_batch_dedupe(const uint64_t* __restrict__ acc,
                                                         const unsigned long long* __restrict__ counters,
                                                         uint64_t acc_cap,
                                                         const int32_t* __restrict__ xperm,
                                                         const int32_t* __restrict__ yperm,
                                                         unsigned long long* __restrict__ bc,
                                                         uint64_t* __restrict__ out,
                                                         uint32_t* __restrict__ out_n)
{
    __shared__ uint64_t s_k[kGraphSortCap];
    __shared__ uint32_t s_w[kWaves];
    const uint64_t m = counters[3];
    if (m > acc_cap || m > (uint64_t)kGraphSortCap) {
        if (threadIdx.x == 0) {
            bc[3] |= (m > acc_cap ? 4ull : 0ull) | 8ull;
            *out_n = 0;
        }
        return;
    }
    uint32_t N = 1;
    while (N < (uint32_t)m) N <<= 1;
    for (uint32_t k = threadIdx.x; k < N; k += kBlock) {
        uint64_t key = ~0ull;
        if (k < (uint32_t)m) {
            const uint64_t v = acc[k];
            const uint32_t a = (uint32_t)xperm[v >> 32];
            const uint32_t b = (uint32_t)yperm[v & 0xffffffffu];
            key = ((uint64_t)a << 32) | b;
        }
        s_k[k] = key;
    }
    __syncthreads();
    for (uint32_t kk = 2; kk <= N; kk <<= 1) {
        for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < N; i += kBlock) {
                const uint32_t ixj = i ^ j;
                if (ixj > i) {
                    const uint64_t a = s_k[i], b = s_k[ixj];
                    const bool up = (i & kk) == 0;
                    if ((a > b) == up) {
                        s_k[i] = b;
                        s_k[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    uint32_t carry = 0;
    for (uint32_t base = 0; base < N; base += kBlock) {
        const uint32_t k = base + threadIdx.x;
        const uint32_t f = (k < (uint32_t)m && (k == 0 || s_k[k] != s_k[k - 1])) ? 1u : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(f, s_w, &tot);
        if (f) out[carry + ex] = s_k[k];
        carry += tot;
    }
    if (threadIdx.x == 0) *out_n = carry;
}

template <int W>
static void graph_verify_short(const GraphBatch& G, hipStream_t s)
{
    verify_batched_w<W>(G.verify, G.first, 0, G.verify_grid, s);
    if (G.y_count) {
        const ProbeParams& P = G.probe;
        const unsigned grid = G.y_count < 65536 ? G.y_count : 65536;
        hipLaunchKernelGGL((k_short<W>), dim3(grid), dim3(kBlock), 0, s, P.x_arena, P.x_slen,
                           P.x_lenstart, P.x_gbase, kLenMax, G.y_arena, G.y_slen, G.y_lenstart,
                           G.y_gbase, G.y_first, G.y_count, P.tau, 0, P.q_tau, G.verify.out,
                           G.verify.out_cap, G.verify.counters);
    }
}

hipError_t launch_graph_batch(const GraphBatch& G, hipStream_t s)
{
    if (!G.probe.nx_dev || !G.verify.dev_counts || G.probe_grid < 1 || G.verify_grid < 1)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, G.probe.counters, 8, 0ull);
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, G.bcounts, 4, 0ull);
    hipLaunchKernelGGL(k_probe<false>, dim3(G.probe_grid), dim3(kBlock), 0, s, G.probe,
                       make_div(G.probe.tau + 1));
    hipLaunchKernelGGL(k_batch_prefix, dim3(1), dim3(kBlock), 0, s, G.probe.hits,
                       G.probe.counters, G.probe.hit_cap,
                       const_cast<unsigned long long*>(G.verify.prefix), G.bcounts, G.chunk_cap);
    hipLaunchKernelGGL(k_chunk_starts_dev, dim3(8), dim3(kBlock), 0, s, G.verify.prefix,
                       G.bcounts, G.first);
    const int w = G.verify.tau + 1;
    if (w <= 9) graph_verify_short<9>(G, s);
    else if (w <= 17) graph_verify_short<17>(G, s);
    else if (w <= 33) graph_verify_short<33>(G, s);
    else graph_verify_short<64>(G, s);
    hipLaunchKernelGGL(k_batch_dedupe, dim3(1), dim3(kBlock), 0, s, G.verify.out,
                       G.verify.counters, G.verify.out_cap, G.xperm, G.yperm, G.bcounts, G.out,
                       G.out_n);
    return hipGetLastError();
}

hipError_t launch_pairs_to_keys(const uint64_t* acc, uint64_t m, const int32_t* xperm,
                                const int32_t* yperm, int self, int bbits, uint64_t* keys,
                                hipStream_t s)
{
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pairs_to_keys, dim3(blocks_for(m)), dim3(kBlock), 0, s, acc, m, xperm,
                       yperm, self, bbits, keys);
    return hipGetLastError();
}

hipError_t launch_unique_flags(const uint64_t* keys, uint64_t m, uint32_t* flags, hipStream_t s)
{
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_unique_flags, dim3(blocks_for(m)), dim3(kBlock), 0, s, keys, m, flags);
    return hipGetLastError();
}

hipError_t launch_compact_pairs(const uint64_t* keys, const uint32_t* flags, const uint32_t* pos,
                                uint64_t m, int bbits, int32_t* a, int32_t* b, hipStream_t s)
{
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_compact_pairs, dim3(blocks_for(m)), dim3(kBlock), 0, s, keys, flags, pos,
                       m, bbits, a, b);
    return hipGetLastError();
}

// Streamed self-joins: a window's result pairs (window-local ids) as global sort keys
// ids[a] << bbits | ids[b].  With min_len > 0 a pair of two strings shorter than min_len (both
// in the window's halo, found again by the window that owns them) becomes the sentinel, all
// ones in 2 * bbits bits, which no pair (a < b) reaches and which sorts after every pair; the
// sentinels are counted.
__global__ __launch_bounds__(kBlock) void k_window_keys(const int32_t* __restrict__ a,
                                                       const int32_t* __restrict__ b, uint64_t m,
                                                       const int32_t* __restrict__ ids,
                                                       const int32_t* __restrict__ offs,
                                                       int min_len, int bbits,
                                                       uint64_t* __restrict__ keys,
                                                       unsigned long long* __restrict__ dropped)
{
    const uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    bool drop = false;
    if (k < m) {
        const int32_t la = a[k], lb = b[k];
        if (min_len > 0) {
            const int na = offs[la + 1] - offs[la], nb = offs[lb + 1] - offs[lb];
            drop = (na > nb ? na : nb) < min_len;
        }
        keys[k] = drop ? ((2 * bbits >= 64) ? ~0ull : (1ull << (2 * bbits)) - 1ull)
                       : ((uint64_t)(uint32_t)ids[la] << bbits) | (uint64_t)(uint32_t)ids[lb];
    }
    const uint64_t dm = __ballot(drop);
    if ((threadIdx.x & 63) == 0 && dm) atomicAdd(dropped, (unsigned long long)__popcll(dm));
}

__global__ __launch_bounds__(kBlock) void k_split_keys(const uint64_t* __restrict__ keys,
                                                      uint64_t m, int bbits,
                                                      int32_t* __restrict__ a,
                                                      int32_t* __restrict__ b)
{
    const uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < m) {
        const uint64_t v = keys[k];
        a[k] = (int32_t)(v >> bbits);
        b[k] = (int32_t)(v & ((1ull << bbits) - 1));
    }
}

hipError_t launch_window_keys(const int32_t* a, const int32_t* b, uint64_t m, const int32_t* ids,
                              const int32_t* offs, int min_len, int bbits, uint64_t* keys,
                              unsigned long long* dropped, hipStream_t s)
{
    if (m == 0) return hipSuccess;
    if (bbits < 1 || bbits > 31) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_window_keys, dim3(blocks_for(m)), dim3(kBlock), 0, s, a, b, m, ids, offs,
                       min_len, bbits, keys, dropped);
    return hipGetLastError();
}

hipError_t launch_split_keys(const uint64_t* keys, uint64_t m, int bbits, int32_t* a, int32_t* b,
                             hipStream_t s)
{
    if (m == 0) return hipSuccess;
    if (bbits < 1 || bbits > 31) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_split_keys, dim3(blocks_for(m)), dim3(kBlock), 0, s, keys, m, bbits, a, b);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_fill_words(uint32_t* __restrict__ p, uint64_t n,
                                                       uint32_t v)
{
    for (uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x; k < n;
         k += (uint64_t)gridDim.x * kBlock)
        p[k] = v;
}

hipError_t launch_fill_words(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const unsigned grid = (unsigned)std::min<uint64_t>(blocks_for(n), 4096);
    hipLaunchKernelGGL(k_fill_words, dim3(grid), dim3(kBlock), 0, s, p, n, v);
    return hipGetLastError();
}

// Checksum of a device string set: offsets[0 .. n] and bytes[0 .. min(offsets[n], cap)), each
// element mixed with its index (SplitMix64's finaliser) and summed.  A plan compares it with the
// value taken when it was made; cap (the bytes allocation measured then) bounds the reads
// whatever offsets[n] holds now.
__global__ __launch_bounds__(kBlock) void k_set_checksum(const int32_t* __restrict__ offs, int64_t n,
                                                         const uint8_t* __restrict__ bytes,
                                                         int64_t cap,
                                                         unsigned long long* __restrict__ sum)
{
    const int64_t last = offs[n];
    const int64_t total = bytes ? (last < 0 ? 0 : (last < cap ? last : cap)) : 0;
    uint64_t acc = 0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k <= n; k += stride)
        acc += mix64((uint64_t)(uint32_t)offs[k] ^ ((uint64_t)k << 32) ^ 0x243F6A8885A308D3ull);
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < total; k += stride)
        acc += mix64((uint64_t)bytes[k] ^ ((uint64_t)k << 8) ^ 0x13198A2E03707344ull);
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0 && acc) atomicAdd(sum, (unsigned long long)acc);
}

hipError_t launch_set_checksum(const int32_t* offs, int64_t n, const uint8_t* bytes, int64_t cap,
                               unsigned long long* sum, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_words, dim3(1), dim3(kBlock), 0, s, (uint32_t*)sum, (uint64_t)2, 0u);
    const unsigned grid = (unsigned)std::max<uint64_t>(
        1, std::min<uint64_t>(blocks_for((uint64_t)n + 1), 2048));
    hipLaunchKernelGGL(k_set_checksum, dim3(grid), dim3(kBlock), 0, s, offs, n, bytes, cap, sum);
    return hipGetLastError();
}

hipError_t launch_gather_i32(const int32_t* in, const int32_t* perm, int64_t n, int32_t* out,
                             hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_i32, dim3(blocks_for(n)), dim3(kBlock), 0, s, in, perm, n, out);
    return hipGetLastError();
}

}  // namespace pj
