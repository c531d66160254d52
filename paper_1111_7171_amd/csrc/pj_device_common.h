// pj_device_common.h -- device helpers of libpassjoin: even partition, multi-match windows,
// segment hashing, index keys, bucket-table lookup and the banded verification DP.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pj_internal.h"

namespace pj {

// Division by d <= 64 of l < 2048 by multiply-shift: q = (l * m) >> 21 with m = ceil(2^21 / d)
// is exact because l * (m - 2^21/d) / 2^21 < 2^-10 < 1/d.
struct Div {
    uint32_t d, m;
    __host__ __device__ inline int operator()(int l) const { return (int)(((uint32_t)l * m) >> 21); }
};

inline Div make_div(int d)
{
    Div v;
    v.d = (uint32_t)d;
    v.m = (uint32_t)(((1u << 21) + (uint32_t)d - 1) / (uint32_t)d);
    return v;
}

// Segment i (1-based) of a length-l string under the even partition into tau+1 segments
// (Sec. 3.1): with q = floor(l/(tau+1)) and k = l - q(tau+1), the first tau+1-k segments have
// length q and the last k have length q+1; p is the 1-based start.
struct Seg {
    int p, len;
};

__device__ inline Seg partition_seg(int l, int i, int tau, Div div)
{
    const int T1 = tau + 1;
    const int q = div(l);
    const int k = l - q * T1;
    Seg s;
    s.len = q + (i > T1 - k ? 1 : 0);
    const int extra = i - 1 - (T1 - k);
    s.p = 1 + (i - 1) * q + (extra > 0 ? extra : 0);
    return s;
}

// Multi-match-aware window (Sec. 4.2): start positions p of x[p, l_i] selected for L_l^i,
// intersecting the left-side bounds p_i -/+ (i-1) and the right-side bounds
// p_i + Delta -/+ (tau+1-i), Delta = n - l, within [1, n - l_i + 1].
__device__ inline void multimatch_window(int n, int l, int tau, int i, Seg sg, int* lo, int* hi)
{
    const int delta = n - l;
    const int last = n - sg.len + 1;
    const int r = tau + 1 - i;
    int bl = sg.p - (i - 1), tl = sg.p + (i - 1);
    int br = sg.p + delta - r, tr = sg.p + delta + r;
    int a = bl > br ? bl : br;
    int b = tl < tr ? tl : tr;
    if (a < 1) a = 1;
    if (b > last) b = last;
    *lo = a;
    *hi = b;
}

// Start-position window of a selection method other than multi-match (PJ_SELECT_POSITION,
// _SHIFT, _LENGTH; Sec. 4 and 4.1), restricted to [1, n - l_i + 1]: position-aware
// [p_i - floor((tau-Delta)/2), p_i + floor((tau+Delta)/2)], shift-based [p_i - tau, p_i + tau],
// length-based every start position.  |Delta| <= tau here, so the halvings are of
// non-negative values.
__device__ inline void select_window(int method, int n, int l, int tau, int i, Seg sg, int* lo,
                                     int* hi)
{
    if (method == 0) {
        multimatch_window(n, l, tau, i, sg, lo, hi);
        return;
    }
    const int delta = n - l;
    const int last = n - sg.len + 1;
    int a = 1, b = last;
    if (method == 1) {
        a = sg.p - ((tau - delta) >> 1);
        b = sg.p + ((tau + delta) >> 1);
    } else if (method == 2) {
        a = sg.p - tau;
        b = sg.p + tau;
    }
    *lo = a < 1 ? 1 : a;
    *hi = b > last ? last : b;
}

// Polynomial segment hash h = sum (c_k + 1) * B^(L-1-k) mod 2^64 (Horner form), rolled across
// consecutive start positions.  Equal segments always hash equal; unequal ones that collide are
// rejected by the byte comparison done before verification.
constexpr uint64_t kHashBase = 0x9E3779B97F4A7C15ull;

__device__ inline uint64_t seg_hash(const uint8_t* w, int len)
{
    uint64_t h = 0;
    for (int k = 0; k < len; ++k) h = h * kHashBase + (uint64_t)w[k] + 1ull;
    return h;
}

__device__ inline uint64_t pow_hash(int len)   // B^(len-1)
{
    uint64_t r = 1, b = kHashBase;
    int e = len - 1;
    while (e > 0) {
        if (e & 1) r *= b;
        b *= b;
        e >>= 1;
    }
    return r;
}

__device__ inline uint64_t roll_hash(uint64_t h, uint8_t out, uint8_t in, uint64_t top)
{
    return (h - ((uint64_t)out + 1ull) * top) * kHashBase + (uint64_t)in + 1ull;
}

// SplitMix64 finaliser (Steele, Lea, Flood 2014), used to spread hash bits.
__host__ __device__ inline uint64_t mix64(uint64_t x)
{
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

// Segment code: the packed symbol codes when len <= exact_len (sym: the indexed set's symbol
// map, `bits` per symbol), else the polynomial hash of the bytes.  Both roll across consecutive
// start positions.
__device__ inline uint64_t seg_code(const uint8_t* w, int len, const uint16_t* sym, int bits,
                                    int exact_len)
{
    uint64_t h = 0;
    if (len <= exact_len) {
        for (int k = 0; k < len; ++k) h = (h << bits) | (uint64_t)sym[w[k]];
    } else {
        // eight bytes read before they enter the hash, so a segment waits on len / 8 reads
        int k = 0;
        for (; k + 8 <= len; k += 8) {
            uint32_t c[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) c[u] = w[k + u];
#pragma unroll
            for (int u = 0; u < 8; ++u) h = h * kHashBase + (uint64_t)c[u] + 1ull;
        }
        for (; k < len; ++k) h = h * kHashBase + (uint64_t)w[k] + 1ull;
    }
    return h;
}

__device__ inline uint64_t roll_code(uint64_t h, int len, uint8_t out, uint8_t in, uint64_t top,
                                     const uint16_t* sym, int bits, int exact_len)
{
    if (len <= exact_len) {
        const int nb = len * bits;                      // <= kHashBits
        return ((h << bits) | (uint64_t)sym[in]) & ((1ull << nb) - 1ull);
    }
    return roll_hash(h, out, in, top);
}

__device__ inline uint64_t make_key(int l, int i, int tau, int len, uint64_t code, int exact_len)
{
    const uint64_t grp = (uint64_t)(l - (tau + 1)) * (uint64_t)(tau + 1) + (uint64_t)(i - 1);
    const uint64_t c = (len <= exact_len) ? code : (mix64(code) >> (64 - kHashBits));
    return (grp << kHashBits) | c;
}

__device__ inline uint64_t table_slot(uint64_t key) { return mix64(key ^ 0x5851F42D4C957F2Dull); }

// Key filter, blocked by (l, i) group: group g owns the words [dir[g], dir[g+1]) of the filter,
// a power of two of them (about 16 bits per list of the group, at least one word), so the keys
// a wave looks up for one probe string and a few (l, i) share one or two cache lines.  A key
// sets two bits of one word of its group's block, all from the slot hash's bits 30.. (the table
// uses the low bits): the word (h >> 45) & (block words - 1), the bits below.
__device__ inline uint32_t filter_bits(uint64_t h)
{
    return (1u << ((uint32_t)(h >> 35) & 31u)) | (1u << ((uint32_t)(h >> 30) & 31u));
}
__device__ inline uint32_t filter_word_in(uint64_t h, uint32_t block_mask)
{
    return (uint32_t)(h >> 45) & block_mask;
}

// The open-addressing lookup from a given slot on (linear probing).
__device__ inline bool table_lookup_from(const uint4* __restrict__ table, uint64_t mask,
                                         uint64_t key, uint64_t slot, uint32_t* start,
                                         uint32_t* count)
{
    while (true) {
        const uint4 v = table[slot];
        const uint64_t k = (uint64_t)v.x | ((uint64_t)v.y << 32);
        if (k == key) {
            *start = v.z;
            *count = v.w;
            return true;
        }
        if (k == kEmptyKey) return false;
        slot = (slot + 1) & mask;
    }
}

__device__ inline bool table_lookup(const uint4* __restrict__ table, uint64_t mask, uint64_t key,
                                    uint32_t* start, uint32_t* count)
{
    uint64_t slot = table_slot(key) & mask;
    while (true) {
        const uint4 v = table[slot];
        const uint64_t k = (uint64_t)v.x | ((uint64_t)v.y << 32);
        if (k == key) {
            *start = v.z;
            *count = v.w;
            return true;
        }
        if (k == kEmptyKey) return false;
        slot = (slot + 1) & mask;
    }
}

// VerifyStringPair (Sec. 5.1; function of Algorithm 3): min(t+1, ED(r, s)) with the length-aware
// band and the expected-edit-distance early termination (Lemma 4).  r is the indexed string's
// part and s the probe string's part; the shorter one gives the rows (r when equal).  With
// Delta = |cols| - |rows| (> t: return t+1), row i keeps the cells j in
// [i - floor((t-Delta)/2), i + floor((t+Delta)/2)], held in registers R[k], j = i - a + k.
// Cells out of the band or the matrix are infinite; values saturate at t+1.  After each row,
// E(i,j) = M(i,j) + |Delta + a - k| (the length gap of the remaining suffixes) is reduced to its
// minimum; above t the pair cannot be within t.  *cells counts recurrence cells (j >= 1).
// MAXW >= t+1 bounds the band width at compile time.
template <int MAXW>
__device__ inline int vsp_global(const uint8_t* r, int lr, const uint8_t* s, int ls, int t,
                                 int* cells)
{
    const uint8_t* A;
    const uint8_t* B;
    int nr, nc;
    if (lr <= ls) { A = r; nr = lr; B = s; nc = ls; }
    else          { A = s; nr = ls; B = r; nc = lr; }
    const int delta = nc - nr;
    *cells = 0;
    if (delta > t) return t + 1;
    const int a = (t - delta) >> 1;
    const int b = (t + delta) >> 1;
    const int W = a + b + 1;
    const int INF = t + 1;
    int R[MAXW];
#pragma unroll
    for (int k = 0; k < MAXW; ++k) {
        const int j = k - a;
        R[k] = (k < W && j >= 0 && j <= nc) ? (j < INF ? j : INF) : INF;
    }
    int ncell = 0;
    for (int i = 1; i <= nr; ++i) {
        const int ai = A[i - 1];
        int left = INF;
        int emin = 1 << 20;
#pragma unroll
        for (int k = 0; k < MAXW; ++k) {
            if (k < W) {
                const int j = i - a + k;
                int v = INF;
                if (j >= 0 && j <= nc) {
                    if (j == 0) {
                        v = i < INF ? i : INF;
                    } else {
                        const int up = (k + 1 < MAXW && k + 1 < W) ? R[(k + 1) < MAXW ? k + 1 : k] : INF;
                        const int d = (ai != (int)B[j - 1]) ? 1 : 0;
                        const int m1 = (up < left ? up : left) + 1;
                        const int m2 = R[k] + d;
                        v = m1 < m2 ? m1 : m2;
                        v = v < INF ? v : INF;
                        ++ncell;
                    }
                    const int dd = delta + a - k;
                    const int e = v + (dd < 0 ? -dd : dd);
                    emin = e < emin ? e : emin;
                }
                R[k] = v;
                left = v;
            }
        }
        if (emin > t) {
            *cells = ncell;
            return t + 1;
        }
    }
    *cells = ncell;
    int res = INF;
#pragma unroll
    for (int k = 0; k < MAXW; ++k)
        if (k == delta + a) res = R[k];
    return res;
}

// Cells of rows 1..s of the band (closed form, defined below).
__device__ inline int band_cells(int s, int nc, int a, int b);

// VerifyStringPair for the batched path (one candidate per lane, each lane with its own
// strings and band): the same orientation, band, early stop, result and cell count as
// vsp_global, computed as vsp_lane does, on expected distances D = M + |kfin - k| with the
// neighbour adjustments cu, cl (0 or 2) and no masks (the argument given for vsp_seg covers the
// BIG borders, the unmasked band indices past a + b and the characters outside 1..nc, which
// read as 256 here).  The band's column characters sit in a register window that shifts by one
// per row; the character entering it and the next row character are loaded a row ahead.  The
// cells of the rows evaluated follow in closed form.  P is a byte pointer into global memory
// or LDS.
template <int MAXW, typename P>
__device__ inline int vsp_fast(P r, int lr, P s, int ls, int t, int* cells)
{
    P A;
    P B;
    int nr, nc;
    if (lr <= ls) { A = r; nr = lr; B = s; nc = ls; }
    else          { A = s; nr = ls; B = r; nc = lr; }
    const int delta = nc - nr;
    *cells = 0;
    if (delta > t) return t + 1;
    const int a = (t - delta) >> 1;
    const int b = (t + delta) >> 1;              // kfin: band index of cell (nr, nc)
    constexpr int BIG = 1 << 20;
    int D[MAXW], w[MAXW], cu[MAXW], cl[MAXW];
#pragma unroll
    for (int k = 0; k < MAXW; ++k) {
        const int j = k - a;                     // column of band index k in row 0
        const int ek = b > k ? b - k : k - b;
        D[k] = (j >= 0 && j <= min(nc, b)) ? j + ek : BIG;
        w[k] = ((unsigned)j < (unsigned)nc) ? (int)B[j] : 256;   // B index of row 1's column
        cu[k] = k < b ? 2 : 0;
        cl[k] = k > b ? 2 : 0;
    }
    int idx_in = MAXW - a;                       // B index entering the window after row 1
    int cin = ((unsigned)idx_in < (unsigned)nc) ? (int)B[idx_in] : 256;
    int ai = nr > 0 ? (int)A[0] : 256;
    int ai_next = nr > 1 ? (int)A[1] : 256;
    int rows = nr;
    bool failed = false;
    for (int i = 1; i <= nr; ++i) {
        // loads for the next row first, so their latency overlaps this row's arithmetic
        const int idx2 = idx_in + 1;
        const int cin_next = ((unsigned)idx2 < (unsigned)nc) ? (int)B[idx2] : 256;
        const int ai_next2 = (i + 1 < nr) ? (int)A[i + 1] : 256;
        int left = BIG;
#pragma unroll
        for (int k = 0; k < MAXW; ++k) {
            const int up = (k + 1 < MAXW) ? D[(k + 1) < MAXW ? k + 1 : k] : BIG;
            const int dg = D[k] + ((ai != w[k]) ? 1 : 0);
            // no left neighbour for the band's first cell, no upper one for its last
            const int v = k == 0 ? (MAXW == 1 ? dg : min(up + cu[k], dg))
                                 : (k + 1 == MAXW ? min(left + cl[k], dg)
                                                  : min(min(up + cu[k], left + cl[k]), dg));
            D[k] = v;
            left = v;
        }
        int emin = D[0];
#pragma unroll
        for (int k = 1; k < MAXW; ++k) emin = min(emin, D[k]);
        if (emin > t) {
            rows = i;
            failed = true;
            break;
        }
#pragma unroll
        for (int k = 0; k + 1 < MAXW; ++k) w[k] = w[k + 1];
        w[MAXW - 1] = cin;
        cin = cin_next;
        idx_in = idx2;
        ai = ai_next;
        ai_next = ai_next2;
    }
    *cells = band_cells(rows, nc, a, b);
    if (failed) return t + 1;
    int out = BIG;
#pragma unroll
    for (int k = 0; k < MAXW; ++k) out = (k == b) ? D[k] : out;
    return min(out, t + 1);
}

// VerifyStringPair for a wave whose lanes share the probe string's part and the band geometry
// (all lanes verify members of one inverted list against the same x): same results and cell
// counts as vsp_global.  U reads the shared part (x's) at wave-uniform positions, V the lane's
// own part (y's); the part lengths lu, lv and t are wave-uniform, so the band bounds, the
// interior/edge decision of each row and the row's cell count are all scalar work, and the
// lanes differ only in the cell values and in the row where they stop.  YROWS tells which part
// gives the rows (the shorter one; y's when equal): with YROWS the column window holds shared
// characters (scalar registers), otherwise the row character is the shared one.

// Bytes of a string read at wave-uniform positions through the scalar cache (loads only).
// A string's slot is 16-byte aligned and a multiple of 16 bytes long, so the aligned dword
// around any byte of the string lies inside the slot.
struct UniformChars {
    const uint8_t* p;
    __device__ inline int operator[](int k) const
    {
        const uintptr_t ad = (uintptr_t)(p + k);
        const uint32_t w =
            *(const __attribute__((address_space(4))) uint32_t*)(ad & ~(uintptr_t)3);
        return (int)((w >> ((ad & 3u) * 8u)) & 0xffu);
    }
};

struct GlobalChars {
    const uint8_t* p;
    __device__ inline int operator[](int k) const { return (int)p[k]; }
};

// The lane's whole string in registers, 4 bytes each (at most 64 bytes), read at a
// wave-uniform position (the wave shares the part's offset and the row).
struct RegChars {
    const uint32_t* r;
    int off;             // part offset within the string (wave-uniform)
    __device__ inline int operator[](int k) const
    {
        const int q = off + k;
        return (int)((r[q >> 2] >> ((q & 3) * 8)) & 0xffu);
    }
};

// Character k of two register strings (same part offset) as the low and high 16-bit halves
// of one word: one byte permute picks byte q & 3 of each string's word q >> 2.
__device__ inline uint32_t reg_pair(const RegChars (&V)[2], int k)
{
    const int q = V[0].off + k;
    const uint32_t d0 = V[0].r[q >> 2], d1 = V[1].r[q >> 2];
    // selector bytes: 0..3 take bytes of d0, 4..7 bytes of d1, 12 gives zero
    return __builtin_amdgcn_perm(d1, d0, 0x0c040c00u + (uint32_t)(q & 3) * 0x10001u);
}

// Bytes of the probe string staged in the wave's LDS buffer, read at wave-uniform positions
// (a broadcast read; no bank conflicts).
struct LdsChars {
    const __attribute__((address_space(3))) uint8_t* p;
    __device__ inline int operator[](int k) const { return (int)p[k]; }
};

// The row loop exits on a wave vote, so the row index, the band bounds and the shared
// characters stay wave-uniform, and every row runs the same unmasked recurrence:
//  * cells left of column 0 start at BIG and only ever see BIG or larger inputs;
//  * column 0 needs no special case: from M(0,0) = 0 the recurrence gives M(i,0) = i;
//  * cells right of column nc are never an input of a cell inside the matrix, and their
//    expected distance exceeds that of cell (i, nc), which is in the band whenever they are,
//    so they change neither a row's stop test nor the result;
//  * band indices W..MAXW-1 (right of the band, when MAXW > W) are computed like the others,
//    without a mask: the values are then those of a DP restricted to a wider band, at most the
//    banded ones.  Reaching a cell at diagonal offset j - i > b costs at least j - i, so its
//    expected distance is at least (j - i) + |delta - (j - i)| >= t + 1, and any value that
//    improves on the banded one through such a cell inherits that bound: every row's test,
//    and the result once saturated at t+1, are those of the band of Lemma 4;
//  * the outer neighbours (left of index 0, above index MAXW-1) read as BIG, or (vsp_lane,
//    vsp_fast) are left out of the minimum: a value that starts at BIG or above grows by at
//    most 2 per row (rows <= 2047), so it stays far below overflow and above every value
//    reached from row 0, and whether it is BIG or a little more changes no minimum that has
//    a value from row 0 among its inputs, no stop test and no result.
// So the characters of columns outside 1..nc are never needed: a window slot there may hold any
// byte (the probe string's LDS buffer is padded so that such reads stay inside it).
// Values are not saturated at t+1: min(v, t+1) commutes with the recurrence, so stop rows
// and verdicts are those of the saturated form.  The expected distance M + |delta + a - k|
// never decreases along a step of the recurrence, so once a row has no cell with expected
// distance <= t no later row has one: a lane is live exactly while its current row passes,
// and it stops at its first failing row.  A lane therefore only counts the rows it passed
// (rows evaluated = passes + 1 if it stopped, nr if it passed them all), and a candidate
// that is not active starts with every band cell at BIG, so it never passes a row.
// Large value of the two-candidate DP's 16-bit cells: it and every value that grows from it
// (at most one per row, rows <= 2047, plus a distance offset <= 63) stay below 2^16, and it
// exceeds every value reached from row 0 of the band.
constexpr uint32_t kBig16 = 0x4000u;

// Row 0, the expected-distance offsets |kfin - k| and (rows from y) the first column window of
// one part's band, as a table in the wave's LDS: entry k of each row of TS ints.  Written once
// per hit by lanes k < TS (every lane computes its entry), then read by every candidate's DP
// with broadcast loads.  Unpacked tables have three more rows for vsp_lane: row 0 plus the
// offsets (BIG outside the band), and the neighbour adjustments 1 + ek(k) - ek(k + 1) and
// 1 + ek(k) - ek(k - 1) (each 0 or 2); with ct > 0 they are followed by ct entries holding the
// band's cells in rows 1..s for s = 0 .. ct-1 (s <= nr), from which a DP reads its count.
__device__ inline void band_table(LdsChars U, int lu, int lv, int t, int lane, int ts,
                                  bool packed, __attribute__((address_space(3))) int* tab,
                                  int ct = 0)
{
    const bool yrows = lv <= lu;
    const int nr = yrows ? lv : lu;
    const int nc = yrows ? lu : lv;
    const int delta = nc - nr;                   // > t: the part fails without a DP
    const int a = (t - delta) >> 1;
    const int b = (t + delta) >> 1;
    const int kfin = delta + a;
    const int jl = lane - a;
    const int r0 = ((unsigned)jl <= (unsigned)min(nc, b)) ? jl : (1 << 20);
    const int ek = kfin - lane < 0 ? lane - kfin : kfin - lane;
    const int w0 = (yrows && (unsigned)jl < (unsigned)nc) ? U[jl] : 256;
    if (lane < ts) {
        if (packed) {
            // both 16-bit halves (two candidates per lane), BIG lowered to kBig16
            const uint32_t r16 = r0 == (1 << 20) ? kBig16 : (uint32_t)r0;
            tab[lane] = (int)(r16 * 0x10001u);
            tab[ts + lane] = (int)((uint32_t)ek * 0x10001u);
            tab[2 * ts + lane] = (int)((uint32_t)w0 * 0x10001u);
        } else {
            tab[lane] = r0;
            tab[ts + lane] = ek;
            tab[2 * ts + lane] = w0;
            tab[3 * ts + lane] = r0 == (1 << 20) ? r0 : r0 + ek;
            tab[4 * ts + lane] = kfin > lane ? 2 : 0;
            tab[5 * ts + lane] = kfin < lane ? 2 : 0;
        }
    }
    if (ct > 0 && delta <= t) {
        for (int s = lane; s < ct && s <= nr; s += 64) tab[6 * ts + s] = band_cells(s, nc, a, b);
    }
}

// Cells of rows 1..s of the band of Lemma 4 (a cells left of the diagonal, b right of it),
// clipped to columns 1..nc: the sum over rows i of |[max(1, i - a), min(nc, i + b)]|, in closed
// form.  Rows i <= nc - b reach the right end i + b; rows i <= a + 1 start at column 1.
__device__ inline int band_cells(int s, int nc, int a, int b)
{
    // every operand is in [0, 2047] (|delta| <= t keeps a, b >= 0), so the full-rate 24-bit
    // multiplier is exact; the halved terms are even and non-negative
    const unsigned us = s, unc = nc, ua = a, ub = b;
    const unsigned c1 = min(max(nc - b, 0), s);  // rows whose right end is i + b
    const unsigned hi = (__umul24(c1, c1 + 1) >> 1) + __umul24(ub, c1) + __umul24(us - c1, unc);
    const unsigned c2 = min(a + 1, s);           // rows whose left end is column 1
    const unsigned lo =
        c2 + ((__umul24(us, us + 1) - __umul24(c2, c2 + 1)) >> 1) - __umul24(ua, us - c2);
    return (int)(hi - lo + us);
}

// NC candidates per lane (members of the same list, so the same probe-string part and band):
// the scalar work of a row (band bounds, shared characters, cell count, loop control) is shared
// by all of them.  A candidate with act[c] false is dead from the start (cells 0, result t+1).
template <int MAXW, bool YROWS, int NC, int TS, typename LaneChars>
__device__ inline void vsp_seg(LdsChars U, int lu, const LaneChars (&V)[NC], int lv, int t,
                               const __attribute__((address_space(3))) int* tab,
                               const bool (&act)[NC], int (&cells)[NC], int (&res)[NC])
{
    static_assert(MAXW <= 64, "one band index per lane");
    const int nr = YROWS ? lv : lu;
    const int nc = YROWS ? lu : lv;
    const int delta = nc - nr;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        cells[c] = 0;
        res[c] = t + 1;
    }
    if (delta > t) return;
    const int a = (t - delta) >> 1;
    const int b = (t + delta) >> 1;
    const int kfin = delta + a;                  // band index of the last cell (nr, nc)
    constexpr int BIG = 1 << 20;
    constexpr int NW = YROWS ? 1 : NC;           // column windows: shared (YROWS) or per candidate
    int R[NC][MAXW], w[NW][MAXW], ek[MAXW];
#pragma unroll
    for (int k = 0; k < MAXW; ++k) {
        const int r0 = tab[k];
#pragma unroll
        for (int c = 0; c < NC; ++c) R[c][k] = act[c] ? r0 : BIG;
        // wide bands keep the offsets in scalar registers (vector registers are scarce there)
        ek[k] = MAXW <= 9 ? tab[TS + k] : __builtin_amdgcn_readfirstlane(tab[TS + k]);
        if (YROWS) {
            w[0][k] = tab[2 * TS + k];
        } else {
            const int idx = k - a;
#pragma unroll
            for (int c = 0; c < NW; ++c)
                w[c][k] = ((unsigned)idx < (unsigned)nc) ? V[c][idx] : 256;
        }
    }
    int idx_in = MAXW - a;                       // column character entering after row 1
    int ai_pre = (!YROWS && nr > 0) ? U[0] : 256;
    int passes[NC];                              // rows passed (a prefix of the rows)
#pragma unroll
    for (int c = 0; c < NC; ++c) passes[c] = 0;
    // Narrow bands unroll the row loop MAXW times and rotate the column window by renaming:
    // at unrolled step u band index k reads slot (u + k) % MAXW, and the entering column
    // character replaces slot u, so no register moves per row.  Wider bands shift the window.
    constexpr bool ROT = MAXW <= 9;
    constexpr int UNROLL = ROT ? MAXW : 1;
    int row = 1;
    bool go = nr > 0;
    while (go) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            // the row index is uniform (the loop exits on a wave vote), but the compiler does
            // not see it; as a scalar, register-array reads at it stay single moves
            const int i = __builtin_amdgcn_readfirstlane(row);
            // row characters: the lanes' own (registers) or the shared one, read a row ahead
            // (U[nr] lies inside the padded buffer)
            int ai[NC];
            if (YROWS) {
#pragma unroll
                for (int c = 0; c < NC; ++c) ai[c] = V[c][i - 1];
            } else {
#pragma unroll
                for (int c = 0; c < NC; ++c) ai[c] = ai_pre;
                ai_pre = U[i];
            }
            int cin[NW];                         // column characters entering after the row
            if (YROWS) {
                cin[0] = U[idx_in];              // past nc: any byte of the padded buffer
            } else {
                const bool cin_ok = (unsigned)idx_in < (unsigned)nc;
#pragma unroll
                for (int c = 0; c < NW; ++c) cin[c] = cin_ok ? V[c][idx_in] : 256;
            }
            bool anyc = false;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int* wc = w[YROWS ? 0 : c];
                int left = BIG;
                int e[MAXW];
#pragma unroll
                for (int k = 0; k < MAXW; ++k) {
                    const int up = (k + 1 < MAXW) ? R[c][(k + 1) < MAXW ? k + 1 : k] : BIG;
                    // min(up + 1, left + 1, diag + d) as min(up, left, diag - [match]) + 1
                    const int dg = R[c][k] - ((ai[c] == wc[(u + k) % MAXW]) ? 1 : 0);
                    const int v = min(min(up, left), dg) + 1;
                    e[k] = v + ek[k];
                    R[c][k] = v;
                    left = v;
                }
                int emin = e[0];
#pragma unroll
                for (int k = 1; k + 1 < MAXW; k += 2) emin = min(emin, min(e[k], e[k + 1]));
                if ((MAXW & 1) == 0) emin = min(emin, e[MAXW - 1]);
                const bool pass = emin <= t;
                passes[c] += pass ? 1 : 0;
                anyc = anyc || pass;
            }
            if (__builtin_amdgcn_ballot_w64(anyc) == 0 || i == nr) {
                go = false;
                break;
            }
#pragma unroll
            for (int c = 0; c < NW; ++c) {
                if (ROT) {
                    w[c][u] = cin[c];
                } else {
#pragma unroll
                    for (int k = 0; k + 1 < MAXW; ++k) w[c][k] = w[c][k + 1];
                    w[c][MAXW - 1] = cin[c];
                }
            }
            ++idx_in;
            ++row;
        }
    }
    const int kf = __builtin_amdgcn_readfirstlane(kfin);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        // branch-free: every lane takes the same path
        const bool all = passes[c] == nr;
        const int nrows = all ? nr : passes[c] + 1;
        const int out = min(R[c][kf], t + 1);
        cells[c] = act[c] ? band_cells(nrows, nc, a, b) : 0;
        res[c] = (act[c] && all) ? out : t + 1;
    }
}

// A lane's own copy of its indexed string in the wave's LDS (one slot per lane), read at
// wave-uniform offsets: no register-array indexing.  Bytes before and after the string are
// other lanes' bytes or padding, which the band DP may read wherever any byte will do.
struct LdsLaneChars {
    const __attribute__((address_space(3))) uint8_t* p;
    __device__ inline int operator[](int k) const { return (int)p[k]; }
};

// The band DP of vsp_seg in the form that keeps each cell's expected distance
// D(i, k) = M(i, k) + |kfin - k| instead of M: the recurrence keeps its shape,
//   D(i, k) = min(D(i-1, k) + [mismatch], D(i-1, k+1) + cu(k), D(i, k-1) + cl(k)),
// with cu(k) = 1 + ek(k) - ek(k+1) = 2 left of band index kfin (else 0) and
// cl(k) = 1 + ek(k) - ek(k-1) = 2 right of it (else 0), since adjacent diagonals' offsets
// differ by exactly one; a row passes when its smallest D is at most t (Lemma 4), and the
// distance is D at band index kfin, whose offset is 0.  Every cell is the M of vsp_seg plus a
// constant of its band index, so the rows evaluated and the verdicts are those of vsp_seg
// (which argues the unmasked band, the BIG borders and the pass counting).  KF >= 0 is kfin
// as a constant (the adjustments become adds of 2 on one side only); KF < 0 reads the
// adjustments from the table.  Member characters come from the lane's LDS copy, the probe's
// from the shared buffer; the row limit is folded into the last row's threshold, so a row
// costs one wave vote.
template <int MAXW, int KF, bool YROWS, int TS>
__device__ inline void vsp_lane(LdsChars U, int lu, LdsLaneChars V, int lv, int t,
                                const __attribute__((address_space(3))) int* tab, bool act,
                                int& cells, int& res)
{
    static_assert(MAXW <= 9 && KF < MAXW, "rotating window of at most 9 columns");
    const int nr = YROWS ? lv : lu;
    const int nc = YROWS ? lu : lv;
    const int delta = nc - nr;
    cells = 0;
    res = t + 1;
    if (delta > t) return;
    const int a = (t - delta) >> 1;
    const int b = (t + delta) >> 1;              // kfin: band index of cell (nr, nc)
    constexpr int BIG = 1 << 20;
    int D[MAXW], w[MAXW], cu[MAXW], cl[MAXW];
#pragma unroll
    for (int k = 0; k < MAXW; ++k) {
        D[k] = act ? tab[3 * TS + k] : BIG;
        if (KF < 0) {
            cu[k] = __builtin_amdgcn_readfirstlane(tab[4 * TS + k]);
            cl[k] = __builtin_amdgcn_readfirstlane(tab[5 * TS + k]);
        }
        // column window before row 1: column k - a (any byte outside 1..nc)
        w[k] = YROWS ? tab[2 * TS + k] : V[k - a];
    }
    int passes = 0;                              // rows passed before row nr
    if (nr > 0) {
        int done_rows = 0;
        for (;;) {
            // rows s+1 .. s+MAXW: row characters at s + u, entering column characters at
            // MAXW - a + s + u; the rotating window as in vsp_seg
            const int s = __builtin_amdgcn_readfirstlane(done_rows);
            const int lim = nr - 1 - s;          // steps u < lim are rows before row nr
            const auto rp = YROWS ? V.p + s : U.p + s;
            const auto cp = YROWS ? U.p + (MAXW - a) + s : V.p + (MAXW - a) + s;
            // the block's characters are read up front, so one LDS round trip serves MAXW rows
            // (past row nr they are padding or other lanes' bytes, never used)
            int rc[MAXW], cc[MAXW];
#pragma unroll
            for (int u = 0; u < MAXW; ++u) {
                rc[u] = rp[u];
                cc[u] = cp[u];
            }
            bool stop = false;
#pragma unroll
            for (int u = 0; u < MAXW; ++u) {
                const int ai = rc[u];
                const int cin = cc[u];
                int left = BIG;
#pragma unroll
                for (int k = 0; k < MAXW; ++k) {
                    const int up = (k + 1 < MAXW) ? D[(k + 1) < MAXW ? k + 1 : k] : BIG;
                    const int dg = D[k] + ((ai != w[(u + k) % MAXW]) ? 1 : 0);
                    int upa, lfa;
                    if constexpr (KF >= 0) {
                        upa = k < KF ? up + 2 : up;
                        lfa = k > KF ? left + 2 : left;
                    } else {
                        upa = up + cu[k];
                        lfa = left + cl[k];
                    }
                    // the band's first cell has no left neighbour and its last no upper one
                    // (both outside the band): those terms drop instead of entering as BIG
                    const int v = k == 0 ? (MAXW == 1 ? dg : min(upa, dg))
                                         : (k + 1 == MAXW ? min(lfa, dg) : min(min(upa, lfa), dg));
                    D[k] = v;
                    left = v;
                }
                int emin = D[0];
#pragma unroll
                for (int k = 1; k + 1 < MAXW; k += 2) emin = min(emin, min(D[k], D[k + 1]));
                if ((MAXW & 1) == 0) emin = min(emin, D[MAXW - 1]);
                // row nr counts as failed: the vote then ends the loop there
                const int th = u < lim ? t : -1;
                const bool pass = emin <= th;
                passes += pass ? 1 : 0;
                if (__builtin_amdgcn_ballot_w64(pass) == 0) {
                    stop = true;
                    break;
                }
                w[u] = cin;
            }
            if (stop) break;
            done_rows = s + MAXW;
        }
    }
    // a lane that passed every row before row nr evaluated all nr rows and its distance is D
    // at kfin; otherwise it evaluated the rows it passed and one more (cells from the table)
    const int rows = min(passes + 1, nr);
    int dk;
    if constexpr (KF >= 0) dk = D[KF];
    else dk = D[__builtin_amdgcn_readfirstlane(b)];
    res = (act && passes >= nr - 1) ? min(dk, t + 1) : t + 1;
    cells = act ? tab[6 * TS + rows] : 0;
}

// Two candidates per lane (members of one list, so one band geometry), packed as the low and
// high 16-bit halves of every cell: the same recurrence as vsp_seg, in packed 16-bit integer
// operations (the cost form min(up + 1, left + 1, diag + [mismatch]) keeps every value
// non-negative).  Cells start at kBig16 where vsp_seg starts at BIG; everything said there about
// the band, the wave vote and the pass counts holds per half.
typedef unsigned short pj_u16x2 __attribute__((ext_vector_type(2)));

__device__ inline pj_u16x2 as_u16x2(uint32_t x) { return __builtin_bit_cast(pj_u16x2, x); }
__device__ inline uint32_t as_u32(pj_u16x2 x) { return __builtin_bit_cast(uint32_t, x); }

template <int MAXW, bool YROWS, int TS>
__device__ inline void vsp_seg2(LdsChars U, int lu, const RegChars (&V)[2], int lv, int t,
                                const __attribute__((address_space(3))) int* tab,
                                const bool (&act)[2], int (&cells)[2], int (&res)[2])
{
    static_assert(MAXW <= 64, "one band index per table entry");
    const int nr = YROWS ? lv : lu;
    const int nc = YROWS ? lu : lv;
    const int delta = nc - nr;
    cells[0] = cells[1] = 0;
    res[0] = res[1] = t + 1;
    if (delta > t) return;
    const int a = (t - delta) >> 1;
    const int b = (t + delta) >> 1;
    const int kfin = delta + a;
    // 1 in both halves, opaque to the compiler: min(x, 1) stays one packed min instead of two
    // compares and selects
    uint32_t one_bits = 0x10001u;
    asm volatile("" : "+v"(one_bits));
    const pj_u16x2 ONE = as_u16x2(one_bits);
    const pj_u16x2 BIG = as_u16x2(kBig16 * 0x10001u);
    constexpr uint32_t NOCHAR = 256u * 0x10001u;  // matches no byte
    // halves of inactive candidates start at kBig16: they never pass a row
    const uint32_t keep = (act[0] ? 0x0000ffffu : 0u) | (act[1] ? 0xffff0000u : 0u);
    pj_u16x2 R[MAXW], ek[MAXW];
    uint32_t w[MAXW];
#pragma unroll
    for (int k = 0; k < MAXW; ++k) {
        const uint32_t r0 = (uint32_t)tab[k];
        R[k] = as_u16x2((r0 & keep) | (kBig16 * 0x10001u & ~keep));
        ek[k] = as_u16x2((uint32_t)tab[TS + k]);
        if (YROWS) {
            w[k] = (uint32_t)tab[2 * TS + k];
        } else {
            const int idx = k - a;
            w[k] = ((unsigned)idx < (unsigned)nc) ? reg_pair(V, idx) : NOCHAR;
        }
    }
    int idx_in = MAXW - a;
    uint32_t ai_pre = (!YROWS && nr > 0) ? (uint32_t)U[0] * 0x10001u : NOCHAR;
    int passes0 = 0, passes1 = 0;
    constexpr bool ROT = MAXW <= 9;
    constexpr int UNROLL = ROT ? MAXW : 1;
    int row = 1;
    bool go = nr > 0;
    while (go) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int i = __builtin_amdgcn_readfirstlane(row);
            uint32_t ai;
            if (YROWS) {
                ai = reg_pair(V, i - 1);
            } else {
                ai = ai_pre;
                ai_pre = (uint32_t)U[i] * 0x10001u;   // U[nr]: inside the padded buffer
            }
            uint32_t cin;
            if (YROWS) {
                cin = (uint32_t)U[idx_in] * 0x10001u;
            } else {
                cin = ((unsigned)idx_in < (unsigned)nc) ? reg_pair(V, idx_in) : NOCHAR;
            }
            pj_u16x2 left = BIG, emin = BIG;
#pragma unroll
            for (int k = 0; k < MAXW; ++k) {
                const pj_u16x2 up = (k + 1 < MAXW) ? R[(k + 1) < MAXW ? k + 1 : k] : BIG;
                // [mismatch] per half: min(a ^ b, 1)
                const pj_u16x2 d =
                    __builtin_elementwise_min(as_u16x2(ai ^ w[(u + k) % MAXW]), ONE);
                const pj_u16x2 v =
                    __builtin_elementwise_min(__builtin_elementwise_min(up, left) + ONE,
                                              R[k] + d);
                const pj_u16x2 e = v + ek[k];
                emin = k == 0 ? e : __builtin_elementwise_min(emin, e);
                R[k] = v;
                left = v;
            }
            const bool p0 = (int)emin.x <= t, p1 = (int)emin.y <= t;
            passes0 += p0 ? 1 : 0;
            passes1 += p1 ? 1 : 0;
            if (__builtin_amdgcn_ballot_w64(p0 || p1) == 0 || i == nr) {
                go = false;
                break;
            }
            if (ROT) {
                w[u] = cin;
            } else {
#pragma unroll
                for (int k = 0; k + 1 < MAXW; ++k) w[k] = w[k + 1];
                w[MAXW - 1] = cin;
            }
            ++idx_in;
            ++row;
        }
    }
    const int kf = __builtin_amdgcn_readfirstlane(kfin);
    const uint32_t fin = as_u32(R[kf]);
    const int out0 = min((int)(fin & 0xffffu), t + 1), out1 = min((int)(fin >> 16), t + 1);
    const bool all0 = passes0 == nr, all1 = passes1 == nr;
    cells[0] = act[0] ? band_cells(all0 ? nr : passes0 + 1, nc, a, b) : 0;
    cells[1] = act[1] ? band_cells(all1 ? nr : passes1 + 1, nc, a, b) : 0;
    res[0] = (act[0] && all0) ? out0 : t + 1;
    res[1] = (act[1] && all1) ? out1 : t + 1;
}

// ------------------------------------------------------------------------------------------
// Sharing computations on common prefixes (Sec. 5.3)
// ------------------------------------------------------------------------------------------

// Rows of a part's DP a lane keeps for the next member of its chain, as 4-bit values
// min(D, 15): with t <= 8, min(v, 15) commutes with the recurrence (min and non-negative
// additions) and every decision compares with t < 15, so a DP resumed from the clamped row
// takes the same early stop and returns the same min(t+1, distance).
constexpr int kShareRows = 16;

// The last member of a chain whose part DP ran, per side (left / right part).
struct SharePrev {
    const uint8_t* part;   // its part's bytes (nullptr: none yet)
    int rows;              // rows evaluated, including a stopping row
    int failed;            // stopped early (every expected distance of a row above t)
    int result;            // min(t+1, distance) when it did not stop early
    int stored;            // rows 1..stored of its DP are in the lane's matrix
};

// VerifyStringPair (Sec. 5.1, the function of Algorithm 3) of a member's part mp (length lm)
// against the probe string's part xp (length lx), sharing the rows it has in common with the
// previous member of the chain (pv): members of one list have parts of equal length and the
// same band.  With rows = the member's part (lm <= lx), row i depends on the member's first i
// bytes, so the rows within the common prefix c of the two parts are identical; with rows =
// the probe's part, row i reads the member's first min(i + b, lm) bytes, so rows up to c - b
// are.  The shared rows come from the lane's matrix (rows 1..min(shared, stored)) and the DP
// resumes after them; an early stop inside the shared rows, or identical parts, are inherited
// without any row.  Cells and the result are those of the unshared call (vsp_fast's
// recurrence on expected distances); cells of rows taken over are added to shared_cells.
// mat: the lane's matrix for this side, row r (1-based) at mat[(r - 1) * NW * 64 + w * 64].
template <int MAXW>
__device__ inline int share_part(const uint8_t* mp, int lm, const uint8_t* xp, int lx, int t,
                                 SharePrev& pv, __attribute__((address_space(3))) uint32_t* mat,
                                 uint64_t& cells, uint64_t& shared_rows, uint64_t& shared_cells)
{
    constexpr int NW = (MAXW + 7) / 8;
    constexpr int BIG = 1 << 20;
    const bool mrows = lm <= lx;
    const uint8_t* A = mrows ? mp : xp;
    const uint8_t* B = mrows ? xp : mp;
    const int nr = mrows ? lm : lx;
    const int nc = mrows ? lx : lm;
    const int delta = nc - nr;
    if (delta > t) {                          // no row is evaluated (the same for every member)
        pv.part = mp;
        pv.rows = 0;
        pv.failed = 1;
        pv.stored = 0;
        return t + 1;
    }
    const int a = (t - delta) >> 1;
    const int b = (t + delta) >> 1;
    int sh = 0;
    if (pv.part) {
        int c = 0;
        while (c < lm && pv.part[c] == mp[c]) ++c;
        sh = (c >= lm) ? nr : (mrows ? c : max(0, c - b));
        if (pv.failed && pv.rows <= sh) {     // stopped inside the shared rows: so does this one
            const int cl = band_cells(pv.rows, nc, a, b);
            cells += (uint64_t)cl;
            shared_cells += (uint64_t)cl;
            shared_rows += (uint64_t)pv.rows;
            pv.part = mp;
            return t + 1;
        }
        if (!pv.failed && sh >= nr) {         // identical rows throughout: the same distance
            const int cl = band_cells(nr, nc, a, b);
            cells += (uint64_t)cl;
            shared_cells += (uint64_t)cl;
            shared_rows += (uint64_t)nr;
            pv.part = mp;
            return pv.result;
        }
    }
    const int s0 = pv.part ? min(sh, pv.stored) : 0;
    int D[MAXW], w[MAXW], cu[MAXW], cl[MAXW];
    if (s0 == 0) {
#pragma unroll
        for (int k = 0; k < MAXW; ++k) {
            const int j = k - a;
            const int ek = b > k ? b - k : k - b;
            D[k] = (j >= 0 && j <= min(nc, b)) ? j + ek : BIG;
        }
    } else {
        const __attribute__((address_space(3))) uint32_t* row = mat + (s0 - 1) * NW * 64;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            const uint32_t v = row[q * 64];
#pragma unroll
            for (int k = 8 * q; k < MAXW && k < 8 * q + 8; ++k) D[k] = (int)((v >> (4 * (k - 8 * q))) & 15u);
        }
    }
#pragma unroll
    for (int k = 0; k < MAXW; ++k) {
        const int j = s0 - a + k;             // B index of band index k in row s0 + 1
        w[k] = ((unsigned)j < (unsigned)nc) ? (int)B[j] : 256;
        cu[k] = k < b ? 2 : 0;
        cl[k] = k > b ? 2 : 0;
    }
    int idx_in = s0 + MAXW - a;               // B index entering the window after row s0 + 1
    int cin = ((unsigned)idx_in < (unsigned)nc) ? (int)B[idx_in] : 256;
    int ai = (s0 < nr) ? (int)A[s0] : 256;
    int rows = nr;
    bool failed = false;
    for (int i = s0 + 1; i <= nr; ++i) {
        const int idx2 = idx_in + 1;
        const int cin_next = ((unsigned)idx2 < (unsigned)nc) ? (int)B[idx2] : 256;
        const int ai_next = (i < nr) ? (int)A[i] : 256;
        int left = BIG;
#pragma unroll
        for (int k = 0; k < MAXW; ++k) {
            const int up = (k + 1 < MAXW) ? D[(k + 1) < MAXW ? k + 1 : k] : BIG;
            const int dg = D[k] + ((ai != w[k]) ? 1 : 0);
            const int v = min(min(up + cu[k], left + cl[k]), dg);
            D[k] = v;
            left = v;
        }
        int emin = D[0];
#pragma unroll
        for (int k = 1; k < MAXW; ++k) emin = min(emin, D[k]);
        if (emin > t) {
            rows = i;
            failed = true;
            break;
        }
        if (i <= kShareRows) {                // keep the row for the next member
            __attribute__((address_space(3))) uint32_t* row = mat + (i - 1) * NW * 64;
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                uint32_t v = 0;
#pragma unroll
                for (int k = 8 * q; k < MAXW && k < 8 * q + 8; ++k)
                    v |= (uint32_t)min(D[k], 15) << (4 * (k - 8 * q));
                row[q * 64] = v;
            }
        }
#pragma unroll
        for (int k = 0; k + 1 < MAXW; ++k) w[k] = w[k + 1];
        w[MAXW - 1] = cin;
        cin = cin_next;
        idx_in = idx2;
        ai = ai_next;
    }
    const int cl_all = band_cells(rows, nc, a, b);
    const int cl_sh = band_cells(s0, nc, a, b);
    cells += (uint64_t)cl_all;
    shared_cells += (uint64_t)cl_sh;
    shared_rows += (uint64_t)s0;
    int out = BIG;
#pragma unroll
    for (int k = 0; k < MAXW; ++k) out = (k == b) ? D[k] : out;
    const int res = failed ? t + 1 : min(out, t + 1);
    pv.part = mp;
    pv.rows = rows;
    pv.failed = failed ? 1 : 0;
    pv.result = res;
    pv.stored = min(failed ? rows - 1 : rows, kShareRows);
    return res;
}

}  // namespace pj
