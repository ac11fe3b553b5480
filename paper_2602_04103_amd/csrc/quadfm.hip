// QuadFm on gfx950 (paper Appendix D): a count-only FM-index over the DNA alphabet whose rank
// queries run on a QuadRank layout: the 16-bit one by default, or any other QuadRank layout (the
// paper instantiates QuadFm with each of its rank structures).
//
// Index over T$ (length n+1):
//   - BWT of T$ with the single '$' stored as A at row dollar; rank_B(q, A) = rank(q, A) - [q > dollar]
//     corrects it (the sentinel handled by storing its position, Appendix D);
//   - C[c] = 1 + #{text characters < c} ('$' sorts first and occupies row 0's bucket);
//   - a lookup table of the interval of every k-mer (the prefix table for the first k characters
//     the backward search processes, i.e. the pattern's last k), built by k backward steps; k = 8
//     as in the paper by default, up to 12 as a build option.
// Count of pattern P (length m): start from table[P[m-k..m)] (or [0, n+1) when m < k), then for
// i = m-k-1 down to 0 (m-1 down to 0): c = P[i], sp = C[c] + rank_B(sp, c), ep = C[c] + rank_B(ep, c),
// stopping once sp >= ep; the count is ep - sp (0 when empty).  m = 0 counts n+1; a code > 3 counts 0.
//
// Two count kernels:
//   fm_batch_kernel       one lane per pattern; the host launches it once per batch of patterns;
//   fm_persistent_kernel  CUs x waves resident wavefronts pull patterns from a device queue: once
//                         at least `refill` lanes of a wave have finished (a tuning choice), the wave
//                         claims as many new patterns as it has idle lanes with one atomic add on
//                         the queue head, so lanes are refilled in batches while work remains (the
//                         GPU counterpart of the paper's active list with swap-pop).
// Both can write the final BWT interval [sp, ep) instead of its size (the paper's query_batch
// returns intervals).
//
// Locate (the extension the paper's closing section proposes), with a text-position sample of the
// suffix array: row k is marked iff SA[k] is a multiple of the sampling rate s, a BiRank over the
// n+1 mark bits gives each marked row its index into the stored SA values, and SA[k] of an
// unmarked row is found by LF steps, k <- C[B[k]] + rank_B(k, B[k]) (each steps one text position
// back), until a marked row: SA[k] = sample + steps, at most s - 1 steps.  The row of '$' has
// SA = 0 and is always marked, so the walk never steps through '$'.
#include <algorithm>
#include <mutex>
#include <new>

#include "birank_dev.hpp"
#include "common.hpp"
#include "quadrank_dev.hpp"

using namespace qr;

namespace qr {
int quadrank_build_into(const uint64_t *d_packed2, uint64_t n, int layout, uint64_t *lines, void *super,
                        hipStream_t stream);
}

struct qr_quadfm_s {
    int device;
    uint64_t n1;      // BWT length = n + 1
    uint64_t dollar;  // row of '$'
    uint64_t C[4];
    int layout;              // QuadRank layout of the BWT's rank structure (QR_LAYOUT_*)
    uint64_t n_lines, super_bytes;
    uint64_t *lines;
    void *super;             // the layout's offset array (a placeholder of 16 bytes when it has none)
    uint2 *table;                // 4^8 intervals (sp, ep)
    unsigned long long *head;    // device work-queue head
    uint32_t *err;               // sticky device error word (locate)
    qr_tuning tune;              // persistent kernel: block, refill threshold (per_lane), waves per CU
    uint32_t kmer;               // characters resolved by the start table (4^kmer entries)
    // locate support (absent until quadfm_locate_attach)
    qr_birank marks;             // BiRank (16-bit layout) over the n+1 mark bits
    uint32_t *samples;           // SA values of the marked rows, in row order
    uint64_t n_samples;
    uint32_t rate;
};

namespace {

constexpr uint32_t KMER_DEFAULT = 8, KMER_MAX = 12;  // the start table holds 4^k intervals

struct FmDev {
    const uint4 *lines;
    const void *super;
    const uint2 *table;
    uint64_t n1, dollar;
    uint64_t C0, C1, C2, C3;
    uint32_t *err;     // sticky error word: ERR_WALK (locate), ERR_OFFSETS (offsets that decrease or
                       // run past the pattern buffer)
    uint32_t kmer;     // characters resolved by the start table
    uint64_t pat_len;  // bytes of the pattern buffer of this call: no pattern may end beyond it
};

constexpr uint32_t ERR_WALK = 1u, ERR_OFFSETS = 2u;

__device__ __forceinline__ uint64_t fm_C(const FmDev &f, uint32_t c) {
    const uint64_t m1 = 0ull - (c & 1u), m2 = 0ull - ((c >> 1) & 1u);
    const uint64_t lo = (f.C0 & ~m1) | (f.C1 & m1), hi = (f.C2 & ~m1) | (f.C3 & m1);
    return (lo & ~m2) | (hi & m2);
}


template <class L>
__device__ __forceinline__ const typename L::Super *super_of(const FmDev &f) {
    return reinterpret_cast<const typename L::Super *>(f.super);
}

// The search works in 32-bit positions and ranks: the build admits at most 2^32 - 1 BWT rows.
template <class L>
__device__ __forceinline__ uint32_t rank_bwt32(const FmDev &f, const LaneHalf &h, uint32_t q, uint32_t c) {
    uint32_t r = lane_rank<L>(h, lane_slot<L>(q, h.j), c);
    if (c == 0) r -= q > f.dollar;
    return r;
}

// One backward step of the interval [sp, ep) with symbol c.  When sp and ep lie in the same half
// line (most steps once the interval is small) both ranks come from one load: the second load is
// issued only by the lanes whose ep lies elsewhere.
template <class L>
__device__ __forceinline__ void fm_step(const FmDev &f, uint32_t c, uint32_t &sp, uint32_t &ep) {
    LaneHalf a;
    load_lane_half<L>(f.lines, super_of<L>(f), sp, a);
    const uint32_t je = qline_of32<L>(ep);
    const bool same = a.j == je && (lane_slot<L>(sp, a.j) >= L::MID) == (lane_slot<L>(ep, je) >= L::MID);
    const uint32_t base = (uint32_t)fm_C(f, c);
    const uint32_t rs = rank_bwt32<L>(f, a, sp, c);
    uint32_t re;
    if (same) {
        re = rank_bwt32<L>(f, a, ep, c);
    } else {
        LaneHalf b;
        load_lane_half<L>(f.lines, super_of<L>(f), ep, b);
        re = rank_bwt32<L>(f, b, ep, c);
    }
    sp = base + rs;
    ep = base + re;
}

template <class L>
__global__ __launch_bounds__(256) void fm_table_kernel(FmDev f, uint2 *__restrict__ table) {
    const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= (1u << (2 * f.kmer))) return;
    uint32_t sp = 0, ep = (uint32_t)f.n1;
    for (uint32_t k = 0; k < f.kmer && sp < ep; ++k) fm_step<L>(f, (w >> (2 * k)) & 3u, sp, ep);
    if (sp >= ep) sp = ep = 0;
    table[w] = make_uint2((uint32_t)sp, (uint32_t)ep);
}

// Totals of each symbol in the BWT (rank at n+1) with '$' removed from A, and out4[4] = 1 iff
// the row of '$' holds A as the index requires.
template <class L>
__global__ void fm_totals_kernel(FmDev f, unsigned long long *__restrict__ out4) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const uint32_t n1 = (uint32_t)f.n1, d = (uint32_t)f.dollar;
    LaneHalf h, d0, d1;
    load_lane_half<L>(f.lines, super_of<L>(f), n1, h);
    load_lane_half<L>(f.lines, super_of<L>(f), d, d0);
    load_lane_half<L>(f.lines, super_of<L>(f), d + 1, d1);
    const uint32_t p = lane_slot<L>(n1, h.j);
    out4[0] = (uint64_t)lane_rank<L>(h, p, 0) - 1;
    out4[1] = lane_rank<L>(h, p, 1);
    out4[2] = lane_rank<L>(h, p, 2);
    out4[3] = lane_rank<L>(h, p, 3);
    out4[4] = lane_rank<L>(d1, lane_slot<L>(d + 1, d1.j), 0) - lane_rank<L>(d0, lane_slot<L>(d, d0.j), 0);
}

// Per-lane search state.  The backward search over a pattern P reads P from its end; over the
// reverse complement of P it reads P from its start and complements every code (c -> 3 - c).
//
// Patterns come as one byte per code, or (PACKED) as 2-bit codes in a stream of u64 words: base i of
// the stream is bits [2 (i mod 32), +2) of word i / 32, and a pattern is a range of stream bases.
struct Search {
    uint32_t sp, ep;   // the current BWT interval (every row index is below 2^32)
    const uint8_t *P;  // pattern start (PACKED: the stream's first word)
    uint64_t base;     // PACKED: stream index of the pattern's first base
    uint32_t m;        // pattern length
    uint32_t left;     // characters still to process
    uint32_t pos;      // index in P of the next character to read
    uint32_t rc;       // 0: P itself, 1: its reverse complement
    uint32_t acc;      // count of the first strand, when counting both
    uint64_t buf;      // pattern bytes [win, win + wlen) (8 of them, or 1 near the pattern ends);
                       // PACKED: stream word win (32 bases), valid when wlen != 0
    uint32_t win;      // index in P of buf's first byte; ~0u before the first fetch
    uint32_t wlen;     // 8 or 1 (PACKED: 32, or 0 before the first fetch)
};

__device__ __forceinline__ uint32_t strand_code(uint32_t c, uint32_t rc) { return (rc && c <= 3u) ? 3u - c : c; }

// Sum of the two strands' counts, saturating at 2^32 - 1 (reachable only for texts over 2^31 bases).
__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b) {
    const uint64_t t = (uint64_t)a + b;
    return t > 0xffffffffull ? 0xffffffffu : (uint32_t)t;
}

// Next character of the current strand.  Characters are fetched 8 at a time with one aligned load
// when the whole aligned 8-byte window lies inside the pattern [P, P + m), else one byte at a time.
// Packed characters are fetched 32 at a time, one stream word: a word that holds a base of the
// pattern lies inside the stream.  (Words of one pattern differ by less than 2^27, so the low 32
// bits of a word index tell them apart.)
template <bool PACKED>
__device__ __forceinline__ uint32_t next_char(Search &s) {
    const uint32_t i = s.pos;
    if constexpr (PACKED) {
        const uint64_t a = s.base + i;
        const uint32_t w = (uint32_t)(a >> 5);
        if (s.wlen == 0 || w != s.win) {
            s.buf = reinterpret_cast<const uint64_t *>(s.P)[a >> 5];
            s.win = w;
            s.wlen = 32;
        }
        s.pos = s.rc ? i + 1 : i - 1;
        const uint32_t c = (uint32_t)(s.buf >> (2 * (a & 31u))) & 3u;
        return s.rc ? 3u - c : c;
    }
    if (s.win == ~0u || i < s.win || i - s.win >= s.wlen) {
        const uintptr_t lo = (uintptr_t)s.P, a = lo + i;
        const uintptr_t w = a & ~(uintptr_t)7;
        if (w >= lo && w + 8 <= lo + s.m) {
            s.win = (uint32_t)(w - lo);
            s.wlen = 8;
            s.buf = *reinterpret_cast<const uint64_t *>(w);
        } else {
            s.win = i;
            s.wlen = 1;
            s.buf = *reinterpret_cast<const uint8_t *>(a);
        }
    }
    const uint32_t c = (uint32_t)(s.buf >> (8 * (i - s.win))) & 0xffu;
    s.pos = s.rc ? i + 1 : i - 1;
    return strand_code(c, s.rc);
}

// Start the search of one strand; returns true if its count is already known (written to cnt).
template <bool PACKED>
__device__ __forceinline__ bool fm_start(const FmDev &f, Search &s, uint32_t rc, uint32_t &cnt) {
    s.rc = rc;
    s.win = ~0u;
    s.wlen = 0;
    const uint32_t m = s.m;
    const uint32_t K = f.kmer;
    if (m >= K) {
        // The first K characters searched: P[m-K..m) for P, the complement of P[0..K) reversed for
        // rc(P).  Their table index is the sum of code_j * 4^j over the characters in the order the
        // search reads them (j = 0 first), so they are read through the same 8-byte window as the
        // later steps, which then continue from where it stands.
        s.pos = rc ? 0 : m - 1;
        uint32_t w = 0;
        bool bad = false;
        for (uint32_t j = 0; j < K; ++j) {
            const uint32_t c = next_char<PACKED>(s);
            bad |= c > 3;
            w |= (c & 3u) << (2 * j);
        }
        if (bad) {
            cnt = 0;
            return true;
        }
        const uint2 iv = f.table[w];
        s.sp = iv.x;
        s.ep = iv.y;
        s.left = m - K;
    } else {
        s.sp = 0;
        s.ep = (uint32_t)f.n1;
        s.left = m;
        s.pos = rc ? 0 : m - 1;
    }
    if (s.sp >= s.ep || s.left == 0) {
        cnt = s.sp < s.ep ? (uint32_t)(s.ep - s.sp) : 0u;
        return true;
    }
    return false;
}

// Initialise the search for a pattern; returns true if its count is already known (written to cnt).
// The offsets count bytes, or (PACKED) stream bases; f.pat_len is the buffer's length in the same unit.
template <bool BOTH, bool PACKED>
__device__ __forceinline__ bool fm_init(const FmDev &f, const uint8_t *__restrict__ pat, const uint64_t *__restrict__ off,
                                        uint64_t p, Search &s, uint32_t &cnt) {
    const uint64_t o = off[p], e = off[p + 1];
    if (e < o || e > f.pat_len || e - o > 0xffffffffull) {  // not a pattern: nothing of it is read
        atomicOr(f.err, ERR_OFFSETS);
        s.m = 0;
        cnt = 0;
        return true;
    }
    const uint64_t m = e - o;
    s.P = PACKED ? pat : pat + o;
    s.base = o;
    s.m = (uint32_t)m;
    s.acc = 0;
    if (m == 0) {  // the empty pattern matches at every position 0..n (counted once)
        cnt = (uint32_t)f.n1;
        return true;
    }
    if (!fm_start<PACKED>(f, s, 0, cnt)) return false;
    if (!BOTH) return true;
    s.acc = cnt;  // forward strand finished at once: go on with the reverse complement
    if (!fm_start<PACKED>(f, s, 1, cnt)) return false;
    cnt = sat_add(cnt, s.acc);
    return true;
}

// Advance one character; returns true when the pattern's count is final (in cnt).
template <class L, bool BOTH, bool PACKED>
__device__ __forceinline__ bool fm_advance(const FmDev &f, Search &s, uint32_t &cnt) {
    const uint32_t c = next_char<PACKED>(s);
    bool fin;
    if (c > 3) {
        cnt = 0;
        fin = true;
    } else {
        fm_step<L>(f, c, s.sp, s.ep);
        --s.left;
        fin = s.sp >= s.ep || s.left == 0;
        if (fin) cnt = s.sp < s.ep ? (uint32_t)(s.ep - s.sp) : 0u;
    }
    if (!fin) return false;
    if (!BOTH || s.rc) {
        cnt = sat_add(cnt, s.acc);
        return true;
    }
    s.acc = cnt;  // forward strand done: start the reverse complement
    if (!fm_start<PACKED>(f, s, 1, cnt)) return false;
    cnt = sat_add(cnt, s.acc);
    return true;
}

// Write a finished pattern's result: its count, or (IV) its final interval, [0, 0) when empty.
template <bool IV>
__device__ __forceinline__ void emit(const FmDev &f, uint32_t *__restrict__ out, uint64_t p, const Search &s,
                                     uint32_t cnt) {
    if (!IV) {
        out[p] = cnt;
        return;
    }
    uint2 v = make_uint2(0u, 0u);
    if (cnt) v = s.m == 0 ? make_uint2(0u, (uint32_t)f.n1) : make_uint2((uint32_t)s.sp, (uint32_t)s.ep);
    reinterpret_cast<uint2 *>(out)[p] = v;
}

template <class L, bool BOTH, bool IV>
__global__ __launch_bounds__(256) void fm_batch_kernel(FmDev f, const uint8_t *__restrict__ pat,
                                                       const uint64_t *__restrict__ off, uint64_t p0, uint64_t np,
                                                       uint32_t *__restrict__ out) {
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    const uint64_t p = p0 + k;
    Search s;
    uint32_t cnt = 0;
    if (!fm_init<BOTH, false>(f, pat, off, p, s, cnt))
        while (!fm_advance<L, BOTH, false>(f, s, cnt)) {
        }
    emit<IV>(f, out, p, s, cnt);
}

__global__ void fill_zero_u64(unsigned long long *p) { *p = 0ull; }

template <class L, bool BOTH, bool IV, bool PACKED>
__global__ __launch_bounds__(256) void fm_persistent_kernel(FmDev f, const uint8_t *__restrict__ pat,
                                                            const uint64_t *__restrict__ off, uint64_t npat,
                                                            uint32_t *__restrict__ out,
                                                            unsigned long long *__restrict__ head, uint32_t refill_min) {
    const uint32_t lane = __lane_id();
    bool active = false, drained = false;
    uint64_t p = 0;
    Search s;
    s.sp = s.ep = 0;
    s.P = pat;
    s.base = 0;
    s.m = s.left = s.pos = s.rc = s.acc = 0;
    s.buf = 0;
    s.win = ~0u;
    s.wlen = 0;
    while (true) {
        if (!drained) {
            const uint64_t idle = __ballot(!active);
            const uint32_t nidle = __popcll(idle);
            if (nidle != 0 && (nidle >= refill_min || nidle == 64)) {
                const uint32_t leader = __ffsll((unsigned long long)idle) - 1;
                unsigned long long got = 0;
                if (lane == leader) got = atomicAdd(head, (unsigned long long)nidle);
                got = __shfl(got, leader, 64);
                if (got + nidle >= npat) drained = true;
                if (!active) {
                    const uint32_t rank = __popcll(idle & ((1ull << lane) - 1ull));
                    const uint64_t mine = got + rank;
                    if (mine < npat) {
                        p = mine;
                        uint32_t cnt = 0;
                        if (fm_init<BOTH, PACKED>(f, pat, off, p, s, cnt)) emit<IV>(f, out, p, s, cnt);
                        else active = true;
                    }
                }
            }
        }
        if (!__any(active)) {
            if (drained) break;
            continue;
        }
        if (active) {
            uint32_t cnt = 0;
            if (fm_advance<L, BOTH, PACKED>(f, s, cnt)) {
                emit<IV>(f, out, p, s, cnt);
                active = false;
            }
        }
    }
}

// ---- locate ---------------------------------------------------------------------------------------
// start[i] = sum over k < i of (ep_k - sp_k), i = 0..npat, in three passes over tiles of
// ISCAN_TILE intervals without any workspace: (1) each tile's total goes to start[first index of
// the tile]; (2) one workgroup turns those totals into exclusive tile offsets in place and writes
// start[npat]; (3) each tile reads its offset, then scans its intervals over it.
constexpr int ISCAN_BLOCK = 256, ISCAN_ITEMS = 16;
constexpr uint64_t ISCAN_TILE = (uint64_t)ISCAN_BLOCK * ISCAN_ITEMS;

__device__ __forceinline__ uint64_t iv_len(const uint2 *__restrict__ iv, uint64_t i, uint64_t npat) {
    if (i >= npat) return 0;
    const uint2 e = iv[i];
    return e.y > e.x ? e.y - e.x : 0u;
}

// Block-wide exclusive scan of one value per thread; returns the exclusive prefix, total in *tot.
__device__ __forceinline__ uint64_t block_exclusive(uint64_t v, uint64_t *wave_tot, uint64_t *tot) {
    const uint32_t t = threadIdx.x;
    const uint64_t incl = wave_inclusive_scan<uint64_t>(v);
    if (__lane_id() == 63) wave_tot[t / 64] = incl;
    __syncthreads();
    uint64_t before = incl - v, all = 0;
    for (uint32_t w = 0; w < blockDim.x / 64; ++w) {
        if (w < t / 64) before += wave_tot[w];
        all += wave_tot[w];
    }
    *tot = all;
    return before;
}

__global__ __launch_bounds__(ISCAN_BLOCK) void iv_tile_totals(const uint2 *__restrict__ iv, uint64_t npat,
                                                              unsigned long long *__restrict__ start) {
    __shared__ uint64_t wave_tot[ISCAN_BLOCK / 64];
    const uint64_t i0 = blockIdx.x * ISCAN_TILE + (uint64_t)threadIdx.x * ISCAN_ITEMS;
    uint64_t mine = 0;
#pragma unroll
    for (int k = 0; k < ISCAN_ITEMS; ++k) mine += iv_len(iv, i0 + k, npat);
    uint64_t tot;
    (void)block_exclusive(mine, wave_tot, &tot);
    if (threadIdx.x == 0) start[blockIdx.x * ISCAN_TILE] = tot;
}

constexpr int ISCAN_TOP = 1024;

__global__ __launch_bounds__(ISCAN_TOP) void iv_tile_offsets(uint64_t ntiles, uint64_t npat,
                                                             unsigned long long *__restrict__ start) {
    __shared__ uint64_t wave_tot[ISCAN_TOP / 64];
    __shared__ uint64_t chunk_total;
    uint64_t carry = 0;
    for (uint64_t b0 = 0; b0 < ntiles; b0 += ISCAN_TOP) {
        const uint64_t b = b0 + threadIdx.x;
        const uint64_t v = b < ntiles ? start[b * ISCAN_TILE] : 0;
        uint64_t tot;
        const uint64_t before = block_exclusive(v, wave_tot, &tot);
        if (b < ntiles) start[b * ISCAN_TILE] = carry + before;
        if (threadIdx.x == 0) chunk_total = tot;
        __syncthreads();
        carry += chunk_total;
        __syncthreads();
    }
    if (threadIdx.x == 0) start[npat] = carry;
}

__global__ __launch_bounds__(ISCAN_BLOCK) void iv_tile_scan(const uint2 *__restrict__ iv, uint64_t npat,
                                                            unsigned long long *__restrict__ start) {
    __shared__ uint64_t wave_tot[ISCAN_BLOCK / 64];
    __shared__ uint64_t tile_off;
    if (threadIdx.x == 0) tile_off = start[blockIdx.x * ISCAN_TILE];
    __syncthreads();  // the offset is read before this tile overwrites its first entry
    const uint64_t i0 = blockIdx.x * ISCAN_TILE + (uint64_t)threadIdx.x * ISCAN_ITEMS;
    uint64_t v[ISCAN_ITEMS], mine = 0;
#pragma unroll
    for (int k = 0; k < ISCAN_ITEMS; ++k) {
        v[k] = mine;
        mine += iv_len(iv, i0 + k, npat);
    }
    uint64_t tot;
    const uint64_t before = tile_off + block_exclusive(mine, wave_tot, &tot);
#pragma unroll
    for (int k = 0; k < ISCAN_ITEMS; ++k)
        if (i0 + k < npat) start[i0 + k] = before + v[k];
}

struct LocDev {
    const uint4 *mlines;      // BiRank (16-bit layout) over the mark bits
    const uint32_t *msuper;
    const uint32_t *samples;  // SA values of the marked rows
    uint32_t rate;
};

// SA[row] by LF steps to the nearest marked row (at most rate - 1 of them); false if none is
// reached within rate steps, which only inconsistent sample data can cause.
template <class L>
__device__ __forceinline__ bool sa_of_row(const FmDev &f, const LocDev &d, uint64_t row64, uint32_t &pos) {
    if (row64 >= f.n1) return false;
    uint32_t row = (uint32_t)row64;  // rows of an FM-index are below 2^32
    for (uint32_t steps = 0; steps < d.rate && row < f.n1; ++steps) {
        uint32_t marked = 0;
        const uint64_t k = br_rank_bit<BR16>(d.mlines, d.msuper, row, marked);
        if (marked) {
            pos = d.samples[k] + steps;
            return true;
        }
        LaneHalf h;
        load_lane_half<L>(f.lines, super_of<L>(f), row, h);
        const uint32_t c = lane_symbol(h, lane_slot<L>(row, h.j));
        row = (uint32_t)fm_C(f, c) + rank_bwt32<L>(f, h, row, c);
    }
    return false;
}

// One lane per output: output g belongs to the last pattern p with start[p] <= g, and is
// SA[sp_p + g - start[p]].
template <class L>
__global__ __launch_bounds__(256) void fm_locate_kernel(FmDev f, LocDev d, const uint2 *__restrict__ iv,
                                                        const unsigned long long *__restrict__ start, uint64_t npat,
                                                        uint64_t total, uint32_t *__restrict__ pos,
                                                        uint32_t *__restrict__ err) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
        uint64_t lo = 0, hi = npat;  // start[lo] <= g < start[hi]
        while (hi - lo > 1) {
            const uint64_t mid = (lo + hi) >> 1;
            if (start[mid] <= g) lo = mid;
            else hi = mid;
        }
        const uint64_t row = iv[lo].x + (g - start[lo]);
        uint32_t v = 0;
        if (!sa_of_row<L>(f, d, row, v)) {
            v = 0xffffffffu;
            atomicOr(err, ERR_WALK);
        }
        pos[g] = v;
    }
}

// f(L{}) for the trait type of a QuadRank layout the index can use (the 16-bit one by default).
template <class F>
auto fm_layout(int layout, F &&f) {
    switch (layout) {
        case QR_LAYOUT_16P: return f(QR16P{});
        case QR_LAYOUT_32: return f(QR32{});
        case QR_LAYOUT_64: return f(QR64{});
        case QR_LAYOUT_24_8: return f(QR24_8{});
        default: return f(QR16{});
    }
}

bool fm_layout_ok(int layout) {
    return layout == QR_LAYOUT_16 || layout == QR_LAYOUT_16P || layout == QR_LAYOUT_32 || layout == QR_LAYOUT_64 ||
           layout == QR_LAYOUT_24_8;
}

void release(qr_quadfm_s *h) {
    if (!h) return;
    if (h->marks) (void)birank_free(h->marks);
    if (h->samples) (void)hipFree(h->samples);
    if (h->lines) (void)hipFree(h->lines);
    if (h->super) (void)hipFree(h->super);
    if (h->table) (void)hipFree(h->table);
    if (h->head) (void)hipFree(h->head);
    if (h->err) (void)hipFree(h->err);
    delete h;
}

FmDev dev_view(const qr_quadfm_s *h) {
    FmDev f;
    f.lines = reinterpret_cast<const uint4 *>(h->lines);
    f.super = h->super;
    f.table = h->table;
    f.n1 = h->n1;
    f.dollar = h->dollar;
    f.C0 = h->C[0], f.C1 = h->C[1], f.C2 = h->C[2], f.C3 = h->C[3];
    f.err = h->err;
    f.kmer = h->kmer;
    f.pat_len = 0;
    return f;
}

// Pattern buffer length for the calls without one: the caller vouches that the CSR lies inside
// d_pat (unbounded), except that a NULL buffer holds no byte.
uint64_t implied_len(const uint8_t *d_pat) { return d_pat ? ~0ull : 0ull; }

int count_args(qr_quadfm h, const uint8_t *d_pat, uint64_t pat_bytes, const uint64_t *d_off, uint64_t npat,
               uint32_t *d_count, const char *what) {
    if (!h || (npat && (!d_off || !d_count))) {
        set_error("%s: null handle or pointer", what);
        return QR_EINVAL;
    }
    if (!d_pat && pat_bytes) {
        set_error("%s: d_pat is NULL but pat_bytes = %llu", what, (unsigned long long)pat_bytes);
        return QR_EINVAL;
    }
    if (((uintptr_t)d_off & 7) || ((uintptr_t)d_count & 3)) {
        set_error("%s: d_off must be 8-byte and d_count 4-byte aligned", what);
        return QR_EINVAL;
    }
    // d_pat may be NULL when every pattern is empty; the kernels treat any pattern ending beyond
    // pat_bytes like a decreasing offset pair (counted 0, sticky error, nothing read)
    return check_device(h->device);
}

}  // namespace

extern "C" {

int quadfm_build_layout(const uint64_t *d_bwt_packed2, uint64_t n_plus_1, uint64_t dollar_pos, uint32_t kmer,
                        int layout, hipStream_t stream, qr_quadfm *out) {
    if (!out) return QR_EINVAL;
    *out = nullptr;
    if (!fm_layout_ok(layout)) {
        set_error("quadfm_build: layout %d is not a QuadRank layout with one-lane queries (16, 16P, 32, 64, 24_8)",
                  layout);
        return QR_EINVAL;
    }
    if (kmer < 1 || kmer > KMER_MAX) {
        set_error("quadfm_build: the start table resolves 1..%u characters, not %u", KMER_MAX, kmer);
        return QR_EINVAL;
    }
    if (!d_bwt_packed2 || n_plus_1 == 0 || dollar_pos >= n_plus_1 || ((uintptr_t)d_bwt_packed2 & 7)) {
        set_error("quadfm_build: need a BWT of n+1 >= 1 symbols and dollar_pos < n+1");
        return QR_EINVAL;
    }
    if (n_plus_1 > 0xffffffffull) {
        set_error("quadfm_build: n+1 = %llu exceeds the u32 interval limit", (unsigned long long)n_plus_1);
        return QR_ERANGE;
    }
    qr_quadfm_s *h = new (std::nothrow) qr_quadfm_s{};
    if (!h) return QR_ENOMEM;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return QR_EHIP;
    }
    h->n1 = n_plus_1;
    h->dollar = dollar_pos;
    h->kmer = kmer;
    h->layout = layout;
    const uint64_t entries = 1ull << (2 * kmer);
    fm_layout(layout, [&](auto tag) {
        using L = decltype(tag);
        h->n_lines = n_plus_1 / L::DATA + 1;
        const uint64_t n_sb = L::SB_LINES ? (h->n_lines - 1) / L::SB_LINES + 1 : 0;
        h->super_bytes = n_sb * 4 * sizeof(typename L::Super);
        return 0;
    });
    h->tune = qr_tuning{256, 16, 16, 0, 0};
    unsigned long long *tot = nullptr;
    if (hipMalloc(&h->lines, h->n_lines * 128) != hipSuccess ||
        hipMalloc(&h->super, std::max<uint64_t>(h->super_bytes, 16)) != hipSuccess ||
        hipMalloc(&h->table, entries * sizeof(uint2)) != hipSuccess || hipMalloc(&h->head, 8) != hipSuccess ||
        hipMalloc(&h->err, 4) != hipSuccess || hipMalloc(&tot, 40) != hipSuccess) {
        (void)hipGetLastError();
        if (tot) (void)hipFree(tot);
        release(h);
        set_error("quadfm_build: device allocation failed");
        return QR_ENOMEM;
    }
    int rc = quadrank_build_into(d_bwt_packed2, n_plus_1, layout, h->lines, h->super, stream);
    if (rc) {
        (void)hipFree(tot);
        release(h);
        return rc;
    }
    FmDev f = dev_view(h);
    fm_layout(layout, [&](auto tag) {
        hipLaunchKernelGGL(fm_totals_kernel<decltype(tag)>, dim3(1), dim3(64), 0, stream, f, tot);
        return 0;
    });
    unsigned long long t[5] = {0, 0, 0, 0, 0};
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(t, tot, 40, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    (void)hipFree(tot);
    if (e != hipSuccess) {
        set_error("quadfm_build: %s", hipGetErrorString(e));
        release(h);
        return QR_EHIP;
    }
    uint64_t acc = 1;
    for (int c = 0; c < 4; ++c) {
        h->C[c] = acc;
        acc += t[c];
    }
    if (acc != n_plus_1 || t[4] != 1) {
        set_error("quadfm_build: the BWT row dollar_pos must hold A (code 0)");
        release(h);
        return QR_EINVAL;
    }
    f = dev_view(h);
    fm_layout(layout, [&](auto tag) {
        hipLaunchKernelGGL(fm_table_kernel<decltype(tag)>, dim3((uint32_t)((entries + 255) / 256)), dim3(256), 0, stream,
                           f, h->table);
        return 0;
    });
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemsetAsync(h->err, 0, 4, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        set_error("quadfm_build: %s", hipGetErrorString(e));
        release(h);
        return QR_EHIP;
    }
    *out = h;
    return QR_OK;
}

int quadfm_build_ex(const uint64_t *d_bwt_packed2, uint64_t n_plus_1, uint64_t dollar_pos, uint32_t kmer,
                    hipStream_t stream, qr_quadfm *out) {
    return quadfm_build_layout(d_bwt_packed2, n_plus_1, dollar_pos, kmer, QR_LAYOUT_16, stream, out);
}

int quadfm_build(const uint64_t *d_bwt_packed2, uint64_t n_plus_1, uint64_t dollar_pos, hipStream_t stream,
                 qr_quadfm *out) {
    return quadfm_build_layout(d_bwt_packed2, n_plus_1, dollar_pos, KMER_DEFAULT, QR_LAYOUT_16, stream, out);
}

int quadfm_layout_kind(qr_quadfm h) { return h ? h->layout : -1; }

// flags: QUADFM_BOTH_STRANDS; iv: write intervals (uint2 per pattern) instead of counts; packed: the
// patterns are 2-bit codes in a stream of u64 words at d_pat, pat_bytes and the offsets count bases
static int count_persistent(qr_quadfm h, const uint8_t *d_pat, uint64_t pat_bytes, const uint64_t *d_off, uint64_t npat,
                            uint32_t *d_count, unsigned long long *head, uint32_t flags, bool iv, hipStream_t stream,
                            bool packed = false) {
    const int block = h->tune.block ? h->tune.block : 256;
    const uint32_t refill = h->tune.per_lane > 0 ? (uint32_t)h->tune.per_lane : 16u;
    const int wpc = h->tune.grid_waves > 0 ? h->tune.grid_waves : 16;
    uint64_t blocks = (uint64_t)cu_count() * wpc * 64 / block;
    const uint64_t need = (npat + block - 1) / block;  // no more waves than patterns need
    blocks = std::max<uint64_t>(1, std::min(blocks, need));
    hipLaunchKernelGGL(fill_zero_u64, dim3(1), dim3(1), 0, stream, head);
    QR_HIP(hipGetLastError());
    const dim3 g((uint32_t)blocks), b(block);
    FmDev f = dev_view(h);
    f.pat_len = pat_bytes;
    fm_layout(h->layout, [&](auto tag) {
        using L = decltype(tag);
        if (iv)
            hipLaunchKernelGGL((fm_persistent_kernel<L, false, true, false>), g, b, 0, stream, f, d_pat, d_off, npat,
                               d_count, head, refill);
        else if (packed && (flags & QUADFM_BOTH_STRANDS))
            hipLaunchKernelGGL((fm_persistent_kernel<L, true, false, true>), g, b, 0, stream, f, d_pat, d_off, npat,
                               d_count, head, refill);
        else if (packed)
            hipLaunchKernelGGL((fm_persistent_kernel<L, false, false, true>), g, b, 0, stream, f, d_pat, d_off, npat,
                               d_count, head, refill);
        else if (flags & QUADFM_BOTH_STRANDS)
            hipLaunchKernelGGL((fm_persistent_kernel<L, true, false, false>), g, b, 0, stream, f, d_pat, d_off, npat,
                               d_count, head, refill);
        else
            hipLaunchKernelGGL((fm_persistent_kernel<L, false, false, false>), g, b, 0, stream, f, d_pat, d_off, npat,
                               d_count, head, refill);
        return 0;
    });
    QR_HIP(hipGetLastError());
    return QR_OK;
}

int quadfm_count_ex(qr_quadfm h, const uint8_t *d_pat, uint64_t pat_bytes, const uint64_t *d_off, uint64_t npat,
                    uint32_t flags, uint32_t *d_count, void *d_workspace, hipStream_t stream) {
    int rc = count_args(h, d_pat, pat_bytes, d_off, npat, d_count, "quadfm_count_ex");
    if (rc) return rc;
    if (flags & ~QUADFM_BOTH_STRANDS) {
        set_error("quadfm_count_ex: unknown flag bits 0x%x", flags);
        return QR_EINVAL;
    }
    if (d_workspace && ((uintptr_t)d_workspace & 7)) {
        set_error("quadfm_count_ex: d_workspace must be 8-byte aligned");
        return QR_EINVAL;
    }
    if (!npat) return QR_OK;
    unsigned long long *head = d_workspace ? reinterpret_cast<unsigned long long *>(d_workspace) : h->head;
    return count_persistent(h, d_pat, pat_bytes, d_off, npat, d_count, head, flags, false, stream);
}

int quadfm_count_packed(qr_quadfm h, const uint64_t *d_pat2, uint64_t pat_bases, const uint64_t *d_off, uint64_t npat,
                        uint32_t flags, uint32_t *d_count, void *d_workspace, hipStream_t stream) {
    int rc = count_args(h, reinterpret_cast<const uint8_t *>(d_pat2), pat_bases, d_off, npat, d_count,
                        "quadfm_count_packed");
    if (rc) return rc;
    if (flags & ~QUADFM_BOTH_STRANDS) {
        set_error("quadfm_count_packed: unknown flag bits 0x%x", flags);
        return QR_EINVAL;
    }
    if (((uintptr_t)d_pat2 & 7) || (d_workspace && ((uintptr_t)d_workspace & 7))) {
        set_error("quadfm_count_packed: d_pat2 and d_workspace must be 8-byte aligned");
        return QR_EINVAL;
    }
    if (!npat) return QR_OK;
    unsigned long long *head = d_workspace ? reinterpret_cast<unsigned long long *>(d_workspace) : h->head;
    return count_persistent(h, reinterpret_cast<const uint8_t *>(d_pat2), pat_bases, d_off, npat, d_count, head, flags,
                            false, stream, true);
}

int quadfm_intervals(qr_quadfm h, const uint8_t *d_pat, uint64_t pat_bytes, const uint64_t *d_off, uint64_t npat,
                     uint32_t *d_iv, hipStream_t stream) {
    int rc = count_args(h, d_pat, pat_bytes, d_off, npat, d_iv, "quadfm_intervals");
    if (rc) return rc;
    if ((uintptr_t)d_iv & 7) {
        set_error("quadfm_intervals: d_iv must be 8-byte aligned");
        return QR_EINVAL;
    }
    if (!npat) return QR_OK;
    return count_persistent(h, d_pat, pat_bytes, d_off, npat, d_iv, h->head, 0u, true, stream);
}

// ---- quadfm_count_noalloc -------------------------------------------------------------------------
// The persistent count's only memory beyond its inputs and outputs is the 8-byte work-queue head.
// For callers that cannot allocate, the head lives in this file-scope device array: every device
// the library runs on holds its own copy until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the symbol): the device address
// of each device's copy is looked up once, with that device current, and kept.
constexpr uint64_t NOALLOC_SCRATCH_BYTES = 256;  // one queue head is used; the rest pads the array
static __device__ __align__(256) unsigned long long scratch[NOALLOC_SCRATCH_BYTES / 8];

constexpr int NOALLOC_MAX_DEVICES = 64;

// Device address of the current device's scratch array (looked up on the first call per device).
static int scratch_address(unsigned long long **out) {
    static std::mutex mu;
    static unsigned long long *addr[NOALLOC_MAX_DEVICES] = {nullptr};
    int dev = -1;
    QR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        set_error("quadfm_count_noalloc: device %d is beyond the %d devices the library tracks", dev,
                  NOALLOC_MAX_DEVICES);
        return QR_EINVAL;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error("quadfm_count_noalloc: hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
            return QR_EHIP;
        }
        addr[dev] = reinterpret_cast<unsigned long long *>(ptr);
    }
    *out = addr[dev];
    return QR_OK;
}

int quadfm_count_noalloc(qr_quadfm h, const uint8_t *d_pat, uint64_t pat_bytes, const uint64_t *d_off, uint64_t npat,
                         uint32_t flags, uint32_t *d_count, hipStream_t stream) {
    int rc = count_args(h, d_pat, pat_bytes, d_off, npat, d_count, "quadfm_count_noalloc");
    if (rc) return rc;
    if (flags & ~QUADFM_BOTH_STRANDS) {
        set_error("quadfm_count_noalloc: unknown flag bits 0x%x", flags);
        return QR_EINVAL;
    }
    unsigned long long *head = nullptr;
    rc = scratch_address(&head);
    if (rc) return rc;
    if (!npat) return QR_OK;
    // the head is cleared by a one-lane kernel on `stream` (count_persistent), not by a memset
    return count_persistent(h, d_pat, pat_bytes, d_off, npat, d_count, head, flags, false, stream);
}

int quadfm_count(qr_quadfm h, const uint8_t *d_pat, const uint64_t *d_off, uint64_t npat, uint32_t *d_count,
                 hipStream_t stream) {
    return quadfm_count_ex(h, d_pat, implied_len(d_pat), d_off, npat, 0u, d_count, nullptr, stream);
}

int quadfm_count_ws(qr_quadfm h, const uint8_t *d_pat, const uint64_t *d_off, uint64_t npat, uint32_t *d_count,
                    void *d_workspace, hipStream_t stream) {
    if (!d_workspace) {
        set_error("quadfm_count_ws: d_workspace is NULL");
        return QR_EINVAL;
    }
    return quadfm_count_ex(h, d_pat, implied_len(d_pat), d_off, npat, 0u, d_count, d_workspace, stream);
}

int quadfm_count_batched_ex(qr_quadfm h, const uint8_t *d_pat, uint64_t pat_bytes, const uint64_t *d_off, uint64_t npat,
                            uint64_t batch, uint32_t flags, uint32_t *d_count, hipStream_t stream) {
    int rc = count_args(h, d_pat, pat_bytes, d_off, npat, d_count, "quadfm_count_batched");
    if (rc) return rc;
    if (flags & ~QUADFM_BOTH_STRANDS) {
        set_error("quadfm_count_batched_ex: unknown flag bits 0x%x", flags);
        return QR_EINVAL;
    }
    if (!batch) batch = npat;
    FmDev f = dev_view(h);
    f.pat_len = pat_bytes;
    for (uint64_t p0 = 0; p0 < npat; p0 += batch) {
        const uint64_t np = std::min(batch, npat - p0);
        const uint64_t blocks = (np + 255) / 256;
        if (blocks > 0x7fffffffull) {
            set_error("quadfm_count_batched: batch too large");
            return QR_EINVAL;
        }
        fm_layout(h->layout, [&](auto tag) {
            using L = decltype(tag);
            if (flags & QUADFM_BOTH_STRANDS)
                hipLaunchKernelGGL((fm_batch_kernel<L, true, false>), dim3((uint32_t)blocks), dim3(256), 0, stream, f,
                                   d_pat, d_off, p0, np, d_count);
            else
                hipLaunchKernelGGL((fm_batch_kernel<L, false, false>), dim3((uint32_t)blocks), dim3(256), 0, stream, f,
                                   d_pat, d_off, p0, np, d_count);
            return 0;
        });
        QR_HIP(hipGetLastError());
    }
    return QR_OK;
}

int quadfm_count_batched(qr_quadfm h, const uint8_t *d_pat, const uint64_t *d_off, uint64_t npat, uint64_t batch,
                         uint32_t *d_count, hipStream_t stream) {
    return quadfm_count_batched_ex(h, d_pat, implied_len(d_pat), d_off, npat, batch, 0u, d_count, stream);
}

int quadfm_check(qr_quadfm h, hipStream_t stream) {
    if (!h) return QR_EINVAL;
    int rc = check_device(h->device);
    if (rc) return rc;
    uint32_t v = 0;
    QR_HIP(hipStreamSynchronize(stream));
    QR_HIP(hipMemcpy(&v, h->err, 4, hipMemcpyDeviceToHost));
    QR_HIP(hipMemset(h->err, 0, 4));
    if (v & ERR_OFFSETS) {
        set_error("quadfm: a pattern's offsets decrease (d_off[p+1] < d_off[p]) or run past the pattern buffer; "
                  "it was counted as 0");
        return QR_EINVAL;
    }
    if (v & ERR_WALK) {
        set_error("quadfm: a locate walk reached no sampled row (inconsistent mark bits or samples)");
        return QR_ERANGE;
    }
    return QR_OK;
}

int quadfm_locate_attach(qr_quadfm h, const uint64_t *d_mark_bits, const uint32_t *d_samples, uint64_t n_samples,
                         uint32_t rate, hipStream_t stream) {
    if (!h || !d_mark_bits || !d_samples || rate == 0 || ((uintptr_t)d_mark_bits & 7) || ((uintptr_t)d_samples & 3)) {
        set_error("quadfm_locate_attach: null or misaligned pointer, or rate 0");
        return QR_EINVAL;
    }
    int rc = check_device(h->device);
    if (rc) return rc;
    const uint64_t n = h->n1 - 1;
    if (n_samples != n / rate + 1) {
        set_error("quadfm_locate_attach: %llu samples given; rate %u over n = %llu needs %llu",
                  (unsigned long long)n_samples, rate, (unsigned long long)n, (unsigned long long)(n / rate + 1));
        return QR_EINVAL;
    }
    qr_birank marks = nullptr;
    rc = birank_build_ex(d_mark_bits, h->n1, QR_LAYOUT_16, stream, &marks);
    if (rc) return rc;
    // the marks must number n_samples and include the row of '$' (SA = 0)
    uint64_t *dq = nullptr, *dr = nullptr, *samples = nullptr;
    if (hipMalloc(&dq, 24) != hipSuccess || hipMalloc(&dr, 24) != hipSuccess ||
        hipMalloc(&samples, n_samples * 4) != hipSuccess) {
        (void)hipGetLastError();
        if (dq) (void)hipFree(dq);
        if (dr) (void)hipFree(dr);
        (void)birank_free(marks);
        set_error("quadfm_locate_attach: device allocation failed");
        return QR_ENOMEM;
    }
    const uint64_t q[3] = {h->n1, h->dollar, h->dollar + 1};
    uint64_t r[3] = {0, 0, 0};
    hipError_t e = hipMemcpyAsync(dq, q, 24, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) rc = birank_rank(marks, dq, 3, dr, stream);
    if (e == hipSuccess && rc == QR_OK) e = hipMemcpyAsync(r, dr, 24, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess && rc == QR_OK)
        e = hipMemcpyAsync(samples, d_samples, n_samples * 4, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess && rc == QR_OK) e = hipStreamSynchronize(stream);
    (void)hipFree(dq);
    (void)hipFree(dr);
    if (e != hipSuccess || rc != QR_OK || r[0] != n_samples || r[2] - r[1] != 1) {
        (void)hipFree(samples);
        (void)birank_free(marks);
        if (e != hipSuccess) {
            set_error("quadfm_locate_attach: %s", hipGetErrorString(e));
            return QR_EHIP;
        }
        if (rc != QR_OK) return rc;
        set_error("quadfm_locate_attach: %llu rows marked (need %llu) or the row of '$' unmarked",
                  (unsigned long long)r[0], (unsigned long long)n_samples);
        return QR_EINVAL;
    }
    if (h->marks) (void)birank_free(h->marks);
    if (h->samples) (void)hipFree(h->samples);
    h->marks = marks;
    h->samples = reinterpret_cast<uint32_t *>(samples);
    h->n_samples = n_samples;
    h->rate = rate;
    return QR_OK;
}

int quadfm_locate_offsets(qr_quadfm h, const uint32_t *d_iv, uint64_t npat, uint64_t *d_start, hipStream_t stream) {
    if (!h || !d_start || (npat && !d_iv) || ((uintptr_t)d_iv & 7) || ((uintptr_t)d_start & 7)) {
        set_error("quadfm_locate_offsets: null or misaligned pointer");
        return QR_EINVAL;
    }
    int rc = check_device(h->device);
    if (rc) return rc;
    const uint2 *iv = reinterpret_cast<const uint2 *>(d_iv);
    unsigned long long *st = reinterpret_cast<unsigned long long *>(d_start);
    const uint64_t ntiles = (npat + ISCAN_TILE - 1) / ISCAN_TILE;
    if (ntiles > 0x7fffffffull) {
        set_error("quadfm_locate_offsets: npat too large");
        return QR_EINVAL;
    }
    if (ntiles) {
        hipLaunchKernelGGL(iv_tile_totals, dim3((uint32_t)ntiles), dim3(ISCAN_BLOCK), 0, stream, iv, npat, st);
        QR_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(iv_tile_offsets, dim3(1), dim3(ISCAN_TOP), 0, stream, ntiles, npat, st);
    QR_HIP(hipGetLastError());
    if (ntiles) {
        hipLaunchKernelGGL(iv_tile_scan, dim3((uint32_t)ntiles), dim3(ISCAN_BLOCK), 0, stream, iv, npat, st);
        QR_HIP(hipGetLastError());
    }
    return QR_OK;
}

int quadfm_locate(qr_quadfm h, const uint32_t *d_iv, const uint64_t *d_start, uint64_t npat, uint64_t total,
                  uint32_t *d_pos, hipStream_t stream) {
    if (!h || (total && (!d_iv || !d_start || !d_pos || !npat)) || ((uintptr_t)d_iv & 7) || ((uintptr_t)d_start & 7) ||
        ((uintptr_t)d_pos & 3)) {
        set_error("quadfm_locate: null or misaligned pointer, or outputs without patterns");
        return QR_EINVAL;
    }
    if (!h->marks) {
        set_error("quadfm_locate: no suffix-array sample attached (quadfm_locate_attach)");
        return QR_EINVAL;
    }
    int rc = check_device(h->device);
    if (rc) return rc;
    if (!total) return QR_OK;
    const void *ml = nullptr, *ms = nullptr;
    rc = birank_layout(h->marks, &ml, nullptr, &ms, nullptr);
    if (rc) return rc;
    LocDev d;
    d.mlines = reinterpret_cast<const uint4 *>(ml);
    d.msuper = reinterpret_cast<const uint32_t *>(ms);
    d.samples = h->samples;
    d.rate = h->rate;
    const uint64_t blocks = std::max<uint64_t>(1, std::min<uint64_t>((total + 255) / 256, (uint64_t)cu_count() * 32));
    fm_layout(h->layout, [&](auto tag) {
        hipLaunchKernelGGL(fm_locate_kernel<decltype(tag)>, dim3((uint32_t)blocks), dim3(256), 0, stream, dev_view(h), d,
                           reinterpret_cast<const uint2 *>(d_iv), reinterpret_cast<const unsigned long long *>(d_start),
                           npat, total, d_pos, h->err);
        return 0;
    });
    QR_HIP(hipGetLastError());
    return QR_OK;
}

int quadfm_free(qr_quadfm h) {
    release(h);
    return QR_OK;
}

uint64_t quadfm_len(qr_quadfm h) { return h ? h->n1 - 1 : 0; }
uint64_t quadfm_bytes(qr_quadfm h) {
    if (!h) return 0;
    return h->n_lines * 128 + h->super_bytes + (1ull << (2 * h->kmer)) * sizeof(uint2) +
           (h->marks ? birank_bytes(h->marks) + h->n_samples * 4 : 0);
}

int quadfm_set_tuning(qr_quadfm h, const qr_tuning *t) {
    if (!h || !t) return QR_EINVAL;
    if ((t->block && (t->block < 64 || t->block > 256 || t->block % 64)) || t->per_lane < 0 || t->per_lane > 64 ||
        t->grid_waves < 0 || t->grid_waves > 64 || t->sweep != 0) {
        set_error("quadfm_set_tuning: block 64..256 step 64, refill threshold 0..64, waves per CU 0..64, sweep 0");
        return QR_EINVAL;
    }
    h->tune = *t;
    return QR_OK;
}

int quadfm_table(qr_quadfm h, const void **d_table, uint64_t *entries) {
    if (!h) return QR_EINVAL;
    if (d_table) *d_table = h->table;
    if (entries) *entries = 1ull << (2 * h->kmer);
    return QR_OK;
}

int quadfm_export_table(qr_quadfm h, uint32_t *h_pairs) {
    if (!h || !h_pairs) return QR_EINVAL;
    int rc = check_device(h->device);
    if (rc) return rc;
    QR_HIP(hipMemcpy(h_pairs, h->table, (1ull << (2 * h->kmer)) * sizeof(uint2), hipMemcpyDeviceToHost));
    return QR_OK;
}

int quadfm_c_array(qr_quadfm h, uint64_t *h_C4) {
    if (!h || !h_C4) return QR_EINVAL;
    for (int c = 0; c < 4; ++c) h_C4[c] = h->C[c];
    return QR_OK;
}

}  // extern "C"
