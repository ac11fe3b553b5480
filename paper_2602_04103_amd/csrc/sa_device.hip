// Device construction of the FM-index input (the suffix array of T$, its BWT and the locate sample)
// on gfx950, in place of the host SA-IS pass: prefix doubling (Manber-Myers) over a hand-written
// LSD radix sort.
//
// Suffixes of T$ (N = n+1 of them, suffix n being '$' alone) are first sorted by their first 21
// characters, packed 3 bits each ('$' and the end of text as 0, A..T as 1..4).  Sorted positions
// with equal keys form groups; every suffix gets the rank of its group (the sorted index of the
// group's first member).  Doubling step h then sorts by the pair (rank[i], rank[i+h] + 1, or 0 past the
// end), which orders suffixes by their first 2h characters; h doubles from 21 until every group is
// a single suffix.  The sort is stable, so ties keep the previous order, as the method requires.
//
// A suffix alone in its group is in its final place, and its rank (that place) stays consistent
// with every longer prefix, so a step only re-sorts the suffixes of groups with two or more members
// (the "active" ones; discarding finished suffixes, as in Larsson and Sadakane's doubling).  Active
// suffixes are kept as the list of their places in the suffix array, in order.  The members of a
// group hold consecutive places and the sort key leads with the group's rank, so after a step's
// sort the k-th key still belongs to the k-th listed place.
//
// Radix sort: 8-bit digits, least significant first.  Per pass: (1) per tile of 4096 keys a 256-bin
// histogram in LDS, stored digit-major; (2) an exclusive scan of all histograms gives every
// (digit, tile) its output base; (3) each tile walks its keys in order, ranks equal digits within a
// wavefront with 9 ballots (lanes whose digits match), adds the counts of earlier wavefronts and
// earlier rows of the tile, places the keys in LDS in sorted order and writes them out as one
// contiguous run per digit.
//
// Outputs: the packed BWT ('$' stored as A at its row), the row of '$', and optionally the
// suffix-array sample of locate (mark bits of rows whose SA value is a multiple of the rate and
// those SA values in row order).
#include <algorithm>
#include <new>

#include "common.hpp"

using namespace qr;

namespace {

constexpr int BLK = 256, ITEMS = 16;
constexpr uint32_t TILE = BLK * ITEMS;  // 4096
constexpr int TOP = 1024;
constexpr uint32_t KEY_CHARS = 21;      // 63 bits of 3-bit characters

// ---- generic u32 scans (sum or max), three passes over tiles of 4096 --------------------------------
struct OpAdd {
    __device__ static uint32_t id() { return 0u; }
    __device__ static uint32_t f(uint32_t a, uint32_t b) { return a + b; }
};
struct OpMax {
    __device__ static uint32_t id() { return 0u; }
    __device__ static uint32_t f(uint32_t a, uint32_t b) { return a > b ? a : b; }
};

// inclusive scan over the 64 lanes of a wavefront
template <class Op>
__device__ __forceinline__ uint32_t wave_incl(uint32_t v) {
    const uint32_t lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(v, d, 64);
        if (lane >= (uint32_t)d) v = Op::f(v, o);
    }
    return v;
}

// exclusive block scan of one value per thread; *tot receives the block aggregate
template <class Op>
__device__ __forceinline__ uint32_t block_excl(uint32_t v, uint32_t *wsh, uint32_t *tot) {
    const uint32_t t = threadIdx.x, nw = blockDim.x / 64;
    const uint32_t incl = wave_incl<Op>(v);
    const uint32_t excl_w = __shfl_up(incl, 1, 64);
    if (__lane_id() == 63) wsh[t / 64] = incl;
    __syncthreads();
    uint32_t before = Op::id(), all = Op::id();
    for (uint32_t w = 0; w < nw; ++w) {
        if (w < t / 64) before = Op::f(before, wsh[w]);
        all = Op::f(all, wsh[w]);
    }
    __syncthreads();
    *tot = all;
    return __lane_id() == 0 ? before : Op::f(before, excl_w);
}

template <class Op>
__global__ __launch_bounds__(BLK) void scan_tiles(const uint32_t *__restrict__ in, uint64_t n, uint32_t *__restrict__ aux) {
    __shared__ uint32_t wsh[BLK / 64];
    const uint64_t i0 = (uint64_t)blockIdx.x * TILE + (uint64_t)threadIdx.x * ITEMS;
    uint32_t a = Op::id();
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
        if (i0 + k < n) a = Op::f(a, in[i0 + k]);
    uint32_t tot;
    (void)block_excl<Op>(a, wsh, &tot);
    if (threadIdx.x == 0) aux[blockIdx.x] = tot;
}

template <class Op>
__global__ __launch_bounds__(TOP) void scan_aux(uint32_t *__restrict__ aux, uint64_t ntiles) {
    __shared__ uint32_t wsh[TOP / 64];
    uint32_t carry = Op::id();
    for (uint64_t b0 = 0; b0 < ntiles; b0 += TOP) {
        const uint64_t b = b0 + threadIdx.x;
        const uint32_t v = b < ntiles ? aux[b] : Op::id();
        uint32_t tot;
        const uint32_t before = block_excl<Op>(v, wsh, &tot);
        if (b < ntiles) aux[b] = Op::f(carry, before);
        carry = Op::f(carry, tot);
    }
}

template <class Op, bool INCL>
__global__ __launch_bounds__(BLK) void scan_apply(const uint32_t *__restrict__ in, uint64_t n,
                                                  const uint32_t *__restrict__ aux, uint32_t *__restrict__ out) {
    __shared__ uint32_t wsh[BLK / 64];
    const uint64_t i0 = (uint64_t)blockIdx.x * TILE + (uint64_t)threadIdx.x * ITEMS;
    uint32_t v[ITEMS], a = Op::id();
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        v[k] = i0 + k < n ? in[i0 + k] : Op::id();
        a = Op::f(a, v[k]);
    }
    uint32_t tot;
    uint32_t run = Op::f(aux[blockIdx.x], block_excl<Op>(a, wsh, &tot));
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const uint32_t next = Op::f(run, v[k]);
        if (i0 + k < n) out[i0 + k] = INCL ? next : run;
        run = next;
    }
}

template <class Op, bool INCL>
hipError_t scan_u32(const uint32_t *in, uint64_t n, uint32_t *out, uint32_t *aux, hipStream_t s) {
    const uint64_t nt = (n + TILE - 1) / TILE;
    if (!nt) return hipSuccess;
    hipLaunchKernelGGL(scan_tiles<Op>, dim3((uint32_t)nt), dim3(BLK), 0, s, in, n, aux);
    hipLaunchKernelGGL(scan_aux<Op>, dim3(1), dim3(TOP), 0, s, aux, nt);
    hipLaunchKernelGGL((scan_apply<Op, INCL>), dim3((uint32_t)nt), dim3(BLK), 0, s, in, n, aux, out);
    return hipGetLastError();
}

// ---- radix sort of (u64 key, u32 value) pairs ------------------------------------------------------
__global__ __launch_bounds__(BLK) void rs_hist(const uint64_t *__restrict__ keys, uint32_t n, uint32_t shift,
                                               uint32_t *__restrict__ hist, uint32_t ntiles) {
    __shared__ uint32_t h[256];
    const uint32_t t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * TILE;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint64_t i = base + (uint64_t)j * BLK + t;
        if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(uint64_t)t * ntiles + blockIdx.x] = h[t];
}

// Scatter of one tile: its keys are first placed in LDS in sorted (digit, then input) order, then
// written out as contiguous runs per digit, so consecutive lanes store to consecutive addresses.
__global__ __launch_bounds__(BLK) void rs_scatter(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                  uint64_t *__restrict__ kout, uint32_t *__restrict__ vout, uint32_t n,
                                                  uint32_t shift, const uint32_t *__restrict__ hist,
                                                  const uint32_t *__restrict__ offs, uint32_t ntiles) {
    __shared__ uint64_t skey[TILE];
    __shared__ uint32_t sval[TILE];
    __shared__ uint32_t gbase[256];   // global start of this tile's run of each digit
    __shared__ uint32_t lstart[256];  // start of each digit's run inside the tile
    __shared__ uint32_t run[256];     // keys of each digit placed so far
    __shared__ uint32_t wcnt[BLK / 64][256];
    __shared__ uint32_t wsh[BLK / 64];
    const uint32_t t = threadIdx.x, w = t / 64, lane = __lane_id();
    const uint64_t hidx = (uint64_t)t * ntiles + blockIdx.x;
    gbase[t] = offs[hidx];
    uint32_t tot;
    lstart[t] = block_excl<OpAdd>(hist[hidx], wsh, &tot);
    run[t] = 0;
#pragma unroll
    for (int k = 0; k < BLK / 64; ++k) wcnt[k][t] = 0;
    __syncthreads();
    const uint64_t lt = (1ull << lane) - 1ull;
    const uint64_t tile0 = (uint64_t)blockIdx.x * TILE;
    for (int j = 0; j < ITEMS; ++j) {
        const uint64_t i = tile0 + (uint64_t)j * BLK + t;
        const bool valid = i < n;
        const uint64_t key = valid ? kin[i] : 0ull;
        const uint32_t val = valid ? vin[i] : 0u;
        const uint32_t d = valid ? ((uint32_t)(key >> shift) & 255u) : 256u;  // 256: no valid digit
        uint64_t same = ~0ull;  // lanes of this wavefront with the same 9-bit digit
#pragma unroll
        for (int b = 0; b < 9; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            same &= bit ? bal : ~bal;
        }
        const uint32_t rank = __popcll(same & lt);
        if (valid && rank == 0) wcnt[w][d] = __popcll(same);
        __syncthreads();
        if (valid) {
            uint32_t lp = lstart[d] + run[d] + rank;
            for (uint32_t k = 0; k < w; ++k) lp += wcnt[k][d];
            skey[lp] = key;
            sval[lp] = val;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int k = 0; k < BLK / 64; ++k) {
            add += wcnt[k][t];
            wcnt[k][t] = 0;
        }
        run[t] += add;
        __syncthreads();
    }
    const uint32_t cnt = (uint32_t)min<uint64_t>(TILE, (uint64_t)n - tile0);
    for (uint32_t p = t; p < cnt; p += BLK) {
        const uint64_t key = skey[p];
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        const uint32_t pos = gbase[d] + (p - lstart[d]);
        kout[pos] = key;
        vout[pos] = sval[p];
    }
}

// ---- prefix doubling -------------------------------------------------------------------------------
__global__ void check_codes(const uint8_t *__restrict__ text, uint64_t n, uint32_t *__restrict__ bad) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && text[i] > 3) atomicOr(bad, 1u);
}

__global__ void init_keys(const uint8_t *__restrict__ text, uint32_t n, uint64_t *__restrict__ key,
                          uint32_t *__restrict__ val) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;  // N = n + 1 suffixes
    uint64_t k = 0;
#pragma unroll
    for (uint32_t t = 0; t < KEY_CHARS; ++t) {
        const uint64_t p = i + t;
        const uint32_t c = p < n ? (uint32_t)text[p] + 1u : 0u;
        k = (k << 3) | c;
    }
    key[i] = k;
    val[i] = (uint32_t)i;
}

// One pass over the U sorted keys of a step (place pos[i] in the suffix array, suffix v[i]):
// store the suffix at its place; g[i] = its place if key i starts a new group, else 0 (a max-scan
// then gives every key its group's first place); act[i] = 1 unless key i is alone in its group.
__global__ void settle(const uint64_t *__restrict__ key, const uint32_t *__restrict__ v, const uint32_t *__restrict__ pos,
                       uint32_t U, uint32_t *__restrict__ sa, uint32_t *__restrict__ g, uint32_t *__restrict__ act) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= U) return;
    const uint64_t k = key[i];
    const bool head = i == 0 || k != key[i - 1];
    const bool tail = i + 1 == U || k != key[i + 1];
    sa[pos[i]] = v[i];
    g[i] = head ? pos[i] : 0u;
    act[i] = (head && tail) ? 0u : 1u;
}

// rank[v[i]] = first place of key i's group
__global__ void set_rank(const uint32_t *__restrict__ v, const uint32_t *__restrict__ gstart, uint32_t U,
                         uint32_t *__restrict__ rank) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < U) rank[v[i]] = gstart[i];
}

// The places of the keys still active, in order (at[i] = exclusive count of active keys before i);
// the number of them goes to *count.
__global__ void compact_active(const uint32_t *__restrict__ pos, const uint32_t *__restrict__ act,
                               const uint32_t *__restrict__ at, uint32_t U, uint32_t *__restrict__ pos_out,
                               unsigned long long *__restrict__ count) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= U) return;
    if (act[i]) pos_out[at[i]] = pos[i];
    if (i + 1 == U) *count = (unsigned long long)at[i] + act[i];
}

__global__ void iota_u32(uint32_t *__restrict__ x, uint32_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = (uint32_t)i;
}

// key of active suffix i for doubling step h: (rank of the suffix, rank of the suffix h further + 1,
// or 0 past the end)
__global__ void pair_keys(const uint32_t *__restrict__ sa, const uint32_t *__restrict__ pos, const uint32_t *__restrict__ rank,
                          uint32_t U, uint32_t N, uint32_t h, uint64_t *__restrict__ key, uint32_t *__restrict__ val) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= U) return;
    const uint32_t s = sa[pos[i]];
    const uint64_t s2 = (uint64_t)s + h;
    const uint32_t r2 = s2 < N ? rank[s2] + 1u : 0u;
    key[i] = ((uint64_t)rank[s] << 32) | r2;
    val[i] = s;
}

// BWT row k = T[SA[k] - 1], '$' (stored as A) where SA[k] = 0; 32 rows per packed word
__global__ void bwt_pack(const uint32_t *__restrict__ sa, const uint8_t *__restrict__ text, uint32_t N,
                         uint64_t *__restrict__ bwt, unsigned long long *__restrict__ dollar) {
    const uint64_t wd = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t nw = ((uint64_t)N + 31) / 32;
    if (wd >= nw) return;
    uint64_t word = 0;
    for (uint32_t r = 0; r < 32; ++r) {
        const uint64_t k = wd * 32 + r;
        if (k >= N) break;
        const uint32_t s = sa[k];
        uint64_t c = 0;
        if (s == 0) *dollar = k;
        else c = text[s - 1];
        word |= c << (2 * r);
    }
    bwt[wd] = word;
}

// mark bits (row k marked iff SA[k] % rate == 0), 64 rows per wavefront, and the marks per wavefront
__global__ void sample_marks(const uint32_t *__restrict__ sa, uint32_t N, uint32_t rate, uint64_t *__restrict__ marks,
                             uint32_t *__restrict__ wcount) {
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool m = k < N && sa[k] % rate == 0;
    const uint64_t b = __ballot(m);
    const uint64_t g = k / 64;
    if (__lane_id() == 0 && g * 64 < N) {
        marks[g] = b;
        wcount[g] = (uint32_t)__popcll(b);
    }
}

__global__ void sample_write(const uint32_t *__restrict__ sa, uint32_t N, uint32_t rate,
                             const uint32_t *__restrict__ wbase, uint32_t *__restrict__ samples) {
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool m = k < N && sa[k] % rate == 0;
    const uint64_t b = __ballot(m);
    if (m) samples[wbase[k / 64] + __popcll(b & ((1ull << __lane_id()) - 1ull))] = sa[k];
}

uint32_t blocks_for(uint64_t n, uint32_t bs) { return (uint32_t)((n + bs - 1) / bs); }

struct Buffers {
    uint64_t *k0 = nullptr, *k1 = nullptr;
    uint32_t *v0 = nullptr, *v1 = nullptr, *rank = nullptr, *g = nullptr, *hist = nullptr, *offs = nullptr,
             *aux = nullptr, *bad = nullptr, *sa = nullptr, *pos = nullptr, *pos2 = nullptr, *act = nullptr,
             *at = nullptr;
    unsigned long long *cnt = nullptr;
    ~Buffers() {
        for (void *p : {(void *)k0, (void *)k1, (void *)v0, (void *)v1, (void *)rank, (void *)g, (void *)hist,
                        (void *)offs, (void *)aux, (void *)bad, (void *)cnt, (void *)sa, (void *)pos, (void *)pos2,
                        (void *)act, (void *)at})
            if (p) (void)hipFree(p);
    }
};

// sort (k0, v0) by the low `bits` bits of the keys; the result ends in (k0, v0)
hipError_t radix_sort(Buffers &B, uint32_t N, uint32_t bits, hipStream_t s) {
    const uint32_t nt = blocks_for(N, TILE);
    const uint64_t nh = (uint64_t)nt * 256;
    for (uint32_t shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(rs_hist, dim3(nt), dim3(BLK), 0, s, B.k0, N, shift, B.hist, nt);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = scan_u32<OpAdd, false>(B.hist, nh, B.offs, B.aux, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(rs_scatter, dim3(nt), dim3(BLK), 0, s, B.k0, B.v0, B.k1, B.v1, N, shift, B.hist, B.offs, nt);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        std::swap(B.k0, B.k1);
        std::swap(B.v0, B.v1);
    }
    return hipSuccess;
}

// After a step's sort of the U active keys (k0, v0) whose places are pos[0..U): store the suffixes
// at their places, give each its group's first place as rank, and keep in pos the places of the
// suffixes whose groups still have two or more members; returns their number in U.
hipError_t settle_step(Buffers &B, uint32_t &U, hipStream_t s) {
    const uint32_t nb = blocks_for(U, 256);
    hipLaunchKernelGGL(settle, dim3(nb), dim3(256), 0, s, B.k0, B.v0, B.pos, U, B.sa, B.g, B.act);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = scan_u32<OpMax, true>(B.g, U, B.g, B.aux, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(set_rank, dim3(nb), dim3(256), 0, s, B.v0, B.g, U, B.rank);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = scan_u32<OpAdd, false>(B.act, U, B.at, B.aux, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(compact_active, dim3(nb), dim3(256), 0, s, B.pos, B.act, B.at, U, B.pos2, B.cnt);
        e = hipGetLastError();
    }
    unsigned long long c = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&c, B.cnt, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) {
        std::swap(B.pos, B.pos2);
        U = (uint32_t)c;
    }
    return e;
}

uint32_t bit_length(uint64_t x) {
    uint32_t b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

}  // namespace

extern "C" int quadfm_index_device(const uint8_t *d_text, uint64_t n, uint32_t rate, uint64_t *d_bwt_packed2,
                                   uint64_t *dollar_pos, uint64_t *d_mark_bits, uint32_t *d_samples, uint32_t *d_sa,
                                   hipStream_t stream) {
    if ((!d_text && n) || !d_bwt_packed2 || !dollar_pos || ((uintptr_t)d_bwt_packed2 & 7) || ((uintptr_t)d_sa & 3) ||
        (rate && (!d_mark_bits || !d_samples || ((uintptr_t)d_mark_bits & 7) || ((uintptr_t)d_samples & 3)))) {
        set_error("quadfm_index_device: null or misaligned pointer");
        return QR_EINVAL;
    }
    if (n + 1 > 0xffffffffull - TILE) {
        set_error("quadfm_index_device: n = %llu is too large for u32 suffix positions", (unsigned long long)n);
        return QR_ERANGE;
    }
    const uint32_t N = (uint32_t)(n + 1);
    Buffers B;
    const uint32_t nt = blocks_for(N, TILE);
    const uint64_t nh = (uint64_t)nt * 256;
    const uint64_t naux = std::max<uint64_t>((nh + TILE - 1) / TILE, ((uint64_t)N + TILE - 1) / TILE) + 1;
    if (hipMalloc(&B.k0, 8ull * N) != hipSuccess || hipMalloc(&B.k1, 8ull * N) != hipSuccess ||
        hipMalloc(&B.v0, 4ull * N) != hipSuccess || hipMalloc(&B.v1, 4ull * N) != hipSuccess ||
        hipMalloc(&B.rank, 4ull * N) != hipSuccess || hipMalloc(&B.g, 4ull * N + 4) != hipSuccess ||
        hipMalloc(&B.hist, 4 * nh) != hipSuccess || hipMalloc(&B.offs, 4 * nh) != hipSuccess ||
        hipMalloc(&B.aux, 4 * naux) != hipSuccess || hipMalloc(&B.bad, 4) != hipSuccess || hipMalloc(&B.cnt, 8) != hipSuccess ||
        hipMalloc(&B.sa, 4ull * N) != hipSuccess || hipMalloc(&B.pos, 4ull * N) != hipSuccess ||
        hipMalloc(&B.pos2, 4ull * N) != hipSuccess || hipMalloc(&B.act, 4ull * N) != hipSuccess ||
        hipMalloc(&B.at, 4ull * N) != hipSuccess) {
        (void)hipGetLastError();
        set_error("quadfm_index_device: device allocation failed (about %llu bytes)", (unsigned long long)(52ull * N + 8 * nh));
        return QR_ENOMEM;
    }
    hipStream_t s = stream;
    hipError_t e = hipMemsetAsync(B.bad, 0, 4, s);
    if (e == hipSuccess && n) {
        hipLaunchKernelGGL(check_codes, dim3(blocks_for(n, 256)), dim3(256), 0, s, d_text, n, B.bad);
        e = hipGetLastError();
    }
    uint32_t bad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, B.bad, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && bad) {
        set_error("quadfm_index_device: a text code is above 3");
        return QR_EINVAL;
    }
    // initial sort: the first 21 characters, all N suffixes active at places 0..N-1
    if (e == hipSuccess) {
        hipLaunchKernelGGL(init_keys, dim3(blocks_for(N, 256)), dim3(256), 0, s, d_text, (uint32_t)n, B.k0, B.v0);
        hipLaunchKernelGGL(iota_u32, dim3(blocks_for(N, 256)), dim3(256), 0, s, B.pos, N);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = radix_sort(B, N, 3 * KEY_CHARS, s);
    uint32_t U = N;
    if (e == hipSuccess) e = settle_step(B, U, s);
    // doubling steps h = 21, 42, 84, ...: sort the active suffixes by (rank[i], rank[i+h]) until none is left
    const uint32_t rbits = bit_length(N);  // ranks < N; second component < N + 1
    for (uint64_t h = KEY_CHARS; e == hipSuccess && U > 0; h *= 2) {
        if (h > 2ull * N) {
            set_error("quadfm_index_device: prefix doubling did not converge");
            return QR_EHIP;
        }
        hipLaunchKernelGGL(pair_keys, dim3(blocks_for(U, 256)), dim3(256), 0, s, B.sa, B.pos, B.rank, U, N, (uint32_t)h,
                           B.k0, B.v0);
        e = hipGetLastError();
        // low word holds rank2 + 1 <= N in rbits bits; high word the first rank: sort bits [0, 32+rbits)
        if (e == hipSuccess) e = radix_sort(B, U, 32 + rbits, s);
        if (e == hipSuccess) e = settle_step(B, U, s);
    }
    // BWT and the locate sample from the suffix array
    unsigned long long *d_dollar = B.cnt;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(bwt_pack, dim3(blocks_for(((uint64_t)N + 31) / 32, 256)), dim3(256), 0, s, B.sa, d_text, N,
                           d_bwt_packed2, d_dollar);
        e = hipGetLastError();
    }
    unsigned long long dol = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&dol, d_dollar, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && d_sa) e = hipMemcpyAsync(d_sa, B.sa, 4ull * N, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && rate) {
        const uint64_t nwv = ((uint64_t)N + 63) / 64;
        hipLaunchKernelGGL(sample_marks, dim3(blocks_for(N, 256)), dim3(256), 0, s, B.sa, N, rate, d_mark_bits, B.hist);
        e = hipGetLastError();
        if (e == hipSuccess) e = scan_u32<OpAdd, false>(B.hist, nwv, B.offs, B.aux, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(sample_write, dim3(blocks_for(N, 256)), dim3(256), 0, s, B.sa, N, rate, B.offs, d_samples);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        set_error("quadfm_index_device: %s", hipGetErrorString(e));
        return QR_EHIP;
    }
    *dollar_pos = dol;
    return QR_OK;
}
