// Build pass 2: exclusive prefix sums of per-group counts (paper Section 3, parallel
// construction: count per superblock, prefix-sum the counts, then fill the superblocks).
//
// Counts are `ncol` interleaved u32 columns (1 for BiRank, 4 for QuadRank).  The pass writes
//   base[i*ncol + c] = sum_{k < i} cnt[k*ncol + c]            (u64, kept for pass 3)
//   super[i*ncol + c] = base[i*ncol + c] >> shift             (u32, the shifted superblock offset;
//                                                              skipped when super is null)
// The paper's prefix sum is one linear pass; here it is three kernels over tiles of 4096 rows and
// needs no workspace: (1) each tile's column totals go to base[first row of the tile]; (2) one
// workgroup turns those totals into exclusive tile offsets in place; (3) every tile reads its
// offsets, then scans its own rows over them.
#include "common.hpp"

namespace qr {

namespace {

constexpr int SCAN_BLOCK = 256, SCAN_ROWS = 16;  // rows per thread
constexpr uint64_t SCAN_TILE = (uint64_t)SCAN_BLOCK * SCAN_ROWS;
constexpr int SCAN_TOP = 1024;

// Block-wide exclusive scan of one value per thread; the block total goes to *tot.
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
    __syncthreads();  // wave_tot may be rewritten by the caller's next scan
    *tot = all;
    return before;
}

template <int NCOL>
__global__ __launch_bounds__(SCAN_BLOCK) void tile_totals(const uint32_t *__restrict__ cnt, uint64_t nrow,
                                                          uint64_t *__restrict__ base) {
    __shared__ uint64_t wave_tot[SCAN_BLOCK / 64];
    const uint64_t r0 = blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ROWS;
    uint64_t mine[NCOL];
#pragma unroll
    for (int c = 0; c < NCOL; ++c) mine[c] = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ROWS; ++k)
        if (r0 + k < nrow)
#pragma unroll
            for (int c = 0; c < NCOL; ++c) mine[c] += cnt[(r0 + k) * NCOL + c];
#pragma unroll
    for (int c = 0; c < NCOL; ++c) {
        uint64_t tot;
        (void)block_exclusive(mine[c], wave_tot, &tot);
        if (threadIdx.x == 0) base[blockIdx.x * SCAN_TILE * NCOL + c] = tot;
    }
}

template <int NCOL>
__global__ __launch_bounds__(SCAN_TOP) void tile_offsets(uint64_t ntiles, uint64_t *__restrict__ base) {
    __shared__ uint64_t wave_tot[SCAN_TOP / 64];
    for (int c = 0; c < NCOL; ++c) {
        uint64_t carry = 0;
        for (uint64_t b0 = 0; b0 < ntiles; b0 += SCAN_TOP) {
            const uint64_t b = b0 + threadIdx.x;
            const uint64_t v = b < ntiles ? base[b * SCAN_TILE * NCOL + c] : 0;
            uint64_t tot;
            const uint64_t before = block_exclusive(v, wave_tot, &tot);
            if (b < ntiles) base[b * SCAN_TILE * NCOL + c] = carry + before;
            carry += tot;
        }
    }
}

template <int NCOL>
__global__ __launch_bounds__(SCAN_BLOCK) void tile_scan(const uint32_t *__restrict__ cnt, uint64_t nrow, uint32_t shift,
                                                        uint64_t *__restrict__ base, uint32_t *__restrict__ super) {
    __shared__ uint64_t wave_tot[SCAN_BLOCK / 64];
    __shared__ uint64_t tile_off[NCOL];
    if (threadIdx.x < NCOL) tile_off[threadIdx.x] = base[blockIdx.x * SCAN_TILE * NCOL + threadIdx.x];
    __syncthreads();  // the offsets are read before this tile overwrites its first row
    const uint64_t r0 = blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ROWS;
#pragma unroll
    for (int c = 0; c < NCOL; ++c) {
        uint32_t v[SCAN_ROWS];
        uint64_t mine = 0;
#pragma unroll
        for (int k = 0; k < SCAN_ROWS; ++k) {
            v[k] = r0 + k < nrow ? cnt[(r0 + k) * NCOL + c] : 0u;
            mine += v[k];
        }
        uint64_t tot;
        uint64_t run = tile_off[c] + block_exclusive(mine, wave_tot, &tot);
#pragma unroll
        for (int k = 0; k < SCAN_ROWS; ++k) {
            if (r0 + k < nrow) {
                base[(r0 + k) * NCOL + c] = run;
                if (super) super[(r0 + k) * NCOL + c] = (uint32_t)(run >> shift);
            }
            run += v[k];
        }
    }
}

template <int NCOL>
hipError_t launch(const uint32_t *cnt, uint64_t nrow, uint32_t shift, uint64_t *base, uint32_t *super, hipStream_t s) {
    const uint64_t ntiles = (nrow + SCAN_TILE - 1) / SCAN_TILE;
    if (!ntiles) return hipSuccess;
    if (ntiles > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(tile_totals<NCOL>, dim3((uint32_t)ntiles), dim3(SCAN_BLOCK), 0, s, cnt, nrow, base);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(tile_offsets<NCOL>, dim3(1), dim3(SCAN_TOP), 0, s, ntiles, base);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(tile_scan<NCOL>, dim3((uint32_t)ntiles), dim3(SCAN_BLOCK), 0, s, cnt, nrow, shift, base, super);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_scan_counts(const uint32_t *cnt, uint64_t nrow, int ncol, uint32_t shift, uint64_t *base,
                              uint32_t *super, hipStream_t s) {
    if (ncol == 1) return launch<1>(cnt, nrow, shift, base, super, s);
    if (ncol == 4) return launch<4>(cnt, nrow, shift, base, super, s);
    return hipErrorInvalidValue;
}

}  // namespace qr
