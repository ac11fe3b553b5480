// Build pass 2: exclusive prefix sums of per-superblock counts (paper Section 3, parallel
// construction: count per superblock, prefix-sum the counts, then fill the superblocks).
//
// Counts are `ncol` interleaved u32 columns (1 for BiRank, 4 for QuadRank).  The pass writes
//   base[i*ncol + c] = sum_{k < i} cnt[k*ncol + c]            (u64, kept for pass 3)
//   super[i*ncol + c] = base[i*ncol + c] >> shift             (u32, the shifted superblock offset;
//                                                              skipped when super is null)
// A single workgroup handles any length: the rows are split into 1024 contiguous chunks, each
// thread reduces its chunk, the chunk totals are scanned in LDS and each thread then rewrites
// its chunk.  Superblock arrays are small (about 1e6 rows at 2^36 bits) so one CU suffices.
#include "common.hpp"

namespace qr {

constexpr int SCAN_THREADS = 1024;

__global__ __launch_bounds__(SCAN_THREADS) void scan_counts_kernel(const uint32_t *__restrict__ cnt, uint64_t nrow,
                                                                   int ncol, uint32_t shift,
                                                                   uint64_t *__restrict__ base,
                                                                   uint32_t *__restrict__ super) {
    __shared__ uint64_t wave_tot[SCAN_THREADS / 64];
    const int t = threadIdx.x;
    const uint64_t chunk = (nrow + SCAN_THREADS - 1) / SCAN_THREADS;
    const uint64_t r0 = (uint64_t)t * chunk;
    const uint64_t r1 = r0 + chunk < nrow ? r0 + chunk : nrow;
    for (int c = 0; c < ncol; ++c) {
        uint64_t local = 0;
        for (uint64_t r = r0; r < r1; ++r) local += cnt[r * ncol + c];
        // block-wide exclusive scan of `local`
        uint64_t incl = wave_inclusive_scan<uint64_t>(local);
        if (__lane_id() == 63) wave_tot[t / 64] = incl;
        __syncthreads();
        uint64_t before = 0;
        for (int w = 0; w < t / 64; ++w) before += wave_tot[w];
        uint64_t run = before + incl - local;
        for (uint64_t r = r0; r < r1; ++r) {
            base[r * ncol + c] = run;
            if (super) super[r * ncol + c] = (uint32_t)(run >> shift);
            run += cnt[r * ncol + c];
        }
        __syncthreads();
    }
}

hipError_t launch_scan_counts(const uint32_t *cnt, uint64_t nrow, int ncol, uint32_t shift, uint64_t *base,
                              uint32_t *super, hipStream_t s) {
    hipLaunchKernelGGL(scan_counts_kernel, dim3(1), dim3(SCAN_THREADS), 0, s, cnt, nrow, ncol, shift, base, super);
    return hipGetLastError();
}

}  // namespace qr
