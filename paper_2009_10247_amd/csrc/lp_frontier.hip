// lp_frontier.hip -- the least model by pushing newly true atoms through the
// transposed program matrix (semi-naive evaluation of T_P) on gfx950.
//
// The synchronous iteration of Algorithm 1 derives at product t exactly the
// rows whose last missing body atom (AND rows) or first child (OR rows)
// became true at product t - 1. Each row keeps a count of entries still
// false: an AND row starts at its length, an OR row at 1, and a row fires when
// a decrement takes its count from 1 to 0. Level t takes the rows that became
// true at product t (F_0: the fact rows of the initial vector), decrements the
// count of every row that names them, and collects the rows that fire into
// F_{t+1}. A row fires at most once, so over the whole solve every entry of
// the matrix is visited once; the levels are the products of the full sweep,
// and the first empty F_t gives the same product count (at least 1).
#include <hip/hip_runtime.h>

#include "lp_dev.h"
#include "lp_kernels.h"

namespace lp {

namespace {

constexpr int kFrontierBlock = 256;
constexpr int kFrontierWaves = kFrontierBlock / 64;

// One level. The waves take the frontier 64 rows at a time (grid-stride). For
// a chunk, a wave scans the lengths of the 64 rows' occurrence lists and walks
// their concatenation 64 entries per pass, each lane finding the row its
// entry belongs to by a binary search over the scan in LDS, so a long list
// is shared by the whole wave. Rows that fire are appended to the next
// frontier with one atomic per wave and pass.
__global__ __launch_bounds__(kFrontierBlock) void frontier_level_kernel(FrontierParams f) {
    __shared__ int32_t s_excl[kFrontierWaves][64];
    __shared__ int32_t s_start[kFrontierWaves][64];
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t n_in = f.sizes[f.level % kFrontierRing];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        f.sizes[(f.level + 2) % kFrontierRing] = 0;  // the size the level after the next adds to
        f.hist[f.level % kFrontierHist] = (int32_t)n_in;
    }
    if (n_in == 0) return;
    uint32_t *n_out = &f.sizes[(f.level + 1) % kFrontierRing];
    const int64_t waves = (int64_t)gridDim.x * kFrontierWaves;
    for (int64_t c0 = ((int64_t)blockIdx.x * kFrontierWaves + wid) * 64; c0 < n_in; c0 += waves * 64) {
        const int64_t j = c0 + lane;
        int32_t s = 0, len = 0;
        if (j < n_in) {
            const int32_t a = f.in[j];
            s = f.occ_ptr[a];
            len = f.occ_ptr[a + 1] - s;
        }
        const int32_t ex = wave_exclusive_scan(len);
        const int32_t total = __builtin_amdgcn_readlane(ex + len, 63);
        s_excl[wid][lane] = ex;
        s_start[wid][lane] = s;
        __builtin_amdgcn_wave_barrier();
        for (int32_t i0 = 0; i0 < total; i0 += 64) {
            const int32_t i = i0 + lane;
            bool fire = false;
            int32_t r = 0;
            if (i < total) {
                // the last row k of the chunk with s_excl[k] <= i (rows with empty lists share
                // their start with the next row and are skipped by taking the last)
                int32_t lo = 0;
#pragma unroll
                for (int step = 32; step > 0; step >>= 1)
                    if (s_excl[wid][lo + step] <= i) lo += step;
                r = f.occ[s_start[wid][lo] + (i - s_excl[wid][lo])];
                fire = atomicSub(&f.cnt[r], 1) == 1;
                if (fire) atomicOr((unsigned long long *)&f.v[r >> 6], 1ull << (r & 63));
            }
            const uint64_t m = __ballot(fire);
            if (m) {
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(n_out, (uint32_t)__popcll(m));
                base = (uint32_t)__builtin_amdgcn_readfirstlane(base);
                if (fire) f.out[base + (uint32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] = r;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

}  // namespace

hipError_t launch_frontier_level(const FrontierParams &f, int grid, hipStream_t st) {
    hipLaunchKernelGGL(frontier_level_kernel, dim3(grid), dim3(kFrontierBlock), 0, st, f);
    return hipGetLastError();
}

}  // namespace lp
