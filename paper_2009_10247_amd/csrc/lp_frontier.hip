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

// Pushes one frontier: the waves take its n_in rows 64 at a time
// (grid-stride from wave `wave` over `waves` waves). For a chunk, a wave scans
// the lengths of the 64 rows' occurrence lists and walks their concatenation
// 64 entries per pass, each lane finding the row its entry belongs to by a
// binary search over the scan in LDS, so a long list is shared by the whole
// wave. Rows that fire are appended to `out` with one atomic on n_out per wave
// and pass. With LDSQ, `in`, `n_out` and `s_out` are in LDS: a fired row's
// index below `cap` goes to s_out, the rest to `out` in global memory.
template <bool LDSQ>
__device__ __forceinline__ void push_frontier(const FrontierParams &f, const int32_t *in, uint32_t n_in, int32_t *out,
                                              uint32_t *n_out, int64_t wave, int64_t waves, int32_t *s_excl,
                                              int32_t *s_start, int lane, int32_t *s_out = nullptr,
                                              uint32_t cap = 0) {
    for (int64_t c0 = wave * 64; c0 < n_in; c0 += waves * 64) {
        const int64_t j = c0 + lane;
        int32_t s = 0, len = 0;
        if (j < n_in) {
            const int32_t a = in[j];
            s = f.occ_ptr[a];
            len = f.occ_ptr[a + 1] - s;
        }
        const int32_t ex = wave_exclusive_scan(len);
        const int32_t total = __builtin_amdgcn_readlane(ex + len, 63);
        s_excl[lane] = ex;
        s_start[lane] = s;
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
                    if (s_excl[lo + step] <= i) lo += step;
                r = f.occ[s_start[lo] + (i - s_excl[lo])];
                fire = atomicSub(&f.cnt[r], 1) == 1;
                if (fire) atomicOr((unsigned long long *)&f.v[r >> 6], 1ull << (r & 63));
            }
            const uint64_t m = __ballot(fire);
            if (m) {
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(n_out, (uint32_t)__popcll(m));
                base = (uint32_t)__builtin_amdgcn_readfirstlane(base);
                if (fire) {
                    const uint32_t k = base + (uint32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    if (LDSQ && k < cap)  // an LDS store (ds_write), never merged with the global one
                        ((lds_u32 *)s_out)[k] = (uint32_t)r;
                    else
                        out[k] = r;
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// One level, f.level, from f.in to f.out over the whole grid.
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
    push_frontier<false>(f, f.in, n_in, f.out, &f.sizes[(f.level + 1) % kFrontierRing],
                         (int64_t)blockIdx.x * kFrontierWaves + wid, (int64_t)gridDim.x * kFrontierWaves,
                         s_excl[wid], s_start[wid], lane);
}

// Orders the LDS accesses of a workgroup across the barrier, and nothing
// else: a wave's global atomics and stores may still be in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Levels f.level .. f.level + n_levels - 1 in one workgroup, with a workgroup
// barrier between levels in place of a launch: for the long stretches of
// small frontiers (a derivation chain), where a launch per level costs more
// than the level's work. The frontier and its size live in LDS (up to
// kFrontierLoopCap rows), so a level's only global accesses are the
// occurrence lists, the counts and v. The loop takes F_{f.level} from global
// memory (the fact rows at level 0, else q[level & 1]) and ends at the first
// empty frontier (its size recorded, so the host sees the fixpoint) or before
// pushing a frontier of more than kFrontierLoopCap rows. Fired rows past that
// index are stored to global memory as they come, and each level's |F_t| to
// its own history slot; the other global stores are made once, at the end,
// after a full barrier: the frontier left (rows below the cap) into q[t & 1],
// its size into sizes[t % kFrontierRing] (the next slot cleared), and the
// first level not pushed into ctl[0]. So a global location is written at most
// once per launch, and what a later launch reads is exactly what the
// per-level kernels would have left. At most n_levels iterations, none of
// them waiting on another workgroup.
__global__ __launch_bounds__(kFrontierLoopBlock) void frontier_levels_kernel(FrontierParams f, const int32_t *facts,
                                                                              int32_t *q0, int32_t *q1,
                                                                              int32_t n_levels, int32_t *ctl) {
    constexpr int NW = kFrontierLoopBlock / 64;
    constexpr uint32_t cap = kFrontierLoopCap;
    __shared__ int32_t s_excl[NW][64];
    __shared__ int32_t s_start[NW][64];
    __shared__ int32_t s_q[2][kFrontierLoopCap];
    __shared__ uint32_t s_n[4];  // frontier sizes, indexed by level & 3
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int32_t t0 = f.level;
    const uint32_t n0 = f.sizes[t0 % kFrontierRing];
    if (n0 > cap) {  // the full grid takes this level; nothing was changed
        if (threadIdx.x == 0) ctl[0] = t0;
        return;
    }
    const int32_t *in0 = t0 == 0 ? facts : ((t0 & 1) ? q1 : q0);
    for (uint32_t j = threadIdx.x; j < n0; j += kFrontierLoopBlock) s_q[t0 & 1][j] = in0[j];
    if (threadIdx.x == 0) {
        s_n[t0 & 3] = n0;
        s_n[(t0 + 1) & 3] = 0;
    }
    lds_barrier();
    int32_t t = t0;
    const int32_t t_end = t0 + n_levels;
    for (; t < t_end; ++t) {
        const uint32_t n_in = s_n[t & 3];
        if (n_in > cap) break;
        if (threadIdx.x == 0) {
            s_n[(t + 2) & 3] = 0;  // read at level t - 2, appended to at level t + 1
            f.hist[t % kFrontierHist] = (int32_t)n_in;
        }
        if (n_in == 0) break;
        push_frontier<true>(f, s_q[t & 1], n_in, (t & 1) ? q0 : q1, &s_n[(t + 1) & 3], wid, NW, s_excl[wid],
                            s_start[wid], lane, s_q[(t + 1) & 1], cap);
        lds_barrier();
    }
    // F_t is not pushed (t = t_end, or it is too large), or it is empty and
    // its level recorded (t < t_end). Hand F_t over in global memory (the rows
    // from index cap on are there already), ordered after every store of the
    // loop.
    const uint32_t n_in = s_n[t & 3];
    __syncthreads();
    if (t > t0) {
        int32_t *qt = (t & 1) ? q1 : q0;
        const uint32_t n_lds = n_in < cap ? n_in : cap;
        for (uint32_t j = threadIdx.x; j < n_lds; j += kFrontierLoopBlock) qt[j] = s_q[t & 1][j];
    }
    if (threadIdx.x == 0) {
        f.sizes[t % kFrontierRing] = n_in;
        f.sizes[(t + 1) % kFrontierRing] = 0;
        ctl[0] = (t < t_end && n_in == 0) ? t + 1 : t;
    }
}

// Least models of many programs: a workgroup takes the next program from
// the queue, sets its counts to the start counts and its interpretation to
// the fact rows, and pushes frontiers level after level (push_frontier over
// its 16 waves, the frontiers in two global buffers of its own, their sizes in
// LDS), with a workgroup barrier between levels, until a level is empty. The
// level count is the product count of the full sweep. The last workgroup to
// leave rewinds the queue, so graph replays need no memset.
__global__ __launch_bounds__(kFBatchBlock) void frontier_batch_kernel(FBatchParams b) {
    extern __shared__ __attribute__((aligned(16))) uint64_t s_fdyn[];
    constexpr int NW = kFBatchBlock / 64;
    __shared__ int32_t s_excl[NW][64];
    __shared__ int32_t s_start[NW][64];
    __shared__ uint32_t s_n[4];  // frontier sizes by level & 3
    __shared__ int32_t s_item;
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int32_t *q[2] = {b.qbuf + (int64_t)blockIdx.x * 2 * b.qcap, b.qbuf + (int64_t)blockIdx.x * 2 * b.qcap + b.qcap};
    typedef const __attribute__((address_space(4))) int32_t c_i32;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int32_t)atomicAdd(&b.queue[0], 1u);
        __syncthreads();
        const int32_t item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= b.n_items) break;
        const int32_t pi = ((c_i32 *)(const void *)b.order)[item];
        FBatchProg P;
        {
            const __attribute__((address_space(4))) uint32_t *s =
                (const __attribute__((address_space(4))) uint32_t *)(const void *)(b.progs + pi);
            uint32_t *o = reinterpret_cast<uint32_t *>(&P);
#pragma unroll
            for (int i = 0; i < (int)(sizeof(FBatchProg) / 4); ++i) o[i] = s[i];
        }
        // a program of at most lds_rows rows keeps its counts and v in LDS (the
        // pushes reach them through generic pointers, as atomics on LDS), and
        // its v goes to memory once at the end
        const bool in_lds = P.n_rows <= b.lds_rows;
        uint64_t *v = in_lds ? (uint64_t *)s_fdyn : P.v;
        int32_t *cnt = in_lds ? (int32_t *)(s_fdyn + ((b.lds_rows + 63) >> 6)) : P.cnt;
        for (int32_t i = threadIdx.x; i < P.n_rows; i += kFBatchBlock) cnt[i] = P.cnt0[i];
        for (int32_t w = threadIdx.x; w < P.n_words; w += kFBatchBlock) v[w] = 0ull;
        if (threadIdx.x == 0) {
            s_n[0] = (uint32_t)P.n_facts;
            s_n[1] = 0;
        }
        __syncthreads();  // v cleared before the fact bits go in
        for (int32_t j = threadIdx.x; j < P.n_facts; j += kFBatchBlock) {
            const int32_t r = P.facts[j];
            q[0][j] = r;
            atomicOr((unsigned long long *)&v[r >> 6], 1ull << (r & 63));
        }
        __syncthreads();
        FrontierParams f{};
        f.occ_ptr = P.occ_ptr;
        f.occ = P.occ;
        f.cnt = cnt;
        f.v = v;
        int32_t t = 1;  // level t pushes F_{t-1} into F_t
        for (;; ++t) {
            const uint32_t n_in = s_n[(t - 1) & 3];
            if (threadIdx.x == 0) s_n[(t + 1) & 3] = 0;  // read at level t - 2, appended to at level t + 1
            if (n_in > 0)
                push_frontier<false>(f, q[(t - 1) & 1], n_in, q[t & 1], &s_n[t & 3], wid, NW, s_excl[wid],
                                     s_start[wid], lane);
            __syncthreads();
            if (s_n[t & 3] == 0 || t > P.n_rows) break;
        }
        if (threadIdx.x == 0) *P.out_products = s_n[t & 3] == 0 ? t : -1;
        if (in_lds)  // (after the last level's barrier: every push is done)
            for (int32_t w = threadIdx.x; w < P.n_words; w += kFBatchBlock) P.v[w] = v[w];
        __syncthreads();  // s_n, s_item, the queues and the LDS counts are reused by the next program
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&b.queue[1], 1u) == gridDim.x - 1) {
            atomicExch(&b.queue[0], 0u);
            atomicExch(&b.queue[1], 0u);
        }
    }
}

}  // namespace

hipError_t launch_frontier_level(const FrontierParams &f, int grid, hipStream_t st) {
    hipLaunchKernelGGL(frontier_level_kernel, dim3(grid), dim3(kFrontierBlock), 0, st, f);
    return hipGetLastError();
}

hipError_t launch_frontier_levels(const FrontierParams &f, const int32_t *facts, int32_t *q0, int32_t *q1,
                                  int32_t n_levels, int32_t *ctl, hipStream_t st) {
    hipLaunchKernelGGL(frontier_levels_kernel, dim3(1), dim3(kFrontierLoopBlock), 0, st, f, facts, q0, q1, n_levels,
                       ctl);
    return hipGetLastError();
}

hipError_t launch_frontier_batch(const FBatchParams &b, int grid, hipStream_t st) {
    hipLaunchKernelGGL(frontier_batch_kernel, dim3((unsigned)grid), dim3(kFBatchBlock), fbatch_lds_bytes(b.lds_rows),
                       st, b);
    return hipGetLastError();
}

void frontier_kernels_allow_lds(int max_dynamic_lds) {
    (void)hipFuncSetAttribute((const void *)frontier_batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              max_dynamic_lds);
    (void)hipGetLastError();
}

}  // namespace lp
