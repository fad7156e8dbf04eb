// lp_spmm.hip -- stable-model kernels on gfx950: the initial matrix
// (Definition 8), the interpretation-matrix step U = theta(M_P V) of
// Algorithm 2, the consistency test of Algorithm 3 and model extraction.
//
// Every row of the interpretation matrix holds W = 2^log2W consecutive
// uint64 words; bit b of word w of row i is atom i in guess column 64w + b.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lp_kernels.h"

namespace lp {

namespace {

constexpr int kBlock = 256;

__device__ inline uint32_t wave_sum(uint32_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ inline uint64_t valid_mask(int32_t k_eff) {
    return k_eff >= 6 ? ~0ull : ((1ull << (1 << k_eff)) - 1ull);
}

}  // namespace

// Thread g owns word (g & (W-1)) of row (g >> log2W): it ANDs (AND row) or ORs
// (OR row) that word of every row its row names; a grid-stride loop gives each
// thread several such items. (Launched for W < 64; wider matrices take
// spmm_step_wide_kernel below, where a wave covers 64 consecutive words of one
// row per chunk, so each gather is one coalesced 512-byte read and the row's
// CSR entries are wave-uniform loads.)
//
// Columns are independent, so the monotone argument of the least-model step
// holds per column: U contains V, and U = V iff both hold the same number of
// bits. The kernel therefore counts the bits of U (counters[step] = |U|, the
// initial matrix's count is counters[0]) instead of reading V's word again
// for popcount(U & ~V): that read would be a quarter of the kernel's traffic.
// The count takes one atomic per workgroup, and the grid is a few workgroups
// per CU (atomics on one address serialize). Product t changed nothing iff
// counters[t] == counters[t-1]; a launch after such a product returns at once
// and copies the count forward.
__global__ __launch_bounds__(kBlock) void spmm_step_kernel(SpmmParams p) {
    __shared__ uint32_t s_bits;
    const int tid = threadIdx.x;
    if (blockIdx.x == 0 && tid == 0) p.counters[(p.step + 1) & (kRing - 1)] = 0;
    if (p.early_exit && p.step >= 2 &&
        p.counters[(p.step - 1) & (kRing - 1)] == p.counters[(p.step - 2) & (kRing - 1)]) {
        // the fixpoint was reached earlier: carry the count forward so every
        // later launch of the batch also returns at once
        if (blockIdx.x == 0 && tid == 0) p.counters[p.step & (kRing - 1)] = p.counters[(p.step - 1) & (kRing - 1)];
        return;
    }
    if (tid == 0) s_bits = 0;
    __syncthreads();
    uint32_t my_bits = 0;
    const int64_t mask_w = (1ll << p.log2W) - 1;
    for (int64_t g = (int64_t)blockIdx.x * kBlock + tid; g < p.total; g += (int64_t)gridDim.x * kBlock) {
        const int32_t row = (int32_t)(g >> p.log2W);
        const int64_t w = g & mask_w;
        const int32_t s = p.row_ptr[row], e = p.row_ptr[row + 1];
        const bool is_and = (p.and_bits[row >> 6] >> (row & 63)) & 1ull;
        uint64_t acc = is_and ? ~0ull : 0ull;
        for (int32_t i = s; i < e; ++i) {
            const int64_t c = p.col[i];
            const uint64_t x = p.V[(c << p.log2W) + w];
            acc = is_and ? (acc & x) : (acc | x);
        }
        if (s == e) acc = 0;
        my_bits += (uint32_t)__popcll(acc);
        p.U[g] = acc;
    }
    my_bits = wave_sum(my_bits);
    if ((tid & 63) == 0 && my_bits) atomicAdd(&s_bits, my_bits);
    __syncthreads();
    if (tid == 0 && s_bits) atomicAdd(&p.counters[p.step & (kRing - 1)], (unsigned long long)s_bits);
}

// The same step for W >= 64 with more loads in flight: a wave takes one row
// and GC chunks of 64 consecutive words of it (GC x 512 bytes per named row),
// and E entries of the row per pass, so each pass issues E GC coalesced loads
// before it combines any (a row names about three others on average; one load
// in flight per wave left the step waiting on memory latency).
template <int GC, int E>
__global__ __launch_bounds__(kBlock) void spmm_step_wide_kernel(SpmmParams p) {
    __shared__ uint32_t s_bits;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    if (blockIdx.x == 0 && tid == 0) p.counters[(p.step + 1) & (kRing - 1)] = 0;
    if (p.early_exit && p.step >= 2 &&
        p.counters[(p.step - 1) & (kRing - 1)] == p.counters[(p.step - 2) & (kRing - 1)]) {
        if (blockIdx.x == 0 && tid == 0) p.counters[p.step & (kRing - 1)] = p.counters[(p.step - 1) & (kRing - 1)];
        return;
    }
    if (tid == 0) s_bits = 0;
    __syncthreads();
    uint32_t my_bits = 0;
    constexpr int kLog2GC = GC == 8 ? 3 : GC == 4 ? 2 : GC == 2 ? 1 : 0;
    const int32_t log2G = p.log2W - 6 - kLog2GC;  // items per row = W / (64 GC)
    const int64_t n_items = (int64_t)(p.total >> p.log2W) << log2G;
    const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t it = (int64_t)blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane(tid >> 6); it < n_items;
         it += waves) {
        const int32_t row = (int32_t)(it >> log2G);
        const int64_t w0 = ((it & ((1ll << log2G) - 1)) * 64 * GC) + lane;
        const int32_t s = p.row_ptr[row], e = p.row_ptr[row + 1];
        const bool is_and = (p.and_bits[row >> 6] >> (row & 63)) & 1ull;
        uint64_t acc[GC];
#pragma unroll
        for (int k = 0; k < GC; ++k) acc[k] = is_and ? ~0ull : 0ull;
        for (int32_t i = s; i < e; i += E) {
            // entries past the row's end reload its last entry (the same word: AND and OR are idempotent)
            uint64_t x[E][GC];
#pragma unroll
            for (int j = 0; j < E; ++j) {
                const int64_t c = p.col[i + j < e ? i + j : e - 1];
#pragma unroll
                for (int k = 0; k < GC; ++k) x[j][k] = p.V[(c << p.log2W) + w0 + 64 * k];
            }
#pragma unroll
            for (int j = 0; j < E; ++j)
#pragma unroll
                for (int k = 0; k < GC; ++k) acc[k] = is_and ? (acc[k] & x[j][k]) : (acc[k] | x[j][k]);
        }
#pragma unroll
        for (int k = 0; k < GC; ++k) {
            const uint64_t a = s == e ? 0ull : acc[k];
            my_bits += (uint32_t)__popcll(a);
            p.U[((int64_t)row << p.log2W) + w0 + 64 * k] = a;
        }
    }
    my_bits = wave_sum(my_bits);
    if ((tid & 63) == 0 && my_bits) atomicAdd(&s_bits, my_bits);
    __syncthreads();
    if (tid == 0 && s_bits) atomicAdd(&p.counters[p.step & (kRing - 1)], (unsigned long long)s_bits);
}

// ---------------------------------------------------------------- dirty rows
//
// Algorithm 2 by dirty rows. A row's value in product t can differ from its
// value in product t-1 only if a row it names changed in product t-1, so
// product t evaluates only those rows (D_t). The initial matrix is 0 outside
// the fact and qbar rows, so a row that names none of them is 0 after product
// 1 as well: D_1 is the set of rows naming a fact or qbar row
// (spmm_dirty_seed_kernel), with the initial matrix in both buffers.
//
// One launch per product t reads V (holding v_{t-1}) and writes U (holding
// v_{t-2}):
//   - the rows that changed in product t-1 (C_{t-1}) and are not in D_t get
//     their v_{t-1} words copied from V into U (rows of D_t are written by
//     their evaluation instead), so U holds v_t on every row afterwards;
//   - every row of D_t is evaluated into U; a row whose words differ from V
//     is appended once to C_t (an atomic max of t on its mark), and the wave
//     that appends it also appends every row naming it (through the transposed
//     matrix) once to D_{t+1}.
// D_t's marks (t on its rows) and D_{t+1}'s are two arrays taken in turn, so
// the marks product t reads do not change under it.
// The products, their count and the fixpoint are those of the full sweep.
// hist[t mod kDirtyHist] counts C_t (the host reads it); ring slot t mod
// kDirtyRing counts D_t. Product t clears the slots products t+1 and t+2
// append to, and returns at once after a product that changed nothing.
// Product 1 needs no read of the initial matrix: it is 0 in every row other
// than the fact and qbar rows, and those keep their initial values in every
// product, so a row changes in product 1 iff it is another row and its result
// is not 0.

__device__ __forceinline__ void dirty_clear_ahead(const DirtyParams &p) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        p.hist[(p.step + 1) & (kDirtyHist - 1)] = 0;
        p.n_dirty[(p.step + 2) & (kDirtyRing - 1)] = 0;
    }
}

// Appends row (changed in product t) to C_t, and the rows naming it to
// D_{t+1}; called by every lane of one wave.
__device__ __forceinline__ void dirty_push(const DirtyParams &p, int32_t row, int lane) {
    const int32_t t = p.step;
    if (lane == 0) p.changed_out[atomicAdd((uint32_t *)&p.hist[t & (kDirtyHist - 1)], 1u)] = row;
    const int32_t o0 = p.occ_ptr[row], o1 = p.occ_ptr[row + 1];
    for (int32_t j = o0 + lane; j < o1; j += 64) {
        const int32_t r = p.occ[j];
        if (atomicMax(&p.dmark[r], t + 1) < t + 1)
            p.dirty_out[atomicAdd(&p.n_dirty[(t + 1) & (kDirtyRing - 1)], 1u)] = r;
    }
}

// One wave per (row, chunk of 64 GC words); W >= 64 (log2W >= 6). Items are
// the copies of C_{t-1}'s rows first, then the evaluations of D_t's rows.
template <int GC>
__global__ __launch_bounds__(kBlock) void spmm_dirty_product_kernel(DirtyParams p) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int32_t t = p.step;
    dirty_clear_ahead(p);
    const int64_t n_copy = t >= 2 ? (int64_t)(uint32_t)p.hist[(t - 1) & (kDirtyHist - 1)] : 0;
    if (t >= 2 && n_copy == 0) return;
    const int64_t n_rows = (int64_t)p.n_dirty[t & (kDirtyRing - 1)];
    constexpr int kLog2GC = GC == 8 ? 3 : GC == 4 ? 2 : GC == 2 ? 1 : 0;
    const int32_t log2G = p.log2W - 6 - kLog2GC;
    const int64_t n_copy_items = n_copy << log2G;
    const int64_t n_items = n_copy_items + (n_rows << log2G);
    const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t it = (int64_t)blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane(tid >> 6); it < n_items;
         it += waves) {
        if (it < n_copy_items) {
            const int32_t row = p.changed_prev[it >> log2G];
            if (p.dmark_cur[row] == t) continue;  // in D_t: its evaluation writes it
            const int64_t at = ((int64_t)row << p.log2W) + ((it & ((1ll << log2G) - 1)) * 64 * GC) + lane;
            uint64_t x[GC];
#pragma unroll
            for (int k = 0; k < GC; ++k) x[k] = p.V[at + 64 * k];
#pragma unroll
            for (int k = 0; k < GC; ++k) p.U[at + 64 * k] = x[k];
            continue;
        }
        const int64_t e_it = it - n_copy_items;
        const int32_t row = p.dirty[e_it >> log2G];
        const int64_t w0 = ((e_it & ((1ll << log2G) - 1)) * 64 * GC) + lane;
        const int32_t s = p.row_ptr[row], e = p.row_ptr[row + 1];
        const bool is_and = (p.and_bits[row >> 6] >> (row & 63)) & 1ull;
        uint64_t acc[GC];
#pragma unroll
        for (int k = 0; k < GC; ++k) acc[k] = is_and ? ~0ull : 0ull;
        for (int32_t i = s; i < e; i += 2) {
            uint64_t x[2][GC];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int64_t c = p.col[i + j < e ? i + j : e - 1];
#pragma unroll
                for (int k = 0; k < GC; ++k) x[j][k] = p.V[(c << p.log2W) + w0 + 64 * k];
            }
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int k = 0; k < GC; ++k) acc[k] = is_and ? (acc[k] & x[j][k]) : (acc[k] | x[j][k]);
        }
        bool diff = false;
        const bool first_varies = row < p.n_std && !((p.fact_bits[row >> 6] >> (row & 63)) & 1ull);
#pragma unroll
        for (int k = 0; k < GC; ++k) {
            const int64_t at = ((int64_t)row << p.log2W) + w0 + 64 * k;
            const uint64_t a = s == e ? 0ull : acc[k];
            diff |= t == 1 ? (first_varies && a != 0ull) : (a != p.V[at]);
            p.U[at] = a;
        }
        if (__ballot(diff) == 0) continue;
        int32_t first = 0;
        if (lane == 0) first = atomicMax(&p.cmark[row], t) < t;
        if (__builtin_amdgcn_readfirstlane(first)) dirty_push(p, row, lane);
    }
}

// W < 64: one thread per word; the W lanes of a row are consecutive in the
// wave (W divides 64). Copies of C_{t-1}'s rows first, then evaluations; a
// changed row is appended by the lowest lane of the wave holding one, a row
// per pass, and the wave pushes its namers.
__global__ __launch_bounds__(kBlock) void spmm_dirty_product_small_kernel(DirtyParams p) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int32_t t = p.step;
    dirty_clear_ahead(p);
    const int64_t n_copy = t >= 2 ? (int64_t)(uint32_t)p.hist[(t - 1) & (kDirtyHist - 1)] : 0;
    if (t >= 2 && n_copy == 0) return;
    const int64_t n_rows = (int64_t)p.n_dirty[t & (kDirtyRing - 1)];
    const int32_t W = 1 << p.log2W;
    const int64_t copy_total = n_copy << p.log2W;
    const int64_t total = copy_total + (n_rows << p.log2W);
    // whole waves iterate together so the ballot sees every lane of a row
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t g0 = (int64_t)blockIdx.x * kBlock + (tid & ~63); g0 < total; g0 += stride) {
        const int64_t g = g0 + lane;
        bool diff = false;
        int32_t row = -1;
        if (g < copy_total) {
            const int32_t r = p.changed_prev[g >> p.log2W];
            if (p.dmark_cur[r] != t) {
                const int64_t at = ((int64_t)r << p.log2W) + (g & (W - 1));
                p.U[at] = p.V[at];
            }
        } else if (g < total) {
            const int64_t pos = (g - copy_total) >> p.log2W;
            row = p.dirty[pos];
            const int64_t w = g & (W - 1);
            const int32_t s = p.row_ptr[row], e = p.row_ptr[row + 1];
            const bool is_and = (p.and_bits[row >> 6] >> (row & 63)) & 1ull;
            uint64_t acc = is_and ? ~0ull : 0ull;
            for (int32_t i = s; i < e; ++i) {
                const uint64_t x = p.V[((int64_t)p.col[i] << p.log2W) + w];
                acc = is_and ? (acc & x) : (acc | x);
            }
            if (s == e) acc = 0;
            const int64_t at = ((int64_t)row << p.log2W) + w;
            if (t == 1)
                diff = row < p.n_std && !((p.fact_bits[row >> 6] >> (row & 63)) & 1ull) && acc != 0ull;
            else
                diff = acc != p.V[at];
            p.U[at] = acc;
        }
        // one flag per row: its first lane holds whether any of its W words changed
        const uint64_t b = __ballot(diff);
        const uint64_t mine = ((W >= 64) ? ~0ull : ((1ull << W) - 1ull)) << (lane & ~(W - 1));
        const bool lead = row >= 0 && (lane & (W - 1)) == 0 && (b & mine) != 0 && atomicMax(&p.cmark[row], t) < t;
        uint64_t leads = __ballot(lead);
        while (leads) {
            const int src = __builtin_ctzll(leads);
            leads &= leads - 1;
            dirty_push(p, __shfl(row, src, 64), lane);
        }
    }
}

// D_1: the rows naming a fact row or a qbar row (the rows the initial matrix
// does not hold at 0). One wave per such row.
__global__ __launch_bounds__(kBlock) void spmm_dirty_seed_kernel(DirtyParams p, const int32_t *facts, int32_t n_facts) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int64_t n_seed = (int64_t)n_facts + (p.n_rows - p.n_std);
    const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t q = (int64_t)blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane(tid >> 6); q < n_seed;
         q += waves) {
        const int32_t row = q < n_facts ? facts[q] : p.n_std + (int32_t)(q - n_facts);
        const int32_t o0 = p.occ_ptr[row], o1 = p.occ_ptr[row + 1];
        for (int32_t j = o0 + lane; j < o1; j += 64) {
            const int32_t r = p.occ[j];
            if (atomicMax(&p.dmark[r], 1) < 1) p.dirty_out[atomicAdd(&p.n_dirty[1], 1u)] = r;
        }
    }
}

// Back to the initial matrix after a solve by dirty rows: every row that
// changed in some product (C mark > 0; never a fact or qbar row, which keep
// their initial values) is set to 0 in both buffers, and the marks, the |D_t|
// ring and the |C_t| history are cleared. One wave per row; the wave that
// reads a row's mark also clears it. marks: [cmark n | dm0 n | dm1 n | ring |
// hist], n = max(n_rows, 1).
__global__ __launch_bounds__(kBlock) void spmm_dirty_reset_kernel(uint64_t *b0, uint64_t *b1, int32_t log2W,
                                                                  int32_t *marks, int32_t n) {
    const int lane = threadIdx.x & 63;
    const int64_t W = 1ll << log2W;
    const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t r = (int64_t)blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); r < n;
         r += waves) {
        if (marks[r] > 0) {
            const int64_t base = r << log2W;
            for (int64_t w = lane; w < W; w += 64) {
                b0[base + w] = 0ull;
                b1[base + w] = 0ull;
            }
        }
        if (lane == 0) {
            marks[r] = 0;
            marks[n + r] = 0;
            marks[2 * (int64_t)n + r] = 0;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < kDirtyRing + kDirtyHist) marks[3 * (int64_t)n + threadIdx.x] = 0;
}

hipError_t launch_dirty_reset(uint64_t *b0, uint64_t *b1, int32_t log2W, int32_t *marks, int32_t n, int max_grid,
                              hipStream_t st) {
    hipLaunchKernelGGL(spmm_dirty_reset_kernel, dim3((unsigned)std::max(1, max_grid)), dim3(kBlock), 0, st, b0, b1,
                       log2W, marks, n);
    return hipGetLastError();
}

// Word g of the initial matrix (Definition 8), written to V and, unless it is
// null, to U.
// Column j of the compressed guess space: bit pos of j
// is the value of the qbar row whose guess sits at bit pos. Fact rows are all
// ones; qbar rows of a pruned guess and all other rows are 0.
__device__ __forceinline__ void init_m0_word(uint64_t *V, uint64_t *U, int64_t g, int32_t log2W, int32_t n_std,
                                                 const uint64_t *fact_bits, const int32_t *guess_pos,
                                                 int32_t k_eff) {
    const int32_t row = (int32_t)(g >> log2W);
    const int64_t w = g & ((1ll << log2W) - 1);
    const uint64_t valid = valid_mask(k_eff);
    uint64_t x = 0;
    if ((fact_bits[row >> 6] >> (row & 63)) & 1ull) {
        x = valid;
    } else if (row >= n_std) {
        const int pos = guess_pos[row - n_std];
        if (pos >= 6) {
            x = ((w >> (pos - 6)) & 1) ? ~0ull : 0ull;
        } else if (pos >= 0) {
            // bit b of the word is set iff bit pos of b is set
            const uint64_t pat[6] = {0xAAAAAAAAAAAAAAAAull, 0xCCCCCCCCCCCCCCCCull, 0xF0F0F0F0F0F0F0F0ull,
                                     0xFF00FF00FF00FF00ull, 0xFFFF0000FFFF0000ull, 0xFFFFFFFF00000000ull};
            x = pat[pos];
        }
        x &= valid;
    }
    V[g] = x;
    if (U) U[g] = x;
}

// The initial matrix; *count receives its bit count, which has a closed form
// (every fact row holds all 2^k_eff guesses, every guessed qbar row half of
// them), so no reduction is needed.
__global__ __launch_bounds__(kBlock) void init_m0_kernel(uint64_t *V, uint64_t *U, int64_t total, int32_t log2W,
                                                         int32_t n_std, const uint64_t *fact_bits,
                                                         const int32_t *guess_pos, int32_t k_eff,
                                                         unsigned long long *count, unsigned long long bits) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g == 0) *count = bits;
    if (g < total) init_m0_word(V, U, g, log2W, n_std, fact_bits, guess_pos, k_eff);
}

// Initial matrix for explicit guesses (word g, V and U unless null): column j is
// guess j of the caller's list, bit t of guesses[j] the initial value of
// qbar_t (row n_std + t); fact rows are all ones; every other row is 0.
__global__ __launch_bounds__(kBlock) void init_guess_kernel(uint64_t *V, uint64_t *U, int64_t total, int32_t log2W,
                                                            int32_t n_std, int32_t K, const uint64_t *fact_bits,
                                                            const uint64_t *guesses) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= total) return;
    const int32_t row = (int32_t)(g >> log2W);
    const int64_t w = g & ((1ll << log2W) - 1);
    uint64_t x = 0;
    if ((fact_bits[row >> 6] >> (row & 63)) & 1ull) {
        x = ~0ull;
    } else if (row >= n_std && row - n_std < K) {
        const int t = row - n_std;
        const uint64_t *gw = guesses + w * 64;
        for (int b = 0; b < 64; ++b) x |= ((gw[b] >> t) & 1ull) << b;
    }
    V[g] = x;
    if (U) U[g] = x;
}

// The guess each column's fixpoint points to: bit t set iff q_t is false in
// the column (then assuming qbar_t is the consistent choice). A column that
// Algorithm 3 accepts maps to its own guess.
__global__ __launch_bounds__(kBlock) void next_guess_kernel(const uint64_t *V, int32_t log2W, int64_t n_cols,
                                                            const int32_t *q_rows, int32_t K, uint64_t *out) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n_cols) return;
    const int64_t w = j >> 6;
    const int b = (int)(j & 63);
    uint64_t g = 0;
    for (int32_t t = 0; t < K; ++t)
        if (!((V[((int64_t)q_rows[t] << log2W) + w] >> b) & 1ull)) g |= 1ull << t;
    out[j] = g;
}

// Algorithm 3: column j is accepted iff for every negated atom q_t exactly
// one of row q_t and row qbar_t is 1 (a_l + a_j = 1), i.e. their XOR is 1.
__global__ __launch_bounds__(kBlock) void stable_check_kernel(const uint64_t *V, int32_t log2W, int64_t W,
                                                              const int32_t *q_rows, int32_t n_std, int32_t K,
                                                              int32_t k_eff, uint64_t *accept,
                                                              unsigned long long *count) {
    const int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    uint32_t c = 0;
    if (w < W) {
        uint64_t ok = valid_mask(k_eff);
        for (int32_t t = 0; t < K; ++t)
            ok &= V[((int64_t)q_rows[t] << log2W) + w] ^ V[((int64_t)(n_std + t) << log2W) + w];
        accept[w] = ok;
        c = (uint32_t)__popcll(ok);
    }
    c = wave_sum(c);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, (unsigned long long)c);
}

// Models: column cols[m] of rows [0, n_atoms) as bytes.
__global__ __launch_bounds__(kBlock) void extract_kernel(const uint64_t *V, int32_t log2W, const int64_t *cols,
                                                         int64_t n_models, int32_t n_atoms, uint8_t *out) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= n_models * (int64_t)n_atoms) return;
    const int64_t mi = g / n_atoms;
    const int32_t a = (int32_t)(g - mi * n_atoms);
    const int64_t j = cols[mi];
    out[g] = (uint8_t)((V[((int64_t)a << log2W) + (j >> 6)] >> (j & 63)) & 1ull);
}

static unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

hipError_t launch_spmm_step(const SpmmParams &p, int max_grid, hipStream_t st) {
    const unsigned grid = std::max(1u, std::min(blocks_for(p.total), (unsigned)std::max(1, max_grid)));
    // chunks per item, measured at W = 1,024 (16 negated atoms): 8 chunks 113 us per product,
    // 4 chunks 119 us, one chunk and one entry at a time 148 us; 4 entries per pass were slower
    // than 2 (rows name about three others, so more entries reload the last one more often)
    if (p.log2W >= 9)
        hipLaunchKernelGGL((spmm_step_wide_kernel<8, 2>), dim3(grid), dim3(kBlock), 0, st, p);
    else if (p.log2W == 8)
        hipLaunchKernelGGL((spmm_step_wide_kernel<4, 2>), dim3(grid), dim3(kBlock), 0, st, p);
    else if (p.log2W == 7)
        hipLaunchKernelGGL((spmm_step_wide_kernel<2, 2>), dim3(grid), dim3(kBlock), 0, st, p);
    else if (p.log2W == 6)
        hipLaunchKernelGGL((spmm_step_wide_kernel<1, 2>), dim3(grid), dim3(kBlock), 0, st, p);
    else
        hipLaunchKernelGGL(spmm_step_kernel, dim3(grid), dim3(kBlock), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_dirty_seed(const DirtyParams &p, const int32_t *facts, int32_t n_facts, int max_grid,
                             hipStream_t st) {
    hipLaunchKernelGGL(spmm_dirty_seed_kernel, dim3((unsigned)std::max(1, max_grid)), dim3(kBlock), 0, st, p, facts,
                       n_facts);
    return hipGetLastError();
}

hipError_t launch_dirty_product(const DirtyParams &p, int max_grid, hipStream_t st) {
    const unsigned grid = (unsigned)std::max(1, max_grid);
    if (p.log2W >= 9)
        hipLaunchKernelGGL((spmm_dirty_product_kernel<8>), dim3(grid), dim3(kBlock), 0, st, p);
    else if (p.log2W == 8)
        hipLaunchKernelGGL((spmm_dirty_product_kernel<4>), dim3(grid), dim3(kBlock), 0, st, p);
    else if (p.log2W == 7)
        hipLaunchKernelGGL((spmm_dirty_product_kernel<2>), dim3(grid), dim3(kBlock), 0, st, p);
    else if (p.log2W == 6)
        hipLaunchKernelGGL((spmm_dirty_product_kernel<1>), dim3(grid), dim3(kBlock), 0, st, p);
    else
        hipLaunchKernelGGL(spmm_dirty_product_small_kernel, dim3(grid), dim3(kBlock), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_init_m0(uint64_t *V, uint64_t *U, int64_t total, int32_t log2W, int32_t n_std,
                          const uint64_t *fact_bits, const int32_t *guess_pos, int32_t k_eff,
                          unsigned long long *count, unsigned long long bits, hipStream_t st) {
    hipLaunchKernelGGL(init_m0_kernel, dim3(blocks_for(total)), dim3(kBlock), 0, st, V, U, total, log2W, n_std,
                       fact_bits, guess_pos, k_eff, count, bits);
    return hipGetLastError();
}

hipError_t launch_init_guess(uint64_t *V, uint64_t *U, int64_t total, int32_t log2W, int32_t n_std, int32_t K,
                             const uint64_t *fact_bits, const uint64_t *guesses, hipStream_t st) {
    hipLaunchKernelGGL(init_guess_kernel, dim3(blocks_for(total)), dim3(kBlock), 0, st, V, U, total, log2W, n_std, K,
                       fact_bits, guesses);
    return hipGetLastError();
}

hipError_t launch_next_guess(const uint64_t *V, int32_t log2W, int64_t n_cols, const int32_t *q_rows, int32_t K,
                             uint64_t *out, hipStream_t st) {
    hipLaunchKernelGGL(next_guess_kernel, dim3(blocks_for(n_cols)), dim3(kBlock), 0, st, V, log2W, n_cols, q_rows, K,
                       out);
    return hipGetLastError();
}

hipError_t launch_stable_check(const uint64_t *V, int32_t log2W, int64_t W, const int32_t *q_rows, int32_t n_std,
                               int32_t K, int32_t k_eff, uint64_t *accept, unsigned long long *count,
                               hipStream_t st) {
    hipLaunchKernelGGL(stable_check_kernel, dim3(blocks_for(W)), dim3(kBlock), 0, st, V, log2W, W, q_rows, n_std, K,
                       k_eff, accept, count);
    return hipGetLastError();
}

hipError_t launch_extract(const uint64_t *V, int32_t log2W, const int64_t *cols, int64_t n_models, int32_t n_atoms,
                          uint8_t *out, hipStream_t st) {
    hipLaunchKernelGGL(extract_kernel, dim3(blocks_for(n_models * (int64_t)n_atoms)), dim3(kBlock), 0, st, V,
                       log2W, cols, n_models, n_atoms, out);
    return hipGetLastError();
}

}  // namespace lp
