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
// thread several such items. With W >= 64 a wave covers 64 consecutive words
// of one row, so each gather is one coalesced 512-byte read and the row's CSR
// entries are wave-uniform loads.
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
template <bool WIDE>
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
        int32_t row = (int32_t)(g >> p.log2W);
        if (WIDE) row = __builtin_amdgcn_readfirstlane(row);
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

// Word g of the initial matrix (Definition 8), written to both buffers.
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
    U[g] = x;
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
    if (p.log2W >= 6)
        hipLaunchKernelGGL((spmm_step_kernel<true>), dim3(grid), dim3(kBlock), 0, st, p);
    else
        hipLaunchKernelGGL((spmm_step_kernel<false>), dim3(grid), dim3(kBlock), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_init_m0(uint64_t *V, uint64_t *U, int64_t total, int32_t log2W, int32_t n_std,
                          const uint64_t *fact_bits, const int32_t *guess_pos, int32_t k_eff,
                          unsigned long long *count, unsigned long long bits, hipStream_t st) {
    hipLaunchKernelGGL(init_m0_kernel, dim3(blocks_for(total)), dim3(kBlock), 0, st, V, U, total, log2W, n_std,
                       fact_bits, guess_pos, k_eff, count, bits);
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
