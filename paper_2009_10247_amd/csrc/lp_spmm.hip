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
// The sets are bitmaps over rows (bit r & 31 of 32-bit word r >> 5), filled
// with atomic ORs whose results are not waited for. One launch per product t
// reads V (holding v_{t-1}) and writes U (holding v_{t-2}):
//   - the rows of C_{t-1} (changed in product t-1) outside D_t get their
//     v_{t-1} words copied from V into U (rows of D_t are written by their
//     evaluation instead), so U holds v_t on every row afterwards;
//   - every row of D_t is evaluated into U; a row whose words differ from V
//     goes into C_t and into the cumulative set of changed rows, and every
//     row naming it (through the transposed matrix) into D_{t+1}.
// Bitmaps come in threes by product mod 3: product t reads D_t and C_{t-1},
// sets D_{t+1} and C_t, and clears the ones products t+1 and t+2 set (D_{t+2},
// C_{t+1}), which no product running at the same time reads. hist[t mod
// kDirtyHist] = 1 iff product t changed a row (the host reads it); product t
// clears the next slot, and returns at once after a product that changed
// nothing. The products, their count and the fixpoint are those of the full
// sweep. Product 1 needs no read of the initial matrix: it is 0 in every row
// other than the fact and qbar rows, and those keep their initial values in
// every product, so a row changes in product 1 iff it is another row and its
// result is not 0.

__device__ __forceinline__ void bit_or(uint32_t *bits, int64_t row) {
    __hip_atomic_fetch_or(&bits[row >> 5], 1u << (row & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Row `row` changed in product t: into C_t and the cumulative set (by lane
// 0), and every row naming it into D_{t+1} (all lanes of the wave).
__device__ __forceinline__ void dirty_changed(const DirtyParams &p, int32_t row, int lane) {
    if (lane == 0) {
        bit_or(p.ccur, row);
        bit_or(p.call, row);
    }
    const int32_t o0 = p.occ_ptr[row], o1 = p.occ_ptr[row + 1];
    for (int32_t j = o0 + lane; j < o1; j += 64) bit_or(p.dnext, p.occ[j]);
}

__device__ __forceinline__ void dirty_clear_ahead(const DirtyParams &p) {
    const int64_t threads = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < p.nb; i += threads) {
        p.dclear[i] = 0u;
        p.cclear[i] = 0u;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) p.hist[(p.step + 1) & (kDirtyHist - 1)] = 0;
}

// Evaluates words [w0, w0 + 64 GC) of NR rows (W >= 64) into U, their loads
// interleaved; bit k of the result (in every lane) is set if a word of
// rows[k] changed, and then that row's sets are updated (the waves of the
// row's other chunks may do the same: the sets are ORed).
template <int GC, int NR>
__device__ __forceinline__ uint32_t dirty_eval_chunk(const DirtyParams &p, const int32_t *rows, int64_t w0, int lane) {
    const int32_t t = p.step;
    const int64_t w = w0 + lane;
    int32_t s[NR], e[NR];
    bool is_and[NR];
    int32_t most = 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        s[r] = p.row_ptr[rows[r]];
        e[r] = p.row_ptr[rows[r] + 1];
        is_and[r] = (p.and_bits[rows[r] >> 6] >> (rows[r] & 63)) & 1ull;
        most = e[r] - s[r] > most ? e[r] - s[r] : most;
    }
    uint64_t acc[NR][GC];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int k = 0; k < GC; ++k) acc[r][k] = is_and[r] ? ~0ull : 0ull;
    // the entries of each row, 64 at a time, one per lane (lanes past the
    // row's end hold its last entry), so a pass reads them with readlane
    // instead of waiting for a load of each
    int32_t cl[NR];
    auto load_entries = [&](int32_t i0) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int32_t at = s[r] + i0 + lane;
            cl[r] = e[r] > s[r] ? p.col[at < e[r] ? at : e[r] - 1] : 0;  // (an empty row reads nothing)
        }
    };
    load_entries(0);
    // two entries of every row per pass; a row shorter than the longest
    // repeats its last entry (harmless for AND and OR alike)
    for (int32_t i = 0; i < most; i += 2) {
        if (i > 0 && (i & 63) == 0) load_entries(i);  // (i even: a pass never straddles two loads)
        uint64_t x[NR][2][GC];
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int64_t c = __builtin_amdgcn_readlane(cl[r], (i + j) & 63);
#pragma unroll
                for (int k = 0; k < GC; ++k) x[r][j][k] = e[r] > s[r] ? p.V[(c << p.log2W) + w + 64 * k] : 0ull;
            }
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int k = 0; k < GC; ++k)
                    acc[r][k] = is_and[r] ? (acc[r][k] & x[r][j][k]) : (acc[r][k] | x[r][j][k]);
    }
    uint32_t changed = 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int32_t row = rows[r];
        const bool first_varies = row < p.n_std && !((p.fact_bits[row >> 6] >> (row & 63)) & 1ull);
        bool diff = false;
#pragma unroll
        for (int k = 0; k < GC; ++k) {
            const int64_t at = ((int64_t)row << p.log2W) + w + 64 * k;
            const uint64_t a = s[r] == e[r] ? 0ull : acc[r][k];
            diff |= t == 1 ? (first_varies && a != 0ull) : (a != p.V[at]);
            p.U[at] = a;
        }
        if (__ballot(diff) != 0) {
            dirty_changed(p, row, lane);
            changed |= 1u << r;
        }
    }
    return changed;
}

// W >= 64: a wave takes a quarter of a bitmap word (8 rows) and one chunk of
// 64 GC words of each of its rows at a time, so rows close together are
// spread over waves.
template <int GC>
__global__ __launch_bounds__(kBlock) void spmm_dirty_product_kernel(DirtyParams p) {
    const int lane = threadIdx.x & 63;
    const int32_t t = p.step;
    dirty_clear_ahead(p);
    if (t >= 2 && p.hist[(t - 1) & (kDirtyHist - 1)] == 0) return;
    constexpr int kLog2GC = GC == 8 ? 3 : GC == 4 ? 2 : GC == 2 ? 1 : 0;
    const int32_t log2G = p.log2W - 6 - kLog2GC;  // chunks per row
    const int64_t n_items = (p.nb << log2G) << 2;
    const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
    bool any = false;
    for (int64_t it = (int64_t)blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
         it < n_items; it += waves) {
        const int q = (int)(it & 3);
        const int64_t ic = it >> 2;
        const int64_t i = ic >> log2G;
        const int64_t w0 = (ic & ((1ll << log2G) - 1)) * 64 * GC;
        const uint32_t quarter = 0xFFu << (8 * q);
        const uint32_t d = p.dcur[i];
        uint32_t dw = d & quarter;
        uint32_t cw = t >= 2 ? (p.cprev[i] & ~d & quarter) : 0u;
        const int64_t row0 = i * 32;
        while (cw) {
            const int b = __builtin_ctz(cw);
            cw &= cw - 1;
            const int64_t base = ((row0 + b) << p.log2W) + w0 + lane;
            uint64_t x[GC];
#pragma unroll
            for (int k = 0; k < GC; ++k) x[k] = p.V[base + 64 * k];
#pragma unroll
            for (int k = 0; k < GC; ++k) p.U[base + 64 * k] = x[k];
        }
        while (dw) {  // two rows at a time, their loads interleaved
            int32_t rows[2];
            rows[0] = (int32_t)(row0 + __builtin_ctz(dw));
            dw &= dw - 1;
            if (dw) {
                rows[1] = (int32_t)(row0 + __builtin_ctz(dw));
                dw &= dw - 1;
                any |= dirty_eval_chunk<GC, 2>(p, rows, w0, lane) != 0u;
            } else {
                any |= dirty_eval_chunk<GC, 1>(p, rows, w0, lane) != 0u;
            }
        }
    }
    if (any && lane == 0) p.hist[t & (kDirtyHist - 1)] = 1;
}

// W < 64: a wave takes p.wpi bitmap words (32 p.wpi rows; the host picks 1 to
// 8 so that the grid's waves all get work) at a time and evaluates their rows
// 64 / W per pass, one lane per word (the W lanes of a row are consecutive in
// the wave).
__global__ __launch_bounds__(kBlock) void spmm_dirty_product_small_kernel(DirtyParams p) {
    const int lane = threadIdx.x & 63;
    const int32_t t = p.step;
    dirty_clear_ahead(p);
    if (t >= 2 && p.hist[(t - 1) & (kDirtyHist - 1)] == 0) return;
    const int32_t W = 1 << p.log2W;
    const int R = 64 >> p.log2W;  // rows per pass
    const int slot = lane >> p.log2W, w = lane & (W - 1);
    const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
    const int64_t gw = (int64_t)blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    bool any = false;
    const int64_t wpi = p.wpi;
    for (int64_t i0 = gw * wpi; i0 < p.nb; i0 += waves * wpi) {
        const int64_t i = i0 + lane;
        uint32_t d = 0, c = 0;
        if (lane < wpi && i < p.nb) {
            d = p.dcur[i];
            c = t >= 2 ? (p.cprev[i] & ~d) : 0u;
        }
        uint64_t m = __ballot((d | c) != 0u);
        while (m) {
            const int src = __builtin_ctzll(m);
            m &= m - 1;
            const int64_t row0 = (i0 + src) * 32;
            uint32_t cw = __builtin_amdgcn_readlane(c, src), dw = __builtin_amdgcn_readlane(d, src);
            while (cw) {  // copies, R rows per pass
                int32_t row = -1;
                for (int sl = 0; sl < R && cw; ++sl) {
                    const int b = __builtin_ctz(cw);
                    cw &= cw - 1;
                    if (sl == slot) row = (int32_t)(row0 + b);
                }
                if (row >= 0) {
                    const int64_t at = ((int64_t)row << p.log2W) + w;
                    p.U[at] = p.V[at];
                }
            }
            while (dw) {  // evaluations, R rows per pass
                int32_t row = -1;
                for (int sl = 0; sl < R && dw; ++sl) {
                    const int b = __builtin_ctz(dw);
                    dw &= dw - 1;
                    if (sl == slot) row = (int32_t)(row0 + b);
                }
                bool diff = false;
                if (row >= 0) {
                    const int32_t s = p.row_ptr[row], e = p.row_ptr[row + 1];
                    const bool is_and = (p.and_bits[row >> 6] >> (row & 63)) & 1ull;
                    uint64_t acc = is_and ? ~0ull : 0ull;
                    // four entries per pass, their loads issued together (the last one repeats past the end)
                    for (int32_t k = s; k < e; k += 4) {
                        int64_t cc[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) cc[q] = p.col[k + q < e ? k + q : e - 1];
                        uint64_t x[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) x[q] = p.V[(cc[q] << p.log2W) + w];
#pragma unroll
                        for (int q = 0; q < 4; ++q) acc = is_and ? (acc & x[q]) : (acc | x[q]);
                    }
                    if (s == e) acc = 0;
                    const int64_t at = ((int64_t)row << p.log2W) + w;
                    if (t == 1)
                        diff = row < p.n_std && !((p.fact_bits[row >> 6] >> (row & 63)) & 1ull) && acc != 0ull;
                    else
                        diff = acc != p.V[at];
                    p.U[at] = acc;
                }
                // a row changed iff one of its W lanes saw a difference; its first lane leads
                const uint64_t b = __ballot(diff);
                const uint64_t mine = ((W >= 64) ? ~0ull : ((1ull << W) - 1ull)) << (lane & ~(W - 1));
                uint64_t leads = __ballot(row >= 0 && w == 0 && (b & mine) != 0);
                any |= leads != 0;
                while (leads) {
                    const int l = __builtin_ctzll(leads);
                    leads &= leads - 1;
                    dirty_changed(p, __shfl(row, l, 64), lane);
                }
            }
        }
    }
    if (any && lane == 0) p.hist[t & (kDirtyHist - 1)] = 1;
}

// D_1: the rows naming a fact row or a qbar row (the rows the initial matrix
// does not hold at 0); the cumulative set of changed rows cleared. One wave
// per fact row; the qbar rows' occurrences
// (one contiguous range of the transposed matrix, since the qbar rows are the
// last rows) are split 64 entries per wave over the grid, as a qbar row can
// be named by a large share of all rows.
__global__ __launch_bounds__(kBlock) void spmm_dirty_seed_kernel(DirtyParams p, const int32_t *facts, int32_t n_facts) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
    const int64_t wave = (int64_t)blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // the cumulative set of changed rows starts empty (the previous solve's reset read it)
    const int64_t threads = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < p.nb; i += threads) p.call[i] = 0u;
    for (int64_t q = wave; q < n_facts; q += waves) {
        const int32_t row = facts[q];
        const int32_t o0 = p.occ_ptr[row], o1 = p.occ_ptr[row + 1];
        for (int32_t j = o0 + lane; j < o1; j += 64) bit_or(p.dnext, p.occ[j]);
    }
    const int64_t b0 = p.occ_ptr[p.n_std], b1 = p.occ_ptr[p.n_rows];
    for (int64_t j = b0 + wave * 64 + lane; j < b1; j += waves * 64) bit_or(p.dnext, p.occ[j]);
}

// Back to the initial matrix after a solve by dirty rows: every row that
// changed in some product (the cumulative set; never a fact or qbar row,
// which keep their initial values) is set to 0 in both buffers, and the D and
// C sets and the history are cleared (the cumulative set is cleared by the
// next solve's seed, as waves here read it until the end). sets: [D0 | D1 |
// D2 | C0 | C1 | C2 | changed], nb words each, then the history. A wave takes
// one bitmap word and 64 words of each of its rows at a time.
__global__ __launch_bounds__(kBlock) void spmm_dirty_reset_kernel(uint64_t *b0, uint64_t *b1, int32_t log2W,
                                                                  uint32_t *sets, int64_t nb) {
    const int lane = threadIdx.x & 63;
    const int32_t log2G = log2W > 6 ? log2W - 6 : 0;  // 64-word chunks per row
    const int64_t n_items = nb << log2G;
    const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
    const uint32_t *call = sets + 6 * nb;
    for (int64_t it = (int64_t)blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
         it < n_items; it += waves) {
        const int64_t i = it >> log2G;
        const int64_t w = ((it & ((1ll << log2G) - 1)) << 6) + lane;
        uint32_t bits = call[i];
        while (bits) {
            const int b = __builtin_ctz(bits);
            bits &= bits - 1;
            if (w < (1ll << log2W)) {
                const int64_t at = ((i * 32 + b) << log2W) + w;
                b0[at] = 0ull;
                b1[at] = 0ull;
            }
        }
    }
    const int64_t threads = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < 6 * nb + kDirtyHist; i += threads) {
        if (i < 6 * nb)
            sets[i] = 0u;
        else
            sets[7 * nb + (i - 6 * nb)] = 0u;
    }
}

hipError_t launch_dirty_reset(uint64_t *b0, uint64_t *b1, int32_t log2W, uint32_t *sets, int64_t nb, int max_grid,
                              hipStream_t st) {
    hipLaunchKernelGGL(spmm_dirty_reset_kernel, dim3((unsigned)std::max(1, max_grid)), dim3(kBlock), 0, st, b0, b1,
                       log2W, sets, nb);
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

// ---------------------------------------------------------------- batches
//
// Stable models of several programs (Algorithms 2 and 3 per program) with one
// launch per product for all of them: the items of the launches are the
// union of the programs' row-words, each program's in whole chunks of
// kSBatchChunk from its chunk0, so every chunk names one program (found by a
// binary search over the descriptors, which the host wrote and the kernels
// read through the constant address space). Per program the product is that
// of spmm_step_kernel, with its bit count in the program's own ring; a
// program whose previous product changed nothing is skipped.

typedef const __attribute__((address_space(4))) SBatchProg csbatch;

__device__ __forceinline__ const csbatch *sbatch_progs(const SBatchParams &b) {
    return (const csbatch *)(const void *)b.progs;
}

__device__ __forceinline__ int32_t sbatch_prog_of(const SBatchParams &b, int64_t c) {
    const csbatch *P = sbatch_progs(b);
    int32_t lo = 0, hi = b.n_progs - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (P[mid].chunk0 <= c) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ uint32_t block_sum(uint32_t x, uint32_t *s_red) {
    x = wave_sum(x);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = x;
    __syncthreads();
    uint32_t s = 0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kBlock / 64; ++k) s += s_red[k];
    __syncthreads();
    return s;  // in thread 0
}

// Both buffers of every program at the initial matrix; count slot 0 its bit
// count (closed form) and slot 1 cleared.
__global__ __launch_bounds__(kBlock) void sbatch_init_kernel(SBatchParams b) {
    static_assert(kSBatchChunk == kBlock, "one chunk per workgroup pass");
    const int tid = threadIdx.x;
    for (int64_t c = blockIdx.x; c < b.n_chunks; c += gridDim.x) {
        const csbatch &P = sbatch_progs(b)[sbatch_prog_of(b, c)];
        const int64_t g = (c - P.chunk0) * kSBatchChunk + tid;
        if (g < P.total) init_m0_word(P.buf[0], P.buf[1], g, P.log2W, P.n_std, P.fact_bits, P.guess_pos, P.k_eff);
        if (c == P.chunk0 && tid == 0) {
            P.count[0] = P.m0_bits;
            P.count[1] = 0;
        }
    }
}

// Product b.step of every program still changing.
__global__ __launch_bounds__(kBlock) void sbatch_step_kernel(SBatchParams b) {
    __shared__ uint32_t s_red[kBlock / 64];
    const int tid = threadIdx.x;
    const int32_t t = b.step;
    for (int64_t c = blockIdx.x; c < b.n_chunks; c += gridDim.x) {
        const csbatch &P = sbatch_progs(b)[sbatch_prog_of(b, c)];
        unsigned long long *cnt = P.count;
        const bool first = c == P.chunk0;
        if (t >= 2 && cnt[(t - 1) & (kRing - 1)] == cnt[(t - 2) & (kRing - 1)]) {
            // the program reached its fixpoint earlier: carry the count forward
            if (first && tid == 0) cnt[t & (kRing - 1)] = cnt[(t - 1) & (kRing - 1)];
            continue;
        }
        if (first && tid == 0) cnt[(t + 1) & (kRing - 1)] = 0;
        const uint64_t *V = P.buf[(t - 1) & 1];
        uint64_t *U = P.buf[t & 1];
        const int32_t log2W = P.log2W;
        const int64_t g = (c - P.chunk0) * kSBatchChunk + tid;
        uint32_t bits = 0;
        if (g < P.total) {
            const int32_t row = (int32_t)(g >> log2W);
            const int64_t w = g & ((1ll << log2W) - 1);
            const int32_t s = P.row_ptr[row], e = P.row_ptr[row + 1];
            const bool is_and = (P.and_bits[row >> 6] >> (row & 63)) & 1ull;
            uint64_t acc = is_and ? ~0ull : 0ull;
            for (int32_t i = s; i < e; ++i) {
                const uint64_t x = V[((int64_t)P.col[i] << log2W) + w];
                acc = is_and ? (acc & x) : (acc | x);
            }
            if (s == e) acc = 0;
            bits = (uint32_t)__popcll(acc);
            U[g] = acc;
        }
        bits = block_sum(bits, s_red);
        if (tid == 0 && bits) atomicAdd(&cnt[t & (kRing - 1)], (unsigned long long)bits);
    }
}

// Algorithm 3 (as stable_check_kernel) and the model of the first accepted
// column, one workgroup per program (W <= 64 words: one lane per word); both
// buffers hold the fixpoint.
__global__ __launch_bounds__(kBlock) void sbatch_outputs_kernel(SBatchParams b) {
    __shared__ int64_t s_first;
    const int tid = threadIdx.x;
    for (int32_t pi = blockIdx.x; pi < b.n_progs; pi += gridDim.x) {
        const csbatch &P = sbatch_progs(b)[pi];
        const uint64_t *V = P.buf[0];
        const int32_t log2W = P.log2W;
        if (tid < 64) {
            uint64_t ok = 0;
            if (tid < (1 << log2W)) {
                ok = valid_mask(P.k_eff);
                for (int32_t q = 0; q < P.K; ++q)
                    ok &= V[((int64_t)P.q_rows[q] << log2W) + tid] ^ V[((int64_t)(P.n_std + q) << log2W) + tid];
                P.accepted[tid] = ok;
            }
            const uint32_t n = wave_sum((uint32_t)__popcll(ok));
            const uint64_t nz = __ballot(ok != 0ull);
            const int l = nz ? __builtin_ctzll(nz) : 0;
            const uint32_t lo = __shfl((uint32_t)ok, l, 64), hi = __shfl((uint32_t)(ok >> 32), l, 64);
            if (tid == 0) {
                *P.n_models = n;
                s_first = nz ? (int64_t)l * 64 + (lo ? __builtin_ctz(lo) : 32 + __builtin_ctz(hi)) : -1;
            }
        }
        __syncthreads();
        const int64_t j = s_first;
        for (int32_t a = tid; a < P.n_atoms; a += kBlock)
            P.model[a] = j >= 0 ? (uint8_t)((V[((int64_t)a << log2W) + (j >> 6)] >> (j & 63)) & 1ull) : (uint8_t)0;
        __syncthreads();
    }
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
    if (p.log2W < 6) {
        hipLaunchKernelGGL(spmm_dirty_product_small_kernel, dim3(grid), dim3(kBlock), 0, st, p);
        return hipGetLastError();
    }
    // chunks of up to 64 x 4 words: more chunks per row put a changed row's
    // words on more waves, which beat keeping more loads in flight per wave
    // (8 words per lane and chunk: 0.272 / 0.296 / 0.681 ms per solve at 15 /
    // 16 / 18 negated atoms on 10,000 atoms; 4: 0.233 / 0.273 / 0.681; 2 at
    // 16: 0.298)
    const int log2GC = std::min(2, p.log2W - 6);
    switch (log2GC) {
        case 2: hipLaunchKernelGGL((spmm_dirty_product_kernel<4>), dim3(grid), dim3(kBlock), 0, st, p); break;
        case 1: hipLaunchKernelGGL((spmm_dirty_product_kernel<2>), dim3(grid), dim3(kBlock), 0, st, p); break;
        default: hipLaunchKernelGGL((spmm_dirty_product_kernel<1>), dim3(grid), dim3(kBlock), 0, st, p); break;
    }
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

hipError_t launch_sbatch_init(const SBatchParams &b, int max_grid, hipStream_t st) {
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(b.n_chunks, std::max(1, max_grid)));
    hipLaunchKernelGGL(sbatch_init_kernel, dim3(grid), dim3(kBlock), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_sbatch_step(const SBatchParams &b, int max_grid, hipStream_t st) {
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(b.n_chunks, std::max(1, max_grid)));
    hipLaunchKernelGGL(sbatch_step_kernel, dim3(grid), dim3(kBlock), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_sbatch_outputs(const SBatchParams &b, hipStream_t st) {
    hipLaunchKernelGGL(sbatch_outputs_kernel, dim3((unsigned)std::max(1, b.n_progs)), dim3(kBlock), 0, st, b);
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
