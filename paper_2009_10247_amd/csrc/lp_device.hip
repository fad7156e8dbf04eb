// lp_device.hip -- gfx950 kernels and the C-ABI entry points that drive them.
//
// Interpretations are bit-packed: bit (i & 63) of word (i >> 6) is row i.
// For the stable-model fixpoint every row holds W = 2^max(K-6,0) words, one
// bit per guess column (row-major, rows of W consecutive words).
//
// The T_P step u = theta(M v) (Definition 5, Algorithm 1) is evaluated
// exactly: an AND row fires iff every entry of v it names is 1, an OR row iff
// at least one is. The fixpoint loop is the synchronous (Jacobi) iteration of
// Algorithms 1 and 2: every product reads v_t and writes a second buffer.
//
// Monotonicity: from the initial vector (facts) or initial matrix, v_t is a
// subset of v_{t+1}. The step therefore ORs its result into the buffer that
// holds v_{t-1}, a subset of the exact result, and the number of new bits is
// popcount(u & ~v); the fixpoint is reached when that count is 0.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lp_internal.h"

namespace lp {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

// ------------------------------------------------------------------ memory

static void *(*g_alloc)(size_t, void *, void *) = nullptr;
static void (*g_release)(void *, void *, void *) = nullptr;
static void *g_alloc_ctx = nullptr;

static lp_status hip_fail(hipError_t e, const char *what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return LP_E_DEVICE;
}

#define LP_HIP(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

static lp_status dev_alloc(void **p, size_t bytes, hipStream_t st) {
    *p = nullptr;
    if (bytes == 0) bytes = 8;
    if (g_alloc) {
        *p = g_alloc(bytes, (void *)st, g_alloc_ctx);
        if (!*p) {
            set_error("device allocation of " + std::to_string(bytes) + " bytes failed");
            return LP_E_NOMEM;
        }
        return LP_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        set_error("hipMalloc of " + std::to_string(bytes) + " bytes: out of memory");
        return LP_E_NOMEM;
    }
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    return LP_OK;
}

static void dev_free(void *p, hipStream_t st) {
    if (!p) return;
    if (g_release) g_release(p, (void *)st, g_alloc_ctx);
    else (void)hipFree(p);
}

// RAII list of device buffers of one call.
struct Scratch {
    hipStream_t st;
    std::vector<void *> ptrs;
    explicit Scratch(hipStream_t s) : st(s) {}
    template <class T>
    lp_status get(T **p, size_t count) {
        void *q;
        lp_status rc = dev_alloc(&q, count * sizeof(T), st);
        if (rc) return rc;
        ptrs.push_back(q);
        *p = (T *)q;
        return LP_OK;
    }
    ~Scratch() {
        if (!ptrs.empty()) (void)hipStreamSynchronize(st);
        for (void *p : ptrs) dev_free(p, st);
    }
};

// Small pinned host buffer per thread for change counters.
constexpr int kRing = 256;
static unsigned long long *pinned_ring() {
    static thread_local unsigned long long *p = nullptr;
    if (!p) {
        if (hipHostMalloc((void **)&p, sizeof(unsigned long long) * kRing, hipHostMallocDefault) != hipSuccess) {
            p = nullptr;
        }
    }
    return p;
}

// ------------------------------------------------------------------ kernels

constexpr int kBlock = 256;   // 4 waves of 64
constexpr int kWavesPerBlock = kBlock / 64;

struct StepParams {
    const int32_t *row_ptr;     // block CSR (long rows empty)
    const int32_t *col;
    const uint64_t *and_bits;   // AND-row bits (long rows cleared)
    const LongSeg *segs;
    const int32_t *long_col;
    uint32_t *and_cnt;          // [2][n_long_and]
    const uint64_t *v;
    uint64_t *u;
    unsigned long long *counters;  // ring of change counts, slot = product index & (kRing-1)
    int32_t n_rows;
    int32_t n_blocks;           // workgroups of the 64-row block part
    int32_t n_long_and;
    int32_t step;               // 1-based product index
    int32_t early_exit;         // 1: return at once if the previous product changed nothing
    int32_t n_segs;             // long-row segments
    int32_t lds_words;          // words of v staged in LDS (LDS-staged kernel)
};

__device__ inline uint64_t range_mask(int s, int t) {  // bits [s, t), 0 <= s < t <= 64
    const uint64_t hi = (t >= 64) ? ~0ull : ((1ull << t) - 1ull);
    return hi & ~((1ull << s) - 1ull);
}

__device__ inline uint32_t wave_sum(uint32_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// One full T_P step. Workgroups [0, n_blocks) each evaluate 4 blocks of 64
// consecutive rows, one wave per block: the wave streams the block's column
// indices 64 at a time (coalesced), gathers one bit of v per entry, and a
// ballot gives each row-owner lane the bits of its own entries in that chunk.
// Workgroups from n_blocks on each evaluate one segment of a long row.
__global__ __launch_bounds__(kBlock) void tp_step_kernel(StepParams p) {
    __shared__ uint32_t s_new;
    const int tid = threadIdx.x;
    if (blockIdx.x == 0 && tid == 0) p.counters[(p.step + 1) & (kRing - 1)] = 0;
    if (p.early_exit && p.step >= 2 && p.counters[(p.step - 1) & (kRing - 1)] == 0) return;
    if (tid == 0) s_new = 0;
    __syncthreads();
    uint32_t my_new = 0;
    if ((int)blockIdx.x < p.n_blocks) {
        const int lane = tid & 63;
        const int64_t word = (int64_t)blockIdx.x * kWavesPerBlock + (tid >> 6);
        const int64_t r0 = word * 64;
        if (r0 < p.n_rows) {
            const int64_t r = r0 + lane;
            const bool valid = r < p.n_rows;
            const int64_t rlast = r0 + 64 < p.n_rows ? r0 + 64 : p.n_rows;
            const int32_t e0 = p.row_ptr[r0];
            const int32_t e1 = p.row_ptr[rlast];
            const int32_t start = valid ? p.row_ptr[r] : e1;
            const int32_t end = valid ? p.row_ptr[r + 1] : e1;
            const uint64_t vw = p.v[word];
            const bool is_and = (p.and_bits[word] >> lane) & 1ull;
            bool acc = is_and;
            for (int32_t base = e0 & ~63; base < e1; base += 64) {
                const int32_t e = base + lane;
                bool b = false;
                if (e >= e0 && e < e1) {
                    const int32_t c = p.col[e];
                    b = (p.v[c >> 6] >> (c & 63)) & 1ull;
                }
                const uint64_t B = __ballot(b);
                const int s = start - base > 0 ? start - base : 0;
                const int t = end - base < 64 ? end - base : 64;
                if (s < t) {
                    const uint64_t m = range_mask(s, t);
                    acc = is_and ? (acc && ((B & m) == m)) : (acc || ((B & m) != 0));
                }
            }
            const uint64_t res = __ballot(acc && valid);
            if (lane == 0) {
                if (res) atomicOr((unsigned long long *)&p.u[word], (unsigned long long)res);
                my_new = (uint32_t)__popcll(res & ~vw);
            }
        }
    } else {
        const LongSeg sg = p.segs[blockIdx.x - p.n_blocks];
        int any = 0, all = 1;
        for (int32_t i = tid; i < sg.len; i += kBlock) {
            const int32_t c = p.long_col[sg.begin + i];
            const int b = (int)((p.v[c >> 6] >> (c & 63)) & 1ull);
            any |= b;
            all &= b;
        }
        any = __syncthreads_or(any);
        all = __syncthreads_and(all);
        if (tid == 0) {
            bool fire;
            if (!sg.is_and) {
                fire = any != 0;
            } else if (sg.nseg == 1) {
                fire = all != 0;
            } else {
                uint32_t *cnt = p.and_cnt + (size_t)(p.step & 1) * p.n_long_and + sg.and_slot;
                fire = all && atomicAdd(cnt, 1u) == (uint32_t)(sg.nseg - 1);
                if (sg.seg == 0)  // first segment clears the count of the next product
                    p.and_cnt[(size_t)((p.step + 1) & 1) * p.n_long_and + sg.and_slot] = 0;
            }
            if (fire) {
                const uint64_t bit = 1ull << (sg.row & 63);
                const uint64_t old = atomicOr((unsigned long long *)&p.u[sg.row >> 6], (unsigned long long)bit);
                if (!(old & bit) && !(p.v[sg.row >> 6] & bit)) my_new = 1;
            }
        }
    }
    my_new = wave_sum(my_new);
    if ((tid & 63) == 0 && my_new) atomicAdd(&s_new, my_new);
    __syncthreads();
    if (tid == 0 && s_new) atomicAdd(&p.counters[p.step & (kRing - 1)], (unsigned long long)s_new);
}

constexpr int kLdsBlock = 1024;            // 16 waves: one workgroup per CU
constexpr int kLdsWaves = kLdsBlock / 64;
constexpr int kUnroll = 8;                  // column chunks in flight per wave

// Same step as tp_step_kernel, for a grid of one workgroup per CU. Each
// workgroup first copies the leading lds_words words of v (the original
// atoms, which are the only atoms rule bodies name) into LDS, so the random
// one-bit gathers of AND rows hit LDS instead of pulling a cache line from L2
// per entry. Waves then take 64-row blocks in a grid-stride loop, issuing
// kUnroll coalesced column-chunk loads before consuming any of them. Long-row
// segments follow, one wave per segment.
// Blocks and long-row segments of one step, with the leading lds_words words
// of v already in s_v. Returns this thread's count of new bits (nonzero only
// on lane 0 of a wave).
__device__ __forceinline__ uint32_t lds_step_body(const StepParams &p, const uint64_t *s_v) {
    const int tid = threadIdx.x;
    const int32_t lw = p.lds_words;
    const int32_t lds_bits = lw * 64;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t n_words = ((int64_t)p.n_rows + 63) >> 6;
    const int64_t wstride = (int64_t)gridDim.x * kLdsWaves;
    uint32_t my_new = 0;
    for (int64_t word = (int64_t)blockIdx.x * kLdsWaves + wave; word < n_words; word += wstride) {
        const int64_t r0 = word * 64;
        const int64_t r = r0 + lane;
        const bool valid = r < p.n_rows;
        const int64_t rlast = r0 + 64 < p.n_rows ? r0 + 64 : p.n_rows;
        const int32_t e1 = p.row_ptr[rlast];
        const int32_t start = valid ? p.row_ptr[r] : e1;
        const int32_t end = valid ? p.row_ptr[r + 1] : e1;
        const int32_t e0 = __builtin_amdgcn_readfirstlane(start);
        const uint64_t vw = word < lw ? s_v[word] : p.v[word];
        const bool is_and = (p.and_bits[word] >> lane) & 1ull;
        bool acc = is_and;
        for (int32_t base = e0 & ~63; base < e1; base += 64 * kUnroll) {
            int32_t c[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int32_t e = base + 64 * u + lane;
                c[u] = (e >= e0 && e < e1) ? p.col[e] : -1;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                bool b = false;
                if (c[u] >= 0) {
                    const uint64_t w = c[u] < lds_bits ? s_v[c[u] >> 6] : p.v[c[u] >> 6];
                    b = (w >> (c[u] & 63)) & 1ull;
                }
                const uint64_t B = __ballot(b);
                const int32_t cb = base + 64 * u;
                const int s = start - cb > 0 ? start - cb : 0;
                const int t = end - cb < 64 ? end - cb : 64;
                if (s < t) {
                    const uint64_t m = range_mask(s, t);
                    acc = is_and ? (acc && ((B & m) == m)) : (acc || ((B & m) != 0));
                }
            }
        }
        const uint64_t res = __ballot(acc && valid);
        if (lane == 0) {
            if (res) atomicOr((unsigned long long *)&p.u[word], (unsigned long long)res);
            my_new += (uint32_t)__popcll(res & ~vw);
        }
    }
    for (int64_t si = (int64_t)blockIdx.x * kLdsWaves + wave; si < p.n_segs; si += wstride) {
        const LongSeg sg = p.segs[si];
        bool any = false, all = true;
        for (int32_t i0 = 0; i0 < sg.len; i0 += 64 * kUnroll) {
            int32_t c[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int32_t i = i0 + 64 * u + lane;
                c[u] = i < sg.len ? p.long_col[sg.begin + i] : -1;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                if (c[u] >= 0) {
                    const uint64_t w = c[u] < lds_bits ? s_v[c[u] >> 6] : p.v[c[u] >> 6];
                    const bool b = (w >> (c[u] & 63)) & 1ull;
                    any |= b;
                    all &= b;
                }
            }
        }
        any = __ballot(any) != 0;
        all = __ballot(!all) == 0;
        if (lane == 0) {
            bool fire;
            if (!sg.is_and) {
                fire = any;
            } else if (sg.nseg == 1) {
                fire = all;
            } else {
                uint32_t *cnt = p.and_cnt + (size_t)(p.step & 1) * p.n_long_and + sg.and_slot;
                fire = all && atomicAdd(cnt, 1u) == (uint32_t)(sg.nseg - 1);
                if (sg.seg == 0) p.and_cnt[(size_t)((p.step + 1) & 1) * p.n_long_and + sg.and_slot] = 0;
            }
            if (fire) {
                const uint64_t bit = 1ull << (sg.row & 63);
                const uint64_t old = atomicOr((unsigned long long *)&p.u[sg.row >> 6], (unsigned long long)bit);
                if (!(old & bit) && !(p.v[sg.row >> 6] & bit)) my_new += 1;
            }
        }
    }
    return my_new;
}

// Adds this workgroup's count of new bits to the product's counter.
__device__ __forceinline__ void add_new_bits(uint32_t my_new, uint32_t *s_new, unsigned long long *slot) {
    my_new = wave_sum(my_new);
    if ((threadIdx.x & 63) == 0 && my_new) atomicAdd(s_new, my_new);
    __syncthreads();
    if (threadIdx.x == 0 && *s_new) atomicAdd(slot, (unsigned long long)*s_new);
}

__global__ __launch_bounds__(kLdsBlock) void tp_step_lds_kernel(StepParams p) {
    extern __shared__ uint64_t s_v[];
    __shared__ uint32_t s_new;
    const int tid = threadIdx.x;
    if (blockIdx.x == 0 && tid == 0) p.counters[(p.step + 1) & (kRing - 1)] = 0;
    if (p.early_exit && p.step >= 2 && p.counters[(p.step - 1) & (kRing - 1)] == 0) return;
    if (tid == 0) s_new = 0;
    for (int32_t i = tid; i < p.lds_words; i += kLdsBlock) s_v[i] = p.v[i];
    __syncthreads();
    const uint32_t my_new = lds_step_body(p, s_v);
    add_new_bits(my_new, &s_new, &p.counters[p.step & (kRing - 1)]);
}

struct PersistParams {
    StepParams p;
    uint64_t *buf0;
    uint64_t *buf1;
    unsigned int *bar;   // [0] arrivals, [1] generation
    int32_t max_steps;
    int32_t *result;     // products, or -1 if max_steps was reached
};

// Grid-wide barrier for a cooperative launch (every workgroup resident).
// Release before arriving, acquire after leaving: the next product reads the
// buffer other XCDs just wrote.
__device__ __forceinline__ void grid_barrier(unsigned int *bar, unsigned int n_groups) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned int arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == n_groups - 1) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen)
                __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// The whole Algorithm 1 loop in one launch. Each product: stage v in LDS,
// evaluate every row, add the new-bit count, grid barrier, read the count.
// Every workgroup reads the same count after the barrier, so all leave the
// loop on the same product; max_steps (n_rows + 1 bounds a monotone
// iteration) guarantees the loop ends.
__global__ __launch_bounds__(kLdsBlock) void tp_fixpoint_persistent_kernel(PersistParams q) {
    extern __shared__ uint64_t s_v[];
    __shared__ uint32_t s_new;
    StepParams p = q.p;
    const int tid = threadIdx.x;
    for (int32_t step = 1;; ++step) {
        p.step = step;
        p.v = (step & 1) ? q.buf0 : q.buf1;
        p.u = (step & 1) ? q.buf1 : q.buf0;
        unsigned long long *slot = &p.counters[step & (kRing - 1)];
        if (blockIdx.x == 0 && tid == 0) p.counters[(step + 1) & (kRing - 1)] = 0;
        if (tid == 0) s_new = 0;
        for (int32_t i = tid; i < p.lds_words; i += kLdsBlock) s_v[i] = p.v[i];
        __syncthreads();
        const uint32_t my_new = lds_step_body(p, s_v);
        add_new_bits(my_new, &s_new, slot);
        grid_barrier(q.bar, gridDim.x);
        const unsigned long long changed = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (changed == 0 || step >= q.max_steps) {
            if (blockIdx.x == 0 && tid == 0) *q.result = changed == 0 ? step : -1;
            return;
        }
    }
}

struct SpmmParams {
    const int32_t *row_ptr;
    const int32_t *col;
    const uint64_t *and_bits;
    const uint64_t *V;
    uint64_t *U;
    unsigned long long *counters;
    int64_t total;       // n_rows << log2W
    int32_t log2W;
    int32_t step;
    int32_t early_exit;
};

// Interpretation-matrix step U = theta(M_P V) (Algorithm 2). Thread g owns
// word (g & (W-1)) of row (g >> log2W): it ANDs (AND row) or ORs (OR row) the
// same word of every row its row names. With W >= 64 a wave covers 64
// consecutive words of one row, so every gather is one coalesced 512-byte read.
template <bool WIDE>
__global__ __launch_bounds__(kBlock) void spmm_step_kernel(SpmmParams p) {
    __shared__ uint32_t s_new;
    const int tid = threadIdx.x;
    if (blockIdx.x == 0 && tid == 0) p.counters[(p.step + 1) & (kRing - 1)] = 0;
    if (p.early_exit && p.step >= 2 && p.counters[(p.step - 1) & (kRing - 1)] == 0) return;
    if (tid == 0) s_new = 0;
    __syncthreads();
    uint32_t my_new = 0;
    const int64_t g = (int64_t)blockIdx.x * kBlock + tid;
    if (g < p.total) {
        int32_t row = (int32_t)(g >> p.log2W);
        if (WIDE) row = __builtin_amdgcn_readfirstlane(row);
        const int64_t w = g & ((1ll << p.log2W) - 1);
        const int32_t s = p.row_ptr[row], e = p.row_ptr[row + 1];
        const bool is_and = (p.and_bits[row >> 6] >> (row & 63)) & 1ull;
        uint64_t acc = is_and ? ~0ull : 0ull;
        for (int32_t i = s; i < e; ++i) {
            const int64_t c = p.col[i];
            const uint64_t x = p.V[(c << p.log2W) + w];
            acc = is_and ? (acc & x) : (acc | x);
        }
        if (s == e) acc = 0;
        const int64_t idx = ((int64_t)row << p.log2W) + w;
        my_new = (uint32_t)__popcll(acc & ~p.V[idx]);
        p.U[idx] = acc;
    }
    my_new = wave_sum(my_new);
    if ((tid & 63) == 0 && my_new) atomicAdd(&s_new, my_new);
    __syncthreads();
    if (tid == 0 && s_new) atomicAdd(&p.counters[p.step & (kRing - 1)], (unsigned long long)s_new);
}

// Initial matrix (Definition 8). Column j of the compressed guess space: bit
// pos of j is the value of the qbar row whose guess sits at bit pos. Fact
// rows are all ones; qbar rows with a pruned guess and all other rows are 0.
__global__ __launch_bounds__(kBlock) void init_m0_kernel(uint64_t *V, uint64_t *U, int64_t total, int32_t log2W,
                                                         int32_t n_std, const uint64_t *fact_bits,
                                                         const int32_t *guess_pos, int32_t k_eff) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= total) return;
    const int32_t row = (int32_t)(g >> log2W);
    const int64_t w = g & ((1ll << log2W) - 1);
    const uint64_t valid = k_eff >= 6 ? ~0ull : ((1ull << (1 << k_eff)) - 1ull);
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

// Algorithm 3: column j is accepted iff for every negated atom q_t exactly
// one of row q_t and row qbar_t is 1 (a_l + a_j = 1), i.e. their XOR is 1.
__global__ __launch_bounds__(kBlock) void stable_check_kernel(const uint64_t *V, int32_t log2W, int64_t W,
                                                              const int32_t *q_rows, int32_t n_std, int32_t K,
                                                              int32_t k_eff, uint64_t *accept,
                                                              unsigned long long *count) {
    const int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    uint32_t c = 0;
    if (w < W) {
        uint64_t ok = k_eff >= 6 ? ~0ull : ((1ull << (1 << k_eff)) - 1ull);
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

// ------------------------------------------------------------------ upload

static int64_t n_words_of(int64_t rows) { return (rows + 63) / 64; }

static std::vector<uint64_t> pack_bits(const std::vector<uint8_t> &x, int64_t words) {
    std::vector<uint64_t> w(words ? words : 1, 0);
    for (size_t i = 0; i < x.size(); ++i)
        if (x[i]) w[i >> 6] |= 1ull << (i & 63);
    return w;
}

template <class T>
static lp_status upload(T **d, const T *h, size_t count, hipStream_t st, int64_t *bytes) {
    lp_status rc = dev_alloc((void **)d, count * sizeof(T), st);
    if (rc) return rc;
    *bytes += (int64_t)(count * sizeof(T));
    if (count) LP_HIP(hipMemcpyAsync(*d, h, count * sizeof(T), hipMemcpyHostToDevice, st));
    return LP_OK;
}

static void free_device(Matrix &m, hipStream_t st) {
    DeviceMatrix &d = m.dev;
    void *ps[] = {d.row_ptr, d.col, d.and_bits, d.fact_bits, d.segs, d.long_col,
                  d.full_row_ptr, d.full_col, d.q_rows, d.guess_pos};
    for (void *p : ps) dev_free(p, st);
    d = DeviceMatrix{};
}

static lp_status upload_matrix(Matrix &m, hipStream_t st) {
    DeviceMatrix &d = m.dev;
    LP_HIP(hipGetDevice(&d.device));
    const int64_t W = n_words_of(m.n_rows);
    std::vector<uint64_t> fact = pack_bits(m.fact, W);
    lp_status rc;
    if ((rc = upload(&d.fact_bits, fact.data(), fact.size(), st, &d.bytes))) return rc;
    if (m.K == 0) {
        // block CSR with long rows emptied, long rows split in segments
        std::vector<int32_t> rp(m.n_rows + 1);
        std::vector<int32_t> col;
        std::vector<int32_t> lcol;
        std::vector<LongSeg> segs;
        std::vector<uint8_t> kind_short(m.kind);
        col.reserve(m.col.size());
        int32_t n_long_and = 0;
        for (int32_t i = 0; i < m.n_rows; ++i) {
            rp[i] = (int32_t)col.size();
            const int32_t s = m.row_ptr[i], e = m.row_ptr[i + 1], len = e - s;
            if (len > kLongRow) {
                kind_short[i] = 0;
                const int32_t nseg = (len + kSegLen - 1) / kSegLen;
                const int32_t slot = (m.kind[i] && nseg > 1) ? n_long_and++ : -1;
                for (int32_t q = 0; q < nseg; ++q) {
                    LongSeg sg{};
                    sg.row = i;
                    sg.is_and = m.kind[i];
                    sg.begin = (int64_t)lcol.size() + (int64_t)q * kSegLen;
                    sg.len = std::min(kSegLen, len - q * kSegLen);
                    sg.nseg = nseg;
                    sg.and_slot = slot;
                    sg.seg = q;
                    segs.push_back(sg);
                }
                lcol.insert(lcol.end(), m.col.begin() + s, m.col.begin() + e);
            } else {
                col.insert(col.end(), m.col.begin() + s, m.col.begin() + e);
            }
        }
        rp[m.n_rows] = (int32_t)col.size();
        std::vector<uint64_t> andb = pack_bits(kind_short, W);
        d.short_nnz = (int64_t)col.size();
        d.long_nnz = (int64_t)lcol.size();
        d.n_segs = (int32_t)segs.size();
        d.n_long_and = n_long_and;
        if ((rc = upload(&d.row_ptr, rp.data(), rp.size(), st, &d.bytes))) return rc;
        if ((rc = upload(&d.col, col.data(), col.size(), st, &d.bytes))) return rc;
        if ((rc = upload(&d.and_bits, andb.data(), andb.size(), st, &d.bytes))) return rc;
        if ((rc = upload((LongSeg **)&d.segs, segs.data(), segs.size(), st, &d.bytes))) return rc;
        if ((rc = upload(&d.long_col, lcol.data(), lcol.size(), st, &d.bytes))) return rc;
    } else {
        std::vector<uint64_t> andb = pack_bits(m.kind, W);
        std::vector<int32_t> qrows(m.neg_atoms);
        if ((rc = upload(&d.full_row_ptr, m.row_ptr.data(), m.row_ptr.size(), st, &d.bytes))) return rc;
        if ((rc = upload(&d.full_col, m.col.data(), m.col.size(), st, &d.bytes))) return rc;
        if ((rc = upload(&d.and_bits, andb.data(), andb.size(), st, &d.bytes))) return rc;
        if ((rc = upload(&d.q_rows, qrows.data(), qrows.size(), st, &d.bytes))) return rc;
        if ((rc = upload(&d.guess_pos, m.guess_pos.data(), m.guess_pos.size(), st, &d.bytes))) return rc;
    }
    LP_HIP(hipStreamSynchronize(st));
    m.info.device_bytes = d.bytes;
    return LP_OK;
}

// ------------------------------------------------------------------ drivers

struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    explicit DeviceGuard(int dev) {
        if (dev >= 0 && hipGetDevice(&prev) == hipSuccess && prev != dev) {
            changed = hipSetDevice(dev) == hipSuccess;
        }
    }
    ~DeviceGuard() {
        if (changed) (void)hipSetDevice(prev);
    }
};

struct DevProps {
    int n_cu = 0;
    int max_lds = 0;
};

static lp_status dev_props(int dev, DevProps *out) {
    static std::mutex mu;
    static DevProps cache[64];
    std::lock_guard<std::mutex> lock(mu);
    if (dev < 0 || dev >= 64) {
        set_error("device id out of range");
        return LP_E_DEVICE;
    }
    if (cache[dev].n_cu == 0) {
        DevProps d;
        LP_HIP(hipDeviceGetAttribute(&d.n_cu, hipDeviceAttributeMultiprocessorCount, dev));
        LP_HIP(hipDeviceGetAttribute(&d.max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        const int dyn = d.max_lds - 256;
        if (dyn > 0) {
            (void)hipFuncSetAttribute((const void *)tp_step_lds_kernel,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
            (void)hipFuncSetAttribute((const void *)tp_fixpoint_persistent_kernel,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
        }
        (void)hipGetLastError();
        cache[dev] = d;
    }
    *out = cache[dev];
    return LP_OK;
}

// Launch configuration of one T_P step, fixed for a whole solve.
struct StepLaunch {
    int variant = LP_STEP_LDS;
    int grid = 0;
    size_t lds_bytes = 0;
};

static lp_status plan_step(const Matrix &m, const lp_schedule *sched, StepParams &p, StepLaunch *L) {
    int variant = sched ? sched->variant : LP_STEP_AUTO;
    if (variant == LP_STEP_AUTO) variant = LP_STEP_LDS;
    L->variant = variant;
    const int64_t n_words = n_words_of(m.n_rows);
    if (variant == LP_STEP_GLOBAL) {
        L->grid = p.n_blocks + p.n_segs;
        L->lds_bytes = 0;
        p.lds_words = 0;
        return LP_OK;
    }
    if (variant != LP_STEP_LDS) {
        set_error("unknown step variant");
        return LP_E_INVAL;
    }
    DevProps d;
    lp_status rc = dev_props(m.dev.device, &d);
    if (rc) return rc;
    const int64_t cap = std::max<int64_t>(0, (d.max_lds - 256) / 8);
    p.lds_words = (int32_t)std::min<int64_t>({cap, n_words_of(m.n_atoms), n_words});
    L->lds_bytes = (size_t)p.lds_words * 8;
    const int64_t want = (n_words + p.n_segs + kLdsWaves - 1) / kLdsWaves;
    int grid = sched && sched->grid > 0 ? sched->grid : d.n_cu;
    L->grid = (int)std::max<int64_t>(1, std::min<int64_t>(grid, want));
    return LP_OK;
}

static void launch_step(const StepLaunch &L, const StepParams &p, hipStream_t st) {
    if (L.variant == LP_STEP_GLOBAL)
        tp_step_kernel<<<L.grid, kBlock, 0, st>>>(p);
    else
        tp_step_lds_kernel<<<L.grid, kLdsBlock, L.lds_bytes, st>>>(p);
}

static StepParams step_params(const Matrix &m) {
    const DeviceMatrix &d = m.dev;
    StepParams p{};
    p.row_ptr = d.row_ptr;
    p.col = d.col;
    p.and_bits = d.and_bits;
    p.segs = (const LongSeg *)d.segs;
    p.long_col = d.long_col;
    p.n_rows = m.n_rows;
    p.n_blocks = (int32_t)((n_words_of(m.n_rows) + kWavesPerBlock - 1) / kWavesPerBlock);
    p.n_long_and = d.n_long_and;
    p.n_segs = d.n_segs;
    p.early_exit = 1;
    return p;
}

// Launch plan of the persistent fixpoint: the LDS-staged step, at most as
// many workgroups as can be resident at once (the grid barrier needs all of
// them running). *grid = 0 if not even one fits.
static lp_status plan_persistent(const Matrix &m, const lp_schedule *sched, StepParams &p, StepLaunch *L,
                                 int *grid) {
    lp_schedule s2 = sched ? *sched : lp_schedule{};
    s2.variant = LP_STEP_LDS;
    lp_status rc = plan_step(m, &s2, p, L);
    if (rc) return rc;
    int per_cu = 0;
    LP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, tp_fixpoint_persistent_kernel, kLdsBlock,
                                                        L->lds_bytes));
    DevProps d;
    if ((rc = dev_props(m.dev.device, &d))) return rc;
    const int64_t resident = (int64_t)per_cu * d.n_cu;
    *grid = (int)std::min<int64_t>(L->grid, resident);
    return LP_OK;
}

static lp_status launch_persistent(const Matrix &m, const StepParams &p, const StepLaunch &L, int grid,
                                   uint64_t *const buf[2], unsigned int *bar, int32_t *res, hipStream_t st) {
    PersistParams q{};
    q.p = p;
    q.buf0 = buf[0];
    q.buf1 = buf[1];
    q.bar = bar;
    q.max_steps = (int32_t)std::min<int64_t>((int64_t)m.n_rows + 1, INT32_MAX - 1);
    q.result = res;
    void *args[] = {&q};
    LP_HIP(hipLaunchCooperativeKernel((const void *)tp_fixpoint_persistent_kernel, dim3(grid), dim3(kLdsBlock),
                                      args, (unsigned int)L.lds_bytes, st));
    return LP_OK;
}

// Least-model fixpoint. On success *out points at the device buffer holding
// the fixpoint (one of bufs[0..1]).
static lp_status least_fixpoint(const Matrix &m, const lp_schedule *sched, hipStream_t st, Scratch &S,
                                uint64_t **out, int32_t *products) {
    const int64_t W = n_words_of(m.n_rows);
    uint64_t *buf[2];
    unsigned long long *counters;
    uint32_t *and_cnt;
    lp_status rc;
    if ((rc = S.get(&buf[0], W)) || (rc = S.get(&buf[1], W)) || (rc = S.get(&counters, kRing)) ||
        (rc = S.get(&and_cnt, 2 * (size_t)m.dev.n_long_and)))
        return rc;
    LP_HIP(hipMemsetAsync(counters, 0, sizeof(unsigned long long) * kRing, st));
    if (m.dev.n_long_and) LP_HIP(hipMemsetAsync(and_cnt, 0, sizeof(uint32_t) * 2 * m.dev.n_long_and, st));
    LP_HIP(hipMemcpyAsync(buf[0], m.dev.fact_bits, W * 8, hipMemcpyDeviceToDevice, st));
    LP_HIP(hipMemcpyAsync(buf[1], m.dev.fact_bits, W * 8, hipMemcpyDeviceToDevice, st));
    if (m.n_rows == 0) {
        *out = buf[0];
        *products = 1;
        return LP_OK;
    }
    int driver = sched ? sched->driver : LP_DRIVER_AUTO;
    StepParams p = step_params(m);
    p.counters = counters;
    p.and_cnt = and_cnt;
    StepLaunch L;
    if (driver == LP_DRIVER_PERSISTENT || driver == LP_DRIVER_AUTO) {
        int grid = 0;
        if ((rc = plan_persistent(m, sched, p, &L, &grid))) return rc;
        if (grid >= 1) {
            unsigned int *bar;
            int32_t *res;
            if ((rc = S.get(&bar, 2)) || (rc = S.get(&res, 1))) return rc;
            LP_HIP(hipMemsetAsync(bar, 0, sizeof(unsigned int) * 2, st));
            if ((rc = launch_persistent(m, p, L, grid, buf, bar, res, st))) return rc;
            int32_t prods = 0;
            LP_HIP(hipMemcpyAsync(&prods, res, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            LP_HIP(hipStreamSynchronize(st));
            if (prods < 1) {
                set_error("fixpoint not reached within n_rows+1 products");
                return LP_E_INTERNAL;
            }
            *products = prods;
            *out = buf[prods & 1];
            return LP_OK;
        }
        if (driver == LP_DRIVER_PERSISTENT) {
            set_error("the persistent step does not fit on this device");
            return LP_E_DEVICE;
        }
    }
    int batch = 1;
    if (driver == LP_DRIVER_BATCHED || driver == LP_DRIVER_AUTO) {
        batch = (sched && sched->steps_per_sync > 0) ? sched->steps_per_sync : 32;
    }
    batch = std::max(1, std::min(batch, kRing / 2 - 1));
    if ((rc = plan_step(m, sched, p, &L))) return rc;
    unsigned long long *h = pinned_ring();
    if (!h) {
        set_error("pinned host allocation failed");
        return LP_E_NOMEM;
    }
    const int64_t limit = (int64_t)m.n_rows + 1;
    for (int64_t t = 0;; t += batch) {
        for (int i = 1; i <= batch; ++i) {
            p.step = (int32_t)(t + i);
            p.v = buf[(p.step - 1) & 1];
            p.u = buf[p.step & 1];
            launch_step(L, p, st);
        }
        LP_HIP(hipGetLastError());
        LP_HIP(hipMemcpyAsync(h, counters, sizeof(unsigned long long) * kRing, hipMemcpyDeviceToHost, st));
        LP_HIP(hipStreamSynchronize(st));
        for (int i = 1; i <= batch; ++i) {
            const int64_t s = t + i;
            if (h[s & (kRing - 1)] == 0) {
                *products = (int32_t)s;
                *out = buf[s & 1];
                return LP_OK;
            }
        }
        if (t + batch > limit) {
            set_error("fixpoint not reached within n_rows+1 products");
            return LP_E_INTERNAL;
        }
    }
}

static void unpack_model(const uint64_t *bits, int32_t n, uint8_t *model) {
    for (int32_t a = 0; a < n; ++a) model[a] = (uint8_t)((bits[a >> 6] >> (a & 63)) & 1ull);
}

static lp_status least_model_impl(const Matrix &m, uint8_t *model, int32_t *products, const lp_schedule *sched,
                                  hipStream_t st) {
    Scratch S(st);
    uint64_t *fix = nullptr;
    int32_t prods = 0;
    lp_status rc = least_fixpoint(m, sched, st, S, &fix, &prods);
    if (rc) return rc;
    const int64_t Wn = n_words_of(m.n_atoms);
    std::vector<uint64_t> hb(Wn ? Wn : 1);
    if (Wn) LP_HIP(hipMemcpyAsync(hb.data(), fix, Wn * 8, hipMemcpyDeviceToHost, st));
    LP_HIP(hipStreamSynchronize(st));
    unpack_model(hb.data(), m.n_atoms, model);
    if (products) *products = prods;
    return LP_OK;
}

static int ilog2(int64_t x) {
    int l = 0;
    while ((1ll << l) < x) ++l;
    return l;
}

static lp_status stable_impl(const Matrix &m, uint64_t *accepted, int64_t *n_models, uint8_t *models,
                             int64_t max_models, uint64_t *interp, int32_t *products, hipStream_t st) {
    const int K = m.K;
    const int64_t H_full = 1ll << K;
    const int64_t W_full = (H_full + 63) / 64;
    if (K == 0) {
        // definite program: exactly one stable model, the least model
        std::vector<uint8_t> lm(m.n_atoms ? m.n_atoms : 1);
        lp_status rc = least_model_impl(m, lm.data(), products, nullptr, st);
        if (rc) return rc;
        accepted[0] = 1;
        *n_models = 1;
        if (models && max_models >= 1) std::memcpy(models, lm.data(), m.n_atoms);
        if (interp)
            for (int32_t a = 0; a < m.n_atoms; ++a) interp[a] = lm[a];
        if (models && max_models < 1) return LP_E_TRUNCATED;
        return LP_OK;
    }
    if (interp && m.K_eff != K) {
        set_error("interp output needs a matrix built without LP_PRUNE_FACT_GUESSES");
        return LP_E_INVAL;
    }
    const int keff = m.K_eff;
    const int64_t H = 1ll << keff;
    const int64_t W = (H + 63) / 64;
    const int log2W = ilog2(W);
    const int64_t total = (int64_t)m.n_rows * W;
    // memory check before any launch
    size_t free_b = 0, total_b = 0;
    LP_HIP(hipMemGetInfo(&free_b, &total_b));
    const double need = 2.0 * (double)total * 8.0 + (double)W * 8.0 + 4096.0;
    if (need > (double)free_b) {
        set_error("stable models need " + std::to_string((long long)need) + " bytes of device memory, " +
                  std::to_string((long long)free_b) + " free");
        return LP_E_NOMEM;
    }
    Scratch S(st);
    uint64_t *buf[2];
    uint64_t *acc_d;
    unsigned long long *counters;
    lp_status rc;
    if ((rc = S.get(&buf[0], total)) || (rc = S.get(&buf[1], total)) || (rc = S.get(&acc_d, W)) ||
        (rc = S.get(&counters, kRing)))
        return rc;
    LP_HIP(hipMemsetAsync(counters, 0, sizeof(unsigned long long) * kRing, st));
    const int64_t blocks = (total + kBlock - 1) / kBlock;
    init_m0_kernel<<<(unsigned)blocks, kBlock, 0, st>>>(buf[0], buf[1], total, log2W, m.n_std, m.dev.fact_bits,
                                                      m.dev.guess_pos, keff);
    LP_HIP(hipGetLastError());
    SpmmParams p{};
    p.row_ptr = m.dev.full_row_ptr;
    p.col = m.dev.full_col;
    p.and_bits = m.dev.and_bits;
    p.counters = counters;
    p.total = total;
    p.log2W = log2W;
    p.early_exit = 1;
    unsigned long long *h = pinned_ring();
    if (!h) {
        set_error("pinned host allocation failed");
        return LP_E_NOMEM;
    }
    const int batch = 8;
    int32_t prods = -1;
    uint64_t *fix = nullptr;
    const int64_t limit = (int64_t)m.n_rows + 1;
    for (int64_t t = 0; prods < 0; t += batch) {
        for (int i = 1; i <= batch; ++i) {
            p.step = (int32_t)(t + i);
            p.V = buf[(p.step - 1) & 1];
            p.U = buf[p.step & 1];
            if (log2W >= 6) spmm_step_kernel<true><<<(unsigned)blocks, kBlock, 0, st>>>(p);
            else spmm_step_kernel<false><<<(unsigned)blocks, kBlock, 0, st>>>(p);
        }
        LP_HIP(hipGetLastError());
        LP_HIP(hipMemcpyAsync(h, counters, sizeof(unsigned long long) * kRing, hipMemcpyDeviceToHost, st));
        LP_HIP(hipStreamSynchronize(st));
        for (int i = 1; i <= batch; ++i) {
            const int64_t s = t + i;
            if (h[s & (kRing - 1)] == 0) {
                prods = (int32_t)s;
                fix = buf[s & 1];
                break;
            }
        }
        if (prods < 0 && t + batch > limit) {
            set_error("fixpoint not reached within n_rows+1 products");
            return LP_E_INTERNAL;
        }
    }
    // Algorithm 3
    unsigned long long *cnt_d = counters;  // slot 0 is free once the loop is done
    LP_HIP(hipMemsetAsync(cnt_d, 0, sizeof(unsigned long long), st));
    stable_check_kernel<<<(unsigned)((W + kBlock - 1) / kBlock), kBlock, 0, st>>>(
        fix, log2W, W, m.dev.q_rows, m.n_std, K, keff, acc_d, cnt_d);
    LP_HIP(hipGetLastError());
    std::vector<uint64_t> acc_h(W);
    unsigned long long nm = 0;
    LP_HIP(hipMemcpyAsync(acc_h.data(), acc_d, W * 8, hipMemcpyDeviceToHost, st));
    LP_HIP(hipMemcpyAsync(&nm, cnt_d, 8, hipMemcpyDeviceToHost, st));
    LP_HIP(hipStreamSynchronize(st));
    // accepted guesses in the full guess space (deposit compressed bits)
    std::memset(accepted, 0, sizeof(uint64_t) * W_full);
    std::vector<int64_t> cols;
    for (int64_t w = 0; w < W; ++w) {
        uint64_t x = acc_h[w];
        while (x) {
            const int b = __builtin_ctzll(x);
            x &= x - 1;
            const int64_t jc = w * 64 + b;
            int64_t jf = 0;
            for (int t = 0; t < K; ++t)
                if (m.guess_pos[t] >= 0 && ((jc >> m.guess_pos[t]) & 1)) jf |= 1ll << t;
            accepted[jf >> 6] |= 1ull << (jf & 63);
            if (models && (int64_t)cols.size() < max_models) cols.push_back(jc);
        }
    }
    *n_models = (int64_t)nm;
    if (interp && m.n_atoms) {
        LP_HIP(hipMemcpyAsync(interp, fix, sizeof(uint64_t) * (size_t)m.n_atoms * W, hipMemcpyDeviceToHost, st));
    }
    if (models && !cols.empty() && m.n_atoms) {
        int64_t *cols_d;
        uint8_t *out_d;
        const int64_t nb = (int64_t)cols.size() * m.n_atoms;
        if ((rc = S.get(&cols_d, cols.size())) || (rc = S.get(&out_d, nb))) return rc;
        LP_HIP(hipMemcpyAsync(cols_d, cols.data(), cols.size() * 8, hipMemcpyHostToDevice, st));
        extract_kernel<<<(unsigned)((nb + kBlock - 1) / kBlock), kBlock, 0, st>>>(fix, log2W, cols_d,
                                                                                 (int64_t)cols.size(),
                                                                                 m.n_atoms, out_d);
        LP_HIP(hipGetLastError());
        LP_HIP(hipMemcpyAsync(models, out_d, nb, hipMemcpyDeviceToHost, st));
    }
    LP_HIP(hipStreamSynchronize(st));
    if (products) *products = prods;
    if (models && (int64_t)nm > max_models) return LP_E_TRUNCATED;
    return LP_OK;
}

static lp_status bench_step_impl(const Matrix &m, const lp_schedule *sched, int32_t reps, float *avg_ms,
                               hipStream_t st) {
    Scratch S(st);
    uint64_t *fix = nullptr;
    int32_t prods = 0;
    lp_status rc = least_fixpoint(m, sched, st, S, &fix, &prods);
    if (rc) return rc;
    const int64_t W = n_words_of(m.n_rows);
    uint64_t *dst;
    unsigned long long *counters;
    uint32_t *and_cnt;
    if ((rc = S.get(&dst, W)) || (rc = S.get(&counters, kRing)) ||
        (rc = S.get(&and_cnt, 2 * (size_t)m.dev.n_long_and)))
        return rc;
    StepParams p = step_params(m);
    p.counters = counters;
    p.and_cnt = and_cnt;
    StepLaunch L;
    hipEvent_t e0, e1;
    LP_HIP(hipEventCreate(&e0));
    LP_HIP(hipEventCreate(&e1));
    float total = 0.f;
    if (sched && sched->driver == LP_DRIVER_PERSISTENT) {
        // each launch runs the whole fixpoint from the initial vector
        int grid = 0;
        if ((rc = plan_persistent(m, sched, p, &L, &grid))) return rc;
        if (grid < 1) {
            set_error("the persistent step does not fit on this device");
            return LP_E_DEVICE;
        }
        uint64_t *buf[2] = {fix, dst};
        unsigned int *bar;
        int32_t *res;
        if ((rc = S.get(&bar, 2)) || (rc = S.get(&res, 1))) return rc;
        for (int i = 0; i < reps; ++i) {
            LP_HIP(hipMemcpyAsync(buf[0], m.dev.fact_bits, W * 8, hipMemcpyDeviceToDevice, st));
            LP_HIP(hipMemcpyAsync(buf[1], m.dev.fact_bits, W * 8, hipMemcpyDeviceToDevice, st));
            LP_HIP(hipMemsetAsync(counters, 0, sizeof(unsigned long long) * kRing, st));
            if (m.dev.n_long_and)
                LP_HIP(hipMemsetAsync(and_cnt, 0, sizeof(uint32_t) * 2 * m.dev.n_long_and, st));
            LP_HIP(hipMemsetAsync(bar, 0, sizeof(unsigned int) * 2, st));
            LP_HIP(hipEventRecord(e0, st));
            if ((rc = launch_persistent(m, p, L, grid, buf, bar, res, st))) return rc;
            LP_HIP(hipEventRecord(e1, st));
            LP_HIP(hipEventSynchronize(e1));
            float ms = 0;
            LP_HIP(hipEventElapsedTime(&ms, e0, e1));
            total += ms;
        }
    } else {
        LP_HIP(hipMemcpyAsync(dst, fix, W * 8, hipMemcpyDeviceToDevice, st));
        LP_HIP(hipMemsetAsync(counters, 0, sizeof(unsigned long long) * kRing, st));
        if (m.dev.n_long_and) LP_HIP(hipMemsetAsync(and_cnt, 0, sizeof(uint32_t) * 2 * m.dev.n_long_and, st));
        p.early_exit = 0;
        p.v = fix;
        p.u = dst;
        if ((rc = plan_step(m, sched, p, &L))) return rc;
        LP_HIP(hipEventRecord(e0, st));
        for (int i = 0; i < reps; ++i) {
            p.step = 2 + (i & 127);
            launch_step(L, p, st);
        }
        LP_HIP(hipGetLastError());
        LP_HIP(hipEventRecord(e1, st));
        LP_HIP(hipEventSynchronize(e1));
        LP_HIP(hipEventElapsedTime(&total, e0, e1));
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = reps > 0 ? total / reps : 0.f;
    return LP_OK;
}

}  // namespace lp

// ------------------------------------------------------------------ C ABI

using namespace lp;

#define LP_GUARD_BEGIN try {
#define LP_GUARD_END                                              \
    }                                                             \
    catch (const std::bad_alloc &) {                              \
        set_error("host allocation failed");                      \
        return LP_E_NOMEM;                                        \
    }                                                             \
    catch (...) {                                                 \
        set_error("unexpected exception");                        \
        return LP_E_INTERNAL;                                     \
    }

extern "C" {

lp_status lp_build_matrix(int32_t n_atoms, int32_t n_rules, const int32_t *head, const int64_t *body_ptr,
                          const int32_t *body_lit, uint32_t flags, void *hip_stream, lp_matrix **out) {
    LP_GUARD_BEGIN
    if (!out) {
        set_error("out must be non-NULL");
        return LP_E_INVAL;
    }
    *out = nullptr;
    lp_matrix *mx = new lp_matrix();
    lp_status rc = build_host(n_atoms, n_rules, head, body_ptr, body_lit, flags, &mx->m);
    if (rc == LP_OK && !(flags & LP_BUILD_HOST_ONLY)) {
        rc = upload_matrix(mx->m, (hipStream_t)hip_stream);
        if (rc) free_device(mx->m, (hipStream_t)hip_stream);
    }
    if (rc) {
        delete mx;
        return rc;
    }
    *out = mx;
    return LP_OK;
    LP_GUARD_END
}

lp_status lp_free_matrix(lp_matrix *m) {
    LP_GUARD_BEGIN
    if (!m) return LP_OK;
    if (!(m->m.flags & LP_BUILD_HOST_ONLY)) {
        DeviceGuard g(m->m.dev.device);
        (void)hipDeviceSynchronize();
        free_device(m->m, nullptr);
    }
    delete m;
    return LP_OK;
    LP_GUARD_END
}

lp_status lp_matrix_info(const lp_matrix *m, lp_info *out) {
    if (!m || !out) {
        set_error("NULL argument");
        return LP_E_INVAL;
    }
    *out = m->m.info;
    return LP_OK;
}

lp_status lp_matrix_neg_atoms(const lp_matrix *m, int32_t *out) {
    if (!m || (!out && m->m.K)) {
        set_error("NULL argument");
        return LP_E_INVAL;
    }
    if (m->m.K) std::memcpy(out, m->m.neg_atoms.data(), sizeof(int32_t) * m->m.K);
    return LP_OK;
}

lp_status lp_matrix_csr(const lp_matrix *m, int32_t *row_ptr, int32_t *col, uint8_t *kind, uint8_t *fact) {
    if (!m) {
        set_error("NULL matrix");
        return LP_E_INVAL;
    }
    const Matrix &M = m->m;
    if (row_ptr) std::memcpy(row_ptr, M.row_ptr.data(), sizeof(int32_t) * M.row_ptr.size());
    if (col && M.nnz) std::memcpy(col, M.col.data(), sizeof(int32_t) * M.nnz);
    if (kind && M.n_rows) std::memcpy(kind, M.kind.data(), M.n_rows);
    if (fact && M.n_rows) std::memcpy(fact, M.fact.data(), M.n_rows);
    return LP_OK;
}

static lp_status check_solvable(const lp_matrix *m) {
    if (!m) {
        set_error("NULL matrix");
        return LP_E_INVAL;
    }
    if (m->m.flags & LP_BUILD_HOST_ONLY) {
        set_error("matrix was built with LP_BUILD_HOST_ONLY");
        return LP_E_HOST_ONLY;
    }
    return LP_OK;
}

lp_status lp_least_model(const lp_matrix *m, uint8_t *model, int32_t *products, const lp_schedule *sched,
                         void *hip_stream) {
    LP_GUARD_BEGIN
    lp_status rc = check_solvable(m);
    if (rc) return rc;
    if (m->m.K) {
        set_error("the program has negative literals; the least model is defined for definite programs");
        return LP_E_NEGATION;
    }
    if (!model && m->m.n_atoms) {
        set_error("model must be non-NULL");
        return LP_E_INVAL;
    }
    DeviceGuard g(m->m.dev.device);
    return least_model_impl(m->m, model, products, sched, (hipStream_t)hip_stream);
    LP_GUARD_END
}

lp_status lp_stable_models(const lp_matrix *m, uint64_t *accepted, int64_t *n_models, uint8_t *models,
                           int64_t max_models, uint64_t *interp, int32_t *products, void *hip_stream) {
    LP_GUARD_BEGIN
    lp_status rc = check_solvable(m);
    if (rc) return rc;
    if (m->m.K > LP_MAX_NEG_ATOMS) {
        set_error("too many negated atoms: " + std::to_string(m->m.K));
        return LP_E_TOO_MANY_GUESSES;
    }
    if (!accepted || !n_models || max_models < 0) {
        set_error("accepted and n_models must be non-NULL, max_models >= 0");
        return LP_E_INVAL;
    }
    DeviceGuard g(m->m.dev.device);
    return stable_impl(m->m, accepted, n_models, models, max_models, interp, products, (hipStream_t)hip_stream);
    LP_GUARD_END
}

lp_status lp_least_model_batch(const lp_matrix *const *ms, int32_t count, uint8_t *const *models,
                               int32_t *products, const lp_schedule *sched, void *hip_stream) {
    LP_GUARD_BEGIN
    if (count < 0 || (count > 0 && (!ms || !models))) {
        set_error("bad batch arguments");
        return LP_E_INVAL;
    }
    for (int32_t i = 0; i < count; ++i) {
        int32_t pr = 0;
        lp_status rc = lp_least_model(ms[i], models[i], &pr, sched, hip_stream);
        if (rc) return rc;
        if (products) products[i] = pr;
    }
    return LP_OK;
    LP_GUARD_END
}

lp_status lp_bench_step(const lp_matrix *m, const lp_schedule *sched, int32_t reps, float *avg_ms,
                        void *hip_stream) {
    LP_GUARD_BEGIN
    lp_status rc = check_solvable(m);
    if (rc) return rc;
    if (m->m.K || !avg_ms || reps < 1) {
        set_error("lp_bench_step needs a definite program, avg_ms and reps >= 1");
        return LP_E_INVAL;
    }
    DeviceGuard g(m->m.dev.device);
    return bench_step_impl(m->m, sched, reps, avg_ms, (hipStream_t)hip_stream);
    LP_GUARD_END
}

lp_status lp_set_allocator(void *(*alloc)(size_t, void *, void *), void (*release)(void *, void *, void *),
                           void *ctx) {
    if ((alloc == nullptr) != (release == nullptr)) {
        set_error("alloc and release must both be set or both be NULL");
        return LP_E_INVAL;
    }
    g_alloc = alloc;
    g_release = release;
    g_alloc_ctx = ctx;
    return LP_OK;
}

const char *lp_last_error(void) { return g_err.c_str(); }

}  // extern "C"
