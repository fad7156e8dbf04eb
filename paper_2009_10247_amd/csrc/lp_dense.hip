// lp_dense.hip -- the dense-matrix form of the T_P products, the third method
// of the paper's experiments (Section 4): the program matrix is stored as an
// n' x n' matrix of bytes (1 where the row names the column) and every product
// reads all of it. It computes the same theta(M v) as the sparse kernels and
// exists to measure what the sparse form saves.
//
// Interpretations are bytes, 0 or 1. A least-model vector is v[ld]; the
// interpretation matrix of the stable-model method is stored guess-major,
// Vt[j][i] = atom i in column j, so that both operands of the matrix product
// run along the atom index in memory. Row i fires iff its count of true
// entries reaches thr[i]: the row length for AND rows (a count never exceeds
// it), 1 for OR rows. Padded rows and columns hold zeros and thr = 1, so they
// never fire.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lp_kernels.h"

namespace lp {
namespace {

typedef int32_t v4i __attribute__((ext_vector_type(4)));

constexpr int kDenseBlock = 256;

__device__ inline uint32_t dense_wave_sum(uint32_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Adds the workgroup's change count to counter blockIdx % kDenseCounters
// (each on its own 128-byte line; the host sums them): one atomic per
// workgroup, spread over several addresses, because same-address atomics
// from every wave serialize. ch: the wave's count, read from its first lane.
// Every thread of the workgroup must call it.
__device__ __forceinline__ void add_changes(uint32_t ch, unsigned long long *changed) {
    __shared__ uint32_t s_ch[8];
    if ((threadIdx.x & 63) == 0) s_ch[threadIdx.x >> 6] = ch;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (uint32_t w = 0; w < (blockDim.x >> 6); ++w) t += s_ch[w];
        if (t) atomicAdd(changed + (blockIdx.x % kDenseCounters) * kDenseCounterStride, (unsigned long long)t);
    }
}

// Number of byte positions where both a and b hold 1 (every byte is 0 or 1).
__device__ __forceinline__ uint32_t and_count(uint4 a, uint4 b) {
    return __builtin_popcount(a.x & b.x) + __builtin_popcount(a.y & b.y) + __builtin_popcount(a.z & b.z) +
           __builtin_popcount(a.w & b.w);
}

// Row i of the dense matrix gets a 1 at every column of row i of the CSR
// matrix (which the caller has cleared). One wave per row.
__global__ __launch_bounds__(kDenseBlock) void dense_scatter_kernel(uint8_t *M, int64_t ld, const int32_t *row_ptr,
                                                                   const int32_t *col, int32_t n_rows) {
    const int32_t row = (int32_t)(blockIdx.x * (kDenseBlock / 64) + (threadIdx.x >> 6));
    if (row >= n_rows) return;
    uint8_t *r = M + (int64_t)row * ld;
    const int32_t e1 = row_ptr[row + 1];
    for (int32_t e = row_ptr[row] + (int32_t)(threadIdx.x & 63); e < e1; e += 64) r[col[e]] = 1;
}

// u = theta(M v) (Algorithm 1's product). Each wave takes kGemvRows
// consecutive rows; lane l reads bytes [16 l, 16 l + 16) of every 1024-byte
// chunk of v and of those rows, so each chunk of v serves all of them. The
// wave's first lane writes the rows' results; the number of rows that
// changed goes to the change counters.
constexpr int kGemvRows = 8;

__global__ __launch_bounds__(kDenseBlock) void dense_gemv_kernel(const uint8_t *M, int64_t ld, const uint8_t *v,
                                                                uint8_t *u, const int32_t *thr,
                                                                unsigned long long *changed) {
    const int lane = threadIdx.x & 63;
    const int64_t r0 = ((int64_t)blockIdx.x * (kDenseBlock / 64) + (threadIdx.x >> 6)) * kGemvRows;
    const uint8_t *a = M + r0 * ld + lane * 16;
    const uint8_t *x = v + lane * 16;
    uint32_t c[kGemvRows];
#pragma unroll
    for (int r = 0; r < kGemvRows; ++r) c[r] = 0;
    const int64_t chunks = ld >> 10;
#pragma unroll 2
    for (int64_t k = 0; k < chunks; ++k) {
        const uint4 xv = *(const uint4 *)(x + (k << 10));
#pragma unroll
        for (int r = 0; r < kGemvRows; ++r) c[r] += and_count(*(const uint4 *)(a + r * ld + (k << 10)), xv);
    }
#pragma unroll
    for (int r = 0; r < kGemvRows; ++r) c[r] = dense_wave_sum(c[r]);
    uint32_t ch = 0;
    if (lane == 0) {
#pragma unroll
        for (int h = 0; h < kGemvRows / 4; ++h) {
            const int4 t = *(const int4 *)(thr + r0 + 4 * h);
            const uint32_t word = (uint32_t)(c[4 * h] >= (uint32_t)t.x) | ((uint32_t)(c[4 * h + 1] >= (uint32_t)t.y) << 8) |
                                  ((uint32_t)(c[4 * h + 2] >= (uint32_t)t.z) << 16) |
                                  ((uint32_t)(c[4 * h + 3] >= (uint32_t)t.w) << 24);
            ch += __builtin_popcount(word ^ *(const uint32_t *)(v + r0 + 4 * h));
            *(uint32_t *)(u + r0 + 4 * h) = word;
        }
    }
    add_changes(ch, changed);
}

// Ut = theta(M V) (Algorithm 2's product) on the int8 matrix cores: counts
// C[i][j] = sum_k M[i][k] Vt[j][k] by v_mfma_i32_16x16x64_i8. A workgroup of
// 2 x NWN waves computes a 128 x 64 NWN tile of C (each wave 64 x 64), K in
// stages of 128 bytes staged through two LDS buffers. Both operands are
// K-contiguous in memory, so lane l's 16 bytes of an A fragment (row l % 16)
// and of a B fragment (column l % 16) cover the same 16 values of k,
// (l / 16) * 16 onwards; the instruction pairs them position by position, so
// its internal order of k does not matter. Result lane l, element e of a
// 16 x 16 tile: row 4 (l / 16) + e, column l % 16.
constexpr int kGT = 128;         // rows of M per tile
constexpr int kGK = 128;         // bytes of k per stage
constexpr int kGRow = kGK + 16;  // LDS row pitch: 16 rows at one k start 36 banks apart
constexpr int kGroupM = 8;       // row tiles per group of the tile order

template <int NWN>
constexpr int gemm_stage_bytes() { return (kGT + 64 * NWN) * kGRow; }

// Workgroup b runs on XCD b % 8; give consecutive logical tiles to one XCD so
// that tiles sharing rows of M share its L2.
__device__ __forceinline__ int32_t xcd_order(int32_t b, int32_t nb) {
    const int32_t xcd = b & 7, local = b >> 3, base = nb >> 3, rem = nb & 7;
    return xcd * base + (xcd < rem ? xcd : rem) + local;
}

// With splits > 1 (few tiles: too few workgroups to keep enough loads in
// flight), workgroup (tile, s) sums only k-stages [s nk / splits, (s + 1) nk /
// splits) and writes its raw counts to partial[s][column][row]; then
// dense_theta_kernel adds the slices and applies theta.
template <int NWN>
__global__ __launch_bounds__(128 * NWN) void dense_gemm_kernel(const uint8_t *M, const uint8_t *Vt, uint8_t *Ut,
                                                              int64_t ld, int64_t hp, int32_t splits,
                                                              int32_t *partial, const int32_t *thr,
                                                              unsigned long long *changed) {
    constexpr int kThreads = 128 * NWN;
    constexpr int BN = 64 * NWN;                         // columns per tile
    constexpr int kAP = kGT * (kGK / 16) / kThreads;     // 16-byte pieces of A per thread and stage
    constexpr int kBP = BN * (kGK / 16) / kThreads;      // and of B
    constexpr int kStage = gemm_stage_bytes<NWN>();
    extern __shared__ __attribute__((aligned(16))) uint8_t s_dense[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int32_t m_tiles = (int32_t)(ld / kGT), n_tiles = (int32_t)(hp / BN);
    const int32_t L = xcd_order((int32_t)blockIdx.x, m_tiles * n_tiles * splits);
    int32_t mt, nt, split = 0;
    if (splits == 1) {
        // groups of kGroupM row tiles, row tile fastest inside a group
        const int32_t per_group = kGroupM * n_tiles;
        const int32_t first_m = (L / per_group) * kGroupM;
        const int32_t gsize = min(kGroupM, m_tiles - first_m);
        const int32_t in_group = L - (L / per_group) * per_group;
        mt = first_m + in_group % gsize;
        nt = in_group / gsize;
    } else {
        // column tile fastest, so the tiles that share rows of M run side by side
        nt = L % n_tiles;
        split = (L / n_tiles) % splits;
        mt = L / (n_tiles * splits);
    }
    const int32_t nk = (int32_t)(ld / kGK) / splits;
    const int64_t kbase = (int64_t)split * nk * kGK;

    const uint8_t *Ag = M + (int64_t)mt * kGT * ld + kbase;
    const uint8_t *Bg = Vt + (int64_t)nt * BN * ld + kbase;
    // staging: 16-byte piece c = tid + kThreads s of a stage: row c / 8,
    // bytes 16 (c % 8) onwards, in global memory and in LDS
    int64_t ga[kAP], gb[kBP];
    int la[kAP], lb[kBP];
#pragma unroll
    for (int s = 0; s < kAP; ++s) {
        const int c = tid + kThreads * s;
        ga[s] = (int64_t)(c >> 3) * ld + (c & 7) * 16;
        la[s] = (c >> 3) * kGRow + (c & 7) * 16;
    }
#pragma unroll
    for (int s = 0; s < kBP; ++s) {
        const int c = tid + kThreads * s;
        gb[s] = (int64_t)(c >> 3) * ld + (c & 7) * 16;
        lb[s] = (kGT + (c >> 3)) * kGRow + (c & 7) * 16;
    }
    v4i ra[kAP], rb[kBP];  // native vectors: arrays of them stay in registers
    v4i acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4i{0, 0, 0, 0};
    const int wm = (wave / NWN) * 64, wn = (wave % NWN) * 64;
    const int fr = lane & 15, fk = (lane >> 4) * 16;
#pragma unroll
    for (int s = 0; s < kAP; ++s) ra[s] = *(const v4i *)(Ag + ga[s]);
#pragma unroll
    for (int s = 0; s < kBP; ++s) rb[s] = *(const v4i *)(Bg + gb[s]);
#pragma unroll
    for (int s = 0; s < kAP; ++s) *(v4i *)(s_dense + la[s]) = ra[s];
#pragma unroll
    for (int s = 0; s < kBP; ++s) *(v4i *)(s_dense + lb[s]) = rb[s];
    __syncthreads();
    for (int32_t kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        const bool more = kt + 1 < nk;
        if (more) {
            const int64_t k0 = (int64_t)(kt + 1) * kGK;
#pragma unroll
            for (int s = 0; s < kAP; ++s) ra[s] = *(const v4i *)(Ag + ga[s] + k0);
#pragma unroll
            for (int s = 0; s < kBP; ++s) rb[s] = *(const v4i *)(Bg + gb[s] + k0);
        }
        const uint8_t *A = s_dense + cur * kStage;
        const uint8_t *B = A + kGT * kGRow;
#pragma unroll
        for (int kk = 0; kk < kGK; kk += 64) {
            v4i a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = *(const v4i *)(A + (wm + 16 * i + fr) * kGRow + kk + fk);
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = *(const v4i *)(B + (wn + 16 * j + fr) * kGRow + kk + fk);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        // the other buffer was last read before the previous barrier
        if (more) {
            uint8_t *Nb = s_dense + (cur ^ 1) * kStage;
#pragma unroll
            for (int s = 0; s < kAP; ++s) *(v4i *)(Nb + la[s]) = ra[s];
#pragma unroll
            for (int s = 0; s < kBP; ++s) *(v4i *)(Nb + lb[s]) = rb[s];
        }
        __syncthreads();
    }
    // theta, the change count against the input, and the store: element e of
    // tile (i, j) is row rr + e, column cc; four rows of one column are four
    // consecutive bytes of Ut.
    uint32_t ch = 0;
    const int64_t row0 = (int64_t)mt * kGT + wm + 4 * (lane >> 4);
    const int64_t col0 = (int64_t)nt * BN + wn + fr;
    if (splits > 1) {
        int32_t *P = partial + (int64_t)split * hp * ld;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) *(v4i *)(P + (col0 + 16 * j) * ld + row0 + 16 * i) = acc[i][j];
        return;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t rr = row0 + 16 * i;
        const int4 t = *(const int4 *)(thr + rr);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t at = (col0 + 16 * j) * ld + rr;
            const v4i s = acc[i][j];
            const uint32_t word = (uint32_t)(s.x >= t.x) | ((uint32_t)(s.y >= t.y) << 8) |
                                  ((uint32_t)(s.z >= t.z) << 16) | ((uint32_t)(s.w >= t.w) << 24);
            ch += __builtin_popcount(word ^ *(const uint32_t *)(Vt + at));
            *(uint32_t *)(Ut + at) = word;
        }
    }
    add_changes(dense_wave_sum(ch), changed);
}

// Adds the splits slices of partial counts and applies theta: four rows of
// one column per thread; the change count as in dense_gemm_kernel.
__global__ __launch_bounds__(kDenseBlock) void dense_theta_kernel(const int32_t *partial, int32_t splits,
                                                                 const uint8_t *Vt, uint8_t *Ut, int64_t ld,
                                                                 int64_t hp, const int32_t *thr,
                                                                 unsigned long long *changed) {
    const int64_t g = (int64_t)blockIdx.x * kDenseBlock + threadIdx.x;
    const int64_t per_col = ld >> 2;
    uint32_t ch = 0;
    if (g < hp * per_col) {
        const int64_t at = g * 4;  // column g / per_col, rows 4 (g % per_col) onwards
        const int64_t slice = hp * ld;
        v4i s = *(const v4i *)(partial + at);
        for (int32_t k = 1; k < splits; ++k) s += *(const v4i *)(partial + k * slice + at);
        const int4 t = *(const int4 *)(thr + (at % ld));
        const uint32_t word = (uint32_t)(s.x >= t.x) | ((uint32_t)(s.y >= t.y) << 8) |
                              ((uint32_t)(s.z >= t.z) << 16) | ((uint32_t)(s.w >= t.w) << 24);
        ch = __builtin_popcount(word ^ *(const uint32_t *)(Vt + at));
        *(uint32_t *)(Ut + at) = word;
    }
    add_changes(dense_wave_sum(ch), changed);
}

// Initial matrix of Definition 8, guess-major: column j < h has 1 in the fact
// rows and bit t of j in row n_std + t (qbar_t); everything else is 0,
// padded columns included. One thread per 16 bytes.
__global__ __launch_bounds__(kDenseBlock) void dense_init_kernel(uint8_t *V, int64_t ld, int64_t h, int64_t hp,
                                                                const uint8_t *fact, int32_t n_std, int32_t K) {
    const int64_t g = (int64_t)blockIdx.x * kDenseBlock + threadIdx.x;
    const int64_t per_col = ld >> 4;
    if (g >= hp * per_col) return;
    const int64_t j = g / per_col;
    const int64_t i0 = (g - j * per_col) * 16;
    uint32_t w[4] = {0, 0, 0, 0};
    if (j < h) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int64_t i = i0 + q;
            uint32_t b = fact[i];
            if (!b && i >= n_std && i < (int64_t)n_std + K) b = (uint32_t)((j >> (i - n_std)) & 1);
            w[q >> 2] |= b << (8 * (q & 3));
        }
    }
    *(uint4 *)(V + j * ld + i0) = uint4{w[0], w[1], w[2], w[3]};
}

// Algorithm 3 on column j: accepted iff exactly one of q_t and qbar_t holds
// for every t. Bit j % 64 of accept[j / 64]; *count gets the accepted total.
__global__ __launch_bounds__(kDenseBlock) void dense_check_kernel(const uint8_t *V, int64_t ld, int64_t h,
                                                                 const int32_t *q_rows, int32_t n_std, int32_t K,
                                                                 uint64_t *accept, unsigned long long *count) {
    const int64_t j = (int64_t)blockIdx.x * kDenseBlock + threadIdx.x;
    bool ok = false;
    if (j < h) {
        const uint8_t *col = V + j * ld;
        ok = true;
        for (int32_t t = 0; t < K; ++t) ok = ok && (col[q_rows[t]] ^ col[n_std + t]) != 0;
    }
    const uint64_t bal = __ballot(ok);
    const int64_t j0 = j - (threadIdx.x & 63);
    if ((threadIdx.x & 63) == 0 && j0 < h) {
        accept[j0 >> 6] = bal;
        if (bal) atomicAdd(count, (unsigned long long)__popcll(bal));
    }
}

// Models: bytes [0, n_atoms) of columns cols[0..n).
__global__ __launch_bounds__(kDenseBlock) void dense_gather_kernel(const uint8_t *V, int64_t ld, const int64_t *cols,
                                                                  int64_t n, int32_t n_atoms, uint8_t *out) {
    const int64_t g = (int64_t)blockIdx.x * kDenseBlock + threadIdx.x;
    if (g >= n * (int64_t)n_atoms) return;
    const int64_t m = g / n_atoms;
    out[g] = V[cols[m] * ld + (g - m * n_atoms)];
}

unsigned dense_blocks(int64_t n) { return (unsigned)((n + kDenseBlock - 1) / kDenseBlock); }

}  // namespace

static_assert(kDenseColAlign == 128 && kDenseAlign % (kGK * kDenseMaxSplits) == 0 && kDenseAlign % kGT == 0 &&
                  kDenseAlign % (kGemvRows * (kDenseBlock / 64)) == 0,
              "dense padding must cover the kernels' tiles");

hipError_t launch_dense_scatter(uint8_t *M, int64_t ld, const int32_t *row_ptr, const int32_t *col, int32_t n_rows,
                                hipStream_t st) {
    if (n_rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(dense_scatter_kernel, dim3((unsigned)((n_rows + 3) / 4)), dim3(kDenseBlock), 0, st, M, ld,
                       row_ptr, col, n_rows);
    return hipGetLastError();
}

hipError_t launch_dense_gemv(const uint8_t *M, int64_t ld, const uint8_t *v, uint8_t *u, const int32_t *thr,
                             unsigned long long *changed, hipStream_t st) {
    if (ld <= 0 || ld % kDenseAlign) return hipErrorInvalidValue;
    hipLaunchKernelGGL(dense_gemv_kernel, dim3((unsigned)(ld / (kGemvRows * (kDenseBlock / 64)))), dim3(kDenseBlock),
                       0, st, M, ld, v, u, thr, changed);
    return hipGetLastError();
}

// Tiles 128 columns wide (NWN = 2). Tiles of 256 columns (NWN = 4, M read
// once per 256 columns) measured slower on both the 256- and the
// 65,536-column products: their 110 KB of LDS leaves one workgroup per CU.
static int gemm_nwn(int64_t) { return 2; }

int dense_gemm_splits(int64_t ld, int64_t hp) {
    const int64_t tiles = (ld / kGT) * (hp / (64 * gemm_nwn(hp)));
    int s = 1;
    while (s < kDenseMaxSplits && tiles * s < kDenseSplitTarget) s *= 2;
    return s;
}

template <int NWN>
static hipError_t gemm_launch(const uint8_t *M, const uint8_t *Vt, uint8_t *Ut, int64_t ld, int64_t hp, int splits,
                              int32_t *partial, const int32_t *thr, unsigned long long *changed, hipStream_t st) {
    constexpr size_t lds = 2 * (size_t)gemm_stage_bytes<NWN>();
    static const hipError_t lds_ok = hipFuncSetAttribute((const void *)dense_gemm_kernel<NWN>,
                                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (lds_ok != hipSuccess) return lds_ok;
    const int64_t blocks = (ld / kGT) * (hp / (64 * NWN)) * splits;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(dense_gemm_kernel<NWN>, dim3((unsigned)blocks), dim3(128 * NWN), lds, st, M, Vt, Ut, ld, hp,
                       (int32_t)splits, partial, thr, changed);
    return hipGetLastError();
}

hipError_t launch_dense_gemm(const uint8_t *M, const uint8_t *Vt, uint8_t *Ut, int64_t ld, int64_t hp,
                             int32_t *partial, const int32_t *thr, unsigned long long *changed, hipStream_t st) {
    if (ld <= 0 || ld % kDenseAlign || hp <= 0 || hp % kDenseColAlign) return hipErrorInvalidValue;
    const int splits = dense_gemm_splits(ld, hp);
    if (splits > 1 && !partial) return hipErrorInvalidValue;
    hipError_t e = gemm_launch<2>(M, Vt, Ut, ld, hp, splits, partial, thr, changed, st);
    if (e != hipSuccess || splits == 1) return e;
    hipLaunchKernelGGL(dense_theta_kernel, dim3(dense_blocks(hp * (ld >> 2))), dim3(kDenseBlock), 0, st, partial,
                       (int32_t)splits, Vt, Ut, ld, hp, thr, changed);
    return hipGetLastError();
}

hipError_t launch_dense_init(uint8_t *V, int64_t ld, int64_t h, int64_t hp, const uint8_t *fact, int32_t n_std,
                             int32_t K, hipStream_t st) {
    hipLaunchKernelGGL(dense_init_kernel, dim3(dense_blocks(hp * (ld >> 4))), dim3(kDenseBlock), 0, st, V, ld, h, hp,
                       fact, n_std, K);
    return hipGetLastError();
}

hipError_t launch_dense_check(const uint8_t *V, int64_t ld, int64_t h, const int32_t *q_rows, int32_t n_std,
                              int32_t K, uint64_t *accept, unsigned long long *count, hipStream_t st) {
    hipLaunchKernelGGL(dense_check_kernel, dim3(dense_blocks(h)), dim3(kDenseBlock), 0, st, V, ld, h, q_rows, n_std, K,
                       accept, count);
    return hipGetLastError();
}

hipError_t launch_dense_gather(const uint8_t *V, int64_t ld, const int64_t *cols, int64_t n, int32_t n_atoms,
                               uint8_t *out, hipStream_t st) {
    if (n <= 0 || n_atoms <= 0) return hipSuccess;
    hipLaunchKernelGGL(dense_gather_kernel, dim3(dense_blocks(n * (int64_t)n_atoms)), dim3(kDenseBlock), 0, st, V, ld,
                       cols, n, n_atoms, out);
    return hipGetLastError();
}

}  // namespace lp
