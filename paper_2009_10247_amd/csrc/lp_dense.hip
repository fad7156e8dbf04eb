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
// wave's first lane writes the rows' results and adds the number of rows that
// changed to *changed.
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
    if (lane == 0) {
        uint32_t ch = 0;
#pragma unroll
        for (int h = 0; h < kGemvRows / 4; ++h) {
            const int4 t = *(const int4 *)(thr + r0 + 4 * h);
            const uint32_t word = (uint32_t)(c[4 * h] >= (uint32_t)t.x) | ((uint32_t)(c[4 * h + 1] >= (uint32_t)t.y) << 8) |
                                  ((uint32_t)(c[4 * h + 2] >= (uint32_t)t.z) << 16) |
                                  ((uint32_t)(c[4 * h + 3] >= (uint32_t)t.w) << 24);
            ch += __builtin_popcount(word ^ *(const uint32_t *)(v + r0 + 4 * h));
            *(uint32_t *)(u + r0 + 4 * h) = word;
        }
        if (ch) atomicAdd(changed, (unsigned long long)ch);
    }
}

// Ut = theta(M V) (Algorithm 2's product) on the int8 matrix cores: counts
// C[i][j] = sum_k M[i][k] Vt[j][k] by v_mfma_i32_16x16x64_i8, a 128 x 128 tile
// of C per workgroup (four waves of 64 x 64), K in stages of 128 bytes staged
// through two LDS buffers. Both operands are K-contiguous in memory, so lane
// l's 16 bytes of an A fragment (row l % 16) and of a B fragment (column
// l % 16) cover the same 16 values of k, (l / 16) * 16 onwards; the
// instruction pairs them position by position, so its internal order of k
// does not matter. Result lane l, element e of a 16 x 16 tile: row
// 4 (l / 16) + e, column l % 16.
constexpr int kGT = 128;                  // tile edge (rows of M, columns of V)
constexpr int kGK = 128;                  // bytes of k per stage
constexpr int kGRow = kGK + 16;           // LDS row pitch: 16 rows at one k start 36 banks apart
constexpr int kGStage = 2 * kGT * kGRow;  // A and B tiles of one stage
constexpr int kGroupM = 8;                // row tiles per group of the tile order

// Workgroup b runs on XCD b % 8; give consecutive logical tiles to one XCD so
// that tiles sharing rows of M share its L2.
__device__ __forceinline__ int32_t xcd_order(int32_t b, int32_t nb) {
    const int32_t xcd = b & 7, local = b >> 3, base = nb >> 3, rem = nb & 7;
    return xcd * base + (xcd < rem ? xcd : rem) + local;
}

__global__ __launch_bounds__(kDenseBlock) void dense_gemm_kernel(const uint8_t *M, const uint8_t *Vt, uint8_t *Ut,
                                                                int64_t ld, int32_t m_tiles, int32_t n_tiles,
                                                                const int32_t *thr, unsigned long long *changed) {
    extern __shared__ __attribute__((aligned(16))) uint8_t s_dense[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // tile order: groups of kGroupM row tiles, row tile fastest inside a group
    const int32_t L = xcd_order((int32_t)blockIdx.x, m_tiles * n_tiles);
    const int32_t per_group = kGroupM * n_tiles;
    const int32_t first_m = (L / per_group) * kGroupM;
    const int32_t gsize = min(kGroupM, m_tiles - first_m);
    const int32_t in_group = L - (L / per_group) * per_group;
    const int32_t mt = first_m + in_group % gsize, nt = in_group / gsize;

    const uint8_t *Ag = M + (int64_t)mt * kGT * ld;
    const uint8_t *Bg = Vt + (int64_t)nt * kGT * ld;
    // staging: 16-byte piece c = tid + 256 s of a stage, s < 4: row c / 8,
    // bytes 16 (c % 8) onwards, in global memory and in LDS
    int64_t goff[4];
    int loff[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int c = tid + kDenseBlock * s;
        goff[s] = (int64_t)(c >> 3) * ld + (c & 7) * 16;
        loff[s] = (c >> 3) * kGRow + (c & 7) * 16;
    }
    uint4 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
#define LP_DENSE_GLOAD(k0)                                  \
    ra0 = *(const uint4 *)(Ag + goff[0] + (k0));            \
    ra1 = *(const uint4 *)(Ag + goff[1] + (k0));            \
    ra2 = *(const uint4 *)(Ag + goff[2] + (k0));            \
    ra3 = *(const uint4 *)(Ag + goff[3] + (k0));            \
    rb0 = *(const uint4 *)(Bg + goff[0] + (k0));            \
    rb1 = *(const uint4 *)(Bg + goff[1] + (k0));            \
    rb2 = *(const uint4 *)(Bg + goff[2] + (k0));            \
    rb3 = *(const uint4 *)(Bg + goff[3] + (k0));
#define LP_DENSE_LSTORE(buf)                                \
    {                                                       \
        uint8_t *A_ = s_dense + (buf) * kGStage;            \
        uint8_t *B_ = A_ + kGT * kGRow;                     \
        *(uint4 *)(A_ + loff[0]) = ra0;                     \
        *(uint4 *)(A_ + loff[1]) = ra1;                     \
        *(uint4 *)(A_ + loff[2]) = ra2;                     \
        *(uint4 *)(A_ + loff[3]) = ra3;                     \
        *(uint4 *)(B_ + loff[0]) = rb0;                     \
        *(uint4 *)(B_ + loff[1]) = rb1;                     \
        *(uint4 *)(B_ + loff[2]) = rb2;                     \
        *(uint4 *)(B_ + loff[3]) = rb3;                     \
    }
    v4i acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4i{0, 0, 0, 0};
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int fr = lane & 15, fk = (lane >> 4) * 16;
    const int32_t nk = (int32_t)(ld / kGK);
    LP_DENSE_GLOAD(0)
    LP_DENSE_LSTORE(0)
    __syncthreads();
    for (int32_t kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        const bool more = kt + 1 < nk;
        if (more) {
            const int64_t k0 = (int64_t)(kt + 1) * kGK;
            LP_DENSE_GLOAD(k0)
        }
        const uint8_t *A = s_dense + cur * kGStage;
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
        if (more) LP_DENSE_LSTORE(cur ^ 1)
        __syncthreads();
    }
#undef LP_DENSE_GLOAD
#undef LP_DENSE_LSTORE
    // theta, the change count against the input, and the store: element e of
    // tile (i, j) is row rr + e, column cc; four rows of one column are four
    // consecutive bytes of Ut.
    uint32_t ch = 0;
    const int64_t row0 = (int64_t)mt * kGT + wm + 4 * (lane >> 4);
    const int64_t col0 = (int64_t)nt * kGT + wn + fr;
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
    ch = dense_wave_sum(ch);
    if (lane == 0 && ch) atomicAdd(changed, (unsigned long long)ch);
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

static_assert(kDenseColAlign == kGT && kDenseAlign % kGK == 0 && kDenseAlign % kGT == 0 &&
                  kDenseAlign % (kGemvRows * (kDenseBlock / 64)) == 0,
              "dense padding must cover the kernels' tiles");
static const size_t kDenseGemmLds = 2 * (size_t)kGStage;

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

hipError_t launch_dense_gemm(const uint8_t *M, const uint8_t *Vt, uint8_t *Ut, int64_t ld, int64_t hp,
                             const int32_t *thr, unsigned long long *changed, hipStream_t st) {
    if (ld <= 0 || ld % kDenseAlign || hp <= 0 || hp % kGT) return hipErrorInvalidValue;
    static const hipError_t lds_ok = hipFuncSetAttribute(
        (const void *)dense_gemm_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kDenseGemmLds);
    if (lds_ok != hipSuccess) return lds_ok;
    const int64_t tiles = (ld / kGT) * (hp / kGT);
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(dense_gemm_kernel, dim3((unsigned)tiles), dim3(kDenseBlock), kDenseGemmLds, st, M, Vt, Ut, ld,
                       (int32_t)(ld / kGT), (int32_t)(hp / kGT), thr, changed);
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
