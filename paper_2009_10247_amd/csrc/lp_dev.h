// lp_dev.h -- device helpers shared by the step kernels (lp_step.hip) and the
// batched fixpoint kernel (lp_batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lp {
namespace {

constexpr int kMaxWaves = 16;  // waves of a 1024-thread workgroup

// Pointers into LDS carry the LDS address space so every gather compiles to
// a ds_read rather than a flat load routed through the texture path.
typedef __attribute__((address_space(3))) uint8_t lds_u8;
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(3))) uint64_t lds_u64;
typedef __attribute__((address_space(3))) int32_t lds_i32;

// AND entries are stored encoded as ((c >> 5) << 7) | (c & 31): one shift
// gives the byte address of the 32-bit word of v holding atom c (a multiple
// of 4), and the low five bits are its bit offset in that word, which
// v_bfe_u32 takes as is. Gathers read whole aligned words, so no masking of a
// narrower load is needed.
__device__ __forceinline__ uint32_t entry_byte(int32_t e) { return (uint32_t)e >> 5; }

__device__ __forceinline__ uint32_t entry_word(const lds_u8 *v, int32_t e) {
    return *(const lds_u32 *)(v + entry_byte(e));
}

__device__ __forceinline__ uint32_t entry_word(const uint8_t *v, int32_t e) {
    return *reinterpret_cast<const uint32_t *>(v + entry_byte(e));
}

// Index of this wave in the grid (blockIdx.x * waves + wave in block), made
// visibly wave-uniform so that loop counters derived from it stay scalar.
__device__ __forceinline__ int64_t grid_wave() {
    const int32_t w = (int32_t)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    return (int64_t)__builtin_amdgcn_readfirstlane(w);
}

__device__ inline uint64_t range_mask(int s, int t) {  // bits [s, t), 0 <= s < t <= 64
    const uint64_t hi = (t >= 64) ? ~0ull : ((1ull << t) - 1ull);
    return hi & ~((1ull << s) - 1ull);
}

__device__ inline uint32_t wave_sum(uint32_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Exclusive prefix sum over the 64 lanes of a wave, with DPP: shifts by 1, 2,
// 4 and 8 inside each row of 16 lanes, then row_bcast:15 and row_bcast:31 carry
// the row totals into the rows above.
__device__ inline int32_t wave_exclusive_scan(int32_t x) {
    int32_t t = x;
    t += __builtin_amdgcn_update_dpp(0, t, 0x111, 0xf, 0xf, false);  // row_shr:1
    t += __builtin_amdgcn_update_dpp(0, t, 0x112, 0xf, 0xf, false);  // row_shr:2
    t += __builtin_amdgcn_update_dpp(0, t, 0x114, 0xf, 0xf, false);  // row_shr:4
    t += __builtin_amdgcn_update_dpp(0, t, 0x118, 0xf, 0xf, false);  // row_shr:8
    t += __builtin_amdgcn_update_dpp(0, t, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
    t += __builtin_amdgcn_update_dpp(0, t, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
    return t - x;
}

}  // namespace
}  // namespace lp
