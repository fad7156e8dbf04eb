// lp_kernels.h -- kernel parameter blocks and launchers shared by the kernel
// translation units (lp_step.hip, lp_batch.hip, lp_spmm.hip) and the runtime (lp_runtime.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "lp_internal.h"

namespace lp {

// Change counts live in a ring indexed by product number & (kRing - 1).
constexpr int kRing = 256;

// One least-model T_P step u = theta(M v) over the device layout of a matrix.
struct StepParams {
    const WordMeta *words;         // [n_words]
    const uint8_t *and_len;        // [n_rows]
    const uint32_t *lens4;         // AND lengths of four consecutive words per lane
    const int32_t *col;            // block AND entries
    const int32_t *or_c0;          // [n_or + 1]
    const int32_t *or_row;         // [n_or] row of each OR row, -1 for rows of the segment pass
    const LongSeg *segs;           // [n_segs]
    const int32_t *long_col;
    uint32_t *and_cnt;             // [2][n_long_and] completion counts of split AND rows
    const uint64_t *v;             // [n_words] v_t
    uint64_t *u;                   // [n_words] holds a subset of the result; the step ORs into it
    unsigned long long *counters;  // change-count ring
    const int32_t *wave_part;      // [2 (waves + 1)]: wave k's first word and that word's first AND entry
    int32_t n_rows;
    int32_t n_long_and;
    int32_t n_segs;
    int32_t n_or;
    int32_t and_end;               // number of block AND entries
    int32_t and_max_col;           // largest column of a block AND entry (-1 if none)
    int32_t step;                  // 1-based product index
    int32_t early_exit;            // 1: return at once if product step-1 changed nothing
    int32_t lds_words;             // words of v staged in LDS (LDS shapes), from word stage_off
    int32_t stage_off;             // first staged word (0 unless the layout is sliced)
    // column-sliced layouts (kStepSlice): a product is n_pass launches, pass k
    // over the AND entries whose columns lie in slice k (staged in LDS); pacc
    // holds per word the AND rows whose entries in the passes so far are all
    // true, and_all every block AND row of the word
    uint64_t *pacc;
    const uint64_t *and_all;
    int32_t pass;
    int32_t n_pass;
};

// Forms of the step kernel: gathers of v from global memory; from v staged
// in LDS (every AND entry names a staged atom); mixed (atoms past the staged
// words are read from global memory); or sliced (one pass per column slice of
// the AND entries, each slice's part of v staged in LDS).
enum StepMode : int { kStepGlobal = 0, kStepLds = 1, kStepMixed = 2, kStepSlice = 3 };

// LDS of the staged forms (static, so v sits at LDS address 0): the staged
// words of v, then one ballot slot area per wave (16 waves x (unroll + 1)
// words), then the new-bit count. gfx950 gives a workgroup 160 KB.
constexpr int kStepLdsBytes = 163840;
inline int32_t step_lds_v_words(int unroll) { return kStepLdsBytes / 8 - 16 * (unroll + 1) - 2; }

// Launch shape of the step kernel. A wave owns wpw consecutive 64-row words
// (a super-block) and keeps unroll column chunks of 64 entries in flight.

struct StepShape {
    int mode = kStepLds;  // StepMode; staged forms use 1024-thread workgroups, one per CU
    int wpw = 8;          // words per super-block: 4 or 8
    int unroll = 8;       // 4, 8 or 16
    int block = 1024;     // threads per workgroup
    int grid = 0;         // workgroups (grid-stride loop over super-blocks)
    // kStepSlice: the slices (host array kept with the matrix) and each
    // slice's wave split for this grid
    int n_slices = 0;
    const SliceLayout *slice = nullptr;
    const int32_t *slice_part[kMaxSlices] = {};
};

bool step_shape_supported(const StepShape &s);
hipError_t launch_step(const StepShape &s, const StepParams &p, hipStream_t st);
// One launch of the step kernel with p as given (one pass of a sliced step).
hipError_t launch_step_pass(const StepShape &s, const StepParams &p, hipStream_t st);

// Sets n 32-bit words at p to 0 (a kernel, not a memset node).
hipError_t launch_zero_words(void *p, int64_t n, hipStream_t st);

// Persistent form: the whole fixpoint loop in one cooperative launch.
struct PersistParams {
    StepParams p;
    uint64_t *buf0;
    uint64_t *buf1;
    int32_t max_steps;
    int32_t *result;  // products, -1 if max_steps was reached, -2 if a grid barrier was abandoned
    uint32_t *bar;    // grid barrier arrivals (0 at launch)
    int32_t *abort;   // set when a workgroup gives up waiting at a barrier (0 at launch)
};
hipError_t launch_persistent(const StepShape &s, const PersistParams &q, hipStream_t st);
hipError_t persistent_occupancy(const StepShape &s, int *blocks_per_cu);

// Many least models in one launch: each workgroup runs whole fixpoints of the
// programs it takes from a device work queue, with both buffers in LDS.
struct ProgDesc {
    const WordMeta *words;
    const uint8_t *and_len;
    const uint32_t *lens4;   // the AND lengths by lane, four words per dword (the step kernels' form)
    const int32_t *col;
    const int32_t *or_c0;
    const int32_t *or_row;
    const LongSeg *segs;
    const int32_t *long_col;
    const uint64_t *fact_bits;
    uint64_t *out_bits;      // [ceil(n_atoms / 64)] fixpoint restricted to the first words
    int32_t *out_products;   // products; -1 if the product bound was exceeded; -2 if a team gave up
    uint64_t *xch;           // team programs: three delta buffers of n_words (new rows of product t in t mod 3)
    uint32_t *team;          // team programs: kTeamStateWords words of barrier and count state
    int32_t n_rows;
    int32_t n_atoms;
    int32_t n_or;
    int32_t n_segs;
    int32_t and_end;
    int32_t team_size;       // workgroups that solve this program together (1: one workgroup alone)
    int32_t long_nnz;        // entries of long_col
    int32_t pad;
};

// A program's layout copied into LDS after the two interpretation buffers
// (tp_batch_kernel, programs solved by one workgroup): byte offsets of the
// AND bitmask and first AND entry of every word, the AND lengths, the AND
// entries (with 64 * 16 entries of the zero padding, which chunk loads read
// past the last entry), the OR child ranges and rows, the long-row segments
// and their entries; `end` is the total. Every array starts 16-byte aligned.
struct LdsLayout {
    int64_t andb, base, len, col, or_c0, or_row, segs, long_col, end;
};
__host__ __device__ inline LdsLayout lds_layout(int64_t n_rows, int64_t and_end, int64_t n_or, int64_t n_segs,
                                                int64_t long_nnz) {
    const int64_t n_words = (n_rows + 63) >> 6;
    LdsLayout L;
    int64_t o = 0;
    L.andb = o;
    o += 8 * n_words;
    L.base = o;
    o = (o + 4 * n_words + 15) & ~(int64_t)15;
    L.len = o;
    o = (o + n_rows + 15) & ~(int64_t)15;
    L.col = o;
    o += 4 * (((and_end + 64 * 16) + 3) & ~(int64_t)3);
    L.or_c0 = o;
    o = (o + 4 * (n_or + 1) + 15) & ~(int64_t)15;
    L.or_row = o;
    o = (o + 4 * n_or + 15) & ~(int64_t)15;
    L.segs = o;
    o += (int64_t)sizeof(LongSeg) * n_segs;
    L.long_col = o;
    o = (o + 4 * long_nnz + 15) & ~(int64_t)15;
    L.end = o;
    return L;
}
// Team state: [0] barrier arrivals, [1] abort flag, [2..4] new-bit counts by
// product index mod 3; one 128-byte line per team. Zero between launches.
constexpr int kTeamStateWords = 32;
constexpr int kMaxTeam = 8;
struct BatchParams {
    const ProgDesc *progs;
    const int32_t *order;    // queue position -> program: team members first, then largest first
    const int32_t *member;   // queue position -> member index within the program's team
    unsigned int *queue;     // [0] next position, [1] finished workgroups; zero between launches
    uint32_t *teams;         // n_teams x kTeamStateWords, reset by the last workgroup to finish
    int32_t n_items;         // queue positions
    int32_t n_teams;
    int32_t lds_words;       // words of each of the two LDS buffers
    uint32_t team_polls;     // polls after which a team barrier gives up
    int32_t lds_layout_bytes;// dynamic LDS after the two buffers for a program's layout (0: none)
    int32_t single;          // 1: one program, described by `one` (no queue, grid of one workgroup)
    ProgDesc one;
};
// One small program by tp_tiny_kernel (every lane keeps its rows in
// registers): at most kTinyWords words of 64 rows, kTinyOr OR rows, no long
// rows, and its layout in LDS beside the two buffers.
constexpr int kTinyBlock = 1024;
constexpr int kTinyWords = 64;
constexpr int kTinyOr = 2048;
bool tiny_fits(int64_t n_rows, int64_t n_or, int64_t n_segs);
hipError_t launch_tiny(const ProgDesc &pd, int32_t lds_words, size_t lds_bytes, hipStream_t st);
bool batch_shape_supported(int wpw, int unroll);
hipError_t launch_batch(int wpw, int unroll, int grid, int block, size_t lds_bytes, const BatchParams &b,
                        hipStream_t st);
hipError_t batch_occupancy(int wpw, int unroll, int block, size_t lds_bytes, int *blocks_per_cu);
void batch_kernels_allow_lds(int max_dynamic_lds);

// Stable models (interpretation matrix with W = 2^log2W words per row).
struct SpmmParams {
    const int32_t *row_ptr;
    const int32_t *col;
    const uint64_t *and_bits;  // AND rows of the full matrix
    const uint64_t *V;
    uint64_t *U;
    unsigned long long *counters;  // ring: bit count of the product's result, slot 0 the initial matrix's
    int64_t total;  // n_rows << log2W
    int32_t log2W;
    int32_t step;
    int32_t early_exit;
};
// max_grid: workgroups of 256 threads (grid-stride loop over the items).
hipError_t launch_spmm_step(const SpmmParams &p, int max_grid, hipStream_t st);
// Stable-model products by dirty rows (lp_spmm.hip): one launch per product
// t; see spmm_dirty_product_kernel.
constexpr int kDirtyHist = 128;  // |C_t| by t mod kDirtyHist, read by the host
struct DirtyParams {
    const int32_t *row_ptr;
    const int32_t *col;
    const uint64_t *and_bits;
    const int32_t *occ_ptr;      // transposed matrix: rows naming each row
    const int32_t *occ;
    const uint64_t *V;           // v_{t-1}
    uint64_t *U;                 // result of product t (holds v_{t-2} on entry)
    // row bitmaps (bit r & 31 of word r >> 5), nb words each
    const uint32_t *dcur;        // D_t
    uint32_t *dnext;             // D_{t+1}, set in product t
    uint32_t *dclear;            // D_{t+2}'s, cleared in product t
    const uint32_t *cprev;       // C_{t-1}
    uint32_t *ccur;              // C_t, set in product t
    uint32_t *cclear;            // C_{t+1}'s, cleared in product t
    uint32_t *call;              // rows changed in any product so far
    int32_t *hist;               // [kDirtyHist] 1 iff product t changed a row, by t mod kDirtyHist
    const uint64_t *fact_bits;   // fact rows (constant, like the qbar rows from n_std on)
    int64_t nb;
    int32_t n_rows;
    int32_t n_std;
    int32_t log2W;
    int32_t step;
    int32_t wpi;                 // bitmap words per wave at a time (narrow rows), 1..8
};
hipError_t launch_dirty_product(const DirtyParams &p, int max_grid, hipStream_t st);
// Rows changed during a solve back to 0 in both buffers, sets and history
// cleared (sets: [D0 | D1 | D2 | C0 | C1 | C2 | changed] of nb words, then the history).
hipError_t launch_dirty_reset(uint64_t *b0, uint64_t *b1, int32_t log2W, uint32_t *sets, int64_t nb, int max_grid,
                              hipStream_t st);
// D_1 from the fact rows (facts[0..n_facts)) and the qbar rows.
hipError_t launch_dirty_seed(const DirtyParams &p, const int32_t *facts, int32_t n_facts, int max_grid,
                             hipStream_t st);
// Frontier (semi-naive) least models: one launch per level. occ_ptr/occ is
// the transposed matrix (for each row, the rows whose entries name it); cnt
// holds each row's count of entries still false (an OR row starts at 1).
constexpr int kFrontierRing = 4;     // frontier sizes, indexed by level % kFrontierRing
constexpr int kFrontierHist = 256;   // |F_t| history, indexed by level % kFrontierHist
struct FrontierParams {
    const int32_t *occ_ptr;  // [n_rows + 1]
    const int32_t *occ;      // rows naming each row
    int32_t *cnt;            // [n_rows]
    uint64_t *v;             // [n_words] the interpretation (ORed into)
    const int32_t *in;       // F_level
    int32_t *out;            // F_level+1 (capacity n_rows)
    uint32_t *sizes;         // [kFrontierRing]
    int32_t *hist;           // [kFrontierHist]
    int32_t level;
};
hipError_t launch_frontier_level(const FrontierParams &f, int grid, hipStream_t st);
// Levels f.level .. f.level + n_levels - 1 in one workgroup of
// kFrontierLoopBlock threads (q0, q1: the two frontier buffers by level
// parity; facts: F_0); stops after an empty frontier or before one of more
// than kFrontierLoopCap rows; ctl[0] = first level not pushed.
constexpr int kFrontierLoopBlock = 1024;
constexpr int kFrontierLoopCap = 4096;
hipError_t launch_frontier_levels(const FrontierParams &f, const int32_t *facts, int32_t *q0, int32_t *q1,
                                  int32_t n_levels, int32_t *ctl, hipStream_t st);

// Many least models by frontier levels in one launch (lp_frontier.hip): each
// workgroup takes programs from a device queue and runs all of a program's
// levels itself, with a workgroup barrier between levels.
struct FBatchProg {
    const int32_t *occ_ptr;   // transposed matrix (rows naming each row)
    const int32_t *occ;
    const int32_t *cnt0;      // [n_rows] entries still false at the start
    const int32_t *facts;     // [n_facts] F_0
    int32_t *cnt;             // [n_rows] working counts
    uint64_t *v;              // [n_words] the fixpoint (fact bits and every row that fires)
    int32_t *out_products;    // products; -1 past n_rows + 1
    int32_t n_rows, n_facts, n_words, pad;
};
struct FBatchParams {
    const FBatchProg *progs;
    const int32_t *order;     // queue position -> program
    unsigned int *queue;      // [0] next position, [1] finished workgroups; zero between launches
    int32_t *qbuf;            // two frontier buffers of qcap rows per workgroup
    int64_t qcap;
    int32_t n_items;
    int32_t lds_rows;         // programs of at most this many rows keep counts and v in LDS (0: none)
};
constexpr int kFBatchBlock = 1024;
// Dynamic LDS of the frontier batch kernel: v (8 bytes per 64 rows), then the counts.
inline size_t fbatch_lds_bytes(int32_t lds_rows) {
    return lds_rows > 0 ? 8 * (size_t)((lds_rows + 63) / 64) + 4 * (size_t)lds_rows : 0;
}
hipError_t launch_frontier_batch(const FBatchParams &b, int grid, hipStream_t st);
void frontier_kernels_allow_lds(int max_dynamic_lds);

hipError_t launch_init_m0(uint64_t *V, uint64_t *U, int64_t total, int32_t log2W, int32_t n_std,
                          const uint64_t *fact_bits, const int32_t *guess_pos, int32_t k_eff,
                          unsigned long long *count, unsigned long long bits, hipStream_t st);
hipError_t launch_init_guess(uint64_t *V, uint64_t *U, int64_t total, int32_t log2W, int32_t n_std, int32_t K,
                             const uint64_t *fact_bits, const uint64_t *guesses, hipStream_t st);
hipError_t launch_next_guess(const uint64_t *V, int32_t log2W, int64_t n_cols, const int32_t *q_rows, int32_t K,
                             uint64_t *out, hipStream_t st);
hipError_t launch_stable_check(const uint64_t *V, int32_t log2W, int64_t W, const int32_t *q_rows, int32_t n_std,
                               int32_t K, int32_t k_eff, uint64_t *accept, unsigned long long *count,
                               hipStream_t st);
hipError_t launch_extract(const uint64_t *V, int32_t log2W, const int64_t *cols, int64_t n_models, int32_t n_atoms,
                          uint8_t *out, hipStream_t st);

// Stable models of several programs at once (lp_spmm.hip): every launch
// takes one product of Algorithm 2 for every program of the batch, over the
// union of their interpretation matrices. Each program's items (row-words)
// fill whole 256-item chunks from chunk0 on, so a chunk belongs to one
// program; a program whose previous product changed nothing is skipped.
constexpr int kSBatchChunk = 256;
struct SBatchProg {
    const int32_t *row_ptr;
    const int32_t *col;
    const uint64_t *and_bits;
    const uint64_t *fact_bits;
    const int32_t *guess_pos;
    const int32_t *q_rows;
    uint64_t *buf[2];          // product t reads buf[(t - 1) & 1] and writes buf[t & 1]
    unsigned long long *count; // kRing bit counts of the program's products, slot 0 the initial matrix's
    uint64_t *accepted;        // W words: Algorithm 3's mask (compressed guess space)
    uint8_t *model;            // n_atoms bytes: the first accepted column's model
    unsigned long long *n_models;
    unsigned long long m0_bits;  // |M0| (closed form)
    int64_t chunk0;            // first chunk of the program
    int64_t total;             // n_rows << log2W
    int32_t n_rows, n_std, K, k_eff, log2W, n_atoms;
};
struct SBatchParams {
    const SBatchProg *progs;
    int32_t n_progs;
    int32_t step;
    int64_t n_chunks;
};
hipError_t launch_sbatch_init(const SBatchParams &b, int max_grid, hipStream_t st);
hipError_t launch_sbatch_step(const SBatchParams &b, int max_grid, hipStream_t st);
// Algorithm 3 and the first model of every program; b.step is the last product issued.
hipError_t launch_sbatch_outputs(const SBatchParams &b, hipStream_t st);

// Dense-matrix products (lp_dense.hip). The dense matrix is ld x ld bytes with
// ld = n_rows rounded up to kDenseAlign; interpretation matrices are hp x ld
// bytes (guess-major) with hp = 2^K rounded up to kDenseColAlign.
constexpr int64_t kDenseAlign = 1024;
constexpr int64_t kDenseColAlign = 128;
// A product with fewer than kDenseSplitTarget tiles of 128 x 128 is split
// along k into up to kDenseMaxSplits slices; dense_gemm_splits gives the
// count, and the caller passes a partial-count buffer of splits x hp x ld int32.
constexpr int kDenseMaxSplits = 8;
// The products' change counts: kDenseCounters counters, kDenseCounterStride
// words apart; a product changed nothing iff all are 0.
constexpr int kDenseCounters = 32;
constexpr int kDenseCounterStride = 16;
constexpr int64_t kDenseSplitTarget = 1024;
int dense_gemm_splits(int64_t ld, int64_t hp);
hipError_t launch_dense_scatter(uint8_t *M, int64_t ld, const int32_t *row_ptr, const int32_t *col, int32_t n_rows,
                                hipStream_t st);
hipError_t launch_dense_gemv(const uint8_t *M, int64_t ld, const uint8_t *v, uint8_t *u, const int32_t *thr,
                             unsigned long long *changed, hipStream_t st);
hipError_t launch_dense_gemm(const uint8_t *M, const uint8_t *Vt, uint8_t *Ut, int64_t ld, int64_t hp,
                             int32_t *partial, const int32_t *thr, unsigned long long *changed, hipStream_t st);
hipError_t launch_dense_init(uint8_t *V, int64_t ld, int64_t h, int64_t hp, const uint8_t *fact, int32_t n_std,
                             int32_t K, hipStream_t st);
hipError_t launch_dense_check(const uint8_t *V, int64_t ld, int64_t h, const int32_t *q_rows, int32_t n_std,
                              int32_t K, uint64_t *accept, unsigned long long *count, hipStream_t st);
hipError_t launch_dense_gather(const uint8_t *V, int64_t ld, const int64_t *cols, int64_t n, int32_t n_atoms,
                               uint8_t *out, hipStream_t st);

}  // namespace lp
