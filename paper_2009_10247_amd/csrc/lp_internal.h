// lp_internal.h -- host-side structures shared by the matrix builder
// (lp_build.cpp) and the device runtime (lp_device.hip). Not part of the ABI.
#pragma once

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "lp.h"

namespace lp {

// Least-model device layout. Rows are grouped by 64 (one bit-packed word of
// v). Every row is one of: empty (never true), fact (true from the initial
// vector on, no work), AND (fires iff all of its entries are true) or OR
// (fires iff one child is true). AND bodies name only original atoms; the k
// children of an OR row are the consecutive new atoms of its head, so an OR
// row is a bit range of v and stores no column indices.
constexpr int32_t kLongAnd = 255;       // longer AND rows go to the segment pass
constexpr int32_t kLongOrBits = 512;    // longer OR rows go to the segment pass
constexpr int32_t kSegAnd = 4096;       // entries per AND segment
constexpr int32_t kSegOrBits = 16384;   // bits per OR segment
constexpr int32_t kColPad = 64 * 16;    // zero entries after col: chunk loads past the end stay in bounds
constexpr int32_t kWordPad = 16;        // empty words after the last: super-block loads past the end stay in bounds
constexpr int kBatchWpw = 8;            // default shape of the batch kernel: words per super-block
constexpr int kBatchUnroll = 16;        // and chunks of 64 entries per round

struct WordMeta {
    int32_t and_base;    // offset in col of the word's first AND entry
    int32_t or_idx;      // index in or_c0 of the word's first OR row
    uint64_t and_bits;   // AND rows evaluated by the block pass
    uint64_t or_bits;    // all OR rows (the block pass evaluates those not in long_bits)
    uint64_t long_bits;  // rows evaluated by the segment pass
};

struct LongSeg {
    int32_t row;
    int32_t is_and;
    int64_t begin;   // AND: offset in long_col; OR: first bit of the range in v
    int32_t len;     // AND: entries; OR: bits
    int32_t nseg;    // segments of this row
    int32_t and_slot;// index into the completion counts of split AND rows, -1 otherwise
    int32_t seg;     // index of this segment within its row
};

// Device-resident form of one matrix. All pointers are device memory owned
// by the matrix (released by lp_free_matrix).
// One column slice of a least-model layout: the AND entries of block AND
// rows whose columns lie in [64 first_word, 64 (first_word + lds_words)),
// stored as the layout stores them, with columns relative to the slice.
struct SliceLayout {
    const WordMeta *words;
    const uint8_t *and_len;
    const uint32_t *lens4;
    const int32_t *col;
    int32_t and_end;
    int32_t and_max_col;
    int32_t first_word;
    int32_t lds_words;
};
constexpr int kMaxSlices = 64;

struct DeviceMatrix {
    // least models (definite programs)
    WordMeta *words = nullptr;    // [n_words + kWordPad]
    uint8_t *and_len = nullptr;   // [(n_words + kWordPad) * 64] AND-row length in the block pass, 0 otherwise
    uint32_t *lens4 = nullptr;    // the same lengths by lane: entry 64 q + l holds rows 64 (4q + k) + l, k < 4,
                                  // one byte each (byte k), for the n_words + kWordPad words
    int32_t *col = nullptr;       // block AND entries in row order
    int32_t *or_c0 = nullptr;     // [n_or + 1] first child of each OR row, ascending rows
    int32_t *or_row = nullptr;    // [n_or] row id of each OR row, -1 if evaluated by segments
    uint64_t *fact_bits = nullptr;// [n_words] initial vector
    LongSeg *segs = nullptr;      // [n_segs]
    int32_t *long_col = nullptr;  // entries of long AND rows
    int32_t n_segs = 0;
    int32_t n_long_and = 0;
    int32_t n_or = 0;
    int32_t and_max_col = -1;     // largest column of a block AND entry
    int64_t and_nnz = 0, long_nnz = 0;
    int64_t stream_bytes = 0;     // bytes one full step streams from memory (layout arrays)
    std::vector<int32_t> word_base;  // host: first AND entry of each word, then the entry count [n_words + 1]
    // device splits of the block pass between waves, one per wave count
    // (created on first use by the step planner, under its lock)
    mutable std::vector<std::pair<int32_t, int32_t *>> wave_parts;
    // column-sliced layout of the block AND entries (when the original atoms
    // exceed a workgroup's LDS, or with LP_STEP_SLICES_SMALL): one layout per
    // slice of columns, each slice's word_base (host) and its wave splits by
    // (slice, wave count), and the block AND rows of every word
    std::vector<SliceLayout> slices;
    std::vector<std::vector<int32_t>> slice_base;
    mutable std::vector<std::pair<int64_t, int32_t *>> slice_parts;
    uint64_t *and_all = nullptr;
    // transposed matrix of the frontier driver (built on first use, under its lock)
    mutable int32_t *fr_ptr = nullptr;    // [n_rows + 1]
    mutable int32_t *fr_occ = nullptr;    // rows naming each row, ascending
    mutable int32_t *fr_cnt0 = nullptr;   // [n_rows] entries still false at the start: AND length, OR 1
    mutable int32_t *fr_facts = nullptr;  // fact rows (F_0)
    mutable int32_t fr_n_facts = 0;
    // device bytes of the structures above that were attached after the
    // upload (wave splits, transposed matrix, stable-solve plan), under the same lock
    mutable int64_t lazy_bytes = 0;
    // buffers and captured graph of stable-model solves by dirty rows, kept
    // between solves (created on first use)
    mutable struct StablePlan *splan = nullptr;
    // stable models (normal programs): plain CSR
    int32_t *full_row_ptr = nullptr;
    int32_t *full_col = nullptr;
    uint64_t *full_and_bits = nullptr;  // [n_words] AND rows
    int32_t *q_rows = nullptr;    // [K] row ids of q_t
    int32_t *guess_pos = nullptr; // [K] bit of the compressed guess index, -1 if pruned
    int64_t bytes = 0;
    int device = -1;
};

struct Matrix {
    int32_t n_atoms = 0, n_rules = 0, n_std = 0, n_rows = 0, K = 0, K_eff = 0;
    int64_t nnz = 0;
    uint32_t flags = 0;
    std::vector<int32_t> row_ptr, col;
    std::vector<uint8_t> kind, fact;
    std::vector<int32_t> neg_atoms;  // q_t, ascending
    std::vector<int32_t> guess_pos;  // per t
    lp_info info{};
    DeviceMatrix dev;
};

// Host builder: validation, dedupe, standardization, positive form, CSR.
lp_status build_host(int32_t n_atoms, int32_t n_rules, const int32_t *head, const int64_t *body_ptr,
                     const int32_t *body_lit, uint32_t flags, Matrix *m);

void set_error(const std::string &msg);

// Largest matrix (rows) whose two bit-packed buffers fit in the batch
// kernel's LDS on `device` (0 if the device cannot be queried).
int64_t batch_max_rows(int device);

}  // namespace lp

struct lp_matrix {
    lp::Matrix m;
};
