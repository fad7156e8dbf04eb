// lp_internal.h -- host-side structures shared by the matrix builder
// (lp_build.cpp) and the device runtime (lp_device.hip). Not part of the ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "lp.h"

namespace lp {

// Rows longer than this leave the 64-row block pass of the least-model step
// and are evaluated by split segments (one workgroup per segment).
constexpr int32_t kLongRow = 256;
constexpr int32_t kSegLen = 4096;

// Device-resident form of one matrix. All pointers are device memory owned
// by the matrix (released by lp_free_matrix).
struct DeviceMatrix {
    // Least-model (SpMV) layout: 64-row block CSR with long rows emptied, plus
    // a segment list for the long rows.
    int32_t *row_ptr = nullptr;   // [n_rows+1]
    int32_t *col = nullptr;       // [short nnz]
    uint64_t *and_bits = nullptr; // [n_words]; bit = 1: AND row (long rows cleared)
    uint64_t *fact_bits = nullptr;// [n_words]; initial vector
    void *segs = nullptr;         // LongSeg[n_segs]
    int32_t *long_col = nullptr;  // [long nnz]
    int32_t n_segs = 0;
    int32_t n_long_and = 0;
    int64_t short_nnz = 0, long_nnz = 0;
    // Stable-model (SpMM) layout: plain CSR.
    int32_t *full_row_ptr = nullptr;
    int32_t *full_col = nullptr;
    int32_t *q_rows = nullptr;    // [K] row ids of q_t
    int32_t *guess_pos = nullptr; // [K] bit of the compressed guess index, -1 if pruned
    int64_t bytes = 0;
    int device = -1;
};

struct LongSeg {
    int32_t row;
    int32_t is_and;
    int64_t begin;   // into long_col
    int32_t len;
    int32_t nseg;    // segments of this row
    int32_t and_slot;// index into the completion counts of split AND rows, -1 otherwise
    int32_t seg;     // index of this segment within its row
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

}  // namespace lp

struct lp_matrix {
    lp::Matrix m;
};
