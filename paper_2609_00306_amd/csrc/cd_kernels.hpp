// Parameter blocks shared between the host entry points and the kernels.
#pragma once
#include <stdint.h>
#include "cd_device.hpp"

namespace cdk {

struct Step1Params {
    const RowRec *rows;        // [n_rows]
    const int32_t *act_row;    // [n_act] row of each active slot
    const int64_t *n_act_dev;  // device count of active rows (must equal n_act)
    int64_t n_act;
    double *D_act;             // [n_act] residual diagonal of the active rows
    double *LT_act;            // [n_act][ldT] vectors on the active rows, row-major
    int64_t ldT;               // row stride of LT_act (multiple of 16)
    const int64_t *n_rows_dev; // device count of rows (must equal n_rows)
    double *Cbuf;              // [QMAX][n_act] candidate columns of rows past the LDS copy
    double *Cblk;              // [QMAX][QMAX] candidate block, row i = candidate i
    Nom *noms;                 // [G][CNOM + 1]
    GridSync *gs;
    int64_t *pivots;           // [max_vectors] row index of each pivot
    int32_t *piv_slot;         // [max_vectors] active slot of each pivot
    double *dpiv;              // [max_vectors] pivot values d_K
    int32_t *pivot_of_row;     // [n_rows] vector index whose pivot is this row, or -1
    int64_t *n_vectors;        // [1]
    int32_t *status;           // [1]
    const int64_t *k_start;    // [1] vectors already formed (0, or M1 when resuming; < 0: skip)
    double *pivot_values;      // optional [max_vectors] output copy of dpiv
    double tau;
    const unsigned long long *d1max_bits;  // max D1 (bit pattern)
    int64_t n_rows;            // tau == 0: stop at max D <= n_rows 2^-53 max D1
    int64_t max_vectors;
    double eta;                // span factor: 1 = exact pivoting, < 1 = qualified-set acceptance
    int32_t q;                 // candidate batch size (<= QMAX)
    int32_t slice;             // at most this many active rows per workgroup (dealt round robin)
    uint32_t spin_limit;
    int64_t *timeline;         // optional: [timeline_cap][8] device clock stamps per batch
    int64_t *timeline_count;   // optional: number of batches
    int64_t timeline_cap;
};

// Up to kStep1Batch decompositions share one cooperative launch; problem i
// owns the workgroups [block_begin[i], block_begin[i + 1]) and its own
// barrier, so small molecules run side by side on the GPU.
constexpr int kStep1Batch = 16;
struct Step1Batch {
    int32_t count;
    int32_t block_begin[kStep1Batch + 1];
    Step1Params p[kStep1Batch];
};

// Pivot-row gather and pivot-block inverses of the problems of one
// pivot-selection launch, in one launch each.
struct PivotMol {
    const double *LT;          // active-row vectors, row-major
    int64_t ldT;
    const int32_t *piv_slot;
    const int64_t *pivots;
    const RowRec *rows;
    const int64_t *n_vectors;
    double *Lp;                // [max_vectors][ldp] pivot rows
    int64_t ldp;               // multiple of 16
    RowRec *prow;
    const double *dpiv;
    double *G;                 // inverse-transposed 64 x 64 pivot blocks
    double *Gf;                // inverse-transposed 128 x 128 pivot blocks, solve operand order
    const int64_t *k_start;    // [1] first vector to form (blocks start there)
};

struct PivotBatch {
    int32_t count;
    int32_t gather_begin[kStep1Batch + 1];    // workgroups of the gather, per problem
    int32_t inverse_begin[kStep1Batch + 1];   // workgroups of the block inverses
    int32_t g128_begin[kStep1Batch + 1];      // workgroups of the 128-block composition
    PivotMol m[kStep1Batch];
};

// All-row solve of up to kStep2Batch problems in one launch.
constexpr int kStep2Batch = 16;
struct Step2Mol {
    const RowRec *rows;
    int64_t n_rows;
    const RowRec *prow;
    const double *Lp;
    int64_t ldp;
    const double *Gf;     // [blocks][128 x 128] inverse-transposed pivot blocks (k_block_g128)
    const int32_t *pivot_of_row;
    const int64_t *n_vectors;
    double *L;
    double *diag;              // final residuals out; when resuming also the residuals in
    const int64_t *k_start;    // [1] first vector to form (< 0: nothing to do)
    int32_t resume;            // 1: start from the residuals in diag, else from D1
};
struct Step2Batch {
    int32_t count;
    int32_t tile_begin[kStep2Batch + 1];
    Step2Mol m[kStep2Batch];
    int64_t *timeline;   // optional stamps of the last problem's first tile
    int64_t tl_cap;
};

}  // namespace cdk
