// Internal interface of the batched path.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/spgemm.h"
#include "config.hpp"

namespace spg {

// Bins 1..BAT_TOP (LDS tables of the single-product path) are batched; rows
// of bin BAT_TOP+1 (key bound above WIN_CAP) are out of range.
constexpr int BAT_TOP = 9;
constexpr int BAT_NB = NSB;
constexpr int BATCH_XMAX = WIN_CAP;

// One product of a batch, as the device sees it.
struct BatchDesc {
    int64_t row_off;        // first global row
    int32_t m;              // rows of A
    int32_t ncolsB;         // columns of B (and C)
    uint32_t flags;         // bit 0: sorted output
    int32_t pad;
    const int32_t *rA, *cA;
    const void *vA;
    const int32_t *rB, *cB;
    const void *vB;
};

// Per-row arrays (global row space).
struct BatchRows {
    int32_t *pid;          // product of the row
    uint8_t *bin;          // bin of the row
    uint32_t *kx;          // key bound: min(flop, ncols) for batched rows, else 0
    int32_t *a0, *a1;      // the row's entries of A: [a0, a1)
};

// Per-product and per-bin counters.
struct BatchCounters {
    unsigned long long *pflop, *pbound, *pmax;
    int *pstatus;
    unsigned *err;
    unsigned *bcnt, *bcur, *boff;   // BAT_NB each
};

// Work buffers of a run (scratch and arena).
struct BatchBufs {
    int4 *list;            // rows by bin: {row, product, a0, a1}
    long long *bsum;       // scan block sums (+ total)
    int64_t *gpos;         // output offset per row
    uint32_t *nnz;         // row counts (symbolic phase)
    int64_t K;             // output capacity (entries): the sum of the bounds
    int32_t *ocols;
    void *ovals;
    int64_t *orpts;
    int64_t rpts_base, cols_base, vals_base;   // byte offsets of the outputs in the arena
};

// Row flop, bins and bin lists (once per batch structure).
hipError_t launch_batch_analyse(const BatchDesc *d, int nprod, int64_t mtot, const BatchRows &r,
                                const BatchCounters &c, int4 *list, uint32_t *nnz, hipStream_t s);
// Symbolic counts, their scan, numeric rows in place and results (every run;
// kernels only).
hipError_t launch_batch_run(int dtype, const BatchDesc *d, int nprod, int64_t mtot, const BatchRows &r,
                            const BatchCounters &c, const BatchBufs &w, spgemm_batch_result *res, hipStream_t s,
                            int ncu);

}  // namespace spg
