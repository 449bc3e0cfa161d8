// Internal interface between the C ABI layer and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "config.hpp"

namespace spg {

struct CsrDev {
    int64_t nrows, ncols, nnz;
    const int32_t *rpts;
    const int32_t *cols;
    const void *vals;
};

struct BinOffsets {
    int64_t v[NSB > NNB ? NSB : NNB];
};


hipError_t launch_validate(const CsrDev &a, int *err, hipStream_t s);
hipError_t launch_row_flop(const CsrDev &A, const CsrDev &B, uint32_t *flop, int32_t *longl, int32_t *huge,
                           PlanHdr *hdr, const BinLimits &L, int ncu, hipStream_t s);
hipError_t launch_sym_scatter(int m, const uint32_t *flop, const int32_t *rA, int64_t ncolsB, const BinOffsets &off,
                              int32_t *perm, int2 *prow, int32_t *nnz_row, int32_t *slot_of, WsHdr *wh,
                              const BinLimits &L, hipStream_t s);
hipError_t launch_sym_bin(int bin, unsigned nrows, const int32_t *perm, const int2 *prow, int64_t off, const CsrDev &A,
                          const CsrDev &B, int32_t *nnz_row, WsHdr *wh, HashCfg hc, int ncu, hipStream_t s);
hipError_t launch_sym_segments(unsigned nbm, const int32_t *perm, int64_t off, const CsrDev &A, const CsrDev &B,
                               int nchunks, uint32_t *chunk_cnt, int32_t *nnz_row, uint32_t *bmap, WsHdr *wh,
                               int ncu, hipStream_t s);
hipError_t launch_scan(const int32_t *nnz_row, int m, long long *bsum, int64_t *rpts_C, WsHdr *wh,
                       hipStream_t s);
hipError_t launch_num_reset(WsHdr *wh, hipStream_t s);
hipError_t launch_num_hist(int m, const int32_t *nnz_row, const uint32_t *flop, const int32_t *rA,
                           const int32_t *slot_of, HeavyRow *heavy, WsHdr *wh, const BinLimits &L, hipStream_t s);
hipError_t launch_count_long_b(const CsrDev &B, PlanHdr *hdr, hipStream_t s);
hipError_t launch_windows(unsigned nheavy_max, const HeavyRow *heavy, int nchunks, const uint32_t *chunk_cnt,
                          const int64_t *rpts_C, const int32_t *rA, uint32_t *whist, uint32_t *wcur, WinItem *items,
                          unsigned cap, WsHdr *wh, hipStream_t s);
hipError_t launch_bucket(const CsrDev &B, int32_t *bc, int32_t *bperm, int32_t *bs, int32_t *long_id,
                         int32_t *long_list, int32_t *idx, int nchunks, WsHdr *wh, hipStream_t s);
hipError_t launch_gather_vals(int dtype, int64_t n, const int32_t *bperm, const void *vB, void *bv, hipStream_t s);
hipError_t launch_num_scatter(int m, const int32_t *nnz_row, const uint32_t *flop, const int32_t *rA,
                              const int64_t *rpts_C, const BinOffsets &off, NumRow *rows, WsHdr *wh,
                              const BinLimits &L, hipStream_t s);
hipError_t launch_check_sorted(const CsrDev &B, int *err, hipStream_t s);
hipError_t launch_num_heap(int dtype, unsigned nrows, const NumRow *rows, int64_t off, const CsrDev &A,
                           const CsrDev &B, int32_t *cC, void *vC, WsHdr *wh, hipStream_t s);
hipError_t launch_num_bin(int bin, int dtype, bool sorted, unsigned nrows, const NumRow *rows, int64_t off,
                          const CsrDev &A, const CsrDev &B, int32_t *cC, void *vC, WsHdr *wh, HashCfg hc, int ncu,
                          hipStream_t s);
hipError_t launch_num_window(int dtype, unsigned nitems, const WinItem *items, const CsrDev &A, const int2 *ki,
                             const int32_t *idx, int nchunks, const int32_t *bc, const void *bv, int32_t *cC,
                             void *vC, const uint32_t *bmap, WsHdr *wh, int ncu, hipStream_t s);
hipError_t launch_entry_brow(const CsrDev &A, const CsrDev &B, const int32_t *long_id, int2 *ki, hipStream_t s);
hipError_t launch_masked_product(const CsrDev &A, const CsrDev &B, const CsrDev &M, bool ones, unsigned *next_row,
                                 int64_t *out, int ncu, hipStream_t s);
hipError_t launch_masked_sum(int64_t m, int64_t ncols, const int64_t *rC, const int32_t *cC, const int64_t *vC,
                             const CsrDev &M, int64_t *out, hipStream_t s);
hipError_t launch_stream_copy(void *dst, const void *src, size_t nbytes, hipStream_t s);
hipError_t launch_stanza_read(const void *base, int64_t nwords, const int64_t *start, int64_t nst, int lw,
                              unsigned long long *sum, unsigned long long *skipped, int ncu, hipStream_t s);

}  // namespace spg
