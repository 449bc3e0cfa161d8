// C ABI of the batched path (declared in include/spgemm.h, "batches").
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include <vector>

#include "../../include/spgemm.h"
#include "batched.hpp"

using namespace spg;

namespace {

constexpr size_t BA = 256;
inline size_t al(size_t x) { return (x + BA - 1) & ~(BA - 1); }

// Scratch: batch description, counters and per-row arrays.
struct ScratchLayout {
    size_t descs, pflop, pbound, pmax, pstatus, err, bcnt, bcur, boff;
    size_t pid, bin, kx, a0, a1, list, nnz, gpos, bsum, total;
};

ScratchLayout scratch_layout(int nprod, int64_t mtot) {
    ScratchLayout L{};
    const size_t np = (size_t)nprod, m = (size_t)mtot;
    size_t o = 0;
    L.descs = o; o += al(sizeof(BatchDesc) * np);
    L.pflop = o; o += al(8 * np);
    L.pbound = o; o += al(8 * np);
    L.pmax = o; o += al(8 * np);
    L.pstatus = o; o += al(4 * np);
    L.err = o; o += al(4);
    L.bcnt = o; o += al(4 * BAT_NB);
    L.bcur = o; o += al(4 * BAT_NB);
    L.boff = o; o += al(4 * BAT_NB);
    L.pid = o; o += al(4 * m);
    L.bin = o; o += al(m);
    L.kx = o; o += al(4 * m);
    L.a0 = o; o += al(4 * m);
    L.a1 = o; o += al(4 * m);
    L.list = o; o += al(16 * m);
    L.nnz = o; o += al(4 * m);
    L.gpos = o; o += al(8 * m);
    L.bsum = o; o += al(8 * ((m + 4095) / 4096 + 2));
    L.total = o;
    return L;
}

// Arena: the products' CSR arrays (K = sum of key bounds, an upper bound of
// the entries).
struct ArenaLayout {
    size_t orpts, ocols, ovals, total;
};

ArenaLayout arena_layout(int nprod, int64_t mtot, int64_t K) {
    ArenaLayout L{};
    size_t o = 0;
    L.orpts = o; o += al(8 * (size_t)(mtot + nprod));
    L.ocols = o; o += al(4 * (size_t)K);
    L.ovals = o; o += al(8 * (size_t)K);
    L.total = o;
    return L;
}

bool ok_csr(const spgemm_csr &a) {
    return a.nrows >= 0 && a.ncols >= 0 && a.nnz >= 0 && a.nrows < INT32_MAX && a.ncols < INT32_MAX &&
           a.nnz < INT32_MAX && a.rpts && (a.nnz == 0 || a.cols);
}

// Total rows, or -1 when a count is invalid or the batch exceeds int32 rows.
int64_t total_rows(int nprod, const spgemm_csr *A) {
    int64_t m = 0;
    for (int p = 0; p < nprod; ++p) {
        if (A[p].nrows < 0 || A[p].nrows >= INT32_MAX) return -1;
        m += A[p].nrows;
    }
    return m < INT32_MAX ? m : -1;
}

int device_cus() {
    static int ncu = 0;
    if (ncu == 0) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            ncu = n;
        else
            ncu = 256;
    }
    return ncu;
}

struct Views {
    const BatchDesc *d;
    BatchRows r;
    BatchCounters c;
};

Views views(char *s, const ScratchLayout &L) {
    Views v;
    v.d = (const BatchDesc *)(s + L.descs);
    v.r = BatchRows{(int32_t *)(s + L.pid), (uint8_t *)(s + L.bin), (uint32_t *)(s + L.kx), (int32_t *)(s + L.a0),
                    (int32_t *)(s + L.a1)};
    v.c = BatchCounters{(unsigned long long *)(s + L.pflop), (unsigned long long *)(s + L.pbound),
                        (unsigned long long *)(s + L.pmax), (int *)(s + L.pstatus), (unsigned *)(s + L.err),
                        (unsigned *)(s + L.bcnt), (unsigned *)(s + L.bcur), (unsigned *)(s + L.boff)};
    return v;
}

}  // namespace

extern "C" {

size_t spgemm_batch_scratch_bytes(int nprod, const spgemm_csr *A) {
    if (nprod <= 0 || !A) return 0;
    const int64_t m = total_rows(nprod, A);
    if (m < 0) return 0;
    return scratch_layout(nprod, m).total;
}

int spgemm_batch_prepare(int nprod, const spgemm_csr *A, const spgemm_csr *B, const unsigned *flags,
                         void *scratch, hipStream_t stream) {
    if (nprod <= 0 || !A || !B || !scratch) return SPGEMM_ERR_INVALID_ARG;
    if (total_rows(nprod, A) < 0) return SPGEMM_ERR_INVALID_ARG;
    std::vector<BatchDesc> d((size_t)nprod);
    int64_t off = 0;
    for (int p = 0; p < nprod; ++p) {
        if (!ok_csr(A[p]) || !ok_csr(B[p])) return SPGEMM_ERR_INVALID_ARG;
        if (A[p].ncols != B[p].nrows) return SPGEMM_ERR_SHAPE;
        const unsigned f = flags ? flags[p] : 0u;
        if (f & ~(unsigned)SPGEMM_SORTED) return SPGEMM_ERR_INVALID_ARG;
        d[p] = BatchDesc{off, (int32_t)A[p].nrows, (int32_t)B[p].ncols, f, 0, A[p].rpts, A[p].cols, A[p].vals,
                         B[p].rpts, B[p].cols, B[p].vals};
        off += A[p].nrows;
    }
    const ScratchLayout L = scratch_layout(nprod, off);
    const hipError_t e = hipMemcpyAsync((char *)scratch + L.descs, d.data(), sizeof(BatchDesc) * (size_t)nprod,
                                        hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return SPGEMM_ERR_HIP;
    // the host array must outlive the copy
    return hipStreamSynchronize(stream) == hipSuccess ? SPGEMM_OK : SPGEMM_ERR_HIP;
}

int spgemm_batch_analyse(int nprod, const spgemm_csr *A, void *scratch, int64_t *flop, int64_t *bound,
                         int64_t *max_key, hipStream_t stream) {
    if (nprod <= 0 || !A || !scratch || !flop || !bound) return SPGEMM_ERR_INVALID_ARG;
    const int64_t mtot = total_rows(nprod, A);
    if (mtot < 0) return SPGEMM_ERR_INVALID_ARG;
    const ScratchLayout L = scratch_layout(nprod, mtot);
    char *s = (char *)scratch;
    const Views v = views(s, L);
    hipError_t e = launch_batch_analyse(v.d, nprod, mtot, v.r, v.c, (int4 *)(s + L.list), (uint32_t *)(s + L.nnz),
                                        stream);
    if (e != hipSuccess) return SPGEMM_ERR_HIP;
    std::vector<unsigned long long> h(3 * (size_t)nprod);
    // pflop, pbound and pmax are laid out one after another (each 256-aligned)
    const size_t n8 = 8 * (size_t)nprod;
    e = hipMemcpyAsync(h.data(), s + L.pflop, n8, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data() + nprod, s + L.pbound, n8, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data() + 2 * nprod, s + L.pmax, n8, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return SPGEMM_ERR_HIP;
    for (int p = 0; p < nprod; ++p) {
        flop[p] = (int64_t)h[p];
        // a product with a row out of range takes no arena (its rows are skipped)
        bound[p] = h[2 * nprod + p] > (unsigned long long)BATCH_XMAX ? 0 : (int64_t)h[nprod + p];
        if (max_key) max_key[p] = (int64_t)h[2 * nprod + p];
    }
    return SPGEMM_OK;
}

int spgemm_batch_bin_rows(int nprod, const spgemm_csr *A, void *scratch, int64_t *rows, hipStream_t stream) {
    if (nprod <= 0 || !A || !scratch || !rows) return SPGEMM_ERR_INVALID_ARG;
    const int64_t mtot = total_rows(nprod, A);
    if (mtot < 0) return SPGEMM_ERR_INVALID_ARG;
    const ScratchLayout L = scratch_layout(nprod, mtot);
    unsigned h[BAT_NB];
    hipError_t e = hipMemcpyAsync(h, (char *)scratch + L.bcnt, sizeof(h), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return SPGEMM_ERR_HIP;
    for (int b = 0; b < BAT_NB; ++b) rows[b] = (int64_t)h[b];
    return SPGEMM_OK;
}

size_t spgemm_batch_arena_bytes(int nprod, const spgemm_csr *A, const int64_t *bound) {
    if (nprod <= 0 || !A || !bound) return 0;
    const int64_t mtot = total_rows(nprod, A);
    if (mtot < 0) return 0;
    int64_t K = 0;
    for (int p = 0; p < nprod; ++p) {
        if (bound[p] < 0) return 0;
        K += bound[p];
    }
    return arena_layout(nprod, mtot, K).total;
}

int spgemm_batch_run(int nprod, const spgemm_csr *A, spgemm_dtype dtype, const int64_t *bound, void *scratch,
                     void *arena, size_t arena_bytes, spgemm_batch_result *results, hipStream_t stream) {
    if (nprod <= 0 || !A || !bound || !scratch || !results) return SPGEMM_ERR_INVALID_ARG;
    if (dtype != SPGEMM_F64 && dtype != SPGEMM_I64) return SPGEMM_ERR_INVALID_ARG;
    const int64_t mtot = total_rows(nprod, A);
    if (mtot < 0) return SPGEMM_ERR_INVALID_ARG;
    int64_t K = 0;
    for (int p = 0; p < nprod; ++p) {
        if (bound[p] < 0) return SPGEMM_ERR_INVALID_ARG;
        K += bound[p];
    }
    const ScratchLayout L = scratch_layout(nprod, mtot);
    const ArenaLayout R = arena_layout(nprod, mtot, K);
    if (!arena || arena_bytes < R.total) return SPGEMM_ERR_WORKSPACE;
    char *s = (char *)scratch;
    char *a = (char *)arena;
    const Views v = views(s, L);
    BatchBufs w;
    w.list = (int4 *)(s + L.list);
    w.bsum = (long long *)(s + L.bsum);
    w.gpos = (int64_t *)(s + L.gpos);
    w.nnz = (uint32_t *)(s + L.nnz);
    w.K = K;
    w.ocols = (int32_t *)(a + R.ocols);
    w.ovals = a + R.ovals;
    w.orpts = (int64_t *)(a + R.orpts);
    w.rpts_base = (int64_t)R.orpts;
    w.cols_base = (int64_t)R.ocols;
    w.vals_base = (int64_t)R.ovals;
    const hipError_t e = launch_batch_run((int)dtype, v.d, nprod, mtot, v.r, v.c, w, results, stream, device_cus());
    return e == hipSuccess ? SPGEMM_OK : SPGEMM_ERR_HIP;
}

}  // extern "C"
