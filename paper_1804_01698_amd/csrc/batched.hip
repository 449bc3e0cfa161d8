// Batched products: many small C[p] = A[p]*B[p] through a fixed sequence of
// launches shared by the whole batch, with no host synchronisation inside
// (the sequence can be captured in a HIP graph and replayed).
//
// Rows of all products form one global row space (product p owns rows
// [row_off[p], row_off[p+1])).  Every row is put in a bin by its key bound
// x = min(row flop, ncols) (Fig. 4's row flop, capped by the width of C), with
// the same table sizes as the single-product path.  The two phases of Section
// 2 then run on the device for the whole batch: a persistent kernel per bin
// counts each row's distinct columns in a keys-only LDS table, one scan of the
// counts gives every row its place in C, and a persistent kernel per bin
// accumulates each row in an LDS table of keys and values and writes it there
// (sorted when its product asks for it).  The caller sizes the arena from the
// bounds x (an upper bound of nnz(C)) before the run, so the run itself
// allocates nothing and needs no host round trip.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "batched.hpp"
#include "config.hpp"
#include "device.hpp"

namespace spg {

__device__ __forceinline__ int prod_of(const BatchDesc *__restrict__ d, int nprod, int64_t g) {
    int lo = 0, hi = nprod - 1;      // last p with d[p].row_off <= g
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].row_off <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_bat_zero(BatchCounters c, int nprod) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < nprod) { c.pflop[p] = 0; c.pbound[p] = 0; c.pmax[p] = 0; c.pstatus[p] = 0; }
    if (p < BAT_NB) { c.bcnt[p] = 0; c.bcur[p] = 0; }
    if (p == 0) *c.err = 0;
}

__global__ void k_bat_reset_err(unsigned *err) {
    if (threadIdx.x == 0) *err = 0;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long x) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        const unsigned long long y = __shfl_xor(x, d);
        x = y > x ? y : x;
    }
    return x;
}

// Row flop (Fig. 4 part 1), key bound and bin of every row of every product,
// per-product totals and per-bin row counts.  Eight lanes per row; a wave
// whose rows all belong to one product adds its totals with one atomic each.
__global__ __launch_bounds__(256) void k_bat_flop(const BatchDesc *__restrict__ d, int nprod, int64_t mtot,
                                                  BatchRows r, BatchCounters c) {
    __shared__ unsigned hist[BAT_NB];
    if (threadIdx.x < BAT_NB) hist[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, sub = lane & 7;
    const int64_t gw = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t wb = gw * 8; wb < mtot; wb += nw * 8) {        // uniform over the wave
        const int64_t g = wb + (lane >> 3);
        const bool valid = g < mtot;
        int p = 0, a0 = 0, a1 = 0, ncols = 0;
        unsigned long long f = 0;
        if (valid) {
            p = prod_of(d, nprod, g);
            const BatchDesc &q = d[p];
            const int i = (int)(g - q.row_off);
            ncols = q.ncolsB;
            a0 = q.rA[i];
            a1 = q.rA[i + 1];
            for (int e = a0 + sub; e < a1; e += 8) {
                const int k = q.cA[e];
                f += (unsigned long long)(q.rB[k + 1] - q.rB[k]);
            }
        }
        f += __shfl_xor(f, 1);
        f += __shfl_xor(f, 2);
        f += __shfl_xor(f, 4);
        const unsigned long long x = f < (unsigned long long)ncols ? f : (unsigned long long)ncols;
        const int b = sym_bin(f, ncols);             // 0 empty, 1..9 tables, 10 out of range
        const bool lead = valid && sub == 0;
        if (lead) {
            r.pid[g] = p;
            r.bin[g] = (uint8_t)b;
            r.kx[g] = (b >= 1 && b <= BAT_TOP) ? (uint32_t)x : 0u;
            r.a0[g] = a0;
            r.a1[g] = a1;
            atomicAdd(&hist[b], 1u);
        }
        unsigned long long cf = lead ? f : 0ull;
        unsigned long long cb = (lead && b <= BAT_TOP) ? x : 0ull;
        unsigned long long cm = lead ? x : 0ull;
        const int p0 = __shfl(p, 0);
        if (__all(!valid || p == p0)) {
            cf = wave_sum_u64(cf);
            cb = wave_sum_u64(cb);
            cm = wave_max_u64(cm);
            if (lane == 0 && cf) {
                atomicAdd(&c.pflop[p0], cf);
                atomicAdd(&c.pbound[p0], cb);
                atomicMax(&c.pmax[p0], cm);
            }
        } else if (lead && f) {
            atomicAdd(&c.pflop[p], cf);
            atomicAdd(&c.pbound[p], cb);
            atomicMax(&c.pmax[p], cm);
        }
    }
    __syncthreads();
    if (threadIdx.x < BAT_NB && hist[threadIdx.x]) atomicAdd(&c.bcnt[threadIdx.x], hist[threadIdx.x]);
}

__global__ void k_bat_binscan(BatchCounters c) {
    if (threadIdx.x == 0) {
        unsigned s = 0;
        for (int b = 0; b < BAT_NB; ++b) { c.boff[b] = s; s += c.bcnt[b]; }
    }
}

// Rows go to their bin's list as {row, product, A range}; empty rows and all
// rows of a product with a row out of range get count 0 (the latter mark
// their product unsupported).  bcur ends as the number of rows listed per bin.
__global__ __launch_bounds__(256) void k_bat_scatter(int64_t mtot, BatchRows r, BatchCounters c,
                                                     int4 *__restrict__ list, uint32_t *__restrict__ nnz) {
    __shared__ unsigned hist[BAT_NB], base[BAT_NB];
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (threadIdx.x < BAT_NB) hist[threadIdx.x] = 0;
    __syncthreads();
    int b = -1;
    unsigned rank = 0;
    if (g < mtot) {
        b = r.bin[g];
        const int p = r.pid[g];
        // a product with any row out of range is left to the caller whole
        const bool skip = c.pmax[p] > (unsigned long long)BATCH_XMAX;
        if (b >= 1 && b <= BAT_TOP && !skip) {
            rank = atomicAdd(&hist[b], 1u);
        } else {
            nnz[g] = 0;
            r.kx[g] = 0u;
            if (skip) c.pstatus[p] = SPGEMM_ERR_UNSUPPORTED;
            b = -1;
        }
    }
    __syncthreads();
    if (threadIdx.x >= 1 && threadIdx.x <= BAT_TOP && hist[threadIdx.x])
        base[threadIdx.x] = c.boff[threadIdx.x] + atomicAdd(&c.bcur[threadIdx.x], hist[threadIdx.x]);
    __syncthreads();
    if (b >= 1 && b <= BAT_TOP) list[base[b] + rank] = make_int4((int)g, r.pid[g], r.a0[g], r.a1[g]);
}

// Exclusive scan of per-row 32-bit counts into 64-bit offsets (3 launches).
__global__ __launch_bounds__(1024) void k_bat_scan_reduce(const uint32_t *__restrict__ x, int64_t n,
                                                          long long *__restrict__ bsum) {
    __shared__ long long ws[17];
    const int64_t base = (int64_t)blockIdx.x * 4096;
    long long s = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t i = base + j * 1024 + threadIdx.x;
        if (i < n) s += x[i];
    }
    long long tot;
    block_excl_scan<1024, long long>(s, tot, ws);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_bat_scan_top(long long *__restrict__ bsum, int nb) {
    __shared__ long long ws[17];
    long long carry = 0;
    for (int c0 = 0; c0 < nb; c0 += 1024) {
        const int i = c0 + (int)threadIdx.x;
        const long long v = i < nb ? bsum[i] : 0;
        long long tot;
        const long long ex = block_excl_scan<1024, long long>(v, tot, ws);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(1024) void k_bat_scan_down(const uint32_t *__restrict__ x, int64_t n,
                                                        const long long *__restrict__ bsum,
                                                        int64_t *__restrict__ out) {
    __shared__ long long ws[17];
    const int64_t base = (int64_t)blockIdx.x * 4096 + (int64_t)threadIdx.x * 4;
    long long v[4], s = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        v[j] = base + j < n ? x[base + j] : 0;
        s += v[j];
    }
    long long tot;
    long long run = block_excl_scan<1024, long long>(s, tot, ws) + bsum[blockIdx.x];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
}

// Symbolic phase of one bin, a block of G threads per row (persistent over
// the bin's list): the row's distinct columns are counted in a keys-only LDS
// hash table of T slots (Section 4.2.1), as in the single-product path.
template <int G, int T, int U>
__global__ __launch_bounds__(G) void k_bat_sym(const BatchDesc *__restrict__ d, int bin, BatchCounters c,
                                               const int4 *__restrict__ list, uint32_t *__restrict__ nnz) {
    __shared__ __align__(16) int keys[T];
    __shared__ SegLds<G, false, double> sg;
    const int tid = threadIdx.x;
    const unsigned n = c.bcur[bin];             // rows actually listed
    const int4 *lst = list + c.boff[bin];
    int ovf = 0;
    for (unsigned it = blockIdx.x; it < n; it += gridDim.x) {
        const int4 rec = lst[it];                 // row, product, A range
        const BatchDesc &q = d[rec.y];
        table_clear<G, T, false, double>(keys, nullptr);
        __syncthreads();
        int cnt = 0;
        enum_row<G, U, false, double>(
            rec.z, rec.w, q.cA, nullptr, sg,
            [&](int k, int &lo, int &hi) { lo = q.rB[k]; hi = q.rB[k + 1]; },
            [&](const int (&qq)[U], const bool (&ok)[U], const double (&)[U]) {
                int col[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int cb = q.cB[qq[u]];           // qq is always a valid index
                    col[u] = ok[u] ? cb : 0;
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (ok[u]) cnt += bkt_insert<false, double, 1>(keys, nullptr, T, col[u], 0.0, ovf);
            });
        __syncthreads();
        int total;
        block_excl_scan<G, int>(cnt, total, sg.wsum);
        if (tid == 0) nnz[rec.x] = (uint32_t)total;
        __syncthreads();
    }
    if (ovf) atomicOr(c.err, (unsigned)ERR_PROBE);
}

// Numeric phase of one bin: the row is accumulated into an LDS table of keys
// and values and leaves the table straight for its place in C (gpos, the scan
// of the symbolic counts), sorted when its product asks for it.  A row whose
// place runs past the arena's capacity of cap_total entries (operands changed
// since the arena was sized) is not written and flags an error.
template <int G, int T, int U, typename V>
__global__ __launch_bounds__(G) void k_bat_num(const BatchDesc *__restrict__ d, int bin, BatchCounters c,
                                               const int4 *__restrict__ list, const uint32_t *__restrict__ nnz,
                                               const int64_t *__restrict__ gpos, int64_t cap_total,
                                               int32_t *__restrict__ ocols, V *__restrict__ ovals) {
    __shared__ __align__(16) int keys[T];
    __shared__ __align__(16) V vals[T];
    __shared__ SegLds<G, true, V> sg;
    const unsigned n = c.bcur[bin];
    const int4 *lst = list + c.boff[bin];
    int ovf = 0;
    for (unsigned it = blockIdx.x; it < n; it += gridDim.x) {
        const int4 rec = lst[it];
        const int64_t g = rec.x;
        const BatchDesc &q = d[rec.y];
        const int64_t o = gpos[g];
        const int cnt = (int)nnz[g];
        table_clear<G, T, true, V>(keys, vals);
        __syncthreads();
        const V *vB = (const V *)q.vB;
        enum_row<G, U, true, V>(
            rec.z, rec.w, q.cA, (const V *)q.vA, sg,
            [&](int k, int &lo, int &hi) { lo = q.rB[k]; hi = q.rB[k + 1]; },
            [&](const int (&qq)[U], const bool (&ok)[U], const V (&av)[U]) {
                int col[U];
                V xv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int cb = q.cB[qq[u]];           // qq is always a valid index
                    const V b = vB[qq[u]];
                    col[u] = ok[u] ? cb : 0;
                    xv[u] = ok[u] ? av[u] * b : V(0);
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (ok[u]) bkt_insert<true, V, 1>(keys, vals, T, col[u], xv[u], ovf);
            });
        __syncthreads();
        const int expected = o + cnt <= cap_total ? cnt : 0;
        if (q.flags & 1u)
            compact_store<G, T, true, V>(keys, vals, sg.wsum, o, expected, ocols, ovals, (int *)c.err);
        else
            compact_store_unsorted<G, T, V>(keys, vals, sg.wsum, o, expected, ocols, ovals, (int *)c.err);
        __syncthreads();
    }
    if (ovf) atomicOr(c.err, (unsigned)ERR_PROBE);
}

// Per-product row pointers (relative to the product's first entry).  Slots:
// product p owns [row_off[p] + p, row_off[p] + m[p] + p] of the region.
__global__ __launch_bounds__(256) void k_bat_rpts(const BatchDesc *__restrict__ d, int nprod, int64_t mtot,
                                                  const int32_t *__restrict__ pid,
                                                  const int64_t *__restrict__ gpos, const long long *tot,
                                                  int64_t *__restrict__ orpts) {
    const int64_t total = *tot;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < mtot + nprod; g += stride) {
        if (g < mtot) {
            const int p = pid[g];
            orpts[g + p] = gpos[g] - gpos[d[p].row_off];
        } else {
            const int p = (int)(g - mtot);
            const int64_t end = p + 1 < nprod ? d[p + 1].row_off : mtot;
            const int64_t first = d[p].row_off < mtot ? gpos[d[p].row_off] : total;
            const int64_t last = end < mtot ? gpos[end] : total;
            orpts[end + p] = last - first;
        }
    }
}

__global__ __launch_bounds__(256) void k_bat_results(const BatchDesc *__restrict__ d, int nprod, int64_t mtot,
                                                     const int64_t *__restrict__ gpos, const long long *tot,
                                                     BatchCounters c, int64_t rpts_base, int64_t cols_base,
                                                     int64_t vals_base, spgemm_batch_result *__restrict__ res) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= nprod) return;
    const int64_t total = *tot;
    const int64_t r0 = d[p].row_off;
    const int64_t r1 = p + 1 < nprod ? d[p + 1].row_off : mtot;
    const int64_t first = r0 < mtot ? gpos[r0] : total;
    const int64_t last = r1 < mtot ? gpos[r1] : total;
    spgemm_batch_result r;
    r.flop = (int64_t)c.pflop[p];
    r.nnz = last - first;
    r.rpts_off = rpts_base + (r0 + p) * 8;
    r.cols_off = cols_base + first * 4;
    r.vals_off = vals_base + first * 8;
    r.status = c.pstatus[p] != 0 ? c.pstatus[p] : (*c.err ? SPGEMM_ERR_INTERNAL : SPGEMM_OK);
    r.pad = 0;
    res[p] = r;
}

static inline unsigned g256(int64_t n) { return (unsigned)((n + 255) / 256); }

static hipError_t scan_u32(const uint32_t *x, int64_t n, long long *bsum, int64_t *out, hipStream_t s) {
    const int nb = (int)((n + 4095) / 4096);
    if (nb > 0) k_bat_scan_reduce<<<nb, 1024, 0, s>>>(x, n, bsum);
    k_bat_scan_top<<<1, 1024, 0, s>>>(bsum, nb);
    if (nb > 0) k_bat_scan_down<<<nb, 1024, 0, s>>>(x, n, bsum, out);
    return hipGetLastError();
}

// Blocks that fit on one CU at once (asked of the runtime once per kernel).
template <class K>
static int occupancy(K kern, int G) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, G, 0) != hipSuccess || occ < 1) occ = 1;
    return occ;
}

// Symbolic and numeric launches of bin b (persistent grids over the bin's
// list; a block of an empty or short list leaves at once).
template <int G, int T>
static void sym_launch(int b, const BatchDesc *d, int64_t mtot, const BatchCounters &c, const int4 *list,
                       uint32_t *nnz, hipStream_t s, int ncu) {
    constexpr int U = u_for(G, T / 2) < 4 ? u_for(G, T / 2) : 4;
    static const int occ = occupancy(k_bat_sym<G, T, U>, G);
    const unsigned grid = (unsigned)std::min<int64_t>(mtot, (int64_t)ncu * occ);
    k_bat_sym<G, T, U><<<grid, G, 0, s>>>(d, b, c, list, nnz);
}

template <int G, int T, typename V>
static void num_launch(int b, const BatchDesc *d, int64_t mtot, const BatchCounters &c, const BatchBufs &w,
                       hipStream_t s, int ncu) {
    constexpr int U = u_for(G, T / 2 + 1) < 4 ? u_for(G, T / 2 + 1) : 4;
    static const int occ = occupancy(k_bat_num<G, T, U, V>, G);
    const unsigned grid = (unsigned)std::min<int64_t>(mtot, (int64_t)ncu * occ);
    k_bat_num<G, T, U, V><<<grid, G, 0, s>>>(d, b, c, w.list, w.nnz, w.gpos, w.K, w.ocols, (V *)w.ovals);
}

hipError_t launch_batch_analyse(const BatchDesc *d, int nprod, int64_t mtot, const BatchRows &r,
                                const BatchCounters &c, int4 *list, uint32_t *nnz, hipStream_t s) {
    k_bat_zero<<<g256(std::max(nprod, BAT_NB)), 256, 0, s>>>(c, nprod);
    if (mtot > 0) {
        const unsigned g = (unsigned)std::min<int64_t>((mtot + 31) / 32, 8192);
        k_bat_flop<<<g, 256, 0, s>>>(d, nprod, mtot, r, c);
        k_bat_binscan<<<1, 64, 0, s>>>(c);
        k_bat_scatter<<<g256(mtot), 256, 0, s>>>(mtot, r, c, list, nnz);
    }
    return hipGetLastError();
}

// Two phases on the device: every bin's symbolic counts, one scan of the
// counts into places in C, then every bin's numeric rows written in place.
template <typename V>
static hipError_t batch_rows_t(const BatchDesc *d, int64_t mtot, const BatchCounters &c, const BatchBufs &w,
                               hipStream_t s, int ncu) {
    sym_launch<SYM_G[1], SYM_T[1]>(1, d, mtot, c, w.list, w.nnz, s, ncu);
    sym_launch<SYM_G[2], SYM_T[2]>(2, d, mtot, c, w.list, w.nnz, s, ncu);
    sym_launch<SYM_G[3], SYM_T[3]>(3, d, mtot, c, w.list, w.nnz, s, ncu);
    sym_launch<SYM_G[4], SYM_T[4]>(4, d, mtot, c, w.list, w.nnz, s, ncu);
    sym_launch<SYM_G[5], SYM_T[5]>(5, d, mtot, c, w.list, w.nnz, s, ncu);
    sym_launch<SYM_G[6], SYM_T[6]>(6, d, mtot, c, w.list, w.nnz, s, ncu);
    sym_launch<SYM_G[7], SYM_T[7]>(7, d, mtot, c, w.list, w.nnz, s, ncu);
    sym_launch<SYM_G[8], SYM_T[8]>(8, d, mtot, c, w.list, w.nnz, s, ncu);
    sym_launch<SYM_G[9], SYM_T[9]>(9, d, mtot, c, w.list, w.nnz, s, ncu);
    hipError_t e = scan_u32(w.nnz, mtot, w.bsum, w.gpos, s);
    if (e != hipSuccess) return e;
    num_launch<NUM_G[1], NUM_T[1], V>(1, d, mtot, c, w, s, ncu);
    num_launch<NUM_G[2], NUM_T[2], V>(2, d, mtot, c, w, s, ncu);
    num_launch<NUM_G[3], NUM_T[3], V>(3, d, mtot, c, w, s, ncu);
    num_launch<NUM_G[4], NUM_T[4], V>(4, d, mtot, c, w, s, ncu);
    num_launch<NUM_G[5], NUM_T[5], V>(5, d, mtot, c, w, s, ncu);
    num_launch<NUM_G[6], NUM_T[6], V>(6, d, mtot, c, w, s, ncu);
    num_launch<NUM_G[7], NUM_T[7], V>(7, d, mtot, c, w, s, ncu);
    num_launch<NUM_G[8], NUM_T[8], V>(8, d, mtot, c, w, s, ncu);
    num_launch<NUM_G[9], NUM_T[9], V>(9, d, mtot, c, w, s, ncu);
    return hipGetLastError();
}

hipError_t launch_batch_run(int dtype, const BatchDesc *d, int nprod, int64_t mtot, const BatchRows &r,
                            const BatchCounters &c, const BatchBufs &w, spgemm_batch_result *res, hipStream_t s,
                            int ncu) {
    k_bat_reset_err<<<1, 64, 0, s>>>(c.err);
    if (mtot > 0) {
        const hipError_t e = dtype == SPGEMM_F64 ? batch_rows_t<double>(d, mtot, c, w, s, ncu)
                                                 : batch_rows_t<unsigned long long>(d, mtot, c, w, s, ncu);
        if (e != hipSuccess) return e;
    } else {
        const hipError_t e = scan_u32(w.nnz, 0, w.bsum, w.gpos, s);   // sets the total (0) the results read
        if (e != hipSuccess) return e;
    }
    // the total entry count is the scan total bsum[nb], read on the device
    const long long *tot = w.bsum + (mtot + 4095) / 4096;
    if (mtot > 0)
        k_bat_rpts<<<(unsigned)std::min<int64_t>(g256(mtot + nprod), 4096), 256, 0, s>>>(d, nprod, mtot, r.pid,
                                                                                         w.gpos, tot, w.orpts);
    k_bat_results<<<g256(nprod), 256, 0, s>>>(d, nprod, mtot, w.gpos, tot, c, w.rpts_base, w.cols_base, w.vals_base,
                                              res);
    return hipGetLastError();
}

}  // namespace spg
