// gfx950 kernels of the two-phase hash SpGEMM and their launchers.
//
// Phase map (paper Section 2 two-phase method; Section 4.2.1, Fig. 5):
//   k_row_flop       row flop (Fig. 4 part 1) + per-bin row counts
//   k_sym_scatter    rows grouped by flop (GPU counterpart of Fig. 4 part 2)
//   k_sym_hash<G,T>  symbolic phase: keys-only LDS hash table per row
//   k_sym_bitmap<W>  symbolic phase for rows above the LDS table range: one
//                    bit per output column in LDS, plus per-chunk counts
//   k_scan_*         exclusive scan of row counts into int64 row pointers
//   k_num_hist       rows grouped by exact nnz(c_i) for the numeric phase
//   k_windows        column windows of the rows too large for one LDS table
//   k_bucket_*       B rows reordered by 4096-column chunk (for windows)
//   k_num_hash       numeric phase: LDS hash table of keys + values per row,
//                    compacted (and sorted if asked) into C
//   k_num_window     numeric phase of one column window of a heavy row
//   k_masked_sum     sum of C over the positions of a mask (triangle count)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "config.hpp"
#include "device.hpp"
#include "launch.hpp"

namespace spg {

constexpr int U_ENUM = 4;   // products per lane per batch (memory-level parallelism)

// ----------------------------------------------------------------------- validate

__global__ __launch_bounds__(256) void k_validate(int64_t nrows, int64_t ncols, int64_t nnz,
                                                  const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ c, int *err) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrows; i += stride) {
        if (rp[i] > rp[i + 1]) bad = 1;
        if (i == 0 && rp[0] != 0) bad = 1;
        if (i == nrows - 1 && (int64_t)rp[nrows] != nnz) bad = 1;
    }
    if (nrows == 0 && blockIdx.x == 0 && threadIdx.x == 0 && (rp[0] != 0 || nnz != 0)) bad = 1;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += stride) {
        const int32_t x = c[p];
        if (x < 0 || (int64_t)x >= ncols) bad = 1;
    }
    if (bad) atomicOr(err, ERR_CSR);
}

// ----------------------------------------------------------------------- row flop

// 256 consecutive rows per block; the block's A entries are walked flat, each
// lane locating its row by binary search over the block's row pointers.
__global__ __launch_bounds__(256) void k_row_flop(int m, const int32_t *__restrict__ rA,
                                                  const int32_t *__restrict__ cA,
                                                  const int32_t *__restrict__ rB, int64_t ncolsB,
                                                  uint32_t *__restrict__ flop_out, PlanHdr *hdr) {
    __shared__ int s_rp[257];
    __shared__ unsigned long long s_f[256];
    __shared__ unsigned long long s_rows[NSB], s_flop[NSB], s_nnza[NSB];
    __shared__ unsigned long long s_tot, s_max;
    const int tid = threadIdx.x;
    const int r0 = blockIdx.x * 256;
    const int nr = min(256, m - r0);
    for (int t = tid; t <= nr; t += 256) s_rp[t] = rA[r0 + t];
    s_f[tid] = 0;
    if (tid < NSB) { s_rows[tid] = 0; s_flop[tid] = 0; s_nnza[tid] = 0; }
    if (tid == 0) { s_tot = 0; s_max = 0; }
    __syncthreads();
    const int p0 = s_rp[0], p1 = s_rp[nr];
    for (int p = p0 + tid; p < p1; p += 256) {
        int lo = 0, hi = nr;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_rp[mid] <= p) lo = mid; else hi = mid - 1;
        }
        const int k = cA[p];
        atomicAdd(&s_f[lo], (unsigned long long)(rB[k + 1] - rB[k]));
    }
    __syncthreads();
    if (tid < nr) {
        const unsigned long long f = s_f[tid];
        flop_out[r0 + tid] = f > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)f;
        const int b = sym_bin(f, ncolsB);
        atomicAdd(&s_rows[b], 1ull);
        atomicAdd(&s_flop[b], f);
        atomicAdd(&s_nnza[b], (unsigned long long)(s_rp[tid + 1] - s_rp[tid]));
        atomicAdd(&s_tot, f);
        atomicMax(&s_max, f);
    }
    __syncthreads();
    if (tid < NSB && s_rows[tid]) {
        atomicAdd(&hdr->sym_rows[tid], s_rows[tid]);
        atomicAdd(&hdr->sym_flop[tid], s_flop[tid]);
        atomicAdd(&hdr->sym_nnza[tid], s_nnza[tid]);
    }
    if (tid == 0) {
        atomicAdd(&hdr->total_flop, s_tot);
        atomicMax(&hdr->max_flop, s_max);
    }
}

// ----------------------------------------------------------------------- binning

__global__ __launch_bounds__(256) void k_sym_scatter(int m, const uint32_t *__restrict__ flop,
                                                     int64_t ncolsB, BinOffsets off,
                                                     int32_t *__restrict__ perm,
                                                     int32_t *__restrict__ nnz_row, WsHdr *wh) {
    __shared__ unsigned int s_cnt[NSB], s_base[NSB];
    const int tid = threadIdx.x;
    if (tid < NSB) s_cnt[tid] = 0;
    __syncthreads();
    const int i = blockIdx.x * 256 + tid;
    int b = -1;
    unsigned int r = 0;
    if (i < m) {
        b = sym_bin(flop[i], ncolsB);
        if (b == 0) nnz_row[i] = 0;
        else r = atomicAdd(&s_cnt[b], 1u);
    }
    __syncthreads();
    if (tid < NSB && s_cnt[tid]) s_base[tid] = atomicAdd(&wh->sym_cursor[tid], s_cnt[tid]);
    __syncthreads();
    if (b > 0) perm[off.v[b] + s_base[b] + r] = i;
}

__global__ __launch_bounds__(256) void k_num_hist(int m, const int32_t *__restrict__ nnz_row,
                                                  const uint32_t *__restrict__ flop,
                                                  const int32_t *__restrict__ rA, WsHdr *wh) {
    __shared__ unsigned long long s_rows[NNB], s_flop[NNB], s_nnza[NNB], s_nnzc[NNB];
    const int tid = threadIdx.x;
    if (tid < NNB) { s_rows[tid] = 0; s_flop[tid] = 0; s_nnza[tid] = 0; s_nnzc[tid] = 0; }
    __syncthreads();
    const int i = blockIdx.x * 256 + tid;
    if (i < m) {
        const int nz = nnz_row[i];
        const int b = num_bin(nz);
        atomicAdd(&s_rows[b], 1ull);
        atomicAdd(&s_flop[b], (unsigned long long)flop[i]);
        atomicAdd(&s_nnza[b], (unsigned long long)(rA[i + 1] - rA[i]));
        atomicAdd(&s_nnzc[b], (unsigned long long)nz);
    }
    __syncthreads();
    if (tid < NNB && s_rows[tid]) {
        atomicAdd(&wh->num_rows[tid], s_rows[tid]);
        atomicAdd(&wh->num_flop[tid], s_flop[tid]);
        atomicAdd(&wh->num_nnza[tid], s_nnza[tid]);
        atomicAdd(&wh->num_nnzc[tid], s_nnzc[tid]);
    }
}

__global__ __launch_bounds__(256) void k_num_scatter(int m, const int32_t *__restrict__ nnz_row,
                                                     BinOffsets off, int32_t *__restrict__ perm,
                                                     WsHdr *wh) {
    __shared__ unsigned int s_cnt[NNB], s_base[NNB];
    const int tid = threadIdx.x;
    if (tid < NNB) s_cnt[tid] = 0;
    __syncthreads();
    const int i = blockIdx.x * 256 + tid;
    int b = -1;
    unsigned int r = 0;
    if (i < m) {
        b = num_bin(nnz_row[i]);
        if (b > 0 && b < NUM_HEAVY_BIN) r = atomicAdd(&s_cnt[b], 1u);
        else b = -1;
    }
    __syncthreads();
    if (tid < NNB && s_cnt[tid]) s_base[tid] = atomicAdd(&wh->num_cursor[tid], s_cnt[tid]);
    __syncthreads();
    if (b > 0) perm[off.v[b] + s_base[b] + r] = i;
}

// ----------------------------------------------------------------------- symbolic

template <int G, int T>
__global__ __launch_bounds__(G) void k_sym_hash(const int32_t *__restrict__ perm, int64_t perm_off,
                                                const int32_t *__restrict__ rA,
                                                const int32_t *__restrict__ cA,
                                                const int32_t *__restrict__ rB,
                                                const int32_t *__restrict__ cB,
                                                int32_t *__restrict__ nnz_row, WsHdr *wh) {
    __shared__ int tab[T];
    __shared__ SegLds<G, false, double> sg;
    const int tid = threadIdx.x;
    const int row = perm[perm_off + blockIdx.x];
    for (int i = tid; i < T; i += G) tab[i] = -1;
    seg_init(sg);
    __syncthreads();
    int cnt = 0, ovf = 0;
    enum_row<G, U_ENUM, false, double>(
        rA[row], rA[row + 1], cA, nullptr, sg,
        [&](int k, int &lo, int &hi) { lo = rB[k]; hi = rB[k + 1]; },
        [&](const int (&q)[U_ENUM], const bool (&ok)[U_ENUM], const double (&)[U_ENUM]) {
            int col[U_ENUM];
#pragma unroll
            for (int u = 0; u < U_ENUM; ++u) col[u] = ok[u] ? cB[q[u]] : 0;
#pragma unroll
            for (int u = 0; u < U_ENUM; ++u)
                if (ok[u]) cnt += sym_insert(tab, T, col[u], ovf);
        });
    __syncthreads();
    int total;
    block_excl_scan<G, int>(cnt, total, sg.wsum);
    if (tid == 0) nnz_row[row] = total;
    if (ovf) {
        atomicAdd(&wh->probe_overflow, 1u);
        atomicOr(&wh->err, ERR_PROBE);
    }
}

// One bit per column of C (swept in passes of NWORDS*32 columns); the
// per-chunk popcounts are kept for the window split of the numeric phase.
template <int NWORDS>
__global__ __launch_bounds__(1024) void k_sym_bitmap(const int32_t *__restrict__ perm, int64_t perm_off,
                                                     const int32_t *__restrict__ rA,
                                                     const int32_t *__restrict__ cA,
                                                     const int32_t *__restrict__ rB,
                                                     const int32_t *__restrict__ cB, int64_t ncols,
                                                     int nchunks, uint32_t *__restrict__ chunk_cnt,
                                                     HeavyRow *__restrict__ heavy,
                                                     int32_t *__restrict__ nnz_row, WsHdr *wh) {
    constexpr int G = 1024;
    constexpr int NW = G / WAVE;
    constexpr int64_t WIN = (int64_t)NWORDS * 32;
    static_assert(NWORDS % (CHUNK_COLS / 32) == 0, "bitmap pass must hold whole chunks");
    __shared__ uint32_t bm[NWORDS];
    __shared__ SegLds<G, false, double> sg;
    __shared__ int s_total;
    const int tid = threadIdx.x, ln = tid & 63, w = tid >> 6;
    const int slot = blockIdx.x;
    const int row = perm[perm_off + slot];
    seg_init(sg);
    if (tid == 0) s_total = 0;
    const int a0 = rA[row], a1 = rA[row + 1];
    const int npass = (int)((ncols + WIN - 1) / WIN);
    for (int pass = 0; pass < npass; ++pass) {
        const int64_t c0 = (int64_t)pass * WIN;
        const int wcols = (int)(ncols - c0 < WIN ? ncols - c0 : WIN);
        const int nw = (wcols + 31) >> 5;
        for (int i = tid; i < nw; i += G) bm[i] = 0;
        __syncthreads();
        enum_row<G, U_ENUM, false, double>(
            a0, a1, cA, nullptr, sg,
            [&](int k, int &lo, int &hi) { lo = rB[k]; hi = rB[k + 1]; },
            [&](const int (&q)[U_ENUM], const bool (&ok)[U_ENUM], const double (&)[U_ENUM]) {
                int col[U_ENUM];
#pragma unroll
                for (int u = 0; u < U_ENUM; ++u) col[u] = ok[u] ? cB[q[u]] : 0;
#pragma unroll
                for (int u = 0; u < U_ENUM; ++u) {
                    const uint32_t c = (uint32_t)((int64_t)col[u] - c0);
                    if (ok[u] && c < (uint32_t)wcols) atomicOr(&bm[c >> 5], 1u << (c & 31));
                }
            });
        __syncthreads();
        const int nch = (wcols + CHUNK_COLS - 1) >> CHUNK_SHIFT;
        const int chunk0 = (int)(c0 >> CHUNK_SHIFT);
        for (int c = w; c < nch; c += NW) {
            int cw = 0;
            for (int j = ln; j < CHUNK_COLS / 32; j += WAVE) {
                const int wi = c * (CHUNK_COLS / 32) + j;
                if (wi < nw) cw += __popc(bm[wi]);
            }
            cw = wave_sum_i32(cw);
            if (ln == 0) {
                chunk_cnt[(size_t)slot * nchunks + chunk0 + c] = (uint32_t)cw;
                atomicAdd(&s_total, cw);
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        nnz_row[row] = s_total;
        if (s_total > WIN_CAP) {
            const unsigned h = atomicAdd(&wh->n_heavy, 1u);
            heavy[h] = HeavyRow{row, slot};
        }
    }
}

// ----------------------------------------------------------------------- scan

__global__ __launch_bounds__(1024) void k_scan_reduce(const int32_t *__restrict__ nnz, int m,
                                                      long long *__restrict__ bsum) {
    __shared__ long long ws[17];
    const int base = blockIdx.x * 4096;
    long long s = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int i = base + j * 1024 + (int)threadIdx.x;
        if (i < m) s += nnz[i];
    }
    long long tot;
    block_excl_scan<1024, long long>(s, tot, ws);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_top(long long *__restrict__ bsum, int nb,
                                                   int64_t *__restrict__ last, WsHdr *wh) {
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
    if (threadIdx.x == 0) {
        *last = carry;
        wh->nnz_c = (unsigned long long)carry;
    }
}

__global__ __launch_bounds__(1024) void k_scan_down(const int32_t *__restrict__ nnz, int m,
                                                    const long long *__restrict__ bsum,
                                                    int64_t *__restrict__ rpts) {
    __shared__ long long ws[17];
    const int base = blockIdx.x * 4096 + (int)threadIdx.x * 4;
    long long v[4];
    long long s = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        v[j] = base + j < m ? nnz[base + j] : 0;
        s += v[j];
    }
    long long tot;
    long long run = block_excl_scan<1024, long long>(s, tot, ws) + bsum[blockIdx.x];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (base + j < m) rpts[base + j] = run;
        run += v[j];
    }
}

// ----------------------------------------------------------------------- windows

__global__ __launch_bounds__(256) void k_windows(const HeavyRow *__restrict__ heavy, int nchunks,
                                                 const uint32_t *__restrict__ chunk_cnt,
                                                 const int64_t *__restrict__ rpts_C,
                                                 WinItem *__restrict__ items, unsigned int cap,
                                                 WsHdr *wh) {
    const unsigned h = blockIdx.x * 256 + threadIdx.x;
    if (h >= wh->n_heavy) return;
    const HeavyRow hr = heavy[h];
    const uint32_t *cc = chunk_cnt + (size_t)hr.slot * nchunks;
    int nwin = 0, cur = 0;
    for (int c = 0; c < nchunks; ++c) {
        const int x = (int)cc[c];
        if (x > WIN_CAP) atomicOr(&wh->err, ERR_CHUNK);
        if (cur + x > WIN_CAP && cur > 0) { ++nwin; cur = 0; }
        cur += x;
    }
    if (cur > 0) ++nwin;
    const unsigned base = atomicAdd(&wh->n_items, (unsigned)nwin);
    if ((unsigned long long)base + nwin > cap) {
        atomicOr(&wh->err, ERR_ITEMS);
        return;
    }
    int64_t pos = rpts_C[hr.row];
    int start = 0, k = 0;
    cur = 0;
    for (int c = 0; c < nchunks; ++c) {
        const int x = (int)cc[c];
        if (cur + x > WIN_CAP && cur > 0) {
            items[base + k++] = WinItem{hr.row, start, c, cur, pos};
            pos += cur;
            start = c;
            cur = 0;
        }
        cur += x;
    }
    if (cur > 0) items[base + k++] = WinItem{hr.row, start, nchunks, cur, pos};
}

// ----------------------------------------------------------------------- bucket B by chunk

// Rows of at most 64 entries: one wave sorts the row by column (rank count).
template <typename V>
__global__ __launch_bounds__(256) void k_bucket_short(int n, const int32_t *__restrict__ rB,
                                                      const int32_t *__restrict__ cB,
                                                      const V *__restrict__ vB,
                                                      int32_t *__restrict__ bc, V *__restrict__ bv,
                                                      int32_t *__restrict__ long_list, WsHdr *wh) {
    const int row = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    const int ln = threadIdx.x & 63;
    if (row >= n) return;
    const int b0 = rB[row];
    const int len = rB[row + 1] - b0;
    if (len > WAVE) {
        if (ln == 0) long_list[atomicAdd(&wh->n_long, 1u)] = row;
        return;
    }
    const int col = ln < len ? cB[b0 + ln] : 0x7fffffff;
    const V v = ln < len ? vB[b0 + ln] : V(0);
    int rank = 0;
    for (int j = 0; j < len; ++j) {
        const int cj = __shfl(col, j);
        rank += (cj < col) || (cj == col && j < ln);
    }
    if (ln < len) {
        bc[b0 + rank] = col;
        bv[b0 + rank] = v;
    }
}

// Longer rows: counting sort by chunk id with LDS counters (a block per row,
// grid-stride over the list of long rows).
template <typename V>
__global__ __launch_bounds__(1024) void k_bucket_long(const int32_t *__restrict__ long_list,
                                                      const WsHdr *wh, const int32_t *__restrict__ rB,
                                                      const int32_t *__restrict__ cB,
                                                      const V *__restrict__ vB,
                                                      int32_t *__restrict__ bc, V *__restrict__ bv,
                                                      int nchunks) {
    __shared__ int cnt[MAX_CHUNKS];
    __shared__ int ws[17];
    const int tid = threadIdx.x;
    const unsigned nl = wh->n_long;
    for (unsigned li = blockIdx.x; li < nl; li += gridDim.x) {
        const int row = long_list[li];
        const int b0 = rB[row], b1 = rB[row + 1];
        for (int c = tid; c < nchunks; c += 1024) cnt[c] = 0;
        __syncthreads();
        for (int p = b0 + tid; p < b1; p += 1024) atomicAdd(&cnt[cB[p] >> CHUNK_SHIFT], 1);
        __syncthreads();
        int carry = 0;
        for (int c0 = 0; c0 < nchunks; c0 += 1024) {
            const int c = c0 + tid;
            const int v = c < nchunks ? cnt[c] : 0;
            int tot;
            const int ex = block_excl_scan<1024, int>(v, tot, ws);
            if (c < nchunks) cnt[c] = carry + ex;
            carry += tot;
        }
        __syncthreads();
        for (int p = b0 + tid; p < b1; p += 1024) {
            const int col = cB[p];
            const int pos = atomicAdd(&cnt[col >> CHUNK_SHIFT], 1);
            bc[b0 + pos] = col;
            bv[b0 + pos] = vB[p];
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------------- numeric

template <int G, int T, bool SORTED, typename V>
__global__ __launch_bounds__(G) void k_num_hash(const int32_t *__restrict__ perm, int64_t perm_off,
                                                const int32_t *__restrict__ rA,
                                                const int32_t *__restrict__ cA,
                                                const V *__restrict__ vA,
                                                const int32_t *__restrict__ rB,
                                                const int32_t *__restrict__ cB,
                                                const V *__restrict__ vB,
                                                const int64_t *__restrict__ rpts_C,
                                                int32_t *__restrict__ cC, V *__restrict__ vC,
                                                WsHdr *wh) {
    __shared__ int keys[T];
    __shared__ V vals[T];
    __shared__ SegLds<G, true, V> sg;
    const int tid = threadIdx.x;
    const int row = perm[perm_off + blockIdx.x];
    for (int i = tid; i < T; i += G) { keys[i] = -1; vals[i] = V(0); }
    seg_init(sg);
    __syncthreads();
    int ovf = 0;
    enum_row<G, U_ENUM, true, V>(
        rA[row], rA[row + 1], cA, vA, sg,
        [&](int k, int &lo, int &hi) { lo = rB[k]; hi = rB[k + 1]; },
        [&](const int (&q)[U_ENUM], const bool (&ok)[U_ENUM], const V (&av)[U_ENUM]) {
            int col[U_ENUM];
            V bvv[U_ENUM];
#pragma unroll
            for (int u = 0; u < U_ENUM; ++u) {
                col[u] = 0;
                bvv[u] = V(0);
                if (ok[u]) { col[u] = cB[q[u]]; bvv[u] = vB[q[u]]; }
            }
#pragma unroll
            for (int u = 0; u < U_ENUM; ++u)
                if (ok[u]) num_insert<V>(keys, vals, T, col[u], av[u] * bvv[u], ovf);
        });
    __syncthreads();
    if (ovf) {
        atomicAdd(&wh->probe_overflow, 1u);
        atomicOr(&wh->err, ERR_PROBE);
    }
    const int64_t o = rpts_C[row];
    const int expected = (int)(rpts_C[row + 1] - o);
    compact_store<G, T, SORTED, V>(keys, vals, sg.wsum, o, expected, cC, vC, &wh->err);
}

// first p in [lo, hi) whose column lies in chunk >= ch (B row bucketed by chunk)
__device__ __forceinline__ int lower_chunk(const int32_t *__restrict__ bc, int lo, int hi, int ch) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((bc[mid] >> CHUNK_SHIFT) < ch) lo = mid + 1; else hi = mid;
    }
    return lo;
}

template <bool SORTED, typename V>
__global__ __launch_bounds__(1024) void k_num_window(const WinItem *__restrict__ items,
                                                     const int32_t *__restrict__ rA,
                                                     const int32_t *__restrict__ cA,
                                                     const V *__restrict__ vA,
                                                     const int32_t *__restrict__ rB,
                                                     const int32_t *__restrict__ bc,
                                                     const V *__restrict__ bv,
                                                     int32_t *__restrict__ cC, V *__restrict__ vC,
                                                     WsHdr *wh) {
    constexpr int G = 1024;
    constexpr int T = WIN_TABLE;
    __shared__ int keys[T];
    __shared__ V vals[T];
    __shared__ SegLds<G, true, V> sg;
    const int tid = threadIdx.x;
    const WinItem it = items[blockIdx.x];
    for (int i = tid; i < T; i += G) { keys[i] = -1; vals[i] = V(0); }
    seg_init(sg);
    __syncthreads();
    int ovf = 0;
    const int ch_lo = it.ch_lo, ch_hi = it.ch_hi;
    enum_row<G, U_ENUM, true, V>(
        rA[it.row], rA[it.row + 1], cA, vA, sg,
        [&](int k, int &lo, int &hi) {
            const int r0 = rB[k], r1 = rB[k + 1];
            lo = lower_chunk(bc, r0, r1, ch_lo);
            hi = lower_chunk(bc, lo, r1, ch_hi);
        },
        [&](const int (&q)[U_ENUM], const bool (&ok)[U_ENUM], const V (&av)[U_ENUM]) {
            int col[U_ENUM];
            V bvv[U_ENUM];
#pragma unroll
            for (int u = 0; u < U_ENUM; ++u) {
                col[u] = 0;
                bvv[u] = V(0);
                if (ok[u]) { col[u] = bc[q[u]]; bvv[u] = bv[q[u]]; }
            }
#pragma unroll
            for (int u = 0; u < U_ENUM; ++u)
                if (ok[u]) num_insert<V>(keys, vals, T, col[u], av[u] * bvv[u], ovf);
        });
    __syncthreads();
    if (ovf) {
        atomicAdd(&wh->probe_overflow, 1u);
        atomicOr(&wh->err, ERR_PROBE);
    }
    compact_store<G, T, SORTED, V>(keys, vals, sg.wsum, it.out_pos, it.count, cC, vC, &wh->err);
}

// ----------------------------------------------------------------------- masked sum

__device__ __forceinline__ bool lds_contains(const int *tab, uint32_t T, int key) {
    uint32_t s = hash_slot(key, T);
    for (uint32_t n = 0; n < T; ++n) {
        const int cur = tab[s];
        if (cur == key) return true;
        if (cur == -1) return false;
        s = (s + 1 == T) ? 0u : s + 1;
    }
    return false;
}

// One block per row: the mask row goes into an LDS hash set (rows up to 4096
// entries) or, for longer rows, into a bitmap swept over column windows.
__global__ __launch_bounds__(256) void k_masked_sum(int64_t m, int64_t ncols,
                                                    const int64_t *__restrict__ rC,
                                                    const int32_t *__restrict__ cC,
                                                    const unsigned long long *__restrict__ vC,
                                                    const int32_t *__restrict__ rM,
                                                    const int32_t *__restrict__ cM,
                                                    unsigned long long *out) {
    constexpr int G = 256;
    constexpr int T = 8192;
    constexpr int64_t WINC = (int64_t)T * 32;
    __shared__ int tab[T];
    __shared__ unsigned long long ws[G / WAVE + 1];
    const int tid = threadIdx.x;
    const int64_t i = blockIdx.x;
    const int m0 = rM[i], m1 = rM[i + 1];
    const int64_t c0 = rC[i], c1 = rC[i + 1];
    unsigned long long s = 0;
    if (m1 > m0 && c1 > c0) {
        if (m1 - m0 <= T / 2) {
            for (int j = tid; j < T; j += G) tab[j] = -1;
            __syncthreads();
            int ovf = 0;
            for (int p = m0 + tid; p < m1; p += G) sym_insert(tab, T, cM[p], ovf);
            __syncthreads();
            for (int64_t q = c0 + tid; q < c1; q += G)
                if (lds_contains(tab, T, cC[q])) s += vC[q];
        } else {
            uint32_t *bm = (uint32_t *)tab;
            for (int64_t w0 = 0; w0 < ncols; w0 += WINC) {
                for (int j = tid; j < T; j += G) bm[j] = 0;
                __syncthreads();
                for (int p = m0 + tid; p < m1; p += G) {
                    const int64_t x = (int64_t)cM[p] - w0;
                    if (x >= 0 && x < WINC) atomicOr(&bm[x >> 5], 1u << (x & 31));
                }
                __syncthreads();
                for (int64_t q = c0 + tid; q < c1; q += G) {
                    const int64_t x = (int64_t)cC[q] - w0;
                    if (x >= 0 && x < WINC && ((bm[x >> 5] >> (x & 31)) & 1u)) s += vC[q];
                }
                __syncthreads();
            }
        }
    }
    unsigned long long tot;
    block_excl_scan<G, unsigned long long>(s, tot, ws);
    if (tid == 0 && tot) atomicAdd(out, tot);
}

__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long *p) { *p = 0; }

// ----------------------------------------------------------------------- copy

__global__ __launch_bounds__(256) void k_stream_copy(const uint4 *__restrict__ src,
                                                     uint4 *__restrict__ dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// ======================================================================= launchers

static inline unsigned grid1(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

hipError_t launch_validate(const CsrDev &a, int *err, hipStream_t s) {
    const unsigned g = (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, grid1(std::max(a.nrows, a.nnz), 256)));
    k_validate<<<g, 256, 0, s>>>(a.nrows, a.ncols, a.nnz, a.rpts, a.cols, err);
    return hipGetLastError();
}

hipError_t launch_row_flop(const CsrDev &A, const CsrDev &B, uint32_t *flop, PlanHdr *hdr, hipStream_t s) {
    if (A.nrows == 0) return hipSuccess;
    k_row_flop<<<grid1(A.nrows, 256), 256, 0, s>>>((int)A.nrows, A.rpts, A.cols, B.rpts, B.ncols, flop, hdr);
    return hipGetLastError();
}

hipError_t launch_sym_scatter(int m, const uint32_t *flop, int64_t ncolsB, const BinOffsets &off,
                              int32_t *perm, int32_t *nnz_row, WsHdr *wh, hipStream_t s) {
    if (m == 0) return hipSuccess;
    k_sym_scatter<<<grid1(m, 256), 256, 0, s>>>(m, flop, ncolsB, off, perm, nnz_row, wh);
    return hipGetLastError();
}

template <int G, int T>
static void sym_hash_l(unsigned nrows, const int32_t *perm, int64_t off, const CsrDev &A,
                       const CsrDev &B, int32_t *nnz_row, WsHdr *wh, hipStream_t s) {
    k_sym_hash<G, T><<<nrows, G, 0, s>>>(perm, off, A.rpts, A.cols, B.rpts, B.cols, nnz_row, wh);
}

hipError_t launch_sym_bin(int bin, unsigned nrows, const int32_t *perm, int64_t off, const CsrDev &A,
                          const CsrDev &B, int32_t *nnz_row, WsHdr *wh, hipStream_t s) {
    if (nrows == 0) return hipSuccess;
    switch (bin) {
        case 1: sym_hash_l<SYM_G[1], SYM_T[1]>(nrows, perm, off, A, B, nnz_row, wh, s); break;
        case 2: sym_hash_l<SYM_G[2], SYM_T[2]>(nrows, perm, off, A, B, nnz_row, wh, s); break;
        case 3: sym_hash_l<SYM_G[3], SYM_T[3]>(nrows, perm, off, A, B, nnz_row, wh, s); break;
        case 4: sym_hash_l<SYM_G[4], SYM_T[4]>(nrows, perm, off, A, B, nnz_row, wh, s); break;
        case 5: sym_hash_l<SYM_G[5], SYM_T[5]>(nrows, perm, off, A, B, nnz_row, wh, s); break;
        case 6: sym_hash_l<SYM_G[6], SYM_T[6]>(nrows, perm, off, A, B, nnz_row, wh, s); break;
        case 7: sym_hash_l<SYM_G[7], SYM_T[7]>(nrows, perm, off, A, B, nnz_row, wh, s); break;
        case 8: sym_hash_l<SYM_G[8], SYM_T[8]>(nrows, perm, off, A, B, nnz_row, wh, s); break;
        case 9: sym_hash_l<SYM_G[9], SYM_T[9]>(nrows, perm, off, A, B, nnz_row, wh, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int bitmap_words_for(int64_t ncols) {
    const int64_t need = (ncols + 31) / 32;
    if (need <= BM_WORDS_SMALL) return BM_WORDS_SMALL;
    if (need <= BM_WORDS_MID) return BM_WORDS_MID;
    return BM_WORDS_LARGE;
}

hipError_t launch_sym_bitmap(unsigned nrows, const int32_t *perm, int64_t off, const CsrDev &A,
                             const CsrDev &B, int nchunks, uint32_t *chunk_cnt, HeavyRow *heavy,
                             int32_t *nnz_row, WsHdr *wh, hipStream_t s) {
    if (nrows == 0) return hipSuccess;
    const int words = bitmap_words_for(B.ncols);
    if (words == BM_WORDS_SMALL)
        k_sym_bitmap<BM_WORDS_SMALL><<<nrows, 1024, 0, s>>>(perm, off, A.rpts, A.cols, B.rpts, B.cols, B.ncols,
                                                            nchunks, chunk_cnt, heavy, nnz_row, wh);
    else if (words == BM_WORDS_MID)
        k_sym_bitmap<BM_WORDS_MID><<<nrows, 1024, 0, s>>>(perm, off, A.rpts, A.cols, B.rpts, B.cols, B.ncols,
                                                          nchunks, chunk_cnt, heavy, nnz_row, wh);
    else
        k_sym_bitmap<BM_WORDS_LARGE><<<nrows, 1024, 0, s>>>(perm, off, A.rpts, A.cols, B.rpts, B.cols, B.ncols,
                                                            nchunks, chunk_cnt, heavy, nnz_row, wh);
    return hipGetLastError();
}

hipError_t launch_scan(const int32_t *nnz_row, int m, long long *bsum, int64_t *rpts_C, WsHdr *wh,
                       hipStream_t s) {
    const int nb = (int)grid1(m, 4096);
    if (nb > 0) k_scan_reduce<<<nb, 1024, 0, s>>>(nnz_row, m, bsum);
    k_scan_top<<<1, 1024, 0, s>>>(bsum, nb, rpts_C + m, wh);
    if (nb > 0) k_scan_down<<<nb, 1024, 0, s>>>(nnz_row, m, bsum, rpts_C);
    return hipGetLastError();
}

hipError_t launch_num_hist(int m, const int32_t *nnz_row, const uint32_t *flop, const int32_t *rA,
                           WsHdr *wh, hipStream_t s) {
    if (m == 0) return hipSuccess;
    k_num_hist<<<grid1(m, 256), 256, 0, s>>>(m, nnz_row, flop, rA, wh);
    return hipGetLastError();
}

hipError_t launch_windows(unsigned nheavy_max, const HeavyRow *heavy, int nchunks, const uint32_t *chunk_cnt,
                          const int64_t *rpts_C, WinItem *items, unsigned cap, WsHdr *wh, hipStream_t s) {
    if (nheavy_max == 0) return hipSuccess;
    k_windows<<<grid1(nheavy_max, 256), 256, 0, s>>>(heavy, nchunks, chunk_cnt, rpts_C, items, cap, wh);
    return hipGetLastError();
}

template <typename V>
static hipError_t bucket_t(const CsrDev &B, int32_t *bc, void *bv, int32_t *long_list, int nchunks,
                           WsHdr *wh, hipStream_t s) {
    if (B.nrows == 0) return hipSuccess;
    k_bucket_short<V><<<grid1(B.nrows, 4), 256, 0, s>>>((int)B.nrows, B.rpts, B.cols, (const V *)B.vals, bc,
                                                         (V *)bv, long_list, wh);
    k_bucket_long<V><<<1024, 1024, 0, s>>>(long_list, wh, B.rpts, B.cols, (const V *)B.vals, bc, (V *)bv,
                                            nchunks);
    return hipGetLastError();
}

hipError_t launch_bucket(int dtype, const CsrDev &B, int32_t *bc, void *bv, int32_t *long_list, int nchunks,
                         WsHdr *wh, hipStream_t s) {
    if (dtype == 0) return bucket_t<double>(B, bc, bv, long_list, nchunks, wh, s);
    return bucket_t<unsigned long long>(B, bc, bv, long_list, nchunks, wh, s);
}

hipError_t launch_num_scatter(int m, const int32_t *nnz_row, const BinOffsets &off, int32_t *perm, WsHdr *wh,
                              hipStream_t s) {
    if (m == 0) return hipSuccess;
    k_num_scatter<<<grid1(m, 256), 256, 0, s>>>(m, nnz_row, off, perm, wh);
    return hipGetLastError();
}

template <int G, int T, bool SORTED, typename V>
static void num_hash_l(unsigned nrows, const int32_t *perm, int64_t off, const CsrDev &A, const CsrDev &B,
                       const int64_t *rpts_C, int32_t *cC, void *vC, WsHdr *wh, hipStream_t s) {
    k_num_hash<G, T, SORTED, V><<<nrows, G, 0, s>>>(perm, off, A.rpts, A.cols, (const V *)A.vals, B.rpts, B.cols,
                                                     (const V *)B.vals, rpts_C, cC, (V *)vC, wh);
}

template <bool SORTED, typename V>
static hipError_t num_bin_t(int bin, unsigned nrows, const int32_t *perm, int64_t off, const CsrDev &A,
                            const CsrDev &B, const int64_t *rpts_C, int32_t *cC, void *vC, WsHdr *wh,
                            hipStream_t s) {
    switch (bin) {
        case 1: num_hash_l<NUM_G[1], NUM_T[1], SORTED, V>(nrows, perm, off, A, B, rpts_C, cC, vC, wh, s); break;
        case 2: num_hash_l<NUM_G[2], NUM_T[2], SORTED, V>(nrows, perm, off, A, B, rpts_C, cC, vC, wh, s); break;
        case 3: num_hash_l<NUM_G[3], NUM_T[3], SORTED, V>(nrows, perm, off, A, B, rpts_C, cC, vC, wh, s); break;
        case 4: num_hash_l<NUM_G[4], NUM_T[4], SORTED, V>(nrows, perm, off, A, B, rpts_C, cC, vC, wh, s); break;
        case 5: num_hash_l<NUM_G[5], NUM_T[5], SORTED, V>(nrows, perm, off, A, B, rpts_C, cC, vC, wh, s); break;
        case 6: num_hash_l<NUM_G[6], NUM_T[6], SORTED, V>(nrows, perm, off, A, B, rpts_C, cC, vC, wh, s); break;
        case 7: num_hash_l<NUM_G[7], NUM_T[7], SORTED, V>(nrows, perm, off, A, B, rpts_C, cC, vC, wh, s); break;
        case 8: num_hash_l<NUM_G[8], NUM_T[8], SORTED, V>(nrows, perm, off, A, B, rpts_C, cC, vC, wh, s); break;
        case 9: num_hash_l<NUM_G[9], NUM_T[9], SORTED, V>(nrows, perm, off, A, B, rpts_C, cC, vC, wh, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_num_bin(int bin, int dtype, bool sorted, unsigned nrows, const int32_t *perm, int64_t off,
                          const CsrDev &A, const CsrDev &B, const int64_t *rpts_C, int32_t *cC, void *vC,
                          WsHdr *wh, hipStream_t s) {
    if (nrows == 0) return hipSuccess;
    if (dtype == 0)
        return sorted ? num_bin_t<true, double>(bin, nrows, perm, off, A, B, rpts_C, cC, vC, wh, s)
                      : num_bin_t<false, double>(bin, nrows, perm, off, A, B, rpts_C, cC, vC, wh, s);
    return sorted ? num_bin_t<true, unsigned long long>(bin, nrows, perm, off, A, B, rpts_C, cC, vC, wh, s)
                  : num_bin_t<false, unsigned long long>(bin, nrows, perm, off, A, B, rpts_C, cC, vC, wh, s);
}

template <bool SORTED, typename V>
static void num_window_l(unsigned nitems, const WinItem *items, const CsrDev &A, const CsrDev &B,
                         const int32_t *bc, const void *bv, int32_t *cC, void *vC, WsHdr *wh, hipStream_t s) {
    k_num_window<SORTED, V><<<nitems, 1024, 0, s>>>(items, A.rpts, A.cols, (const V *)A.vals, B.rpts, bc,
                                                    (const V *)bv, cC, (V *)vC, wh);
}

hipError_t launch_num_window(int dtype, bool sorted, unsigned nitems, const WinItem *items, const CsrDev &A,
                             const CsrDev &B, const int32_t *bc, const void *bv, int32_t *cC, void *vC,
                             WsHdr *wh, hipStream_t s) {
    if (nitems == 0) return hipSuccess;
    if (dtype == 0) {
        if (sorted) num_window_l<true, double>(nitems, items, A, B, bc, bv, cC, vC, wh, s);
        else num_window_l<false, double>(nitems, items, A, B, bc, bv, cC, vC, wh, s);
    } else {
        if (sorted) num_window_l<true, unsigned long long>(nitems, items, A, B, bc, bv, cC, vC, wh, s);
        else num_window_l<false, unsigned long long>(nitems, items, A, B, bc, bv, cC, vC, wh, s);
    }
    return hipGetLastError();
}

hipError_t launch_masked_sum(int64_t m, int64_t ncols, const int64_t *rC, const int32_t *cC, const int64_t *vC,
                             const CsrDev &M, int64_t *out, hipStream_t s) {
    k_zero_u64<<<1, 1, 0, s>>>((unsigned long long *)out);
    if (m > 0)
        k_masked_sum<<<(unsigned)m, 256, 0, s>>>(m, ncols, rC, cC, (const unsigned long long *)vC, M.rpts, M.cols,
                                                 (unsigned long long *)out);
    return hipGetLastError();
}

hipError_t launch_stream_copy(void *dst, const void *src, size_t nbytes, hipStream_t s) {
    const size_t n = nbytes / 16;
    if (n == 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<size_t>((n + 255) / 256, 256 * 64);
    k_stream_copy<<<g, 256, 0, s>>>((const uint4 *)src, (uint4 *)dst, n);
    return hipGetLastError();
}

}  // namespace spg
