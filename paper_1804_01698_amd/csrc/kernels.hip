// gfx950 kernels of the two-phase hash SpGEMM and their launchers.
//
// Phase map (paper Section 2 two-phase method; Section 4.2.1, Fig. 5):
//   k_row_flop       row flop (Fig. 4 part 1) + per-bin row counts
//   k_sym_scatter    rows grouped by flop (GPU counterpart of Fig. 4 part 2)
//   k_sym_hash<G,T>  symbolic phase: keys-only LDS hash table per row
//   k_sym_bitmap<W>  symbolic phase for rows above the LDS table range
//                    (persistent): one bit per output column in LDS, plus
//                    per-chunk counts and, for heavy rows, the bits
//   k_scan_*         exclusive scan of row counts into int64 row pointers
//   k_num_hist       rows grouped by exact nnz(c_i) for the numeric phase
//   k_win_*          column windows of the rows too large for one LDS table
//   k_bucket_*       B rows reordered by 4096-column chunk, with a chunk index
//   k_gather_vals    B values in that order (numeric phase)
//   k_num_hash       numeric phase: LDS hash table of keys + values per row,
//                    compacted, or ranked in column passes when sorted
//   k_num_window     numeric phase of the column windows of heavy rows
//                    (persistent): occupancy bits, ranks, values and columns
//                    written at their rank
//   k_masked_sum     sum of C over the positions of a mask (triangle count)
//   k_masked_product the same sum without forming C
//   k_stream_copy, k_stanza_read   copy and stanza-read bandwidth probes
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "config.hpp"
#include "device.hpp"
#include "launch.hpp"

namespace spg {

// Products per lane per batch (memory-level parallelism), by kernel family.
constexpr int U_SEG = 16;
constexpr int U_RANK1 = 16;
constexpr int U_RANK2 = 8;

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

// Row flop: the flop of row i is the sum over its entries a_ik of the length
// of B row k.  A first pass takes 256 consecutive rows per block and sums a
// row of at most FLOP_SHORT_ROW entries in its own thread (eight entries'
// loads in flight); longer rows are listed and summed afterwards across the
// whole GPU (k_long_flop: a wave per row; k_huge_flop: a block per row).
// Summing them inside the first pass left the few row blocks where the long
// rows of a skewed matrix crowd together walking dozens of rows per wave
// while every other block had finished.

// Length of the B row that entry p of A selects.
__device__ __forceinline__ uint32_t entry_deg(int p, const int32_t *__restrict__ cA, const int32_t *__restrict__ rB) {
    const int k = cA[p];
    return (uint32_t)(rB[k + 1] - rB[k]);
}

// Row flop, key bound bin and the plan header's per-bin totals of a row.
__device__ __forceinline__ void row_flop_put(int row, unsigned long long f, int na, int64_t ncolsB,
                                             uint32_t *__restrict__ flop_out, unsigned long long *rows,
                                             unsigned long long *flop, unsigned long long *nnza,
                                             unsigned long long *tot, unsigned long long *mx, const BinLimits &L) {
    flop_out[row] = f > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)f;
    const int b = sym_bin_l(f, ncolsB, L);
    atomicAdd(&rows[b], 1ull);
    atomicAdd(&flop[b], f);
    atomicAdd(&nnza[b], (unsigned long long)na);
    atomicAdd(tot, f);
    atomicMax(mx, f);
}

__global__ __launch_bounds__(256) void k_row_flop(int m, const int32_t *__restrict__ rA,
                                                  const int32_t *__restrict__ cA, const int32_t *__restrict__ rB,
                                                  int64_t ncolsB, uint32_t *__restrict__ flop_out,
                                                  int32_t *__restrict__ longl, int32_t *__restrict__ huge,
                                                  PlanHdr *hdr, BinLimits L) {
    __shared__ int s_long[256], s_huge[256];
    __shared__ int s_nlong, s_nhuge, s_lbase, s_hbase;
    __shared__ unsigned long long s_rows[NSB], s_flop[NSB], s_nnza[NSB];
    __shared__ unsigned long long s_tot, s_max;
    const int tid = threadIdx.x;
    const int r0 = blockIdx.x * 256;
    const int nr = min(256, m - r0);
    if (tid < NSB) { s_rows[tid] = 0; s_flop[tid] = 0; s_nnza[tid] = 0; }
    if (tid == 0) { s_tot = 0; s_max = 0; s_nlong = 0; s_nhuge = 0; s_lbase = 0; s_hbase = 0; }
    __syncthreads();
    int a0 = 0, a1 = 0;
    unsigned long long f = 0;
    if (tid < nr) {
        a0 = rA[r0 + tid];
        a1 = rA[r0 + tid + 1];
        if (a1 - a0 <= FLOP_SHORT_ROW) {
            int p = a0;
            for (; p + 8 <= a1; p += 8) {              // eight entries' loads in flight
                unsigned long long d = 0;
#pragma unroll
                for (int u = 0; u < 8; ++u) d += entry_deg(p + u, cA, rB);
                f += d;
            }
            for (; p < a1; ++p) f += entry_deg(p, cA, rB);
        } else if (a1 - a0 <= FLOP_WAVE_ROW) {
            s_long[atomicAdd(&s_nlong, 1)] = r0 + tid;
        } else {
            s_huge[atomicAdd(&s_nhuge, 1)] = r0 + tid;
        }
    }
    __syncthreads();
    // the block's long rows join the lists with one global atomic per list
    if (tid == 0) {
        if (s_nlong) s_lbase = (int)atomicAdd(&hdr->n_long_a, (unsigned)s_nlong);
        if (s_nhuge) s_hbase = (int)atomicAdd(&hdr->n_huge, (unsigned)s_nhuge);
    }
    __syncthreads();
    if (tid < s_nlong) longl[s_lbase + tid] = s_long[tid];
    if (tid < s_nhuge) huge[s_hbase + tid] = s_huge[tid];
    if (tid < nr && a1 - a0 <= FLOP_SHORT_ROW)
        row_flop_put(r0 + tid, f, a1 - a0, ncolsB, flop_out, s_rows, s_flop, s_nnza, &s_tot, &s_max, L);
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

// The listed rows of FLOP_SHORT_ROW+1 .. FLOP_WAVE_ROW entries, a wave each
// over the whole list (a persistent grid; wave j of the grid takes entries j,
// j + waves, ...), 64-entry steps with four steps' loads in flight; the
// per-bin totals are gathered per block and added to the header once.
__global__ __launch_bounds__(256) void k_long_flop(const int32_t *__restrict__ rA, const int32_t *__restrict__ cA,
                                                   const int32_t *__restrict__ rB, int64_t ncolsB,
                                                   const int32_t *__restrict__ longl, uint32_t *__restrict__ flop_out,
                                                   PlanHdr *hdr, BinLimits L) {
    __shared__ unsigned long long s_rows[NSB], s_flop[NSB], s_nnza[NSB];
    __shared__ unsigned long long s_tot, s_max;
    const int tid = threadIdx.x;
    if (tid < NSB) { s_rows[tid] = 0; s_flop[tid] = 0; s_nnza[tid] = 0; }
    if (tid == 0) { s_tot = 0; s_max = 0; }
    __syncthreads();
    const unsigned n = hdr->n_long_a;
    const unsigned nw = gridDim.x * 4;
    const int ln = tid & 63;
    for (unsigned j = blockIdx.x * 4 + (unsigned)(tid >> 6); j < n; j += nw) {   // uniform over the wave
        const int row = longl[j];
        const int b0 = rA[row], b1 = rA[row + 1];
        unsigned long long g = 0;
#pragma unroll 4
        for (int p = b0 + ln; p < b1; p += 64) g += entry_deg(p, cA, rB);
        g = wave_sum_u64(g);
        if (ln == 0) row_flop_put(row, g, b1 - b0, ncolsB, flop_out, s_rows, s_flop, s_nnza, &s_tot, &s_max, L);
    }
    __syncthreads();
    if (tid < NSB && s_rows[tid]) {
        atomicAdd(&hdr->sym_rows[tid], s_rows[tid]);
        atomicAdd(&hdr->sym_flop[tid], s_flop[tid]);
        atomicAdd(&hdr->sym_nnza[tid], s_nnza[tid]);
    }
    if (tid == 0 && s_tot) {
        atomicAdd(&hdr->total_flop, s_tot);
        atomicMax(&hdr->max_flop, s_max);
    }
}

// The listed rows of more than FLOP_WAVE_ROW entries, a block each (blocks
// past the list's length leave at once), 2048 entries' loads in flight.
__global__ __launch_bounds__(256) void k_huge_flop(const int32_t *__restrict__ rA, const int32_t *__restrict__ cA,
                                                   const int32_t *__restrict__ rB, int64_t ncolsB,
                                                   const int32_t *__restrict__ huge, uint32_t *__restrict__ flop_out,
                                                   PlanHdr *hdr, BinLimits L) {
    __shared__ unsigned long long s_g;
    if (blockIdx.x >= hdr->n_huge) return;            // uniform over the block
    const int row = huge[blockIdx.x];
    const int b0 = rA[row], b1 = rA[row + 1];
    if (threadIdx.x == 0) s_g = 0;
    __syncthreads();
    unsigned long long g = 0;
#pragma unroll 8
    for (int p = b0 + (int)threadIdx.x; p < b1; p += 256) g += entry_deg(p, cA, rB);
    g = wave_sum_u64(g);
    if ((threadIdx.x & 63) == 0) atomicAdd(&s_g, g);
    __syncthreads();
    if (threadIdx.x == 0)
        row_flop_put(row, s_g, b1 - b0, ncolsB, flop_out, hdr->sym_rows, hdr->sym_flop, hdr->sym_nnza,
                     &hdr->total_flop, &hdr->max_flop, L);
}

__global__ __launch_bounds__(256) void k_count_long_b(int n, const int32_t *__restrict__ rB, PlanHdr *hdr) {
    __shared__ int ws[5];
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int c = (i < n && rB[i + 1] - rB[i] > SHORT_ROW) ? 1 : 0;
    int tot;
    block_excl_scan<256, int>(c, tot, ws);
    if (threadIdx.x == 0 && tot) atomicAdd(&hdr->n_long_b, (unsigned long long)tot);
}

// ----------------------------------------------------------------------- binning

__global__ __launch_bounds__(256) void k_sym_scatter(int m, const uint32_t *__restrict__ flop,
                                                     const int32_t *__restrict__ rA,
                                                     int64_t ncolsB, BinOffsets off,
                                                     int32_t *__restrict__ perm, int2 *__restrict__ prow,
                                                     int32_t *__restrict__ nnz_row,
                                                     int32_t *__restrict__ slot_of, WsHdr *wh, BinLimits L) {
    __shared__ unsigned int s_cnt[NSB], s_base[NSB];
    const int tid = threadIdx.x;
    if (tid < NSB) s_cnt[tid] = 0;
    __syncthreads();
    const int i = blockIdx.x * 256 + tid;
    int b = -1;
    unsigned int r = 0;
    if (i < m) {
        b = sym_bin_l(flop[i], ncolsB, L);
        if (b == 0) nnz_row[i] = 0;
        else r = atomicAdd(&s_cnt[b], 1u);
    }
    __syncthreads();
    if (tid < NSB && s_cnt[tid]) s_base[tid] = atomicAdd(&wh->sym_cursor[tid], s_cnt[tid]);
    __syncthreads();
    if (b > 0) {
        perm[off.v[b] + s_base[b] + r] = i;
        prow[off.v[b] + s_base[b] + r] = make_int2(rA[i], rA[i + 1]);
    }
    if (b == SYM_BITMAP_BIN) {
        nnz_row[i] = 0;                       // summed over the row's work items
        slot_of[i] = (int32_t)(s_base[b] + r);
    }
}

// Rows grouped by nnz(c_i); rows above WIN_CAP are listed as heavy.
__global__ __launch_bounds__(256) void k_num_hist(int m, const int32_t *__restrict__ nnz_row,
                                                  const uint32_t *__restrict__ flop,
                                                  const int32_t *__restrict__ rA,
                                                  const int32_t *__restrict__ slot_of,
                                                  HeavyRow *__restrict__ heavy, WsHdr *wh, BinLimits L) {
    __shared__ unsigned long long s_rows[NNB], s_flop[NNB], s_nnza[NNB], s_nnzc[NNB];
    const int tid = threadIdx.x;
    if (tid < NNB) { s_rows[tid] = 0; s_flop[tid] = 0; s_nnza[tid] = 0; s_nnzc[tid] = 0; }
    __syncthreads();
    const int i = blockIdx.x * 256 + tid;
    if (i < m) {
        const int nz = nnz_row[i];
        const int b = num_bin_row(nz, flop[i], rA[i + 1] - rA[i], L);
        atomicAdd(&s_rows[b], 1ull);
        atomicAdd(&s_flop[b], (unsigned long long)flop[i]);
        atomicAdd(&s_nnza[b], (unsigned long long)(rA[i + 1] - rA[i]));
        atomicAdd(&s_nnzc[b], (unsigned long long)nz);
        if (b == NUM_HEAVY_BIN) heavy[atomicAdd(&wh->n_heavy, 1u)] = HeavyRow{i, slot_of[i]};
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
                                                     const uint32_t *__restrict__ flop,
                                                     const int32_t *__restrict__ rA,
                                                     const int64_t *__restrict__ rpts_C,
                                                     BinOffsets off, NumRow *__restrict__ rows,
                                                     WsHdr *wh, BinLimits L) {
    __shared__ unsigned int s_cnt[NNB], s_base[NNB];
    const int tid = threadIdx.x;
    if (tid < NNB) s_cnt[tid] = 0;
    __syncthreads();
    const int i = blockIdx.x * 256 + tid;
    int b = -1;
    unsigned int r = 0;
    if (i < m) {
        b = num_bin_row(nnz_row[i], flop[i], rA[i + 1] - rA[i], L);
        if (b > 0 && b != NUM_HEAVY_BIN) r = atomicAdd(&s_cnt[b], 1u);
        else b = -1;
    }
    __syncthreads();
    if (tid < NNB && s_cnt[tid]) s_base[tid] = atomicAdd(&wh->num_cursor[tid], s_cnt[tid]);
    __syncthreads();
    if (b > 0)
        rows[off.v[b] + s_base[b] + r] =
            NumRow{rA[i], rA[i + 1], ((unsigned long long)rpts_C[i] << 16) | (unsigned)nnz_row[i]};
}

// ----------------------------------------------------------------------- row prefetch

// A row of A as a hash block starts it: its range and, when it has at most G
// entries, this thread's entry k (a_ik) with the slice [lo, hi) of B row k.
// Persistent blocks load the next row's entries while the current row's
// products run, and the slices once they are done, so a row starts without
// the dependent chain row -> A range -> k -> B row pointers.
template <typename V>
struct RowPre {
    int row, a0, a1, k, lo, hi;
    V a;
};

template <int G, bool NUM, typename V>
__device__ __forceinline__ RowPre<V> row_pre_entry(int row, int a0, int a1, const int32_t *__restrict__ cA,
                                                   const V *__restrict__ vA) {
    RowPre<V> p{row, a0, a1, -1, 0, 0, V(0)};
    const int e = p.a0 + (int)threadIdx.x;
    if (p.a1 - p.a0 <= G && e < p.a1) {
        p.k = cA[e];
        if constexpr (NUM) p.a = vA[e];
    }
    return p;
}

template <typename V>
__device__ __forceinline__ void row_pre_slice(RowPre<V> &p, const int32_t *__restrict__ rB) {
    if (p.k >= 0) {
        p.lo = rB[p.k];
        p.hi = rB[p.k + 1];
    }
}

template <int G, bool NUM, typename V>
__device__ __forceinline__ RowPre<V> row_pre(int row, int a0, int a1, const int32_t *__restrict__ cA,
                                             const V *__restrict__ vA, const int32_t *__restrict__ rB) {
    RowPre<V> p = row_pre_entry<G, NUM, V>(row, a0, a1, cA, vA);
    row_pre_slice(p, rB);
    return p;
}

// ----------------------------------------------------------------------- symbolic

template <int G, int T, int U, bool PERSIST>
__global__ __launch_bounds__(G) __attribute__((amdgpu_waves_per_eu(8))) void k_sym_hash(const int32_t *__restrict__ perm, const int2 *__restrict__ prow,
                                                int64_t perm_off, unsigned nrows,
                                                const int32_t *__restrict__ cA,
                                                const int32_t *__restrict__ rB,
                                                const int32_t *__restrict__ cB,
                                                int32_t *__restrict__ nnz_row, WsHdr *wh, HashCfg hc) {
    __shared__ __align__(16) int tab[T];
    __shared__ SegLds<G, false, double> sg;
    __shared__ unsigned s_next;
    const int tid = threadIdx.x;
    // persistent over the bin's rows, or one row per block (a single trip)
    unsigned it = blockIdx.x;
    if (it >= nrows) return;                              // uniform over the block
    // persistent: each block's first two rows are blockIdx.x and blockIdx.x +
    // gridDim.x, later ones are claimed from the bin's counter (a fixed stride
    // leaves blocks with unequal work when the bin holds few rows per block);
    // thread 0 issues the claim of the row after next at the top of each row
    unsigned pend = it + gridDim.x;
    // the bin list gives the row and its A range side by side (no dependent load)
    RowPre<double> cur;
    {
        const int2 ar = prow[perm_off + it];
        if constexpr (PERSIST) cur = row_pre<G, false, double>(perm[perm_off + it], ar.x, ar.y, cA, nullptr, rB);
        else cur = RowPre<double>{perm[perm_off + it], ar.x, ar.y, -1, 0, 0, 0.0};
    }
    while (true) {
        const int row = cur.row;
        table_clear<G, T, false, double>(tab, nullptr);
        if (PERSIST && tid == 0) {
            s_next = pend;
            pend = 2 * gridDim.x + atomicAdd(&wh->sym_next[hc.bin], 1u);
        }
        __syncthreads();
        const unsigned nit = PERSIST ? s_next : nrows;
        RowPre<double> nxt{};
        if constexpr (PERSIST)
            if (nit < nrows) {
                const int2 ar = prow[perm_off + nit];
                nxt = row_pre_entry<G, false, double>(perm[perm_off + nit], ar.x, ar.y, cA, nullptr);
            }
        int cnt = 0, ovf = 0;
        unsigned prb = 0;
        auto act = [&](const int (&q)[U], const bool (&ok)[U], const double (&)[U]) {
            int col[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                // lane 0 holds row u's first product: rows with none skip their load
                const int c = __builtin_amdgcn_readfirstlane((int)ok[u]) ? cB[q[u]] : 0;   // q is a valid index
                col[u] = ok[u] ? c : 0;
            }
            if (hc.bq == 1) {
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (ok[u]) cnt += bkt_insert<false, double, 1>(tab, nullptr, T, col[u], 0.0, ovf, hc.mul, 1u, &prb);
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (ok[u]) cnt += bkt_insert<false, double>(tab, nullptr, T, col[u], 0.0, ovf, hc.mul, hc.bq, &prb);
            }
        };
        auto slice = [&](int k, int &lo, int &hi) { lo = rB[k]; hi = rB[k + 1]; };
        if (PERSIST && cur.a1 - cur.a0 <= G) enum_chunk<G, U, false, double>(cur.lo, cur.hi - cur.lo, 0.0, sg, act);
        else if (PERSIST) enum_row<G, U, false, double>(cur.a0, cur.a1, cA, nullptr, sg, slice, act);
        else enum_row<G, U, false, double>(cur.a0, cur.a1, cA, nullptr, sg, slice, act);
        __syncthreads();
        if constexpr (PERSIST)
            if (nit < nrows) row_pre_slice(nxt, rB);
        int total;
        block_excl_scan<G, int>(cnt, total, sg.wsum);
        if (tid == 0) nnz_row[row] = total;
        if (hc.count) {
            const unsigned long long t = wave_sum_u64(prb);
            if ((tid & 63) == 0 && t) atomicAdd(&wh->sym_probes[hc.bin], t);
        }
        if (ovf) {
            atomicAdd(&wh->probe_overflow, 1u);
            atomicOr(&wh->err, ERR_PROBE);
        }
        if (!PERSIST || nit >= nrows) break;
        __syncthreads();                                  // the table is reused by the next row
        it = nit;
        cur = nxt;
    }
}

// Symbolic phase of the bitmap-bin rows: one block per row, one LDS bit per
// column of C (matrices wider than the bitmap are swept in passes of NWORDS*32
// columns), then the popcount of every 4096-column chunk is kept for the
// window split of the numeric phase.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int NWORDS>
__global__ __launch_bounds__(1024) void k_sym_bitmap(const int32_t *__restrict__ perm, int64_t perm_off,
                                                     unsigned nrows,
                                                     const int32_t *__restrict__ rA,
                                                     const int32_t *__restrict__ cA,
                                                     const int32_t *__restrict__ rB,
                                                     const int32_t *__restrict__ cB, int64_t ncols,
                                                     int nchunks, uint32_t *__restrict__ chunk_cnt,
                                                     int32_t *__restrict__ nnz_row,
                                                     uint32_t *__restrict__ bmap, WsHdr *wh) {
    constexpr int G = 1024;
    constexpr int64_t WIN = (int64_t)NWORDS * 32;
    constexpr int Q_PER_CHUNK = WORDS_PER_CHUNK / 4;          // 16-byte quads per chunk
    static_assert(NWORDS % WORDS_PER_CHUNK == 0, "bitmap pass must hold whole chunks");
    static_assert(Q_PER_CHUNK == 32 && G % 4 == 0, "a chunk is counted by four threads of eight quads");
    __shared__ __align__(16) uint32_t bm[NWORDS];
    __shared__ SegLds<G, false, double> sg;
    __shared__ int s_total;
    __shared__ unsigned s_next;
    u32x4 *bm4 = reinterpret_cast<u32x4 *>(bm);
    const int tid = threadIdx.x;
    unsigned slot = blockIdx.x;                               // the row's index in the bin
    if (slot >= nrows) return;                                // uniform over the block
    // Each block's first two rows are blockIdx.x and blockIdx.x + gridDim.x;
    // later rows are claimed one at a time from a counter (row flop in this
    // bin spans three orders of magnitude, so a fixed stride leaves some
    // blocks with far more work than others).  Thread 0 issues the claim of
    // the row after next at the top of each row, so its latency hides behind
    // a whole row.
    unsigned pend = slot + gridDim.x;
    // the bitmap is clear at the start of every pass: cleared once here, then
    // by the last phase that reads it
    for (int i = tid; i < NWORDS / 4; i += G) bm4[i] = u32x4{0u, 0u, 0u, 0u};
    RowPre<double> cur;
    {
        const int r0 = perm[perm_off + slot];
        cur = row_pre<G, false, double>(r0, rA[r0], rA[r0 + 1], cA, nullptr, rB);
    }
    const int npass = (int)((ncols + WIN - 1) / WIN);
    auto slice = [&](int k, int &lo, int &hi) { lo = rB[k]; hi = rB[k + 1]; };
    while (true) {
        const int row = cur.row;
        if (tid == 0) {
            s_total = 0;
            s_next = pend;
            pend = 2 * gridDim.x + atomicAdd(&wh->bm_next, 1u);
        }
        __syncthreads();
        // the next row's A entries are loaded while this row's products run
        const unsigned nslot = s_next;
        RowPre<double> nxt{};
        if (nslot < nrows) {
            const int r1 = perm[perm_off + nslot];
            nxt = row_pre_entry<G, false, double>(r1, rA[r1], rA[r1 + 1], cA, nullptr);
        }
        for (int pass = 0; pass < npass; ++pass) {
            const int64_t c0 = (int64_t)pass * WIN;
            const uint32_t wcols = (uint32_t)(ncols - c0 < WIN ? ncols - c0 : WIN);
            const int nch = (int)((wcols + CHUNK_COLS - 1) >> CHUNK_SHIFT);
            const int nq = nch * Q_PER_CHUNK;                // whole chunks, 16 bytes at a time
            const int chunk0 = (int)(c0 >> CHUNK_SHIFT);
            auto act = [&](const int (&q)[U_SEG], const bool (&ok)[U_SEG], const double (&)[U_SEG]) {
                int col[U_SEG];
#pragma unroll
                for (int u = 0; u < U_SEG; ++u) {
                    const int c = cB[q[u]];                   // q is always a valid index
                    col[u] = ok[u] ? c : -1;
                }
#pragma unroll
                for (int u = 0; u < U_SEG; ++u) {
                    const uint32_t off = (uint32_t)((int64_t)col[u] - c0);
                    if (ok[u] && off < wcols) atomicOr(&bm[off >> 5], 1u << (off & 31));
                }
            };
            if (cur.a1 - cur.a0 <= G) enum_chunk<G, U_SEG, false, double>(cur.lo, cur.hi - cur.lo, 0.0, sg, act);
            else enum_row<G, U_SEG, false, double>(cur.a0, cur.a1, cA, nullptr, sg, slice, act);
            __syncthreads();
            // per-chunk counts: four threads per chunk of 32 quads, eight quads
            // each, read in an order rotated by the thread so that the lanes of
            // a wave fall on different banks
            for (int t = tid; t < nch * 4; t += G) {
                int c = 0;
#pragma unroll
                for (int j = 0; j < Q_PER_CHUNK / 4; ++j) {
                    const u32x4 v = bm4[t * (Q_PER_CHUNK / 4) + ((j + t) & (Q_PER_CHUNK / 4 - 1))];
                    c += __popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w);
                }
                c += dpp_move<0xB1, 0xF>(c);          // quad lanes (1,0,3,2): xor 1
                c += dpp_move<0x4E, 0xF>(c);          // quad lanes (2,3,0,1): xor 2
                if ((t & 3) == 0) {
                    chunk_cnt[(size_t)slot * nchunks + chunk0 + t / 4] = (uint32_t)c;
                    atomicAdd(&s_total, c);
                }
            }
            __syncthreads();
            // the row's bits are kept for the numeric windows (whole chunks); a
            // one-pass row that ends up with at most WIN_CAP entries takes a
            // hash table instead and needs none.  The bitmap is cleared behind.
            if (bmap && (npass > 1 || s_total > WIN_CAP)) {
                u32x4 *dst = reinterpret_cast<u32x4 *>(bmap + ((size_t)slot * nchunks + chunk0) * WORDS_PER_CHUNK);
                for (int i = tid; i < nq; i += G) {
                    __builtin_nontemporal_store(bm4[i], &dst[i]);
                    bm4[i] = u32x4{0u, 0u, 0u, 0u};
                }
            } else {
                for (int i = tid; i < nq; i += G) bm4[i] = u32x4{0u, 0u, 0u, 0u};
            }
            __syncthreads();
        }
        if (tid == 0) nnz_row[row] = s_total;
        if (nslot >= nrows) break;
        row_pre_slice(nxt, rB);
        slot = nslot;
        cur = nxt;
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

// Column windows of the heavy rows.  Greedy split of a row's chunks: a window
// opens at the first non-empty chunk and takes chunks while its LDS footprint
// fits RANK_BUDGET words (in half words: 256 per chunk for its 128 bit/rank
// words, 3 per entry for the value word and a half-word staging slot); its
// first chunk is always taken.  The windows are laid out sorted by first
// chunk so that the blocks running side by side read the same column slices
// of the shared B rows.
// One wave per heavy row: the row's chunk counts are read 64 at a time
// (coalesced) and their footprints prefix-summed across the wave; a window's
// end is then the first lane whose running footprint overflows (a ballot), so
// the split costs a few wave operations per window, not a step per chunk.
// f(lo, hi, cnt) is called by every lane of the wave for every window.
template <class F>
__device__ __forceinline__ void wave_windows(const uint32_t *__restrict__ cc, int nchunks, F f) {
    constexpr int CAP = 2 * RANK_BUDGET;
    const int ln = threadIdx.x & 63;
    bool open = false;                   // wave-uniform state of the window being built
    int start = 0, units = 0, cnt = 0;
    for (int t = 0; t < nchunks; t += WAVE) {
        const int n = min(WAVE, nchunks - t);
        const int x = ln < n ? (int)cc[t + ln] : 0;
        const int pu = wave_incl_scan<int>(ln < n ? 2 * WORDS_PER_CHUNK + 3 * x : 0);
        const int px = wave_incl_scan<int>(x);
        int pos = 0;                     // first chunk of the tile not yet placed
        while (pos < n) {
            int first = pos;             // lanes from here on may end the window
            if (!open) {
                const uint64_t ne = __ballot(ln >= pos && x > 0);
                if (ne == 0) break;
                pos = __ffsll((unsigned long long)ne) - 1;
                open = true;
                start = t + pos;
                units = 0;
                cnt = 0;
                first = pos + 1;
            }
            const int ub = pos > 0 ? __builtin_amdgcn_readlane(pu, pos - 1) : 0;
            const int xb = pos > 0 ? __builtin_amdgcn_readlane(px, pos - 1) : 0;
            const uint64_t over = __ballot(ln >= first && ln < n && units + pu - ub > CAP);
            if (over == 0) {
                units += __builtin_amdgcn_readlane(pu, n - 1) - ub;
                cnt += __builtin_amdgcn_readlane(px, n - 1) - xb;
                pos = n;
            } else {
                const int e = __ffsll((unsigned long long)over) - 1;   // e > pos, or the window spans tiles
                cnt += (e > 0 ? __builtin_amdgcn_readlane(px, e - 1) : 0) - xb;
                f(start, t + e, cnt);
                open = false;
                pos = e;
            }
        }
    }
    if (open) f(start, nchunks, cnt);
}

// Blocks of 16 heavy rows (one per wave); window counts per first chunk are
// gathered in LDS first (one global atomic per chunk and block) when the
// chunks fit LDS_WIN_CHUNKS.
constexpr int LDS_WIN_CHUNKS = 4096;

__global__ __launch_bounds__(1024) void k_win_count(const HeavyRow *__restrict__ heavy, int nchunks,
                                                    const uint32_t *__restrict__ chunk_cnt,
                                                    uint32_t *__restrict__ whist, WsHdr *wh) {
    __shared__ uint32_t hist[LDS_WIN_CHUNKS];
    __shared__ unsigned s_items;
    const bool lds = nchunks <= LDS_WIN_CHUNKS;
    const int tid = threadIdx.x, ln = tid & 63;
    if (lds)
        for (int c = tid; c < nchunks; c += 1024) hist[c] = 0u;
    if (tid == 0) s_items = 0;
    __syncthreads();
    const unsigned h = blockIdx.x * 16 + (tid >> 6);
    if (h < wh->n_heavy) {
        const uint32_t *cc = chunk_cnt + (size_t)heavy[h].slot * nchunks;
        bool wide = false;
        for (int c = ln; c < nchunks; c += WAVE) wide |= cc[c] > (uint32_t)CHUNK_COLS;
        if (wide) atomicOr(&wh->err, ERR_CHUNK);
        unsigned n = 0;
        wave_windows(cc, nchunks, [&](int lo, int, int) {
            if (ln == 0) {
                if (lds) atomicAdd(&hist[lo], 1u);
                else atomicAdd(&whist[lo], 1u);
            }
            ++n;
        });
        if (ln == 0) atomicAdd(&s_items, n);
    }
    __syncthreads();
    if (lds)
        for (int c = tid; c < nchunks; c += 1024)
            if (hist[c]) atomicAdd(&whist[c], hist[c]);
    if (tid == 0 && s_items) atomicAdd(&wh->n_items, s_items);
}

// exclusive scan of the per-chunk window counts (one block)
__global__ __launch_bounds__(1024) void k_win_scan(uint32_t *__restrict__ whist, int nchunks,
                                                   unsigned cap, WsHdr *wh) {
    __shared__ int ws[17];
    int carry = 0;
    for (int c0 = 0; c0 < nchunks; c0 += 1024) {
        const int c = c0 + (int)threadIdx.x;
        const int v = c < nchunks ? (int)whist[c] : 0;
        int tot;
        const int ex = block_excl_scan<1024, int>(v, tot, ws);
        if (c < nchunks) whist[c] = (uint32_t)(carry + ex);
        carry += tot;
    }
    if (threadIdx.x == 0 && (unsigned)carry > cap) atomicOr(&wh->err, ERR_ITEMS);
}

// Windows laid out sorted by first chunk: a window's slot is its chunk's
// start (wpos) plus a block base reserved with one atomic per chunk and block
// plus its rank within the block (LDS), or one global atomic per window when
// the chunks do not fit LDS.
__global__ __launch_bounds__(1024) void k_win_emit(const HeavyRow *__restrict__ heavy, int nchunks,
                                                   const uint32_t *__restrict__ chunk_cnt,
                                                   const int64_t *__restrict__ rpts_C,
                                                   const int32_t *__restrict__ rA,
                                                   const uint32_t *__restrict__ wpos, uint32_t *__restrict__ wcur,
                                                   WinItem *__restrict__ items, unsigned cap, WsHdr *wh) {
    __shared__ uint32_t cntl[LDS_WIN_CHUNKS], basel[LDS_WIN_CHUNKS];
    if (wh->err & ERR_ITEMS) return;                 // uniform over the grid
    const bool lds = nchunks <= LDS_WIN_CHUNKS;
    const int tid = threadIdx.x, ln = tid & 63;
    const unsigned h = blockIdx.x * 16 + (tid >> 6);
    const bool mine = h < wh->n_heavy;
    HeavyRow hr{0, 0};
    const uint32_t *cc = chunk_cnt;
    if (mine) {
        hr = heavy[h];
        cc = chunk_cnt + (size_t)hr.slot * nchunks;
    }
    if (lds) {
        for (int c = tid; c < nchunks; c += 1024) cntl[c] = 0u;
        __syncthreads();
        if (mine)
            wave_windows(cc, nchunks, [&](int lo, int, int) {
                if (ln == 0) atomicAdd(&cntl[lo], 1u);
            });
        __syncthreads();
        for (int c = tid; c < nchunks; c += 1024) {
            const uint32_t k = cntl[c];
            if (k) basel[c] = atomicAdd(&wcur[c], k);
            cntl[c] = 0u;
        }
        __syncthreads();
    }
    if (!mine) return;
    int64_t pos = rpts_C[hr.row];
    const int a0 = rA[hr.row], a1 = rA[hr.row + 1];
    wave_windows(cc, nchunks, [&](int lo, int hi, int cnt) {
        if (ln == 0) {
            const unsigned at = wpos[lo] + (lds ? basel[lo] + atomicAdd(&cntl[lo], 1u) : atomicAdd(&wcur[lo], 1u));
            if (at < cap) items[at] = WinItem{hr.row, lo, hi, cnt, pos, a0, a1, hr.slot, 0};
        }
        pos += cnt;
    });
}

// ----------------------------------------------------------------------- bucket B by chunk

// Multiplier of the scrambled order of a row of len > 1 entries: odd, near
// len times the golden ratio's fractional part, coprime to len, so that
// t -> t*K mod len is a permutation that sends neighbours far apart.
__device__ inline int scramble_mul(int len) {
    int k = (int)((double)len * 0.6180339887498949) | 1;
    for (;; k += 2) {
        if (k >= len) return 1;
        int a = len, b = k;
        while (b) { const int t = a % b; a = b; b = t; }
        if (a == 1) return k;
    }
}

// Besides the bucketed copy, every row of B is also written in a scrambled
// order (bs: entry t of the row goes to position t*K mod len).  The symbolic
// bitmap reads that copy: consecutive lanes then carry columns from all over
// the row even when the input rows are sorted, so the LDS atomic ORs of a
// wave rarely meet in one word.
// Rows of at most SHORT_ROW entries keep their order in bc (windows read them
// whole and filter by column); longer rows are listed for k_bucket_long.
// bperm[p] is the original position of the entry now at p of bc (values
// follow in numeric).
__global__ __launch_bounds__(256) void k_bucket_short(int n, const int32_t *__restrict__ rB,
                                                      const int32_t *__restrict__ cB,
                                                      int32_t *__restrict__ bc, int32_t *__restrict__ bperm,
                                                      int32_t *__restrict__ bs,
                                                      int32_t *__restrict__ long_id,
                                                      int32_t *__restrict__ long_list, WsHdr *wh) {
    const int row = blockIdx.x * 256 + (int)threadIdx.x;
    if (row >= n) return;
    const int b0 = rB[row], b1 = rB[row + 1];
    if (b1 - b0 > SHORT_ROW) {
        const int li = (int)atomicAdd(&wh->n_long, 1u);
        long_id[row] = li;
        long_list[li] = row;
        return;
    }
    long_id[row] = -1;
    const int len = b1 - b0;
    const int K = len > 1 ? scramble_mul(len) : 1;
    int j = 0;
    for (int p = b0; p < b1; ++p) {
        const int c = cB[p];
        bc[p] = c;
        bperm[p] = p;
        bs[b0 + j] = c;
        j += K;
        if (j >= len) j -= len;
    }
}

// Longer rows: counting sort by chunk id with LDS counters, and the chunk
// offsets (relative to the row start) kept as the row's index:
// idx[li*(nchunks+1) + c] = first position of chunk c, idx[..+nchunks] = len.
// The counting pass also writes the row's scrambled copy into bs.
template <int NCNT>
__global__ __launch_bounds__(256) void k_bucket_long(const int32_t *__restrict__ long_list,
                                                     const WsHdr *wh, const int32_t *__restrict__ rB,
                                                     const int32_t *__restrict__ cB,
                                                     int32_t *__restrict__ bc, int32_t *__restrict__ bperm,
                                                     int32_t *__restrict__ bs,
                                                     int32_t *__restrict__ idx, int nchunks) {
    __shared__ int cnt[NCNT];
    __shared__ int ws[5];
    __shared__ int s_k;
    const int tid = threadIdx.x;
    const unsigned nl = wh->n_long;
    for (unsigned li = blockIdx.x; li < nl; li += gridDim.x) {
        const int row = long_list[li];
        const int b0 = rB[row], b1 = rB[row + 1];
        const int len = b1 - b0;
        for (int c = tid; c < nchunks; c += 256) cnt[c] = 0;
        if (tid == 0) s_k = scramble_mul(len);
        __syncthreads();
        {
            const int K = s_k;
            const int jstep = (int)(((int64_t)256 * K) % len);
            int j = (int)(((int64_t)tid * K) % len);
            for (int p = b0 + tid; p < b1; p += 256) {
                const int col = cB[p];
                atomicAdd(&cnt[col >> CHUNK_SHIFT], 1);
                bs[b0 + j] = col;
                j += jstep;
                if (j >= len) j -= len;
            }
        }
        __syncthreads();
        int32_t *ix = idx + (size_t)li * (nchunks + 1);
        int carry = 0;
        for (int c0 = 0; c0 < nchunks; c0 += 256) {
            const int c = c0 + tid;
            const int v = c < nchunks ? cnt[c] : 0;
            int tot;
            const int ex = block_excl_scan<256, int>(v, tot, ws);
            if (c < nchunks) {
                cnt[c] = carry + ex;
                ix[c] = carry + ex;
            }
            carry += tot;
        }
        if (tid == 0) ix[nchunks] = len;
        __syncthreads();
        for (int p = b0 + tid; p < b1; p += 256) {
            const int col = cB[p];
            const int pos = atomicAdd(&cnt[col >> CHUNK_SHIFT], 1);
            bc[b0 + pos] = col;
            bperm[b0 + pos] = p;
        }
        __syncthreads();
    }
}

template <typename V>
__global__ __launch_bounds__(256) void k_gather_vals(int64_t n, const int32_t *__restrict__ bperm,
                                                     const V *__restrict__ vB, V *__restrict__ bv) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += stride) bv[p] = vB[bperm[p]];
}

// What the window kernel needs of the B row an entry a_ik selects, per entry
// of A (so that a window's slices are one load plus the chunk index away from
// its A range, not three): ki[e] = {start of B row k, its chunk-index id}, or
// for a row without an index {start, -1 - length}.
__global__ __launch_bounds__(256) void k_entry_brow(int64_t nnz, const int32_t *__restrict__ cA,
                                                    const int32_t *__restrict__ rB,
                                                    const int32_t *__restrict__ long_id, int2 *__restrict__ ki) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nnz; e += stride) {
        const int k = cA[e];
        const int r0 = rB[k], li = long_id[k];
        ki[e] = make_int2(r0, li >= 0 ? li : -1 - (rB[k + 1] - r0));
    }
}

// ----------------------------------------------------------------------- numeric

// Column passes of the rank sort of a wide bin before it falls back to the
// bucket sort (measured at 2^20 columns, 13 passes: the 11264-slot bin took
// 13.3 ms ranked and 10.6 ms bucket-sorted).
__host__ __device__ constexpr int rank_passes(int) { return 2; }

// LDS of a numeric hash block besides its table: the enumeration state, and
// (512-thread bins) extra words so that the idle enumeration LDS plus them can
// hold a rank bitmap of 64 K columns per pass for sorted output.
template <int G, typename V>
struct NumLds {
    SegLds<G, true, V> sg;
    uint2 extra[G == 512 ? 1024 : 1];
};

template <int G, int T, int U, bool SORTED, typename V, bool PERSIST>
__global__ __launch_bounds__(G) void k_num_hash(const NumRow *__restrict__ rows, int64_t perm_off, unsigned nrows,
                                                const int32_t *__restrict__ cA,
                                                const V *__restrict__ vA,
                                                const int32_t *__restrict__ rB,
                                                const int32_t *__restrict__ cB,
                                                const V *__restrict__ vB,
                                                int32_t *__restrict__ cC, V *__restrict__ vC,
                                                WsHdr *wh, HashCfg hc, int64_t ncolsB) {
    __shared__ __align__(16) int keys[T];
    __shared__ __align__(16) V vals[T];
    __shared__ __align__(16) NumLds<G, V> lds;
    __shared__ int rank_ws[G / WAVE + 1];
    SegLds<G, true, V> &sg = lds.sg;
    __shared__ unsigned s_next;
    const int tid = threadIdx.x;
    // persistent over the bin's rows (the first two blockIdx.x and blockIdx.x
    // + gridDim.x, later ones claimed from the bin's counter, the claim of the
    // row after next issued at the top of each row), or one row per block (a
    // single trip)
    unsigned it = blockIdx.x;
    if (it >= nrows) return;                                  // uniform over the block
    unsigned pend = it + gridDim.x;
    // the bin list gives each row's A range and place in C (no dependent load);
    // RowPre.row carries the list index
    NumRow nr = rows[perm_off + it];
    RowPre<V> cur;
    if constexpr (PERSIST) cur = row_pre<G, true, V>((int)it, nr.a0, nr.a1, cA, vA, rB);
    else cur = RowPre<V>{(int)it, nr.a0, nr.a1, -1, 0, 0, V(0)};
    while (true) {
        table_clear<G, T, true, V>(keys, vals);
        if (PERSIST && tid == 0) {
            s_next = pend;
            pend = 2 * gridDim.x + atomicAdd(&wh->num_next[hc.bin], 1u);
        }
        __syncthreads();
        // the next row's A entries are loaded while this row's products run
        const unsigned nit = PERSIST ? s_next : nrows;
        RowPre<V> nxt{};
        NumRow nnr{};
        if constexpr (PERSIST)
            if (nit < nrows) {
                nnr = rows[perm_off + nit];
                nxt = row_pre_entry<G, true, V>((int)nit, nnr.a0, nnr.a1, cA, vA);
            }
        int ovf = 0;
        unsigned prb = 0;
        auto act = [&](const int (&q)[U], const bool (&ok)[U], const V (&av)[U]) {
            int col[U];
            V x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                // lane 0 holds row u's first product: rows with none skip their loads
                int c = 0;
                V b = V(0);
                if (__builtin_amdgcn_readfirstlane((int)ok[u])) {
                    c = cB[q[u]];                             // q is a valid index
                    b = vB[q[u]];
                }
                col[u] = ok[u] ? c : 0;
                x[u] = ok[u] ? av[u] * b : V(0);
            }
            if (hc.bq == 1) {
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (ok[u]) bkt_insert<true, V, 1>(keys, vals, T, col[u], x[u], ovf, hc.mul, 1u, &prb);
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (ok[u]) bkt_insert<true, V>(keys, vals, T, col[u], x[u], ovf, hc.mul, hc.bq, &prb);
            }
        };
        auto slice = [&](int k, int &lo, int &hi) { lo = rB[k]; hi = rB[k + 1]; };
        if (PERSIST && cur.a1 - cur.a0 <= G) enum_chunk<G, U, true, V>(cur.lo, cur.hi - cur.lo, cur.a, sg, act);
        else if (PERSIST) enum_row<G, U, true, V>(cur.a0, cur.a1, cA, vA, sg, slice, act);
        else enum_row<G, U, true, V>(cur.a0, cur.a1, cA, vA, sg, slice, act);
        __syncthreads();
        if constexpr (PERSIST)
            if (nit < nrows) row_pre_slice(nxt, rB);          // and then the slices of their B rows
        if (ovf) {
            atomicAdd(&wh->probe_overflow, 1u);
            atomicOr(&wh->err, ERR_PROBE);
        }
        if (hc.count) {
            const unsigned long long t = wave_sum_u64(prb);
            if ((tid & 63) == 0 && t) atomicAdd(&wh->num_probes[hc.bin], t);
        }
        const int64_t o = (int64_t)(nr.out_n >> 16);
        const int expected = (int)(nr.out_n & 0xFFFFu);
        bool ranked = false;
        if constexpr (SORTED && G >= 512) {
            // Sorted output of a wide bin by rank instead of a bucket sort: the
            // columns of C are swept in passes of as many columns as a bitmap in
            // the (now idle) enumeration LDS holds; in a pass, the keys inside
            // it set their bit, and an exclusive popcount prefix per word plus
            // the keys of the earlier passes gives each its rank.  Each thread
            // holds its slots (lane by lane) in registers through the passes;
            // the entries then move to their ranks inside the table and leave
            // in coalesced runs (stores straight to scattered places of C cost
            // partial-line writes to HBM).  Up to rank_passes(T) passes; wider
            // matrices are bucket-sorted.
            constexpr int RW = (int)(sizeof(NumLds<G, V>) / sizeof(uint2));
            constexpr int64_t PW = (int64_t)RW * 32;
            constexpr int SL = T / G;                             // slots per thread
            static_assert(T % G == 0, "table size a multiple of the block");
            const int npass = (int)((ncolsB + PW - 1) / PW);
            if (npass <= rank_passes(T)) {
                uint2 *rw = reinterpret_cast<uint2 *>(&lds);
                int kr[SL], rk[SL];
#pragma unroll
                for (int j = 0; j < SL; ++j) {
                    kr[j] = keys[j * G + tid];
                    rk[j] = -1;
                }
                int base = 0;
                for (int ps = 0; ps < npass; ++ps) {
                    const int c0 = (int)(ps * PW);
                    const int64_t span = ncolsB - c0 < PW ? ncolsB - c0 : PW;
                    const int nw = (int)((span + 31) >> 5);
                    for (int i = tid; i < nw; i += G) rw[i] = make_uint2(0u, 0u);
                    __syncthreads();
#pragma unroll
                    for (int j = 0; j < SL; ++j) {
                        const uint32_t off = (uint32_t)(kr[j] - c0);
                        if (kr[j] != -1 && off < (uint32_t)span) atomicOr(&rw[off >> 5].x, 1u << (off & 31));
                    }
                    __syncthreads();
                    const int S = (nw + G - 1) / G;
                    const int w0 = tid * S;
                    int c = 0;
                    for (int j = 0; j < S; ++j)
                        if (w0 + j < nw) c += __popc(rw[w0 + j].x);
                    int total;
                    int pre = base + block_excl_scan<G, int>(c, total, rank_ws);
                    for (int j = 0; j < S; ++j)
                        if (w0 + j < nw) {
                            rw[w0 + j].y = (uint32_t)pre;
                            pre += __popc(rw[w0 + j].x);
                        }
                    __syncthreads();
#pragma unroll
                    for (int j = 0; j < SL; ++j) {
                        const uint32_t off = (uint32_t)(kr[j] - c0);
                        if (kr[j] != -1 && off < (uint32_t)span) {
                            const uint2 e = rw[off >> 5];
                            rk[j] = (int)(e.y + __popc(e.x & ((1u << (off & 31)) - 1u)));
                        }
                    }
                    base += total;
                    __syncthreads();                          // the bitmap is reused by the next pass
                }
                // ranks are a permutation of [0, base), base <= T: every entry
                // is read before any moves
                V vr[SL];
#pragma unroll
                for (int j = 0; j < SL; ++j) vr[j] = vals[j * G + tid];
                __syncthreads();
#pragma unroll
                for (int j = 0; j < SL; ++j)
                    if (rk[j] >= 0) {
                        keys[rk[j]] = kr[j];
                        vals[rk[j]] = vr[j];
                    }
                __syncthreads();
                const int n = base < expected ? base : expected;
                for (int i = tid; i < n; i += G) {
                    __builtin_nontemporal_store(keys[i], &cC[o + i]);
                    __builtin_nontemporal_store(vals[i], &vC[o + i]);
                }
                if (base != expected && tid == 0) atomicOr(&wh->err, ERR_COUNT);
                ranked = true;
            }
        }
        if constexpr (!SORTED) compact_store_unsorted<G, T, V>(keys, vals, sg.wsum, o, expected, cC, vC, &wh->err);
        else if (!ranked) compact_store<G, T, SORTED, V>(keys, vals, sg.wsum, o, expected, cC, vC, &wh->err);
        if (!PERSIST || nit >= nrows) break;
        __syncthreads();                                      // the table is reused by the next row
        it = nit;
        cur = nxt;
        nr = nnr;
    }
}

// Claim of the next window for the block (thread 0 only): windows, sorted by
// first chunk, are split into eight contiguous ranges, one per group of blocks
// blockIdx % 8 (workgroups are dealt round-robin over the XCDs, so a group is
// one XCD and the blocks sharing an L2 read the same column slices of B); a
// block takes its group's windows in order and then helps the other groups.
constexpr unsigned WIN_NONE = 0xFFFFFFFFu;

// Claims run one window ahead of their use: the block holds the raw counter
// value of an issued claim (raw) and turns it into a window index only when
// that window is next, so the atomic's latency is not waited for.
__device__ __forceinline__ unsigned win_resolve(WsHdr *wh, unsigned nitems, unsigned g0, unsigned &d,
                                                unsigned &raw) {
    constexpr unsigned NG = 8;
    while (d < NG) {
        const unsigned g = (g0 + d) % NG;
        const unsigned lo = (unsigned)((unsigned long long)nitems * g / NG);
        const unsigned hi = (unsigned)((unsigned long long)nitems * (g + 1) / NG);
        if (lo + raw < hi) return lo + raw;
        if (++d < NG) raw = atomicAdd(&wh->win_next[(g0 + d) % NG], 1u);   // this group is done
    }
    return WIN_NONE;
}

__device__ __forceinline__ void win_issue(WsHdr *wh, unsigned g0, unsigned d, unsigned &raw) {
    if (d < 8) raw = atomicAdd(&wh->win_next[(g0 + d) % 8], 1u);
}

// Quads (16-byte groups of four bitmap words) of the next window that each
// thread holds in registers while the current window's output leaves: thread
// t takes the contiguous quads [t*S4, t*S4 + S4) of the window, S4 =
// ceil(nwords / (4*G)), which covers the largest window RANK_BUDGET allows.
constexpr int WIN_PRE_QUADS = (RANK_BUDGET + 4 * WIN_G - 1) / (4 * WIN_G);

// Numeric phase of the heavy rows, one column window at a time by a
// persistent grid (one block per CU slot).  A window's output columns are
// marked first (one bit per column in LDS), their ranks are the exclusive
// prefix of the bit counts, and the products are then added straight into a
// dense array of values indexed by rank: no hashing, no probing, and the
// window leaves in ascending column order.  Each product also writes its
// column at its rank (every product of a column writes the same value), so
// the output columns need no separate expansion of the bits: the work is
// spread over the products instead of over words whose bit counts vary from
// 0 to 32 within a wave.  The slice of B row k inside the window is two loads
// from k's chunk index, or the whole row (filtered by column) when the row is
// short.
// When the symbolic phase kept the rows' bits, a window's words are loaded
// into registers (contiguous quads per thread) while the previous window's
// output is being stored, when the registers of the products are free; the
// window then starts with one pass that counts each thread's bits, scans the
// counts across the block and writes every word with its rank prefix to LDS.
// Without stored bits (SPGEMM_LOW_MEMORY) a first pass over the products
// marks them.  For a row of at most G entries of A each thread holds one a_ik
// and its slice; the next window's item and a_ik are loaded before the
// current window's products, its B row pointers and bits before the current
// output stores and its slice after them, so every level of that chain hides
// behind work the block does anyway.  Output stores are left in flight (a
// block barrier does not wait for stores).
template <typename V>
__global__ __launch_bounds__(WIN_G) void k_num_window(const WinItem *__restrict__ items, unsigned nitems,
                                                     const int2 *__restrict__ ki,
                                                     const V *__restrict__ vA,
                                                     const int32_t *__restrict__ idx, int nchunks,
                                                     const int32_t *__restrict__ bc,
                                                     const V *__restrict__ bv,
                                                     int32_t *__restrict__ cC, V *__restrict__ vC,
                                                     const uint32_t *__restrict__ bmap, WsHdr *wh) {
    constexpr int G = WIN_G;
    constexpr int QPC = WORDS_PER_CHUNK / 4;                       // quads per chunk
    __shared__ __align__(16) unsigned long long buf[RANK_BUDGET];   // words, then values
    __shared__ SegLds<G, true, V> sg;
    __shared__ unsigned long long s_wsum[G / WAVE + 1];
    __shared__ unsigned s_claim[2];
    const int tid = threadIdx.x;
    const int nch1 = nchunks + 1;
    const unsigned g0 = blockIdx.x % 8;
    unsigned gd = 0;                     // thread 0: groups done
    unsigned raw = 0;                    // thread 0: raw value of the claim in flight
    bool bad = false;
    int ptotal = 0, pnseg = 0;           // products and segments laid out at the window's start

    // the slice inside chunks [ch_lo, ch_hi) of the B row that entry info b
    // describes (k_entry_brow)
    auto slice_of = [&](int2 b, int ch_lo, int ch_hi, int &lo, int &hi) {
        if (b.y >= 0) {
            const int32_t *ix = idx + (size_t)b.y * nch1;
            lo = b.x + ix[ch_lo];
            hi = b.x + ix[ch_hi];
        } else {
            lo = b.x;
            hi = b.x - 1 - b.y;
        }
    };
    // this thread's quads of window w's stored bits (zero past the window)
    auto load_bits = [&](const WinItem &w, u32x4 (&q)[WIN_PRE_QUADS]) {
        const int nq = (w.ch_hi - w.ch_lo) * QPC;
        const int s4 = (nq + G - 1) / G;
        const u32x4 *src = reinterpret_cast<const u32x4 *>(bmap + ((size_t)w.slot * nchunks + w.ch_lo) *
                                                                      WORDS_PER_CHUNK);
#pragma unroll
        for (int k = 0; k < WIN_PRE_QUADS; ++k) {
            const int qi = tid * s4 + k;
            q[k] = u32x4{0u, 0u, 0u, 0u};
            if (k < s4 && qi < nq) q[k] = __builtin_nontemporal_load(&src[qi]);
        }
    };

    if (tid == 0) {
        win_issue(wh, g0, gd, raw);
        s_claim[0] = win_resolve(wh, nitems, g0, gd, raw);
        win_issue(wh, g0, gd, raw);
    }
    __syncthreads();
    unsigned cur = __builtin_amdgcn_readfirstlane(s_claim[0]);
    u32x4 q[WIN_PRE_QUADS];              // the current window's bits (stored-bits mode)
    int par = 0;
    WinItem it{};
    int lo = 0, hi = 0;
    V a = V(0);
    if (cur != WIN_NONE) {
        it = items[cur];
        if (it.a1 - it.a0 <= G && it.a0 + tid < it.a1) {
            a = vA[it.a0 + tid];
            slice_of(ki[it.a0 + tid], it.ch_lo, it.ch_hi, lo, hi);
        }
        if (bmap) load_bits(it, q);
    }
    while (cur != WIN_NONE) {
        if (tid == 0) {
            s_claim[par ^ 1] = win_resolve(wh, nitems, g0, gd, raw);
            win_issue(wh, g0, gd, raw);
        }
        const bool resident = it.a1 - it.a0 <= G;
        const int ch_lo = it.ch_lo, count = it.count;
        const int nwords = (it.ch_hi - ch_lo) * WORDS_PER_CHUNK;
        const uint32_t span = (uint32_t)nwords * 32u;
        const int c0 = ch_lo << CHUNK_SHIFT;
        uint32_t *w32 = reinterpret_cast<uint32_t *>(buf);   // word w: bits w32[2w], rank prefix w32[2w+1]
        V *vals = reinterpret_cast<V *>(buf + nwords);
        int32_t *stage = reinterpret_cast<int32_t *>(buf + nwords + count);   // columns by rank

        // a row of more than G entries of A: its slices G entries at a time
        auto walk_row = [&](auto &&act, auto tag) {
            constexpr bool NUMW = decltype(tag)::value;
            for (int cb = it.a0; cb < it.a1; cb += G) {
                const int e = cb + tid;
                int l = 0, h = 0;
                V av = V(0);
                if (e < it.a1) {
                    slice_of(ki[e], it.ch_lo, it.ch_hi, l, h);
                    if constexpr (NUMW) av = vA[e];
                }
                if constexpr (NUMW) enum_chunk<G, U_RANK2, true, V>(l, h - l, av, sg, act);
                else enum_chunk<G, U_RANK1, false, V>(l, h - l, V(0), sg, act);
            }
        };
        if (bmap) {
            // ranks: this thread's bit count, its exclusive prefix over the
            // block, then each word with its prefix (two words per 16 bytes).
            // For a row of at most G entries of A the same block scan also
            // lays out the product segments (slice lengths and the count of
            // non-empty slices), packed in one 64-bit value per thread: the
            // bit count in bits 42..63, the slice length in 11..41, the
            // segment flag in 0..10 (window totals stay below 2^22, 2^31 and
            // 2^11).
            const int nq = nwords / 4;
            const int s4 = (nq + G - 1) / G;
            int c = 0;
#pragma unroll
            for (int k = 0; k < WIN_PRE_QUADS; ++k)
                c += __popc(q[k].x) + __popc(q[k].y) + __popc(q[k].z) + __popc(q[k].w);
            const int len = resident ? hi - lo : 0;
            const unsigned long long packed = ((unsigned long long)c << 42) | ((unsigned long long)len << 11) |
                                              (len > 0 ? 1ull : 0ull);
            unsigned long long ptot;
            const unsigned long long pex = block_excl_scan<G, unsigned long long>(packed, ptot, s_wsum);
            int pre = (int)(pex >> 42);
            const int total = (int)(ptot >> 42);
            if (resident) {
                const int pre_ne = (int)(pex & 2047u);
                if (len > 0) {
                    const int po = (int)((pex >> 11) & 0x7FFFFFFFull);
                    sg.base[pre_ne] = lo - po;
                    sg.off[pre_ne] = po;
                    sg.a[pre_ne] = a;
                }
                ptotal = __builtin_amdgcn_readfirstlane((int)((ptot >> 11) & 0x7FFFFFFFull));
                pnseg = __builtin_amdgcn_readfirstlane((int)(ptot & 2047u));
            }
            u32x4 *b4 = reinterpret_cast<u32x4 *>(buf);
#pragma unroll
            for (int k = 0; k < WIN_PRE_QUADS; ++k) {
                const int qi = tid * s4 + k;
                if (k < s4 && qi < nq) {
                    const uint32_t p0 = (uint32_t)pre, p1 = p0 + __popc(q[k].x), p2 = p1 + __popc(q[k].y),
                                   p3 = p2 + __popc(q[k].z);
                    b4[2 * qi] = u32x4{q[k].x, p0, q[k].y, p1};
                    b4[2 * qi + 1] = u32x4{q[k].z, p2, q[k].w, p3};
                    pre = (int)(p3 + __popc(q[k].w));
                }
            }
            if (total != count) bad = true;
            for (int i = tid; i < count; i += G) vals[i] = V(0);
        } else {
            for (int i = tid; i < nwords; i += G) buf[i] = 0ull;
            for (int i = tid; i < count; i += G) vals[i] = V(0);
            __syncthreads();
            // pass 1: occupancy bits from the products
            auto mark = [&](const int (&qq)[U_RANK1], const bool (&ok)[U_RANK1], const V (&)[U_RANK1]) {
                int col[U_RANK1];
#pragma unroll
                for (int u = 0; u < U_RANK1; ++u) {
                    const int cb = bc[qq[u]];                 // qq is always a valid index
                    col[u] = ok[u] ? cb : c0 - 1;
                }
#pragma unroll
                for (int u = 0; u < U_RANK1; ++u) {
                    const uint32_t off = (uint32_t)(col[u] - c0);
                    if (off < span) atomicOr(&w32[2 * (off >> 5)], 1u << (off & 31));
                }
            };
            if (resident) enum_chunk<G, U_RANK1, false, V>(lo, hi - lo, V(0), sg, mark);
            else walk_row(mark, std::false_type{});
            __syncthreads();
            // ranks: exclusive prefix of the bit counts, per word
            const int S = (nwords + G - 1) / G;
            const int w0 = tid * S;
            int c = 0;
            for (int j = 0; j < S; ++j)
                if (w0 + j < nwords) c += __popc(w32[2 * (w0 + j)]);
            int total;
            int pre = block_excl_scan<G, int>(c, total, sg.wsum);
            for (int j = 0; j < S; ++j)
                if (w0 + j < nwords) {
                    w32[2 * (w0 + j) + 1] = (uint32_t)pre;
                    pre += __popc(w32[2 * (w0 + j)]);
                }
            if (total != count) bad = true;
        }
        __syncthreads();

        // next window, stage 1: its item, this thread's a_ik and its B row
        const unsigned nxt = __builtin_amdgcn_readfirstlane(s_claim[par ^ 1]);
        WinItem nit{};
        bool nres = false;
        int2 nb = make_int2(0, -1);
        V na = V(0);
        if (nxt != WIN_NONE) {
            nit = items[nxt];
            if (nit.a1 - nit.a0 <= G && nit.a0 + tid < nit.a1) {
                nres = true;
                nb = ki[nit.a0 + tid];
                na = vA[nit.a0 + tid];
            }
        }

        // products: values added at their rank
        auto add = [&](const int (&qq)[U_RANK2], const bool (&ok)[U_RANK2], const V (&av)[U_RANK2]) {
            int col[U_RANK2];
            V x[U_RANK2];
#pragma unroll
            for (int u = 0; u < U_RANK2; ++u) {
                const int cb = bc[qq[u]];                     // qq is always a valid index
                const V b = bv[qq[u]];
                col[u] = ok[u] ? cb : c0 - 1;
                x[u] = ok[u] ? av[u] * b : V(0);
            }
#pragma unroll
            for (int u = 0; u < U_RANK2; ++u) {
                const uint32_t off = (uint32_t)(col[u] - c0);
                if (off < span) {
                    const uint2 e = reinterpret_cast<const uint2 *>(buf)[off >> 5];
                    const uint32_t rank = e.y + __popc(e.x & ((1u << (off & 31)) - 1u));
                    if (rank < (uint32_t)count) {
                        lds_add(&vals[rank], x[u]);
                        stage[rank] = col[u];   // the same value from every product of the column
                    }
                }
            }
        };
        if (resident && bmap) enum_walk<G, U_RANK2, true, V>(ptotal, pnseg, sg, add);   // laid out above
        else if (resident) enum_chunk<G, U_RANK2, true, V>(lo, hi - lo, a, sg, add);
        else walk_row(add, std::true_type{});
        __syncthreads();

        // next window, stage 2: its slice (the chunk index) and its bits
        int nlo = 0, nhi = 0;
        if (nres) slice_of(nb, nit.ch_lo, nit.ch_hi, nlo, nhi);
        // (every path sets q here: the previous window's bits are dead
        // through the products, so their registers are free there)
#pragma unroll
        for (int k = 0; k < WIN_PRE_QUADS; ++k) q[k] = u32x4{0u, 0u, 0u, 0u};
        if (bmap && nxt != WIN_NONE) load_bits(nit, q);

        // values and columns leave in consecutive runs
        for (int r = tid; r < count; r += G) {
            __builtin_nontemporal_store(stage[r], &cC[it.out_pos + r]);
            __builtin_nontemporal_store(vals[r], &vC[it.out_pos + r]);
        }

        __syncthreads();

        cur = nxt;
        it = nit;
        lo = nlo;
        hi = nhi;
        a = na;
        par ^= 1;
    }
    if (bad) atomicOr(&wh->err, ERR_COUNT);
}

// ----------------------------------------------------------------------- heap merge

// Wave-wide reductions (every lane active).
extern "C" __device__ __attribute__((const)) double __ockl_wfred_add_f64(double);
extern "C" __device__ __attribute__((const)) unsigned long long __ockl_wfred_add_u64(unsigned long long);

__device__ __forceinline__ int wave_min_all(int x) { return __ockl_wfred_min_i32(x); }
__device__ __forceinline__ double wave_add_all(double x) { return __ockl_wfred_add_f64(x); }
__device__ __forceinline__ unsigned long long wave_add_all(unsigned long long x) {
    return __ockl_wfred_add_u64(x);
}

// Rows of B in ascending column order (repeats allowed)?  Sets ERR_UNSORTED_B
// in *err otherwise.
__global__ __launch_bounds__(256) void k_check_sorted(int64_t nnz, const int32_t *__restrict__ rB,
                                                      int64_t nrows, const int32_t *__restrict__ cB, int *err) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    bool bad = false;
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < nrows; r += stride) {
        const int b0 = rB[r], b1 = rB[r + 1];
        for (int p = b0 + 1; p < b1; ++p) bad |= cB[p] < cB[p - 1];
    }
    (void)nnz;
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(err, ERR_UNSORTED_B);
}

// Numeric phase of the heap bin: the priority-queue accumulation of Section
// 4.2.3.  Row c_i is built by repeatedly taking the smallest column among the
// heads of the B rows that the entries a_ik select, adding a_ik*b_kj for every
// head at that column, and advancing those heads; the queue holds one head
// per entry of a_i (O(nnz(a_i)) state, as in the paper).  On the GPU a row is
// one wave: the row's B slices (at most HEAP_FCAP products) are first copied
// to LDS, lane l keeps the heads of the row's entries l, l+64, l+128, l+192
// (a four-slot queue per lane), and the queue's minimum is the wave-wide
// minimum of the lanes' smallest heads (a tournament over the 64 lanes in
// cross-lane reductions).  A column met again in the next round (a repeated
// column inside a B row, or a repeated k) adds into the same entry.  Entries
// leave in ascending column order, 64 per coalesced store.  The B rows must be
// sorted (checked when the plan is made).
template <typename V>
__global__ __launch_bounds__(64) void k_num_heap(const NumRow *__restrict__ rows, int64_t perm_off, unsigned nrows,
                                                 const int32_t *__restrict__ cA,
                                                 const V *__restrict__ vA, const int32_t *__restrict__ rB,
                                                 const int32_t *__restrict__ cB, const V *__restrict__ vB,
                                                 int32_t *__restrict__ cC, V *__restrict__ vC, WsHdr *wh) {
    constexpr int NQ = HEAP_MAX_A / WAVE;       // queue slots per lane
    constexpr int NONE = 0x7FFFFFFF;            // head of an exhausted slice
    __shared__ int scol[HEAP_FCAP];
    __shared__ V sval[HEAP_FCAP];
    __shared__ int soff[HEAP_MAX_A];
    __shared__ int slo[HEAP_MAX_A];
    const int ln = threadIdx.x;
    if (blockIdx.x >= nrows) return;
    const NumRow nr = rows[perm_off + blockIdx.x];
    const int a0 = nr.a0, a1 = nr.a1;
    // the slices of the row's entries, laid end to end in LDS (entry a0 + s
    // owns positions [soff[s], soff[s] + len))
    int cur[NQ], end[NQ];
    V av[NQ];
    int base = 0;
#pragma unroll
    for (int t = 0; t < NQ; ++t) {
        const int e = a0 + t * WAVE + ln;
        int lo = 0, len = 0;
        av[t] = V(0);
        if (e < a1) {
            const int k = cA[e];
            av[t] = vA[e];
            lo = rB[k];
            len = rB[k + 1] - lo;
        }
        const int incl = wave_incl_scan<int>(len);
        cur[t] = base + incl - len;
        end[t] = base + incl;
        soff[t * WAVE + ln] = cur[t];
        slo[t * WAVE + ln] = lo;
        base += wave_last(incl);
    }
    const int F = base;                         // <= HEAP_FCAP (the bin's rule)
    wave_sync();
    for (int p = ln; p < F; p += WAVE) {
        int l = 0, h = HEAP_MAX_A - 1;          // the last slice starting at or before p
        while (l < h) {
            const int mid = (l + h + 1) >> 1;
            if (soff[mid] <= p) l = mid; else h = mid - 1;
        }
        const int src = slo[l] + (p - soff[l]);
        scol[p] = cB[src];
        sval[p] = vB[src];
    }
    wave_sync();
    int head[NQ];
#pragma unroll
    for (int t = 0; t < NQ; ++t) head[t] = cur[t] < end[t] ? scol[cur[t]] : NONE;
    const int64_t o = (int64_t)(nr.out_n >> 16);
    const int expected = (int)(nr.out_n & 0xFFFFu);
    int nout = 0;                               // entries emitted (wave-uniform)
    int last = -1;                              // column of the pending entry (wave-uniform)
    V pend = V(0);
    int rc = 0;                                 // this lane's slot of the 64-entry output run
    V rv = V(0);
    auto emit = [&](int c, V v) {
        if (ln == (nout & (WAVE - 1))) {
            rc = c;
            rv = v;
        }
        ++nout;
        if ((nout & (WAVE - 1)) == 0) {
            const int at = nout - WAVE + ln;
            if (at < expected) {
                __builtin_nontemporal_store(rc, &cC[o + at]);
                __builtin_nontemporal_store(rv, &vC[o + at]);
            }
        }
    };
    for (;;) {
        int lm = head[0];
#pragma unroll
        for (int t = 1; t < NQ; ++t) lm = min(lm, head[t]);
        const int m = wave_min_all(lm);
        if (m == NONE) break;
        V x = V(0);
#pragma unroll
        for (int t = 0; t < NQ; ++t)
            if (head[t] == m) {
                x += av[t] * sval[cur[t]];
                ++cur[t];
                head[t] = cur[t] < end[t] ? scol[cur[t]] : NONE;
            }
        const V sum = wave_add_all(x);
        if (m == last) {
            pend += sum;
        } else {
            if (last >= 0) emit(last, pend);
            last = m;
            pend = sum;
        }
    }
    if (last >= 0) emit(last, pend);
    const int rem = nout & (WAVE - 1);
    if (rem) {
        const int at = nout - rem + ln;
        if (ln < rem && at < expected) {
            __builtin_nontemporal_store(rc, &cC[o + at]);
            __builtin_nontemporal_store(rv, &vC[o + at]);
        }
    }
    if (nout != expected && ln == 0) atomicOr(&wh->err, ERR_COUNT);
}

// ----------------------------------------------------------------------- masked product sum

// Sum of C_ij over the positions (i, j) of a mask M with C = A*B, without
// forming C (the masked product of Section 5.6's triangle count: keep a_ik*b_kj
// only where (i, j) is in M).  A persistent grid claims rows of A; a block sets
// the row's mask columns in an LDS bitmap over a pass of NWORDS*32 columns,
// keeps the products whose column bit is set (int64, wrap-around; all values 1
// when ONES) and clears the bits again.  One atomic per block at the end.
constexpr int U_MASK = 8;

template <int NWORDS, bool ONES>
__global__ __launch_bounds__(1024) void k_masked_product(int m, int64_t ncols, const int32_t *__restrict__ rA,
                                                         const int32_t *__restrict__ cA,
                                                         const unsigned long long *__restrict__ vA,
                                                         const int32_t *__restrict__ rB,
                                                         const int32_t *__restrict__ cB,
                                                         const unsigned long long *__restrict__ vB,
                                                         const int32_t *__restrict__ rM,
                                                         const int32_t *__restrict__ cM, unsigned *next_row,
                                                         unsigned long long *out) {
    constexpr int G = 1024;
    constexpr int64_t WIN = (int64_t)NWORDS * 32;
    using V = unsigned long long;
    __shared__ uint32_t bm[NWORDS];
    __shared__ SegLds<G, !ONES, V> sg;
    __shared__ int s_row;
    __shared__ V s_part[G / WAVE];
    const int tid = threadIdx.x;
    for (int i = tid; i < NWORDS; i += G) bm[i] = 0u;
    V acc = 0;
    const int npass = (int)((ncols + WIN - 1) / WIN);
    for (;;) {
        if (tid == 0) s_row = (int)atomicAdd(next_row, 1u);
        __syncthreads();                               // also orders the bitmap clear
        const int row = s_row;
        __syncthreads();                               // everyone has read s_row
        if (row >= m) break;                           // uniform over the block
        const int a0 = rA[row], a1 = rA[row + 1], m0 = rM[row], m1 = rM[row + 1];
        if (a0 == a1 || m0 == m1) continue;            // uniform: nothing to add
        for (int pass = 0; pass < npass; ++pass) {
            const int64_t c0 = (int64_t)pass * WIN;
            for (int p = m0 + tid; p < m1; p += G) {
                const uint32_t off = (uint32_t)((int64_t)cM[p] - c0);
                if (off < (uint32_t)WIN) atomicOr(&bm[off >> 5], 1u << (off & 31));
            }
            __syncthreads();
            enum_row<G, U_MASK, !ONES, V>(
                a0, a1, cA, vA, sg, [&](int k, int &lo, int &hi) { lo = rB[k]; hi = rB[k + 1]; },
                [&](const int (&q)[U_MASK], const bool (&ok)[U_MASK], const V (&av)[U_MASK]) {
#pragma unroll
                    for (int u = 0; u < U_MASK; ++u) {
                        const int c = cB[q[u]];                   // q is always a valid index
                        V b = 1;
                        if constexpr (!ONES) b = vB[q[u]];
                        const uint32_t off = (uint32_t)((int64_t)c - c0);
                        const bool hit = ok[u] && off < (uint32_t)WIN && ((bm[off >> 5] >> (off & 31)) & 1u);
                        if constexpr (ONES) acc += hit ? 1ull : 0ull;
                        else acc += hit ? av[u] * b : 0ull;
                    }
                });
            __syncthreads();
            for (int p = m0 + tid; p < m1; p += G) {
                const uint32_t off = (uint32_t)((int64_t)cM[p] - c0);
                if (off < (uint32_t)WIN) bm[off >> 5] = 0u;
            }
            __syncthreads();
        }
    }
    acc = wave_sum_u64(acc);
    if ((tid & 63) == 0) s_part[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        V t = 0;
        for (int w = 0; w < G / WAVE; ++w) t += s_part[w];
        if (t) atomicAdd(out, t);
    }
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

// Streaming copy at the rate the GPU sustains: four 16-byte loads in flight
// per lane before their stores, non-temporal on both sides (MI355X, 1 GiB
// each way: 6.1 TB/s with 16384 blocks, against 4.6 TB/s for one plain
// 16-byte load per lane per step).
constexpr int COPY_K = 4;

__global__ __launch_bounds__(256) void k_stream_copy(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                     size_t n) {
    const size_t stride = (size_t)gridDim.x * 256 * COPY_K;
    for (size_t base = (size_t)blockIdx.x * 256 * COPY_K + threadIdx.x; base < n; base += stride) {
        u32x4 v[COPY_K];
#pragma unroll
        for (int k = 0; k < COPY_K; ++k) {
            const size_t i = base + (size_t)k * 256;
            v[k] = u32x4{0u, 0u, 0u, 0u};
            if (i < n) v[k] = __builtin_nontemporal_load(&src[i]);
        }
#pragma unroll
        for (int k = 0; k < COPY_K; ++k) {
            const size_t i = base + (size_t)k * 256;
            if (i < n) __builtin_nontemporal_store(v[k], &dst[i]);
        }
    }
}

// ----------------------------------------------------------------------- stanza probe

// Reads nst stanzas of 2^lw 8-byte words, stanza s starting at word start[s]
// of base (nwords long), and adds every word read into *sum (wrap-around;
// one atomic per block).  Consecutive lanes take consecutive words of a
// stanza, then of the next one, so a short stanza costs its own length plus
// the read of its start, as a row of B costs an SpGEMM.  A stanza that does
// not fit the array is skipped and counted in *skipped.
__global__ __launch_bounds__(256) void k_stanza_read(const unsigned long long *__restrict__ base, int64_t nwords,
                                                     const int64_t *__restrict__ start, int64_t nst, int lw,
                                                     unsigned long long *sum, unsigned long long *skipped) {
    __shared__ unsigned long long s_part[256 / WAVE];
    const int64_t total = nst << lw;
    const int64_t stride = (int64_t)gridDim.x * 256;
    const int64_t wmask = ((int64_t)1 << lw) - 1;
    constexpr int U = 8;                                      // loads in flight per lane
    unsigned long long acc = 0, bad = 0;
    for (int64_t i0 = (int64_t)blockIdx.x * 256 + threadIdx.x; i0 < total; i0 += stride * U) {
        int64_t st[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + u * stride;
            st[u] = i < total ? start[i >> lw] : -1;
        }
        unsigned long long v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + u * stride;
            const bool fits = st[u] >= 0 && st[u] <= nwords - (wmask + 1);
            // every lane loads (word 0 when its stanza does not fit) so that the
            // U loads leave together; the value is dropped afterwards
            const unsigned long long x = __builtin_nontemporal_load(&base[fits ? st[u] + (i & wmask) : 0]);
            v[u] = fits ? x : 0ull;
            bad += (i < total && !fits && (i & wmask) == 0) ? 1ull : 0ull;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc += v[u];
    }
    acc = wave_sum_u64(acc);
    bad = wave_sum_u64(bad);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < 256 / WAVE; ++w) t += s_part[w];
        atomicAdd(sum, t);
    }
    if ((threadIdx.x & 63) == 0 && bad) atomicAdd(skipped, bad);
}

// ======================================================================= launchers

static inline unsigned grid1(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// Blocks of a kernel that fit on one CU at once (asked of the runtime once).
template <class K>
static int blocks_per_cu(K kern, int G) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, G, 0) != hipSuccess || occ < 1) occ = 1;
    return occ;
}

hipError_t launch_validate(const CsrDev &a, int *err, hipStream_t s) {
    const unsigned g = (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, grid1(std::max(a.nrows, a.nnz), 256)));
    k_validate<<<g, 256, 0, s>>>(a.nrows, a.ncols, a.nnz, a.rpts, a.cols, err);
    return hipGetLastError();
}

hipError_t launch_row_flop(const CsrDev &A, const CsrDev &B, uint32_t *flop, int32_t *longl, int32_t *huge,
                           PlanHdr *hdr, const BinLimits &L, int ncu, hipStream_t s) {
    if (A.nrows == 0) return hipSuccess;
    k_row_flop<<<grid1(A.nrows, 256), 256, 0, s>>>((int)A.nrows, A.rpts, A.cols, B.rpts, B.ncols, flop, longl, huge,
                                                    hdr, L);
    // rows that can have more than FLOP_SHORT_ROW entries: four per block,
    // at most eight blocks per CU
    const int64_t cap_long = std::min<int64_t>(A.nrows, A.nnz / (FLOP_SHORT_ROW + 1));
    if (cap_long > 0)
        k_long_flop<<<(unsigned)std::min<int64_t>((cap_long + 3) / 4, (int64_t)ncu * 8), 256, 0, s>>>(
            A.rpts, A.cols, B.rpts, B.ncols, longl, flop, hdr, L);
    const int64_t cap = A.nnz / (FLOP_WAVE_ROW + 1);   // rows that can be that long
    if (cap > 0)
        k_huge_flop<<<(unsigned)cap, 256, 0, s>>>(A.rpts, A.cols, B.rpts, B.ncols, huge, flop, hdr, L);
    return hipGetLastError();
}

hipError_t launch_sym_scatter(int m, const uint32_t *flop, const int32_t *rA, int64_t ncolsB, const BinOffsets &off,
                              int32_t *perm, int2 *prow, int32_t *nnz_row, int32_t *slot_of, WsHdr *wh,
                              const BinLimits &L, hipStream_t s) {
    if (m == 0) return hipSuccess;
    k_sym_scatter<<<grid1(m, 256), 256, 0, s>>>(m, flop, rA, ncolsB, off, perm, prow, nnz_row, slot_of, wh, L);
    return hipGetLastError();
}

template <int G, int T>
static void sym_hash_l(unsigned nrows, const int32_t *perm, const int2 *prow, int64_t off, const CsrDev &A,
                       const CsrDev &B, int32_t *nnz_row, WsHdr *wh, HashCfg hc, int ncu, hipStream_t s) {
    // at most four products per lane keep the kernel within 64 registers
    // (eight waves per SIMD: two 1024-thread blocks per CU)
    constexpr int U = u_for(G, T / 2 + 1) < 4 ? u_for(G, T / 2 + 1) : 4;
    // wide bins (few blocks per CU) run persistent; narrow ones a block per row
    constexpr bool P = G >= 512;
    static const int occ = P ? blocks_per_cu(k_sym_hash<G, T, U, P>, G) : 0;
    const unsigned grid = P ? (unsigned)std::min<int64_t>(nrows, (int64_t)ncu * occ) : nrows;
    k_sym_hash<G, T, U, P><<<grid, G, 0, s>>>(perm, prow, off, nrows, A.cols, B.rpts, B.cols, nnz_row, wh, hc);
}

hipError_t launch_sym_bin(int bin, unsigned nrows, const int32_t *perm, const int2 *prow, int64_t off, const CsrDev &A,
                          const CsrDev &B, int32_t *nnz_row, WsHdr *wh, HashCfg hc, int ncu, hipStream_t s) {
    if (nrows == 0) return hipSuccess;
    switch (bin) {
        case 1: sym_hash_l<SYM_G[1], SYM_T[1]>(nrows, perm, prow, off, A, B, nnz_row, wh, hc, ncu, s); break;
        case 2: sym_hash_l<SYM_G[2], SYM_T[2]>(nrows, perm, prow, off, A, B, nnz_row, wh, hc, ncu, s); break;
        case 3: sym_hash_l<SYM_G[3], SYM_T[3]>(nrows, perm, prow, off, A, B, nnz_row, wh, hc, ncu, s); break;
        case 4: sym_hash_l<SYM_G[4], SYM_T[4]>(nrows, perm, prow, off, A, B, nnz_row, wh, hc, ncu, s); break;
        case 5: sym_hash_l<SYM_G[5], SYM_T[5]>(nrows, perm, prow, off, A, B, nnz_row, wh, hc, ncu, s); break;
        case 6: sym_hash_l<SYM_G[6], SYM_T[6]>(nrows, perm, prow, off, A, B, nnz_row, wh, hc, ncu, s); break;
        case 7: sym_hash_l<SYM_G[7], SYM_T[7]>(nrows, perm, prow, off, A, B, nnz_row, wh, hc, ncu, s); break;
        case 8: sym_hash_l<SYM_G[8], SYM_T[8]>(nrows, perm, prow, off, A, B, nnz_row, wh, hc, ncu, s); break;
        case 9: sym_hash_l<SYM_G[9], SYM_T[9]>(nrows, perm, prow, off, A, B, nnz_row, wh, hc, ncu, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// persistent: a grid of the blocks that fit the CUs at once walks the bin
template <int W>
static void sym_bitmap_l(unsigned nbm, const int32_t *perm, int64_t off, const CsrDev &A, const CsrDev &B,
                         int nchunks, uint32_t *chunk_cnt, int32_t *nnz_row, uint32_t *bmap, WsHdr *wh, int ncu,
                         hipStream_t s) {
    static const int occ = blocks_per_cu(k_sym_bitmap<W>, 1024);
    const unsigned grid = (unsigned)std::min<int64_t>(nbm, (int64_t)ncu * occ);
    k_sym_bitmap<W><<<grid, 1024, 0, s>>>(perm, off, nbm, A.rpts, A.cols, B.rpts, B.cols, B.ncols, nchunks, chunk_cnt,
                                          nnz_row, bmap, wh);
}

hipError_t launch_sym_segments(unsigned nbm, const int32_t *perm, int64_t off, const CsrDev &A, const CsrDev &B,
                               int nchunks, uint32_t *chunk_cnt, int32_t *nnz_row, uint32_t *bmap, WsHdr *wh,
                               int ncu, hipStream_t s) {
    if (nbm == 0) return hipSuccess;
    const int64_t need = (B.ncols + 31) / 32;
    if (need <= BM_WORDS_SMALL)
        sym_bitmap_l<BM_WORDS_SMALL>(nbm, perm, off, A, B, nchunks, chunk_cnt, nnz_row, bmap, wh, ncu, s);
    else if (need <= BM_WORDS_MID)
        sym_bitmap_l<BM_WORDS_MID>(nbm, perm, off, A, B, nchunks, chunk_cnt, nnz_row, bmap, wh, ncu, s);
    else
        sym_bitmap_l<BM_WORDS_LARGE>(nbm, perm, off, A, B, nchunks, chunk_cnt, nnz_row, bmap, wh, ncu, s);
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
                           const int32_t *slot_of, HeavyRow *heavy, WsHdr *wh, const BinLimits &L, hipStream_t s) {
    if (m == 0) return hipSuccess;
    k_num_hist<<<grid1(m, 256), 256, 0, s>>>(m, nnz_row, flop, rA, slot_of, heavy, wh, L);
    return hipGetLastError();
}

hipError_t launch_count_long_b(const CsrDev &B, PlanHdr *hdr, hipStream_t s) {
    if (B.nrows == 0) return hipSuccess;
    k_count_long_b<<<grid1(B.nrows, 256), 256, 0, s>>>((int)B.nrows, B.rpts, hdr);
    return hipGetLastError();
}

hipError_t launch_windows(unsigned nheavy_max, const HeavyRow *heavy, int nchunks, const uint32_t *chunk_cnt,
                          const int64_t *rpts_C, const int32_t *rA, uint32_t *whist, uint32_t *wcur, WinItem *items,
                          unsigned cap, WsHdr *wh, hipStream_t s) {
    if (nheavy_max == 0) return hipSuccess;
    hipError_t e = hipMemsetAsync(whist, 0, sizeof(uint32_t) * 2 * (size_t)nchunks, s);   // whist and wcur
    if (e != hipSuccess) return e;
    k_win_count<<<grid1(nheavy_max, 16), 1024, 0, s>>>(heavy, nchunks, chunk_cnt, whist, wh);
    k_win_scan<<<1, 1024, 0, s>>>(whist, nchunks, cap, wh);
    k_win_emit<<<grid1(nheavy_max, 16), 1024, 0, s>>>(heavy, nchunks, chunk_cnt, rpts_C, rA, whist, wcur, items, cap,
                                                      wh);
    return hipGetLastError();
}

hipError_t launch_bucket(const CsrDev &B, int32_t *bc, int32_t *bperm, int32_t *bs, int32_t *long_id,
                         int32_t *long_list, int32_t *idx, int nchunks, WsHdr *wh, hipStream_t s) {
    if (B.nrows == 0) return hipSuccess;
    k_bucket_short<<<grid1(B.nrows, 256), 256, 0, s>>>((int)B.nrows, B.rpts, B.cols, bc, bperm, bs, long_id,
                                                        long_list, wh);
    if (nchunks <= 1024)
        k_bucket_long<1024><<<4096, 256, 0, s>>>(long_list, wh, B.rpts, B.cols, bc, bperm, bs, idx, nchunks);
    else
        k_bucket_long<MAX_CHUNKS><<<1024, 256, 0, s>>>(long_list, wh, B.rpts, B.cols, bc, bperm, bs, idx, nchunks);
    return hipGetLastError();
}

hipError_t launch_gather_vals(int dtype, int64_t n, const int32_t *bperm, const void *vB, void *bv, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<int64_t>(grid1(n, 256), 256 * 32);
    if (dtype == 0) k_gather_vals<double><<<g, 256, 0, s>>>(n, bperm, (const double *)vB, (double *)bv);
    else k_gather_vals<unsigned long long><<<g, 256, 0, s>>>(n, bperm, (const unsigned long long *)vB,
                                                             (unsigned long long *)bv);
    return hipGetLastError();
}

hipError_t launch_entry_brow(const CsrDev &A, const CsrDev &B, const int32_t *long_id, int2 *ki, hipStream_t s) {
    if (A.nnz == 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<int64_t>(grid1(A.nnz, 256), 256 * 32);
    k_entry_brow<<<g, 256, 0, s>>>(A.nnz, A.cols, B.rpts, long_id, ki);
    return hipGetLastError();
}

hipError_t launch_num_scatter(int m, const int32_t *nnz_row, const uint32_t *flop, const int32_t *rA,
                              const int64_t *rpts_C, const BinOffsets &off, NumRow *rows, WsHdr *wh,
                              const BinLimits &L, hipStream_t s) {
    if (m == 0) return hipSuccess;
    k_num_scatter<<<grid1(m, 256), 256, 0, s>>>(m, nnz_row, flop, rA, rpts_C, off, rows, wh, L);
    return hipGetLastError();
}

template <int G, int T, bool SORTED, typename V>
static void num_hash_l(unsigned nrows, const NumRow *rows, int64_t off, const CsrDev &A, const CsrDev &B,
                       int32_t *cC, void *vC, WsHdr *wh, HashCfg hc, int ncu, hipStream_t s) {
    constexpr int U = u_for(G, T / 2 + 1) < 4 ? u_for(G, T / 2 + 1) : 4;
    // wide bins (few blocks per CU) run persistent; narrow ones a block per row
    constexpr bool P = G >= 512;
    static const int occ = P ? blocks_per_cu(k_num_hash<G, T, U, SORTED, V, P>, G) : 0;
    const unsigned grid = P ? (unsigned)std::min<int64_t>(nrows, (int64_t)ncu * occ) : nrows;
    k_num_hash<G, T, U, SORTED, V, P><<<grid, G, 0, s>>>(rows, off, nrows, A.cols, (const V *)A.vals, B.rpts,
                                                    B.cols, (const V *)B.vals, cC, (V *)vC, wh, hc, B.ncols);
}

template <bool SORTED, typename V>
static hipError_t num_bin_t(int bin, unsigned nrows, const NumRow *rows, int64_t off, const CsrDev &A,
                            const CsrDev &B, int32_t *cC, void *vC, WsHdr *wh, HashCfg hc, int ncu,
                            hipStream_t s) {
    switch (bin) {
        case 1: num_hash_l<NUM_G[1], NUM_T[1], SORTED, V>(nrows, rows, off, A, B, cC, vC, wh, hc, ncu, s); break;
        case 2: num_hash_l<NUM_G[2], NUM_T[2], SORTED, V>(nrows, rows, off, A, B, cC, vC, wh, hc, ncu, s); break;
        case 3: num_hash_l<NUM_G[3], NUM_T[3], SORTED, V>(nrows, rows, off, A, B, cC, vC, wh, hc, ncu, s); break;
        case 4: num_hash_l<NUM_G[4], NUM_T[4], SORTED, V>(nrows, rows, off, A, B, cC, vC, wh, hc, ncu, s); break;
        case 5: num_hash_l<NUM_G[5], NUM_T[5], SORTED, V>(nrows, rows, off, A, B, cC, vC, wh, hc, ncu, s); break;
        case 6: num_hash_l<NUM_G[6], NUM_T[6], SORTED, V>(nrows, rows, off, A, B, cC, vC, wh, hc, ncu, s); break;
        case 7: num_hash_l<NUM_G[7], NUM_T[7], SORTED, V>(nrows, rows, off, A, B, cC, vC, wh, hc, ncu, s); break;
        case 8: num_hash_l<NUM_G[8], NUM_T[8], SORTED, V>(nrows, rows, off, A, B, cC, vC, wh, hc, ncu, s); break;
        case 9: num_hash_l<NUM_G[9], NUM_T[9], SORTED, V>(nrows, rows, off, A, B, cC, vC, wh, hc, ncu, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_num_bin(int bin, int dtype, bool sorted, unsigned nrows, const NumRow *rows, int64_t off,
                          const CsrDev &A, const CsrDev &B, int32_t *cC, void *vC, WsHdr *wh, HashCfg hc, int ncu,
                          hipStream_t s) {
    if (nrows == 0) return hipSuccess;
    if (dtype == 0)
        return sorted ? num_bin_t<true, double>(bin, nrows, rows, off, A, B, cC, vC, wh, hc, ncu, s)
                      : num_bin_t<false, double>(bin, nrows, rows, off, A, B, cC, vC, wh, hc, ncu, s);
    return sorted ? num_bin_t<true, unsigned long long>(bin, nrows, rows, off, A, B, cC, vC, wh, hc, ncu, s)
                  : num_bin_t<false, unsigned long long>(bin, nrows, rows, off, A, B, cC, vC, wh, hc, ncu, s);
}

__global__ void k_zero_u32n(unsigned *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// Claim counters of the numeric phase (windows and persistent hash bins) back
// to zero: the phase may run again on the same symbolic result.
__global__ void k_num_reset(WsHdr *wh) {
    const int t = (int)threadIdx.x;
    if (t < 8) wh->win_next[t] = 0u;
    if (t < NNB) wh->num_next[t] = 0u;
}

hipError_t launch_num_reset(WsHdr *wh, hipStream_t s) {
    k_num_reset<<<1, 64, 0, s>>>(wh);
    return hipGetLastError();
}


// Windows leave in ascending column order, so sorted and unsorted output share it.
hipError_t launch_num_window(int dtype, unsigned nitems, const WinItem *items, const CsrDev &A, const int2 *ki,
                             const int32_t *idx, int nchunks, const int32_t *bc, const void *bv, int32_t *cC,
                             void *vC, const uint32_t *bmap, WsHdr *wh, int ncu, hipStream_t s) {
    if (nitems == 0) return hipSuccess;
    if (dtype == 0) {
        static const int occ = blocks_per_cu(k_num_window<double>, WIN_G);
        const unsigned grid = (unsigned)std::min<int64_t>(nitems, (int64_t)ncu * occ);
        k_num_window<double><<<grid, WIN_G, 0, s>>>(items, nitems, ki, (const double *)A.vals, idx, nchunks, bc,
                                                    (const double *)bv, cC, (double *)vC, bmap, wh);
    } else {
        static const int occ = blocks_per_cu(k_num_window<unsigned long long>, WIN_G);
        const unsigned grid = (unsigned)std::min<int64_t>(nitems, (int64_t)ncu * occ);
        k_num_window<unsigned long long><<<grid, WIN_G, 0, s>>>(
            items, nitems, ki, (const unsigned long long *)A.vals, idx, nchunks, bc, (const unsigned long long *)bv,
            cC, (unsigned long long *)vC, bmap, wh);
    }
    return hipGetLastError();
}

hipError_t launch_check_sorted(const CsrDev &B, int *err, hipStream_t s) {
    if (B.nrows == 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<int64_t>(grid1(B.nrows, 256), 8192);
    k_check_sorted<<<g, 256, 0, s>>>(B.nnz, B.rpts, B.nrows, B.cols, err);
    return hipGetLastError();
}

hipError_t launch_num_heap(int dtype, unsigned nrows, const NumRow *rows, int64_t off, const CsrDev &A,
                           const CsrDev &B, int32_t *cC, void *vC, WsHdr *wh, hipStream_t s) {
    if (nrows == 0) return hipSuccess;
    if (dtype == 0)
        k_num_heap<double><<<nrows, WAVE, 0, s>>>(rows, off, nrows, A.cols, (const double *)A.vals, B.rpts,
                                                  B.cols, (const double *)B.vals, cC, (double *)vC, wh);
    else
        k_num_heap<unsigned long long><<<nrows, WAVE, 0, s>>>(
            rows, off, nrows, A.cols, (const unsigned long long *)A.vals, B.rpts, B.cols,
            (const unsigned long long *)B.vals, cC, (unsigned long long *)vC, wh);
    return hipGetLastError();
}

template <int NWORDS, bool ONES>
static void masked_product_l(const CsrDev &A, const CsrDev &B, const CsrDev &M, unsigned *next_row,
                             unsigned long long *out, int ncu, hipStream_t s) {
    static const int occ = blocks_per_cu(k_masked_product<NWORDS, ONES>, 1024);
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(A.nrows, (int64_t)ncu * occ));
    k_masked_product<NWORDS, ONES><<<grid, 1024, 0, s>>>(
        (int)A.nrows, B.ncols, A.rpts, A.cols, (const unsigned long long *)A.vals, B.rpts, B.cols,
        (const unsigned long long *)B.vals, M.rpts, M.cols, next_row, out);
}

template <bool ONES>
static void masked_product_t(const CsrDev &A, const CsrDev &B, const CsrDev &M, unsigned *next_row,
                             unsigned long long *out, int ncu, hipStream_t s) {
    // bitmap tiers: 64 K, 256 K, 1 M columns per pass (the largest leaves room
    // for the multipliers in LDS)
    const int64_t need = (B.ncols + 31) / 32;
    if (need <= BM_WORDS_SMALL) masked_product_l<BM_WORDS_SMALL, ONES>(A, B, M, next_row, out, ncu, s);
    else if (need <= BM_WORDS_MID) masked_product_l<BM_WORDS_MID, ONES>(A, B, M, next_row, out, ncu, s);
    else masked_product_l<32768, ONES>(A, B, M, next_row, out, ncu, s);
}

hipError_t launch_masked_product(const CsrDev &A, const CsrDev &B, const CsrDev &M, bool ones, unsigned *next_row,
                                 int64_t *out, int ncu, hipStream_t s) {
    k_zero_u64<<<1, 1, 0, s>>>((unsigned long long *)out);
    k_zero_u32n<<<1, 64, 0, s>>>(next_row, 1);
    if (A.nrows == 0) return hipGetLastError();
    if (ones) masked_product_t<true>(A, B, M, next_row, (unsigned long long *)out, ncu, s);
    else masked_product_t<false>(A, B, M, next_row, (unsigned long long *)out, ncu, s);
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

hipError_t launch_stanza_read(const void *base, int64_t nwords, const int64_t *start, int64_t nst, int lw,
                              unsigned long long *sum, unsigned long long *skipped, int ncu, hipStream_t s) {
    k_zero_u64<<<1, 1, 0, s>>>(sum);
    k_zero_u64<<<1, 1, 0, s>>>(skipped);
    const int64_t total = nst << lw;
    if (total == 0) return hipGetLastError();
    const unsigned g = (unsigned)std::min<int64_t>((total + 255) / 256, (int64_t)ncu * 32);
    k_stanza_read<<<g, 256, 0, s>>>((const unsigned long long *)base, nwords, start, nst, lw, sum, skipped);
    return hipGetLastError();
}

hipError_t launch_stream_copy(void *dst, const void *src, size_t nbytes, hipStream_t s) {
    const size_t n = nbytes / 16;
    if (n == 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<size_t>((n + 256 * COPY_K - 1) / (256 * COPY_K), 16384);
    k_stream_copy<<<g, 256, 0, s>>>((const u32x4 *)src, (u32x4 *)dst, n);
    return hipGetLastError();
}

}  // namespace spg
