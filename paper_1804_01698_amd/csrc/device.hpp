// Device building blocks for the gfx950 SpGEMM kernels: wave/block scans, LDS
// hash tables, and the load-balanced enumeration of the products of one row.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "config.hpp"

namespace spg {

constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// Make this wave's LDS writes visible to its other lanes before they read.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint64_t lanemask_le() {
    const int l = lane_id();
    return l == 63 ? ~0ull : ((2ull << l) - 1ull);
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const T y = __shfl_up(x, d);
        if (lane_id() >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d);
    return x;
}

__device__ __forceinline__ int wave_sum_i32(int x) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d);
    return x;
}

// Exclusive scan over a block of G threads (G a multiple of 64, <= 1024).
// wsum needs G/64 + 1 entries of LDS.  Contains block barriers when G > 64.
template <int G, typename T>
__device__ __forceinline__ T block_excl_scan(T x, T &total, T *wsum) {
    constexpr int NW = G / WAVE;
    const T incl = wave_incl_scan<T>(x);
    if constexpr (NW == 1) {
        total = __shfl(incl, 63);
        return incl - x;
    } else {
        const int w = threadIdx.x >> 6;
        if (lane_id() == 63) wsum[w] = incl;
        __syncthreads();
        if (threadIdx.x < WAVE) {
            const T v = threadIdx.x < NW ? wsum[threadIdx.x] : T(0);
            const T vi = wave_incl_scan<T>(v);
            if (threadIdx.x < NW) wsum[threadIdx.x] = vi - v;
            if (threadIdx.x == NW - 1) wsum[NW] = vi;
        }
        __syncthreads();
        const T res = incl - x + wsum[w];
        total = wsum[NW];
        __syncthreads();
        return res;
    }
}

template <int G>
__device__ __forceinline__ void block_sync() {
    if constexpr (G == WAVE) wave_sync();
    else __syncthreads();
}

// ---- LDS hash tables ----------------------------------------------------------
// Keys are column ids (>= 0); an empty slot holds -1.  The slot is the high
// half of (key * 2654435761) * T, a multiplicative hash folded onto any table
// size T; collisions are resolved by linear probing with wrap-around.
__device__ __forceinline__ uint32_t hash_slot(int key, uint32_t T) {
    const uint32_t h = (uint32_t)key * 2654435761u;
    return (uint32_t)(((uint64_t)h * T) >> 32);
}

__device__ __forceinline__ int lds_load(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Insert a key; returns 1 if it was new.  A probe sequence longer than T
// (impossible while the table has a free slot) sets *ovf and gives up.
__device__ __forceinline__ int sym_insert(int *tab, uint32_t T, int key, int &ovf) {
    uint32_t s = hash_slot(key, T);
    for (uint32_t n = 0; n < T; ++n) {
        const int cur = lds_load(&tab[s]);
        if (cur == key) return 0;
        if (cur == -1) {
            const int old = atomicCAS(&tab[s], -1, key);
            if (old == -1) return 1;
            if (old == key) return 0;
        }
        s = (s + 1 == T) ? 0u : s + 1;
    }
    ovf = 1;
    return 0;
}

__device__ __forceinline__ void lds_add(double *p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(unsigned long long *p, unsigned long long v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Insert-or-accumulate (numeric phase).
template <typename V>
__device__ __forceinline__ void num_insert(int *keys, V *vals, uint32_t T, int key, V x, int &ovf) {
    uint32_t s = hash_slot(key, T);
    for (uint32_t n = 0; n < T; ++n) {
        const int cur = lds_load(&keys[s]);
        if (cur == key) { lds_add(&vals[s], x); return; }
        if (cur == -1) {
            const int old = atomicCAS(&keys[s], -1, key);
            if (old == -1 || old == key) { lds_add(&vals[s], x); return; }
        }
        s = (s + 1 == T) ? 0u : s + 1;
    }
    ovf = 1;
}

// ---- product enumeration ---------------------------------------------------
// The products of one row of C are the pairs (a_ik, b_kj) for every stored
// a_ik of the row and every b_kj of a slice of row k of B (the whole row, or
// the part inside a column window).  A block of G threads takes the row's
// A entries G at a time, lays their slices end to end (exclusive scan of the
// slice lengths) and lets its waves pull batches of 64*U consecutive products
// from a shared counter, so a few long B rows are spread over all waves.
// Inside a batch, lane l of a 64-wide step owns product base+l; its segment
// is found from a 64-bit mask of the segments starting in the step (one LDS
// byte per start, read back with a ballot), not by a per-lane search.
template <int G, bool NUM, typename V>
struct SegLds {
    int lo[G];
    int off[G];
    V a[NUM ? G : 1];
    int wsum[G / WAVE + 1];
    int next;
    unsigned char mark[G / WAVE][WAVE];
};

template <int G, bool NUM, typename V>
__device__ __forceinline__ void seg_init(SegLds<G, NUM, V> &sg) {
    (&sg.mark[0][0])[threadIdx.x] = 0;
}

// slice(k, lo, hi): B-row k's products are B entries [lo, hi).
// act(q[U], ok[U], a[U]): process up to U products per lane: B index q,
// multiplier a (numeric phase), ok = valid.
template <int G, int U, bool NUM, typename V, class SliceF, class ActF>
__device__ __forceinline__ void enum_row(int a0, int a1, const int32_t *__restrict__ colsA,
                                         const V *__restrict__ valsA, SegLds<G, NUM, V> &sg,
                                         SliceF slice, ActF act) {
    const int tid = threadIdx.x;
    const int ln = tid & 63;
    const int w = tid >> 6;
    for (int cb = a0; cb < a1; cb += G) {
        const int e = cb + tid;
        int lo = 0, len = 0;
        V a = V(0);
        if (e < a1) {
            int hi = 0;
            slice(colsA[e], lo, hi);
            len = hi - lo;
            if constexpr (NUM) a = valsA[e];
        }
        int total, nseg;
        const int pre_len = block_excl_scan<G, int>(len, total, sg.wsum);
        const int pre_ne = block_excl_scan<G, int>(len > 0 ? 1 : 0, nseg, sg.wsum);
        if (len > 0) {
            sg.lo[pre_ne] = lo;
            sg.off[pre_ne] = pre_len;
            if constexpr (NUM) sg.a[pre_ne] = a;
        }
        if (tid == 0) sg.next = 0;
        block_sync<G>();
        for (;;) {
            int pb = 0;
            if (ln == 0) pb = atomicAdd(&sg.next, WAVE * U);
            pb = __shfl(pb, 0);
            if (pb >= total) break;
            // last segment starting before pb (upper_bound(off, pb-1) - 1)
            int lo_i = 0, hi_i = nseg;
            while (lo_i < hi_i) {
                const int mid = (lo_i + hi_i) >> 1;
                if (sg.off[mid] <= pb - 1) lo_i = mid + 1; else hi_i = mid;
            }
            int e_prev = lo_i - 1;
            int q[U];
            bool ok[U];
            V av[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int base = pb + WAVE * u;
                ok[u] = false;
                q[u] = 0;
                av[u] = V(0);
                if (base < total) {
                    const int cand = e_prev + 1 + ln;
                    if (cand < nseg) {
                        const int so = sg.off[cand];
                        if (so < base + WAVE) sg.mark[w][so - base] = 1;
                    }
                    wave_sync();
                    const uint64_t M = __ballot(sg.mark[w][ln] != 0);
                    sg.mark[w][ln] = 0;
                    int eh = e_prev + __popcll(M & lanemask_le());
                    eh = eh < 0 ? 0 : (eh >= nseg ? nseg - 1 : eh);
                    const int p = base + ln;
                    if (p < total) {
                        ok[u] = true;
                        q[u] = sg.lo[eh] + (p - sg.off[eh]);
                        if constexpr (NUM) av[u] = sg.a[eh];
                    }
                    e_prev += __popcll(M);
                    wave_sync();
                }
            }
            act(q, ok, av);
        }
        block_sync<G>();
    }
}

// Exclusive in-place bitonic sort (ascending keys) of n <= np2 entries held in
// LDS, all compare-exchanges oriented low-to-high so that positions >= n
// behave as +infinity and need no storage.
template <int G, typename V>
__device__ void bitonic_sort_lds(int *keys, V *vals, int n) {
    if (n <= 1) return;
    int lg = 0;
    while ((1 << lg) < n) ++lg;
    const int half_total = 1 << (lg - 1);
    for (int s = 1; s <= lg; ++s) {
        const int hs = s - 1;                  // log2(half block)
        for (int t = threadIdx.x; t < half_total; t += G) {
            const int blk = t >> hs, o = t & ((1 << hs) - 1);
            const int i = (blk << s) + o;
            const int j = (blk << s) + (1 << s) - 1 - o;
            if (j < n) {
                const int ki = keys[i], kj = keys[j];
                if (ki > kj) {
                    keys[i] = kj; keys[j] = ki;
                    const V vi = vals[i]; vals[i] = vals[j]; vals[j] = vi;
                }
            }
        }
        block_sync<G>();
        for (int ls = hs - 1; ls >= 0; --ls) {
            for (int t = threadIdx.x; t < half_total; t += G) {
                const int i = ((t >> ls) << (ls + 1)) + (t & ((1 << ls) - 1));
                const int j = i + (1 << ls);
                if (j < n) {
                    const int ki = keys[i], kj = keys[j];
                    if (ki > kj) {
                        keys[i] = kj; keys[j] = ki;
                        const V vi = vals[i]; vals[i] = vals[j]; vals[j] = vi;
                    }
                }
            }
            block_sync<G>();
        }
    }
}

// Compact the occupied slots of an LDS table to its front (table order),
// optionally sort them, and copy them to the output.  Returns the count.
template <int G, int T, bool SORTED, typename V>
__device__ __forceinline__ int compact_store(int *keys, V *vals, int *wsum, int64_t out_pos,
                                             int expected, int32_t *__restrict__ colsC,
                                             V *__restrict__ valsC, int *err) {
    constexpr int S = (T + G - 1) / G;
    const int tid = threadIdx.x;
    int kk[S];
    V vv[S];
    int c = 0;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int s = tid * S + j;
        kk[j] = -1;
        vv[j] = V(0);
        if (s < T) { kk[j] = keys[s]; vv[j] = vals[s]; }
        c += kk[j] != -1;
    }
    int total;
    int pos = block_excl_scan<G, int>(c, total, wsum);
    block_sync<G>();
#pragma unroll
    for (int j = 0; j < S; ++j)
        if (kk[j] != -1) { keys[pos] = kk[j]; vals[pos] = vv[j]; ++pos; }
    block_sync<G>();
    if constexpr (SORTED) bitonic_sort_lds<G, V>(keys, vals, total);
    const int n = total < expected ? total : expected;
    if (total != expected && tid == 0) atomicOr(err, ERR_COUNT);
    for (int j = tid; j < n; j += G) {
        colsC[out_pos + j] = keys[j];
        valsC[out_pos + j] = vals[j];
    }
    return total;
}

}  // namespace spg
