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

// Value of x from another lane by a DPP move (VALU only, no LDS): lanes
// whose source lies outside the pattern, or whose row is outside ROW_MASK,
// get 0.  CTRL 0x00..0xFF = a permutation inside each quad of lanes (2 bits
// per lane); 0x110+n = shift right by n within each row of 16 lanes; 0x142 =
// lane 15 of each row to the whole next row; 0x143 = lane 31 to the rows
// above it.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_i32(int x) {
    return __builtin_amdgcn_update_dpp(0, x, CTRL, ROW_MASK, 0xF, false);
}
template <int CTRL, int ROW_MASK, typename T>
__device__ __forceinline__ T dpp_move(T x) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit lanes");
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, dpp_i32<CTRL, ROW_MASK>(__builtin_bit_cast(int, x)));
    } else {
        const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
        const unsigned lo = (unsigned)dpp_i32<CTRL, ROW_MASK>((int)(unsigned)u);
        const unsigned hi = (unsigned)dpp_i32<CTRL, ROW_MASK>((int)(unsigned)(u >> 32));
        return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
    }
}

// Inclusive prefix sum over the 64 lanes of a wave (all lanes active):
// Hillis-Steele steps of 1, 2, 4, 8 inside each row of 16 lanes, then the
// row totals are carried upward by two broadcasts.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
    x += dpp_move<0x111, 0xF>(x);
    x += dpp_move<0x112, 0xF>(x);
    x += dpp_move<0x114, 0xF>(x);
    x += dpp_move<0x118, 0xF>(x);
    x += dpp_move<0x142, 0xA>(x);
    x += dpp_move<0x143, 0xC>(x);
    return x;
}

// Value of lane 63 (uniform).
template <typename T>
__device__ __forceinline__ T wave_last(T x) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit lanes");
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 63));
    } else {
        const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
        const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, 63);
        const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), 63);
        return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
    }
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
    return wave_last(wave_incl_scan(x));
}

__device__ __forceinline__ int wave_sum_i32(int x) {
    return wave_last(wave_incl_scan(x));
}

// Exclusive scan over a block of G threads (G a multiple of 64, <= 1024).
// wsum needs G/64 + 1 entries of LDS.  Contains block barriers when G > 64.
template <int G, typename T>
__device__ __forceinline__ T block_excl_scan(T x, T &total, T *wsum) {
    constexpr int NW = G / WAVE;
    const T incl = wave_incl_scan<T>(x);
    if constexpr (NW == 1) {
        total = wave_last(incl);
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
// half of (key * mul mod 2^32) * T, a multiplicative hash (Section 4.2.1:
// the key times a constant) folded onto any table size T; collisions are
// resolved by linear probing with wrap-around.  mul = 0 sends every key to
// slot 0 (a worst case for tests).
__device__ __forceinline__ uint32_t hash_slot(int key, uint32_t T, uint32_t mul = HASH_MUL_DEFAULT) {
    const uint32_t h = (uint32_t)key * mul;
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

// ---- bucketed tables (vector probing) ----------------------------------------
// The table is split into buckets of 4 consecutive slots read with one 16-byte
// LDS load; a key is looked for in its whole bucket at once, a new key takes
// the first empty slot of the bucket (slots fill from the front), and a full
// bucket without the key sends the probe to the next bucket (linear probing
// over buckets).  This is the chunked probing of the paper's HashVector
// (Section 4.2.2) with a 4-slot chunk matched to one ds_read_b128.
constexpr int BKT = 4;

__device__ __forceinline__ int4 lds_load4(const int *p) {
    return *reinterpret_cast<const int4 *>(p);
}

// Slot of key in the bucket (match or first empty), -1 if full without it;
// empty_hit says the slot is empty (needs a CAS).
__device__ __forceinline__ int bucket_pick(int4 k, int key, bool &empty_hit) {
    // selects, not branches: the first match, else the first empty slot
    int m = k.w == key ? 3 : -1;
    m = k.z == key ? 2 : m;
    m = k.y == key ? 1 : m;
    m = k.x == key ? 0 : m;
    int f = k.w == -1 ? 3 : -1;
    f = k.z == -1 ? 2 : f;
    f = k.y == -1 ? 1 : f;
    f = k.x == -1 ? 0 : f;
    empty_hit = m < 0 && f >= 0;
    return m >= 0 ? m : f;
}

// Insert key (and with NUM add x to its value); returns 1 if the key is new.
// A bucket is bq consecutive quads (4 slots each, one 16-byte LDS load): the
// quads of the key's bucket are read front to back, a quad holding the key or
// an empty slot ends the probe (slots, and then quads, fill from the front,
// so a key is never behind an empty slot), and a full bucket sends the probe
// to the next bucket.  bq = 1 is the 4-slot bucket; bq = 2 or 4 the 8- or
// 16-slot chunk of the paper's HashVector (Section 4.2.2), which trades a
// longer scan of a busy bucket for fewer jumps to the next one.  A probe
// that runs past every bucket without room sets ovf and gives up.
// FIXED_BQ > 0 fixes bq at compile time (the default 4-slot buckets compile
// to the plain one-quad probe).
// *probes (if given) counts the quads read: the collision factor of Eq. 2 is
// their number per insertion.
template <bool NUM, typename V, int FIXED_BQ = 0>
__device__ __forceinline__ int bkt_insert(int *keys, V *vals, uint32_t T, int key, V x, int &ovf,
                                          uint32_t mul = HASH_MUL_DEFAULT, uint32_t bq_rt = 1,
                                          unsigned *probes = nullptr) {
    const uint32_t bq = FIXED_BQ > 0 ? (uint32_t)FIXED_BQ : bq_rt;
    const uint32_t W = BKT * bq;                   // slots per bucket
    const uint32_t NB = T / W;
    if (bq == 1) {
        // 4-slot buckets: the key's own slot (inside its bucket) is tried
        // first with one CAS, which settles the insert when that slot was
        // empty or already held the key; otherwise the bucket is scanned.  A
        // key then sits either in its own slot or in the first slot of the
        // bucket that was empty when it arrived, both inside the bucket that
        // every insert of the key reads whole, so no duplicate can arise.
        const uint32_t h = hash_slot(key, T, mul);
        if (probes) ++*probes;
        const int old = atomicCAS(&keys[h], -1, key);
        if (old == -1 || old == key) {
            if constexpr (NUM) lds_add(&vals[h], x);
            return old == -1;
        }
    }
    uint32_t b = hash_slot(key, NB, mul);
    uint32_t q = 0;                                // quad of the bucket being read
    for (uint32_t it = 0; it < T / BKT + T; ++it) {
        __asm__ __volatile__("" ::: "memory");   // re-read the quad every round
        const uint32_t base = b * W + q * BKT;
        const int4 k = lds_load4(&keys[base]);
        if (probes) ++*probes;
        bool e;
        const int j = bucket_pick(k, key, e);
        if (j < 0) {                               // quad full without the key
            if (++q == bq) {
                q = 0;
                b = (b + 1 == NB) ? 0u : b + 1;
            }
            continue;
        }
        int added = 0;
        if (e) {
            const int old = atomicCAS(&keys[base + j], -1, key);
            if (old != -1 && old != key) continue;    // lost the slot: look at this quad again
            added = old == -1;
        }
        if constexpr (NUM) lds_add(&vals[base + j], x);
        return added;
    }
    ovf = 1;
    return 0;
}

// ---- product enumeration ---------------------------------------------------
// The products of one row of C are the pairs (a_ik, b_kj) for every stored
// a_ik of the row and every b_kj of a slice of row k of B (the whole row, or
// the part inside a column window).  A block of G threads takes the row's
// A entries G at a time and lays their slices end to end (exclusive scan of
// the slice lengths).  Wave w then owns the contiguous product range
// [w*P/NW, (w+1)*P/NW), so a few long B rows are spread evenly over all
// waves.  It walks its range in batches of 64*U products: the segments a
// batch touches are found by galloping from the previous batch, and each
// lane locates its U products' segments by U interleaved bisections over
// that (usually tiny) range, so one batch costs a handful of LDS round trips
// and one round of U independent global loads per lane.
template <int G, bool NUM, typename V>
struct SegLds {
    int base[G];      // B index of the segment's product 0 minus its offset: product p reads B at base + p
    int off[G];
    V a[NUM ? G : 1];
    int wsum[G / WAVE + 1];
    uint2 starts[G / WAVE][32];   // per wave: segment-start bits of a batch, prefix counts
};

// One chunk: this thread's entry has slice [lo, lo+len) and multiplier a.
// act(q[U], ok[U], a[U]) processes up to U products per lane: B index q,
// multiplier a (numeric phase), ok = valid.  q is a valid B index even where
// ok is false (the first entry of some segment), so act may load at q
// unconditionally and discard the value.
// The batches of products of segments already laid out in sg (nseg
// segments, total products; see enum_chunk), ending with a block barrier.
template <int G, int U, bool NUM, typename V, bool SNUM, class ActF>
__device__ __forceinline__ void enum_walk(int total, int nseg, SegLds<G, SNUM, V> &sg, ActF act) {
    static_assert(SNUM || !NUM, "numeric enumeration needs room for the multipliers");
    constexpr int NW = G / WAVE;
    const int ln = threadIdx.x & 63;
    const int w = G == WAVE ? 0 : (int)(threadIdx.x >> 6);   // G == 64: one wave of a larger block
    const int P0 = (int)(((long long)w * total) / NW);
    const int P1 = (int)(((long long)(w + 1) * total) / NW);
    if (P0 < P1) {
        // segment of the wave's first product (segment 0 holds product 0)
        int e = 0;
        if (P0 > 0) {
            int hi = nseg - 1;
            while (e < hi) {
                const int mid = (e + hi + 1) >> 1;
                if (sg.off[mid] <= P0) e = mid; else hi = mid - 1;
            }
        }
        for (int pb = P0; pb < P1; pb += WAVE * U) {
            const int last = min(pb + WAVE * U, P1) - 1;
            // segment of the batch's last product: the last segment when the
            // batch ends the row, else by galloping and bisection from e
            int eh = e;
            if (last == total - 1) {
                eh = nseg - 1;
            } else {
                int step = 1;
                while (eh + step < nseg && sg.off[eh + step] <= last) { eh += step; step <<= 1; }
                int top = min(eh + step, nseg) - 1;
                while (eh < top) {
                    const int mid = (eh + top + 1) >> 1;
                    if (sg.off[mid] <= last) eh = mid; else top = mid - 1;
                }
            }
            // lanes past the range read the batch's last product again (a
            // valid index) so that loads need no branch
            int q[U];
            bool ok[U];
            V av[U];
            if (e == eh) {
                // the whole batch lies in one segment: uniform base, no search
                const int base = sg.base[e];
                V a1 = V(0);
                if constexpr (NUM) a1 = sg.a[e];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int p = pb + WAVE * u + ln;
                    ok[u] = p <= last;
                    q[u] = base + min(p, last);
                    av[u] = a1;
                }
            } else {
                // segment of each product of the batch: the wave marks where
                // the segments e+1..eh start inside [pb, pb + 64U) in an LDS
                // bitmap with per-word prefix counts; product p then lies in
                // segment e + (number of starts at or before p).
                static_assert(U * WAVE <= 32 * 32, "batch larger than the start bitmap");
                constexpr int NWD = (U * WAVE + 31) / 32;
                uint2 *sb = sg.starts[w];
                if (ln < NWD) sb[ln].x = 0u;
                wave_sync();
                for (int sidx = e + 1 + ln; sidx <= eh; sidx += WAVE) {
                    const int rel = sg.off[sidx] - pb;
                    atomicOr(&sb[rel >> 5].x, 1u << (rel & 31));
                }
                wave_sync();
                {
                    const uint32_t bits = ln < NWD ? sb[ln].x : 0u;
                    const int c = __popc(bits);
                    const int incl = wave_incl_scan<int>(c);
                    if (ln < NWD) sb[ln].y = (uint32_t)(incl - c);
                }
                wave_sync();
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int rel = WAVE * u + ln;
                    const int p = pb + rel;
                    const uint2 bw = sb[rel >> 5];
                    const uint32_t upto = (uint32_t)((2ull << (rel & 31)) - 1ull);
                    const int seg = e + (int)bw.y + __popc(bw.x & upto);
                    ok[u] = p <= last;
                    q[u] = sg.base[seg] + min(p, last);    // p > last: seg is eh, which holds last
                    av[u] = V(0);
                    if constexpr (NUM) av[u] = sg.a[seg];
                }
                wave_sync();        // the bitmap is reused by the next batch
            }
            act(q, ok, av);
            e = eh;
        }
    }
    block_sync<G>();
}

template <int G, int U, bool NUM, typename V, bool SNUM, class ActF>
__device__ __forceinline__ void enum_chunk(int lo, int len, V a, SegLds<G, SNUM, V> &sg, ActF act) {
    int total, nseg;
    const int pre_len = block_excl_scan<G, int>(len, total, sg.wsum);
    const int pre_ne = block_excl_scan<G, int>(len > 0 ? 1 : 0, nseg, sg.wsum);
    if (len > 0) {
        sg.base[pre_ne] = lo - pre_len;
        sg.off[pre_ne] = pre_len;
        if constexpr (NUM) sg.a[pre_ne] = a;
    }
    block_sync<G>();
    enum_walk<G, U, NUM, V>(total, nseg, sg, act);
}

// All A entries [a0, a1) of a row, G at a time; slice(k, lo, hi) gives the
// B entries [lo, hi) that a_ik multiplies.
template <int G, int U, bool NUM, typename V, bool SNUM, class SliceF, class ActF>
__device__ __forceinline__ void enum_row(int a0, int a1, const int32_t *__restrict__ colsA,
                                         const V *__restrict__ valsA, SegLds<G, SNUM, V> &sg,
                                         SliceF slice, ActF act) {
    for (int cb = a0; cb < a1; cb += G) {
        const int e = cb + (int)(threadIdx.x & (G - 1));
        int lo = 0, hi = 0;
        V a = V(0);
        if (e < a1) {
            slice(colsA[e], lo, hi);
            if constexpr (NUM) a = valsA[e];
        }
        enum_chunk<G, U, NUM, V>(lo, hi - lo, a, sg, act);
    }
}

// Sort the n <= T entries at the front of a T-slot table (distinct keys >= 0)
// in one pass of bucketing: keys are spread over NB = T/2 buckets by their
// place in [min, max] (a monotone map), the bucket counts are scanned, every
// entry is scattered to its bucket, and its rank is its bucket's start plus
// the number of smaller keys in the bucket (a handful on average).  The
// entries wait in registers meanwhile, and the value array serves as the
// counters.  A few LDS operations per entry, against the two LDS round trips
// per stage of a bitonic network or the n comparisons per entry of a rank
// count.  Ends with the sorted entries at [0, n) and a block barrier.
template <int G, int T, typename V>
__device__ void bucket_sort_lds(int *keys, V *vals, int n) {
    static_assert(T % G == 0 && sizeof(V) == 8, "table layout");
    constexpr int E = T / G;                  // entries per thread at most
    constexpr int NB = T / 2;
    constexpr int NW = G / WAVE;
    static_assert(3 * NB + 2 * NW <= 2 * T, "counters fit the value array");
    if (n <= 1) return;                       // uniform over the block
    const int tid = threadIdx.x;
    int k[E], b[E];
    V v[E];
    int lo = INT32_MAX, hi = -1;
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int e = tid + i * G;
        k[i] = e < n ? keys[e] : -1;
        v[i] = e < n ? vals[e] : V(0);
        if (e < n) { lo = min(lo, k[i]); hi = max(hi, k[i]); }
    }
    lo = __ockl_wfred_min_i32(lo);
    hi = __ockl_wfred_max_i32(hi);
    block_sync<G>();                          // every entry read: the arrays are free
    int *cnt = reinterpret_cast<int *>(vals);
    int *start = cnt + NB;
    int *cur = start + NB;
    if constexpr (NW > 1) {
        int *red = cur + NB;                  // per-wave minima, then maxima
        if ((tid & 63) == 0) { red[tid >> 6] = lo; red[NW + (tid >> 6)] = hi; }
    }
    for (int i = tid; i < NB; i += G) { cnt[i] = 0; cur[i] = 0; }
    block_sync<G>();
    if constexpr (NW > 1) {
        const int *red = cur + NB;
        for (int w = 0; w < NW; ++w) { lo = min(lo, red[w]); hi = max(hi, red[NW + w]); }
    }
    // bucket of key x: x - lo when the keys span at most NB values, else
    // (x - lo) * m / 2^32 with m = floor(NB * 2^32 / span): monotone in x, < NB
    const unsigned span = (unsigned)(hi - lo) + 1u;
    const unsigned long long m = span <= (unsigned)NB ? 0ull : ((unsigned long long)NB << 32) / span;
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const unsigned x = (unsigned)(k[i] - lo);
        b[i] = k[i] < 0 ? 0 : (m == 0 ? (int)x : (int)(((unsigned long long)x * m) >> 32));
        if (k[i] >= 0) atomicAdd(&cnt[b[i]], 1);
    }
    block_sync<G>();
    {
        // exclusive scan of the counts: NB/G consecutive buckets per thread
        constexpr int PB = (NB + G - 1) / G;
        int c = 0;
#pragma unroll
        for (int j = 0; j < PB; ++j) {
            const int q = tid * PB + j;
            if (q < NB) c += cnt[q];
        }
        int tot;
        int pre = block_excl_scan<G, int>(c, tot, reinterpret_cast<int *>(keys) + T - (NW + 1));
#pragma unroll
        for (int j = 0; j < PB; ++j) {
            const int q = tid * PB + j;
            if (q < NB) { start[q] = pre; pre += cnt[q]; }
        }
    }
    block_sync<G>();
#pragma unroll
    for (int i = 0; i < E; ++i)
        if (k[i] >= 0) keys[start[b[i]] + atomicAdd(&cur[b[i]], 1)] = k[i];
    block_sync<G>();
    int r[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
        r[i] = -1;
        if (k[i] >= 0) {
            // eight reads in flight: a skewed key set can put many keys in
            // one bucket (R-MAT rows crowd their low columns)
            const int s0 = start[b[i]], s1 = s0 + cnt[b[i]];
            int c = s0, q = s0;
            for (; q + 8 <= s1; q += 8) {
                int t = 0;
#pragma unroll
                for (int u = 0; u < 8; ++u) t += keys[q + u] < k[i];
                c += t;
            }
            for (; q < s1; ++q) c += keys[q] < k[i];
            r[i] = c;
        }
    }
    block_sync<G>();                          // every bucket read before the entries move
    int *kk = keys;
#pragma unroll
    for (int i = 0; i < E; ++i)
        if (r[i] >= 0) { kk[r[i]] = k[i]; vals[r[i]] = v[i]; }
    block_sync<G>();
}

// Compact the occupied slots of an LDS table to its front (slots read lane by
// lane, so in a permuted table order; the sorted output does not see it),
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
        const int s = j * G + tid;                    // lane by lane: no bank conflicts
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
    const int n = total < expected ? total : expected;
    if (total != expected && tid == 0) atomicOr(err, ERR_COUNT);
    if constexpr (SORTED) {
        bucket_sort_lds<G, T, V>(keys, vals, total);
    }
    for (int j = tid; j < n; j += G) {
        __builtin_nontemporal_store(keys[j], &colsC[out_pos + j]);
        __builtin_nontemporal_store(vals[j], &valsC[out_pos + j]);
    }
    return total;
}

// Unsorted output of a finished table: wave w takes the slots [w*T/NW,
// (w+1)*T/NW), read lane by lane (conflict-free), counts its keys from one
// ballot per row of 64 slots, the counts are scanned across the waves, and
// each wave writes its entries in the runs the ballots give: the entries go
// from the table to C with no LDS round trip.  Returns the number of keys.
template <int G, int T, typename V>
__device__ __forceinline__ int compact_store_unsorted(const int *keys, const V *vals, int *wsum, int64_t out_pos,
                                                      int expected, int32_t *__restrict__ colsC,
                                                      V *__restrict__ valsC, int *err) {
    constexpr int NW = G / WAVE;
    static_assert(T % G == 0, "table size a multiple of the block");
    constexpr int S = T / G;
    const int ln = lane_id();
    const int w = NW == 1 ? 0 : (int)(threadIdx.x >> 6);
    const int *kw = keys + w * (T / NW);
    int kk[S];
    unsigned long long m[S];
    int c = 0;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        kk[j] = kw[j * WAVE + ln];
        m[j] = __ballot(kk[j] != -1);
        c += __popcll(m[j]);
    }
    int base = 0, total = c;
    if constexpr (NW > 1) {
        if (ln == 0) wsum[w] = c;
        __syncthreads();
        const int v = ln < NW ? wsum[ln] : 0;
        base = wave_sum_i32(ln < w ? v : 0);
        total = wave_sum_i32(v);
        __syncthreads();                      // wsum is free again
    }
    const V *vw = vals + w * (T / NW);
    const unsigned long long below = (1ull << ln) - 1ull;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int pos = base + __popcll(m[j] & below);
        if (kk[j] != -1 && pos < expected) {
            __builtin_nontemporal_store(kk[j], &colsC[out_pos + pos]);
            __builtin_nontemporal_store(vw[j * WAVE + ln], &valsC[out_pos + pos]);
        }
        base += __popcll(m[j]);
    }
    if (total != expected && threadIdx.x == 0) atomicOr(err, ERR_COUNT);
    return total;
}

// Empty a table of T keys (and with NUM its 8-byte values, zeroed): 16-byte
// LDS stores; both arrays 16-byte aligned.
template <int G, int T, bool NUM, typename V>
__device__ __forceinline__ void table_clear(int *keys, V *vals) {
    static_assert(T % 4 == 0 && sizeof(V) == 8, "table layout");
    int4 *k4 = reinterpret_cast<int4 *>(keys);
    for (int i = (int)threadIdx.x; i < T / 4; i += G) k4[i] = make_int4(-1, -1, -1, -1);
    if constexpr (NUM) {
        ulonglong2 *v2 = reinterpret_cast<ulonglong2 *>(vals);
        for (int i = (int)threadIdx.x; i < T / 2; i += G) v2[i] = make_ulonglong2(0ull, 0ull);
    }
}

}  // namespace spg
