// C ABI of the gfx950 SpGEMM library: plan / symbolic / numeric / free.
//
// Host-side orchestration of the two-phase hash SpGEMM (paper Section 2,
// two-phase method; Section 4.2.1, Fig. 5).  The library never allocates
// device memory: the plan scratch, the workspace and C come from the caller.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/spgemm.h"
#include "config.hpp"
#include "launch.hpp"

using namespace spg;

namespace {

thread_local char g_hip_msg[256] = "";

int hip_fail(hipError_t e, const char *what) {
    snprintf(g_hip_msg, sizeof(g_hip_msg), "HIP error in %s: %s", what, hipGetErrorString(e));
    return SPGEMM_ERR_HIP;
}

#define HIPCK(expr, what)                           \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

struct TimedLaunch {
    std::string name;
    hipEvent_t e0, e1;
    double bytes;
};

struct Prod {
    CsrDev A, B;
    int64_t m = 0;
    // plan scratch
    char *ps = nullptr;
    PlanHdr *phdr = nullptr;
    uint32_t *flop = nullptr;
    PlanHdr h{};
    int64_t sym_off[NSB]{};
    int64_t nbm = 0;          // rows in the bitmap bin
    int nchunks = 0;
    unsigned items_cap = 0;
    // workspace layout (offsets from the product's base)
    size_t ws_base = 0, ws_bytes = 0;
    size_t o_hdr = 0, o_perm_sym = 0, o_prow_sym = 0, o_rows_num = 0, o_nnz = 0, o_bsum = 0;
    size_t o_chunk = 0, o_heavy = 0, o_items = 0, o_bc = 0, o_bv = 0, o_long = 0;
    size_t o_whist = 0, o_long_id = 0, o_idx = 0, o_slot = 0, o_bperm = 0, o_bmap = 0, o_bs = 0, o_ki = 0;
    bool store_bm = false;    // symbolic bitmaps kept for the numeric windows
    // after symbolic
    char *ws = nullptr;
    WsHdr *wh = nullptr;
    WsHdr hw{};
    int64_t *rpts_C = nullptr;
    int64_t num_off[NNB]{};

    template <typename T> T *at(size_t off) const { return (T *)(ws + off); }
};

enum State { PLANNED = 1, SYMBOLIC_DONE = 2 };

}  // namespace

struct spgemm_plan_s {
    int nprod = 0;
    int dtype = 0;
    unsigned flags = 0;
    hipStream_t stream = nullptr;
    int state = 0;
    std::vector<Prod> prods;
    size_t ws_total = 0;
    bool timing = false;
    uint32_t count_probes = 0;
    int ncu = 256;
    BinLimits lim = default_limits();
    std::vector<TimedLaunch> tl;
};

namespace {

template <class F>
hipError_t timed(spgemm_plan_s *p, const char *name, double bytes, F f) {
    if (!p->timing) return f();
    TimedLaunch t{name, nullptr, nullptr, bytes};
    hipError_t e = hipEventCreate(&t.e0);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&t.e1);
    if (e != hipSuccess) return e;
    e = hipEventRecord(t.e0, p->stream);
    if (e != hipSuccess) return e;
    e = f();
    if (e != hipSuccess) return e;
    e = hipEventRecord(t.e1, p->stream);
    p->tl.push_back(t);
    return e;
}

bool csr_ok(const spgemm_csr &a) {
    if (a.nrows < 0 || a.ncols < 0 || a.nnz < 0) return false;
    if (a.nrows >= INT32_MAX || a.ncols >= INT32_MAX || a.nnz >= INT32_MAX) return false;
    if (!a.rpts) return false;
    if (a.nnz > 0 && !a.cols) return false;
    return true;
}

CsrDev dev(const spgemm_csr &a) { return CsrDev{a.nrows, a.ncols, a.nnz, a.rpts, a.cols, a.vals}; }

// Per-bin limits of a config, checked against the table sizes (a limit above
// its table could leave a probe without a free slot).
bool limits_from(const spgemm_config *cfg, BinLimits *L) {
    *L = default_limits();
    if (!cfg) return true;
    for (int b = 1; b <= 9; ++b) {
        const int64_t s = cfg->sym_max[b - 1], n = cfg->num_max[b - 1];
        if (s < 1 || s > SYM_T[b] || s < L->sym[b - 1]) return false;
        if (n < 1 || n > NUM_T[b] || n < L->num[b - 1]) return false;
        L->sym[b] = s;
        L->num[b] = n;
    }
    if (L->sym[9] != WIN_CAP || L->num[9] != WIN_CAP) return false;
    if (cfg->bucket_slots != 4 && cfg->bucket_slots != 8 && cfg->bucket_slots != 16) return false;
    if (cfg->heap > 1) return false;
    L->hmul = cfg->hash_mul;
    L->bq = cfg->bucket_slots / 4;
    L->heap = cfg->heap;
    return true;
}

// header, per-row flop (uint32), the list of rows longer than FLOP_WAVE_ROW,
// the list of rows of FLOP_SHORT_ROW+1 .. FLOP_WAVE_ROW entries (int32 each)
static size_t huge_list_bytes(int64_t nnz) { return align_up((size_t)(nnz / (FLOP_WAVE_ROW + 1)) * 4); }
static size_t long_list_bytes(int64_t m, int64_t nnz) {
    return align_up((size_t)std::min<int64_t>(m, nnz / (FLOP_SHORT_ROW + 1)) * 4);
}
size_t plan_scratch_one(int64_t m, int64_t nnz) {
    return PLAN_HDR_BYTES + align_up((size_t)m * 4) + huge_list_bytes(nnz) + long_list_bytes(m, nnz);
}

// Workspace of spgemm_symbolic_static.  Each GPU the library runs on holds
// its own copy until the process ends; host code reaches it only through
// the address hipGetSymbolAddress gives for the current device.
static __device__ __align__(256) unsigned char scratch[SPGEMM_STATIC_WS_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the static workspace on device dev (which is current),
// resolved on the first call per device.
int static_workspace(int dev, void **out) {
    if (dev < 0 || dev >= MAX_DEVICES) return SPGEMM_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPCK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p) return SPGEMM_ERR_INTERNAL;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SPGEMM_OK;
}

}  // namespace

extern "C" {

size_t spgemm_plan_scratch_bytes(int nprod, const spgemm_csr *A) {
    if (nprod <= 0 || !A) return 0;
    size_t t = 0;
    for (int p = 0; p < nprod; ++p) {
        if (A[p].nrows < 0 || A[p].nnz < 0) return 0;
        t += plan_scratch_one(A[p].nrows, A[p].nnz);
    }
    return t;
}

const char *spgemm_strerror(int status) {
    switch (status) {
        case SPGEMM_OK: return "ok";
        case SPGEMM_ERR_INVALID_ARG: return "invalid argument";
        case SPGEMM_ERR_SHAPE: return "shape mismatch: A.ncols != B.nrows";
        case SPGEMM_ERR_INVALID_CSR: return "malformed CSR input";
        case SPGEMM_ERR_WORKSPACE: return "workspace missing or too small";
        case SPGEMM_ERR_OVERFLOW: return "size exceeds the supported index range";
        case SPGEMM_ERR_STATE: return "call out of order";
        case SPGEMM_ERR_HIP: return g_hip_msg[0] ? g_hip_msg : "HIP runtime error";
        case SPGEMM_ERR_UNSUPPORTED: return "input outside the supported envelope";
        case SPGEMM_ERR_HOST_ALLOC: return "host allocation failed";
        case SPGEMM_ERR_INTERNAL: return "device-side consistency check failed";
        case SPGEMM_ERR_STATIC_LIMIT:
            return "the plan's workspace exceeds the static scratch of spgemm_symbolic_static (64 MiB)";
        default: return "unknown status";
    }
}

void spgemm_config_default(spgemm_config *cfg) {
    if (!cfg) return;
    cfg->hash_mul = HASH_MUL_DEFAULT;
    cfg->bucket_slots = 4;
    cfg->heap = 0;
    for (int b = 1; b <= 9; ++b) {
        cfg->sym_max[b - 1] = (int32_t)SYM_XMAX[b];
        cfg->num_max[b - 1] = (int32_t)NUM_XMAX[b];
    }
}

int spgemm_config_check(const spgemm_config *cfg) {
    BinLimits L;
    return (cfg && limits_from(cfg, &L)) ? SPGEMM_OK : SPGEMM_ERR_INVALID_ARG;
}

int spgemm_plan(spgemm_plan_t *out, int nprod, const spgemm_csr *A, const spgemm_csr *B, spgemm_dtype dtype,
                unsigned flags, void *plan_scratch, hipStream_t stream, size_t *workspace_bytes,
                const spgemm_config *cfg) {
    if (!out) return SPGEMM_ERR_INVALID_ARG;
    *out = nullptr;
    if (nprod <= 0 || !A || !B || !workspace_bytes) return SPGEMM_ERR_INVALID_ARG;
    if (dtype != SPGEMM_F64 && dtype != SPGEMM_I64) return SPGEMM_ERR_INVALID_ARG;
    if (flags & ~(unsigned)(SPGEMM_SORTED | SPGEMM_VALIDATE | SPGEMM_TIMING | SPGEMM_LOW_MEMORY |
                            SPGEMM_PROBE_COUNT))
        return SPGEMM_ERR_INVALID_ARG;
    for (int p = 0; p < nprod; ++p) {
        if (!csr_ok(A[p]) || !csr_ok(B[p])) return SPGEMM_ERR_INVALID_ARG;
        if (A[p].ncols != B[p].nrows) return SPGEMM_ERR_SHAPE;
    }
    if (!plan_scratch) return SPGEMM_ERR_INVALID_ARG;
    BinLimits lim;
    if (!limits_from(cfg, &lim)) return SPGEMM_ERR_INVALID_ARG;
    if (lim.heap && !(flags & SPGEMM_SORTED)) return SPGEMM_ERR_INVALID_ARG;   // the merge emits sorted rows

    spgemm_plan_s *pl = new (std::nothrow) spgemm_plan_s();
    if (!pl) return SPGEMM_ERR_HOST_ALLOC;
    pl->lim = lim;
    pl->nprod = nprod;
    pl->dtype = (int)dtype;
    pl->flags = flags;
    pl->stream = stream;
    pl->timing = (flags & SPGEMM_TIMING) != 0;
    pl->count_probes = (flags & SPGEMM_PROBE_COUNT) ? 1u : 0u;
    {
        int devid = 0, ncu = 0;
        if (hipGetDevice(&devid) == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, devid) == hipSuccess && ncu > 0)
            pl->ncu = ncu;
    }
    pl->prods.resize(nprod);
    auto fail = [&](int st) { delete pl; return st; };

    char *ps = (char *)plan_scratch;
    for (int p = 0; p < nprod; ++p) {
        Prod &q = pl->prods[p];
        q.A = dev(A[p]);
        q.B = dev(B[p]);
        q.m = A[p].nrows;
        q.ps = ps;
        q.phdr = (PlanHdr *)ps;
        q.flop = (uint32_t *)(ps + PLAN_HDR_BYTES);
        ps += plan_scratch_one(q.m, q.A.nnz);
        hipError_t e = hipMemsetAsync(q.phdr, 0, sizeof(PlanHdr), stream);
        if (e != hipSuccess) return fail(hip_fail(e, "hipMemsetAsync(plan header)"));
    }
    if (flags & SPGEMM_VALIDATE) {
        for (int p = 0; p < nprod; ++p) {
            Prod &q = pl->prods[p];
            hipError_t e = launch_validate(q.A, &q.phdr->err, stream);
            if (e == hipSuccess) e = launch_validate(q.B, &q.phdr->err, stream);
            if (e != hipSuccess) return fail(hip_fail(e, "validate"));
        }
        int bad = 0;
        for (int p = 0; p < nprod; ++p) {
            int err = 0;
            hipError_t e = hipMemcpyAsync(&err, &pl->prods[p].phdr->err, sizeof(int), hipMemcpyDeviceToHost, stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return fail(hip_fail(e, "validate readback"));
            bad |= err;
        }
        if (bad) return fail(SPGEMM_ERR_INVALID_CSR);
    }
    for (int p = 0; p < nprod; ++p) {
        Prod &q = pl->prods[p];
        int32_t *huge = (int32_t *)(q.ps + PLAN_HDR_BYTES + align_up((size_t)q.m * 4));   // after the row flop
        int32_t *longl = (int32_t *)((char *)huge + huge_list_bytes(q.A.nnz));
        hipError_t e = timed(pl, "row_flop", 12.0 * q.A.nnz + 8.0 * q.m, [&] {
            return launch_row_flop(q.A, q.B, q.flop, longl, huge, q.phdr, pl->lim, pl->ncu, stream);
        });
        if (e == hipSuccess) e = launch_count_long_b(q.B, q.phdr, stream);
        if (e == hipSuccess && pl->lim.heap) e = launch_check_sorted(q.B, &q.phdr->err, stream);
        if (e != hipSuccess) return fail(hip_fail(e, "row_flop"));
    }
    for (int p = 0; p < nprod; ++p) {
        hipError_t e = hipMemcpyAsync(&pl->prods[p].h, pl->prods[p].phdr, sizeof(PlanHdr), hipMemcpyDeviceToHost,
                                      stream);
        if (e != hipSuccess) return fail(hip_fail(e, "plan readback"));
    }
    {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return fail(hip_fail(e, "plan sync"));
    }

    size_t ws = 0;
    for (int p = 0; p < nprod; ++p) {
        Prod &q = pl->prods[p];
        if (q.h.max_flop > (unsigned long long)INT32_MAX) return fail(SPGEMM_ERR_UNSUPPORTED);
        if (pl->lim.heap && (q.h.err & ERR_UNSORTED_B)) return fail(SPGEMM_ERR_UNSUPPORTED);
        int64_t acc = 0;
        for (int b = 0; b < NSB; ++b) {
            q.sym_off[b] = acc;
            if (b > 0) acc += (int64_t)q.h.sym_rows[b];
        }
        q.nbm = (int64_t)q.h.sym_rows[SYM_BITMAP_BIN];
        q.nchunks = (int)((q.B.ncols + CHUNK_COLS - 1) / CHUNK_COLS);
        if (q.nbm > 0 && q.nchunks > MAX_CHUNKS) return fail(SPGEMM_ERR_UNSUPPORTED);
        const size_t m = (size_t)q.m;
        const size_t nb = (m + 4095) / 4096;
        size_t o = 0;
        q.ws_base = ws;
        q.o_hdr = o; o += align_up(WS_HDR_BYTES);
        q.o_perm_sym = o; o += align_up(4 * m);
        q.o_prow_sym = o; o += align_up(8 * m);
        q.o_rows_num = o; o += align_up(sizeof(NumRow) * m);
        q.o_nnz = o; o += align_up(4 * m);
        q.o_bsum = o; o += align_up(8 * (nb + 1));
        q.o_slot = o; o += align_up(4 * m);
        if (q.nbm > 0) {
            // a closed window uses more than 2*RANK_BUDGET - (256 + 3*4096) half words
            const unsigned long long per = 2ull * RANK_BUDGET - (2 * WORDS_PER_CHUNK + 3 * CHUNK_COLS);
            const unsigned long long cap = 3ull * q.h.total_flop / per +
                                           (unsigned long long)q.nbm *
                                               (2ull * WORDS_PER_CHUNK * q.nchunks / per + 2) + 16;
            if (cap > 0xFFFFFFF0ull) return fail(SPGEMM_ERR_OVERFLOW);
            q.items_cap = (unsigned)cap;

            q.o_chunk = o; o += align_up(4 * (size_t)q.nbm * (size_t)q.nchunks);
            const unsigned long long bm_bytes = 4ull * WORDS_PER_CHUNK * (unsigned long long)q.nbm * q.nchunks;
            q.store_bm = !(flags & SPGEMM_LOW_MEMORY) && bm_bytes <= BM_STORE_MAX;
            if (q.store_bm) { q.o_bmap = o; o += align_up((size_t)bm_bytes); }
            q.o_heavy = o; o += align_up(sizeof(HeavyRow) * (size_t)q.nbm);
            q.o_items = o; o += align_up(sizeof(WinItem) * (size_t)q.items_cap);
            q.o_whist = o; o += align_up(sizeof(uint32_t) * 2 * (size_t)q.nchunks);
            q.o_bperm = o; o += align_up(4 * (size_t)q.B.nnz);
            q.o_bc = o; o += align_up(4 * (size_t)q.B.nnz);
            q.o_bs = o; o += align_up(4 * (size_t)q.B.nnz);
            q.o_bv = o; o += align_up(8 * (size_t)q.B.nnz);
            q.o_long = o; o += align_up(4 * (size_t)q.B.nrows);
            q.o_long_id = o; o += align_up(4 * (size_t)q.B.nrows);
            q.o_idx = o; o += align_up(4 * (size_t)q.h.n_long_b * (size_t)(q.nchunks + 1));
            q.o_ki = o; o += align_up(8 * (size_t)q.A.nnz);
        }
        q.ws_bytes = o;
        ws += o;
    }
    pl->ws_total = ws;
    pl->state = PLANNED;
    *workspace_bytes = ws;
    *out = pl;
    return SPGEMM_OK;
}

int spgemm_symbolic(spgemm_plan_t pl, void *workspace, int64_t *const *rpts_C, int64_t *nnz_C) {
    if (!pl || !rpts_C || !nnz_C) return SPGEMM_ERR_INVALID_ARG;
    if (pl->state < PLANNED) return SPGEMM_ERR_STATE;
    if (pl->ws_total > 0 && !workspace) return SPGEMM_ERR_WORKSPACE;
    hipStream_t s = pl->stream;
    for (int p = 0; p < pl->nprod; ++p) {
        Prod &q = pl->prods[p];
        if (!rpts_C[p]) return SPGEMM_ERR_INVALID_ARG;
        q.ws = (char *)workspace + q.ws_base;
        q.wh = q.at<WsHdr>(q.o_hdr);
        q.rpts_C = rpts_C[p];
        HIPCK(hipMemsetAsync(q.wh, 0, sizeof(WsHdr), s), "hipMemsetAsync(workspace header)");
        const int m = (int)q.m;
        int32_t *perm = q.at<int32_t>(q.o_perm_sym);
        int32_t *nnz = q.at<int32_t>(q.o_nnz);
        BinOffsets off{};
        for (int b = 0; b < NSB; ++b) off.v[b] = q.sym_off[b];
        HIPCK(timed(pl, "sym_scatter", 8.0 * m,
                    [&] {
                        return launch_sym_scatter(m, q.flop, q.A.rpts, q.B.ncols, off, perm, q.at<int2>(q.o_prow_sym),
                                                  nnz, q.at<int32_t>(q.o_slot), q.wh, pl->lim, s);
                    }),
              "sym_scatter");
        if (q.nbm > 0) {
            HIPCK(timed(pl, "bucket_B", 8.0 * q.B.nrows + 16.0 * q.B.nnz,
                        [&] {
                            return launch_bucket(q.B, q.at<int32_t>(q.o_bc), q.at<int32_t>(q.o_bperm),
                                                 q.at<int32_t>(q.o_bs),
                                                 q.at<int32_t>(q.o_long_id), q.at<int32_t>(q.o_long),
                                                 q.at<int32_t>(q.o_idx), q.nchunks, q.wh, s);
                        }),
                  "bucket_B");
            HIPCK(timed(pl, "entry_brow", 20.0 * q.A.nnz,
                        [&] {
                            return launch_entry_brow(q.A, q.B, q.at<int32_t>(q.o_long_id), q.at<int2>(q.o_ki), s);
                        }),
                  "entry_brow");
        }
        // largest tables first: long-running blocks start early
        for (int b = NSB - 1; b >= 1; --b) {
            const unsigned nr = (unsigned)q.h.sym_rows[b];
            if (nr == 0) continue;
            const double rows_bytes = 16.0 * nr + 12.0 * q.h.sym_nnza[b] + 4.0 * q.h.sym_flop[b];
            if (b == SYM_BITMAP_BIN) {
                // B with every row in a scrambled order (see k_bucket_short)
                CsrDev Bb = q.B;
                Bb.cols = q.at<int32_t>(q.o_bs);
                HIPCK(timed(pl, "sym_bitmap", rows_bytes + 4.0 * nr * q.nchunks,
                            [&] {
                                return launch_sym_segments(nr, perm, off.v[b], q.A, Bb, q.nchunks,
                                                           q.at<uint32_t>(q.o_chunk), nnz,
                                                           q.store_bm ? q.at<uint32_t>(q.o_bmap) : nullptr,
                                                           q.wh, pl->ncu, s);
                            }),
                      "sym_bitmap");
            } else {
                char name[32];
                snprintf(name, sizeof(name), "sym_hash_%d", SYM_T[b]);
                HIPCK(timed(pl, name, rows_bytes,
                            [&] { return launch_sym_bin(b, nr, perm, q.at<int2>(q.o_prow_sym), off.v[b], q.A, q.B,
                                                        nnz, q.wh,
                                                              HashCfg{pl->lim.hmul, pl->lim.bq, pl->count_probes, (uint32_t)b},
                                                              pl->ncu, s); }),
                      "sym_hash");
            }
        }
        HIPCK(timed(pl, "scan", 16.0 * m + 8.0,
                    [&] { return launch_scan(nnz, m, q.at<long long>(q.o_bsum), q.rpts_C, q.wh, s); }),
              "scan");
        HIPCK(timed(pl, "num_hist", 12.0 * m,
                    [&] {
                        return launch_num_hist(m, nnz, q.flop, q.A.rpts, q.at<int32_t>(q.o_slot),
                                               q.at<HeavyRow>(q.o_heavy), q.wh, pl->lim, s);
                    }),
              "num_hist");
        if (q.nbm > 0) {
            HIPCK(timed(pl, "windows", 8.0 * q.nbm * q.nchunks,
                        [&] {
                            return launch_windows((unsigned)q.nbm, q.at<HeavyRow>(q.o_heavy), q.nchunks,
                                                  q.at<uint32_t>(q.o_chunk), q.rpts_C, q.A.rpts,
                                                  q.at<uint32_t>(q.o_whist), q.at<uint32_t>(q.o_whist) + q.nchunks,
                                                  q.at<WinItem>(q.o_items), q.items_cap, q.wh, s);
                        }),
                  "windows");
        }
        HIPCK(hipMemcpyAsync(&q.hw, q.wh, sizeof(WsHdr), hipMemcpyDeviceToHost, s), "symbolic readback");
    }
    HIPCK(hipStreamSynchronize(s), "symbolic sync");
    int bad = 0;
    for (int p = 0; p < pl->nprod; ++p) {
        Prod &q = pl->prods[p];
        if (q.hw.err) bad = 1;
        nnz_C[p] = (int64_t)q.hw.nnz_c;
        int64_t acc = 0;
        for (int b = 0; b < NNB; ++b) {
            q.num_off[b] = acc;
            if (b > 0 && b != NUM_HEAVY_BIN) acc += (int64_t)q.hw.num_rows[b];
        }
        BinOffsets off{};
        for (int b = 0; b < NNB; ++b) off.v[b] = q.num_off[b];
        HIPCK(timed(pl, "num_scatter", 8.0 * q.m,
                    [&] {
                        return launch_num_scatter((int)q.m, q.at<int32_t>(q.o_nnz), q.flop, q.A.rpts, q.rpts_C,
                                                  off, q.at<NumRow>(q.o_rows_num), q.wh, pl->lim, s);
                    }),
              "num_scatter");
    }
    if (bad) return SPGEMM_ERR_INTERNAL;
    pl->state = SYMBOLIC_DONE;
    return SPGEMM_OK;
}

int spgemm_symbolic_static(spgemm_plan_t pl, int64_t *const *rpts_C, int64_t *nnz_C) {
    if (!pl || !rpts_C || !nnz_C) return SPGEMM_ERR_INVALID_ARG;
    if (pl->state < PLANNED) return SPGEMM_ERR_STATE;
    if (pl->ws_total > (size_t)SPGEMM_STATIC_WS_BYTES) return SPGEMM_ERR_STATIC_LIMIT;
    int cur = 0, sdev = 0;
    HIPCK(hipGetDevice(&cur), "hipGetDevice");
    HIPCK(hipStreamGetDevice(pl->stream, &sdev), "hipStreamGetDevice");
    if (cur != sdev) return SPGEMM_ERR_INVALID_ARG;
    void *ws = nullptr;
    const int st = static_workspace(cur, &ws);
    if (st != SPGEMM_OK) return st;
    return spgemm_symbolic(pl, ws, rpts_C, nnz_C);
}

int spgemm_numeric(spgemm_plan_t pl, const spgemm_csr *A, const spgemm_csr *B, int32_t *const *cols_C,
                   void *const *vals_C) {
    if (!pl || !A || !B || !cols_C || !vals_C) return SPGEMM_ERR_INVALID_ARG;
    if (pl->state < SYMBOLIC_DONE) return SPGEMM_ERR_STATE;
    hipStream_t s = pl->stream;
    const bool sorted = (pl->flags & SPGEMM_SORTED) != 0;
    for (int p = 0; p < pl->nprod; ++p) {
        Prod &q = pl->prods[p];
        if (A[p].rpts != q.A.rpts || A[p].cols != q.A.cols || B[p].rpts != q.B.rpts || B[p].cols != q.B.cols ||
            A[p].nnz != q.A.nnz || B[p].nnz != q.B.nnz)
            return SPGEMM_ERR_STATE;
        if ((A[p].nnz > 0 && !A[p].vals) || (B[p].nnz > 0 && !B[p].vals)) return SPGEMM_ERR_INVALID_ARG;
        if (q.hw.nnz_c > 0 && (!cols_C[p] || !vals_C[p])) return SPGEMM_ERR_INVALID_ARG;
    }
    for (int p = 0; p < pl->nprod; ++p) {
        Prod &q = pl->prods[p];
        q.A.vals = A[p].vals;
        q.B.vals = B[p].vals;
        const unsigned nitems = q.hw.n_items;
        // claim counters of the windows and of the persistent hash bins (the
        // bins of 512 threads and up: the rule of num_hash_l, which launches
        // them as persistent grids that claim rows)
        bool claims = nitems > 0;
        for (int b = 1; b < NUM_HEAVY_BIN; ++b) claims |= NUM_G[b] >= 512 && q.hw.num_rows[b] > 0;
        if (claims) HIPCK(launch_num_reset(q.wh, s), "num_reset");
        if (nitems > 0) {
            HIPCK(timed(pl, "gather_B_vals", 20.0 * q.B.nnz,
                        [&] {
                            return launch_gather_vals(pl->dtype, q.B.nnz, q.at<int32_t>(q.o_bperm), q.B.vals,
                                                      q.at<void>(q.o_bv), s);
                        }),
                  "gather_B_vals");
        }
        const NumRow *rows = q.at<NumRow>(q.o_rows_num);
        for (int b = NUM_HEAVY_BIN - 1; b >= 1; --b) {
            const unsigned nr = (unsigned)q.hw.num_rows[b];
            if (nr == 0) continue;
            char name[32];
            snprintf(name, sizeof(name), "num_hash_%d", NUM_T[b]);
            const double bytes = 28.0 * nr + 20.0 * q.hw.num_nnza[b] + 12.0 * q.hw.num_flop[b] +
                                 12.0 * q.hw.num_nnzc[b];
            HIPCK(timed(pl, name, bytes,
                        [&] {
                            return launch_num_bin(b, pl->dtype, sorted, nr, rows, q.num_off[b], q.A, q.B,
                                                  cols_C[p], vals_C[p], q.wh,
                                                  HashCfg{pl->lim.hmul, pl->lim.bq, pl->count_probes, (uint32_t)b},
                                                  pl->ncu, s);
                        }),
                  "num_hash");
        }
        if (q.hw.num_rows[NUM_HEAP_BIN] > 0) {
            const int hb = NUM_HEAP_BIN;
            const unsigned nr = (unsigned)q.hw.num_rows[hb];
            const double bytes = 28.0 * nr + 20.0 * q.hw.num_nnza[hb] + 12.0 * q.hw.num_flop[hb] +
                                 12.0 * q.hw.num_nnzc[hb];
            HIPCK(timed(pl, "num_heap", bytes,
                        [&] {
                            return launch_num_heap(pl->dtype, nr, rows, q.num_off[hb], q.A, q.B, cols_C[p],
                                                   vals_C[p], q.wh, s);
                        }),
                  "num_heap");
        }
        if (nitems > 0) {
            const int hb = NUM_HEAVY_BIN;
            const double bytes = 24.0 * nitems + 8.0 * q.hw.num_rows[hb] + 20.0 * q.hw.num_nnza[hb] +
                                 12.0 * q.hw.num_flop[hb] + 12.0 * q.hw.num_nnzc[hb];
            HIPCK(timed(pl, "num_window", bytes,
                        [&] {
                            return launch_num_window(pl->dtype, q.hw.n_items, q.at<WinItem>(q.o_items), q.A,
                                                     q.at<int2>(q.o_ki), q.at<int32_t>(q.o_idx), q.nchunks,
                                                     q.at<int32_t>(q.o_bc), q.at<void>(q.o_bv), cols_C[p],
                                                     vals_C[p], q.store_bm ? q.at<uint32_t>(q.o_bmap) : nullptr,
                                                     q.wh, pl->ncu, s);
                        }),
                  "num_window");
        }
    }
    return SPGEMM_OK;
}

int spgemm_free(spgemm_plan_t pl) {
    if (!pl) return SPGEMM_OK;
    for (auto &t : pl->tl) {
        (void)hipEventDestroy(t.e0);
        (void)hipEventDestroy(t.e1);
    }
    delete pl;
    return SPGEMM_OK;
}

int spgemm_plan_stats(spgemm_plan_t pl, int iprod, spgemm_stats *out) {
    if (!pl || !out || iprod < 0 || iprod >= pl->nprod) return SPGEMM_ERR_INVALID_ARG;
    Prod &q = pl->prods[iprod];
    memset(out, 0, sizeof(*out));
    out->flop = (int64_t)q.h.total_flop;
    out->max_row_flop = (int64_t)q.h.max_flop;
    for (int b = 1; b <= 9; ++b) out->sym_flop[b - 1] = (int64_t)q.h.sym_flop[b];
    if (pl->state >= SYMBOLIC_DONE) {
        WsHdr now{};
        HIPCK(hipMemcpyAsync(&now, q.wh, sizeof(WsHdr), hipMemcpyDeviceToHost, pl->stream), "stats readback");
        HIPCK(hipStreamSynchronize(pl->stream), "stats sync");
        out->nnz_C = (int64_t)now.nnz_c;
        out->heavy_rows = (int64_t)now.n_heavy;
        out->windows = (int64_t)now.n_items;
        out->probe_overflow = (int64_t)now.probe_overflow;
        out->heap_rows = (int64_t)now.num_rows[NUM_HEAP_BIN];
        for (int b = 1; b <= 9; ++b) {
            out->num_flop[b - 1] = (int64_t)now.num_flop[b];
            out->num_probes[b - 1] = (int64_t)now.num_probes[b];
            out->sym_probes[b - 1] = (int64_t)now.sym_probes[b];
        }
        if (now.err & ~ERR_PROBE) return SPGEMM_ERR_INTERNAL;
        if (now.probe_overflow) return SPGEMM_ERR_INTERNAL;
    }
    return SPGEMM_OK;
}

int spgemm_plan_set_timing(spgemm_plan_t pl, int enable) {
    if (!pl) return SPGEMM_ERR_INVALID_ARG;
    pl->timing = enable != 0;
    return SPGEMM_OK;
}

int spgemm_plan_kernel_times(spgemm_plan_t pl, spgemm_kernel_time *out, int cap) {
    if (!pl || (!out && cap > 0) || cap < 0) return SPGEMM_ERR_INVALID_ARG;
    std::vector<spgemm_kernel_time> agg;
    for (auto &t : pl->tl) {
        HIPCK(hipEventSynchronize(t.e1), "event sync");
        float ms = 0.f;
        HIPCK(hipEventElapsedTime(&ms, t.e0, t.e1), "event elapsed");
        auto it = std::find_if(agg.begin(), agg.end(),
                               [&](const spgemm_kernel_time &k) { return t.name == k.name; });
        if (it == agg.end()) {
            spgemm_kernel_time k{};
            snprintf(k.name, sizeof(k.name), "%s", t.name.c_str());
            agg.push_back(k);
            it = agg.end() - 1;
        }
        it->ms += ms;
        it->launches += 1;
        it->alg_bytes += t.bytes;
    }
    for (auto &t : pl->tl) {
        (void)hipEventDestroy(t.e0);
        (void)hipEventDestroy(t.e1);
    }
    pl->tl.clear();
    const int n = (int)std::min<size_t>(agg.size(), (size_t)cap);
    for (int i = 0; i < n; ++i) out[i] = agg[i];
    return n;
}

int spgemm_masked_sum_i64(int64_t nrows, int64_t ncols, const int64_t *rpts_C, const int32_t *cols_C,
                          const int64_t *vals_C, const spgemm_csr *M, int64_t *out, hipStream_t stream) {
    if (!M || !out || !rpts_C || nrows < 0 || ncols < 0) return SPGEMM_ERR_INVALID_ARG;
    if (!csr_ok(*M)) return SPGEMM_ERR_INVALID_ARG;
    if (M->nrows != nrows || M->ncols != ncols) return SPGEMM_ERR_SHAPE;
    if (nrows >= INT32_MAX) return SPGEMM_ERR_OVERFLOW;
    HIPCK(launch_masked_sum(nrows, ncols, rpts_C, cols_C, vals_C, dev(*M), out, stream), "masked_sum");
    return SPGEMM_OK;
}

// compute units of the current device (256 when the runtime cannot say)
static int current_ncu() {
    int devid = 0, n = 0;
    if (hipGetDevice(&devid) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, devid) == hipSuccess && n > 0)
        return n;
    return 256;
}

int spgemm_masked_product_sum_i64(const spgemm_csr *A, const spgemm_csr *B, const spgemm_csr *M, void *workspace,
                                  int64_t *out, hipStream_t stream) {
    if (!A || !B || !M || !workspace || !out) return SPGEMM_ERR_INVALID_ARG;
    if (!csr_ok(*A) || !csr_ok(*B) || !csr_ok(*M)) return SPGEMM_ERR_INVALID_ARG;
    if (A->ncols != B->nrows || M->nrows != A->nrows || M->ncols != B->ncols) return SPGEMM_ERR_SHAPE;
    const bool ones = !A->vals || !B->vals;
    HIPCK(launch_masked_product(dev(*A), dev(*B), dev(*M), ones, (unsigned *)workspace, out, current_ncu(), stream),
          "masked_product");
    return SPGEMM_OK;
}

int spgemm_stream_copy(void *dst, const void *src, size_t nbytes, hipStream_t stream) {
    if ((nbytes % 16) != 0 || (nbytes > 0 && (!dst || !src))) return SPGEMM_ERR_INVALID_ARG;
    HIPCK(launch_stream_copy(dst, src, nbytes, stream), "stream_copy");
    return SPGEMM_OK;
}

int spgemm_stanza_read(const void *base, size_t nbytes, const int64_t *start, int64_t nstanza, int log2_words,
                       unsigned long long *sum, unsigned long long *skipped, hipStream_t stream) {
    if (!base || nbytes < 8 || (nbytes % 8) != 0 || !sum || !skipped) return SPGEMM_ERR_INVALID_ARG;
    if (log2_words < 0 || log2_words > SPGEMM_STANZA_MAX_LOG2 || nstanza < 0 || (nstanza > 0 && !start))
        return SPGEMM_ERR_INVALID_ARG;
    if (nstanza > (INT64_MAX >> SPGEMM_STANZA_MAX_LOG2)) return SPGEMM_ERR_OVERFLOW;
    HIPCK(launch_stanza_read(base, (int64_t)(nbytes / 8), start, nstanza, log2_words, sum, skipped, current_ncu(),
                             stream),
          "stanza_read");
    return SPGEMM_OK;
}

}  // extern "C"
