// Tunables and shared layouts of the gfx950 SpGEMM library (host and device).
#pragma once
#include <stdint.h>

namespace spg {

// ---- heavy rows: column windows --------------------------------------------
// Rows whose output does not fit one LDS table (more than WIN_CAP entries)
// are accumulated window by window; a window is a run of whole 4096-column
// chunks whose LDS footprint (below) fits RANK_BUDGET words, which bounds it
// at about 11.6 K output entries.  WIN_TABLE is the largest numeric hash
// table (bin 9), sized for WIN_CAP entries at a load of at most 0.75.
constexpr int CHUNK_SHIFT = 12;
constexpr int CHUNK_COLS = 1 << CHUNK_SHIFT;
constexpr int WIN_TABLE = 11264;   // 132 KB of keys+values for 8-byte values
constexpr int WIN_CAP = 8448;      // load factor <= 0.75
// A column window of a heavy row holds, in LDS, one 64-bit word per 32
// columns (occupancy bits + exclusive rank prefix), one value per output
// entry and a 4-byte staging slot per entry: 128 words per chunk plus 1.5
// words per entry must fit RANK_BUDGET words.  Windows are worked on by
// blocks of WIN_G threads, one per CU (the LDS of two blocks of 512 threads
// with half the budget each measured 3 % slower at R-MAT scale 20: twice the
// windows, and more rows above the block's resident A entries).
constexpr int WORDS_PER_CHUNK = CHUNK_COLS / 32;
constexpr int WIN_G = 1024;
constexpr int RANK_BUDGET = 17664;
constexpr int MAX_CHUNKS = 32768;  // heavy-row support: ncols <= 2^27
// B rows longer than SHORT_ROW get a chunk-offset index (slice of a window =
// two loads); shorter rows are read whole and filtered by column.
constexpr int SHORT_ROW = 16;

// Symbolic phase of rows whose flop exceeds WIN_CAP: one bit per column of
// C in LDS; wider matrices are swept in passes of BM_WORDS*32 columns.
constexpr int BM_WORDS_SMALL = 2048;    //   8 KB:    65,536 columns
constexpr int BM_WORDS_MID = 8192;      //  32 KB:   262,144 columns
constexpr int BM_WORDS_LARGE = 36864;   // 144 KB: 1,179,648 columns

// ---- bins -------------------------------------------------------------------
// Symbolic bins by x = min(row flop, ncols): bin 0 = empty row, bins 1..9 LDS
// hash tables of T >= 2x keys, bin 10 = bitmap.  Blocks stay narrow up to the
// 512-slot tables (one wave per row): the rows there are latency-bound chains
// of dependent loads, and narrower blocks keep more rows in flight per CU
// (ER 2^20, 256 products per row: 6.7 -> 4.9 ms against 128-thread blocks).
// The same holds up to the 8192-slot table, whose 512-thread blocks fit four
// rows per CU in LDS (R-MAT scale 20: 0.93 -> 0.71 ms against 1024 threads;
// 4096 slots with 256 threads 0.37 -> 0.25 ms, 2048 slots with 128 threads
// 0.20 -> 0.16 ms); the 16384-slot table keeps two 1024-thread rows per CU.
constexpr int NSB = 11;
constexpr int SYM_BITMAP_BIN = 10;
constexpr int SYM_G[NSB] = {0, 64, 64, 64, 64, 128, 128, 256, 512, 1024, 1024};
constexpr int SYM_T[NSB] = {0, 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384, 0};
constexpr int64_t SYM_XMAX[NSB] = {0, 32, 64, 128, 256, 512, 1024, 2048, 4096, WIN_CAP, INT64_MAX};

// Numeric bins by exact nnz(c_i): bin 0 = empty row, bins 1..9 LDS hash
// tables of keys+values, bin 10 = heavy (column windows), bin 11 = heap merge
// (only when a plan asks for it: rows of bins 1..9 with at most HEAP_MAX_A
// entries of A and at most HEAP_FCAP products).
constexpr int NNB = 12;
constexpr int NUM_HEAVY_BIN = 10;
constexpr int NUM_HEAP_BIN = 11;
constexpr int HEAP_MAX_A = 256;
constexpr int HEAP_FCAP = 1024;
constexpr int NUM_G[NNB] = {0, 64, 64, 64, 64, 128, 256, 512, 1024, 1024, 1024, 64};
constexpr int NUM_T[NNB] = {0, 64, 128, 256, 512, 1024, 2048, 4096, 8192, WIN_TABLE, WIN_TABLE, 0};
constexpr int64_t NUM_XMAX[NNB] = {0, 32, 64, 128, 256, 512, 1024, 2048, 4096, WIN_CAP, INT64_MAX, 0};

// Bin limits of one plan (tunable; see spgemm_config): bin b of the symbolic
// phase takes rows with sym[b-1] < min(flop, ncols) <= sym[b], bin b of the
// numeric phase rows with num[b-1] < nnz(c_i) <= num[b].  A limit never
// exceeds its bin's table size (so a probe always finds room); bin 9 ends at
// WIN_CAP in both phases (the heavy-row boundary is structural).  hmul is
// the odd multiplier of the column hash, bq the 4-slot quads per bucket of
// the LDS tables (1: 4-slot buckets; 2 or 4: the wider chunks of the
// paper's HashVector, Section 4.2.2); heap = 1 sends the numeric phase of the
// rows in the heap envelope to the heap merge (Section 4.2.3).
constexpr uint32_t HASH_MUL_DEFAULT = 2654435761u;
struct BinLimits {
    int64_t sym[NSB];
    int64_t num[NNB];
    uint32_t hmul;
    uint32_t bq;
    uint32_t heap;
};

// What a hash kernel needs of the configuration.
struct HashCfg {
    uint32_t mul;   // odd multiplier of the column hash
    uint32_t bq;    // 4-slot quads per bucket: 1, 2 or 4
    uint32_t count; // 1: add the bucket reads of every insert to the bin's probe counter
    uint32_t bin;   // the kernel's bin (index of that counter)
};

__host__ __device__ inline BinLimits default_limits() {
    BinLimits L{};
    for (int b = 0; b < NSB; ++b) L.sym[b] = SYM_XMAX[b];
    for (int b = 0; b < NNB; ++b) L.num[b] = NUM_XMAX[b];
    L.hmul = HASH_MUL_DEFAULT;
    L.bq = 1;
    L.heap = 0;
    return L;
}

__host__ __device__ inline int sym_bin_l(uint64_t flop, int64_t ncols, const BinLimits &L) {
    uint64_t x = flop < (uint64_t)ncols ? flop : (uint64_t)ncols;
    if (x == 0) return 0;
    for (int b = 1; b < SYM_BITMAP_BIN; ++b)
        if (x <= (uint64_t)L.sym[b]) return b;
    return SYM_BITMAP_BIN;
}

__host__ __device__ inline int num_bin_l(int64_t nnz, const BinLimits &L) {
    if (nnz <= 0) return 0;
    for (int b = 1; b < NUM_HEAVY_BIN; ++b)
        if (nnz <= L.num[b]) return b;
    return NUM_HEAVY_BIN;
}

// Numeric bin of a row with nnz(c_i) = nnz, row flop and na entries of A.
__host__ __device__ inline int num_bin_row(int64_t nnz, uint64_t flop, int na, const BinLimits &L) {
    const int b = num_bin_l(nnz, L);
    if (L.heap && b >= 1 && b < NUM_HEAVY_BIN && na <= HEAP_MAX_A && flop <= (uint64_t)HEAP_FCAP)
        return NUM_HEAP_BIN;
    return b;
}

__host__ __device__ inline int sym_bin(uint64_t flop, int64_t ncols) {
    uint64_t x = flop < (uint64_t)ncols ? flop : (uint64_t)ncols;
    if (x == 0) return 0;
    for (int b = 1; b < SYM_BITMAP_BIN; ++b)
        if (x <= (uint64_t)SYM_XMAX[b]) return b;
    return SYM_BITMAP_BIN;
}

// Products per lane per enumeration batch of a hash bin: about the bin's
// largest row per thread, as a power of two <= 8.
__host__ __device__ constexpr int u_for(int G, int64_t xmax) {
    return xmax <= G ? 1 : (xmax <= 2 * (int64_t)G ? 2 : (xmax <= 4 * (int64_t)G ? 4 : 8));
}

__host__ __device__ inline int num_bin(int64_t nnz) {
    if (nnz <= 0) return 0;
    for (int b = 1; b < NUM_HEAVY_BIN; ++b)
        if (nnz <= NUM_XMAX[b]) return b;
    return NUM_HEAVY_BIN;
}

// ---- device-side headers (counters the host reads back) ----------------------
enum : int {
    ERR_PROBE = 1,       // a hash probe sequence ran past the table size
    ERR_COUNT = 2,       // numeric row count differs from the symbolic count
    ERR_ITEMS = 4,       // window item list capacity exceeded
    ERR_CSR = 8,         // malformed CSR (validate mode)
    ERR_CHUNK = 16,      // a heavy row has a chunk wider than a window
    ERR_UNSORTED_B = 32  // a row of B is not in ascending column order
};

struct PlanHdr {
    unsigned long long total_flop;
    unsigned long long max_flop;
    unsigned long long n_long_b;   // rows of B longer than SHORT_ROW
    unsigned long long sym_rows[NSB];
    unsigned long long sym_flop[NSB];
    unsigned long long sym_nnza[NSB];
    int err;
    unsigned n_huge;               // rows of A longer than FLOP_WAVE_ROW (listed for k_huge_flop)
    unsigned n_long_a;             // rows of A of FLOP_SHORT_ROW+1 .. FLOP_WAVE_ROW entries (k_long_flop)
    int pad_[5];
};

// Row flop: a row of A with at most FLOP_SHORT_ROW entries is summed by one
// thread in the pass over all rows; longer rows are listed in the plan
// scratch and summed after it, a wave per row up to FLOP_WAVE_ROW entries
// (at most min(m, nnz(A) / (FLOP_SHORT_ROW + 1)) rows) and a block per row
// beyond (at most nnz(A) / (FLOP_WAVE_ROW + 1) rows).
constexpr int FLOP_SHORT_ROW = 32;
constexpr int FLOP_WAVE_ROW = 4096;

struct WsHdr {
    unsigned long long nnz_c;
    unsigned long long num_rows[NNB];
    unsigned long long num_flop[NNB];
    unsigned long long num_nnza[NNB];
    unsigned long long num_nnzc[NNB];
    unsigned int sym_cursor[NSB];
    unsigned int num_cursor[NNB];
    unsigned int n_heavy;
    unsigned int n_items;
    unsigned int n_long;
    int err;
    unsigned int probe_overflow;
    unsigned int n_groups;
    unsigned int bm_next;       // row claim counter of the bitmap bin (k_sym_bitmap)
    unsigned int pad2_;
    unsigned int win_next[8];   // window claim counters, one per XCD group
    unsigned long long sym_probes[NSB];   // bucket reads of the hash inserts (SPGEMM_PROBE_COUNT)
    unsigned long long num_probes[NNB];
    // row claim counters of the persistent hash bins, per bin: the symbolic
    // ones start at zero with the header, the numeric ones are reset at the
    // start of every numeric phase (k_num_reset)
    unsigned int sym_next[NSB];
    unsigned int num_next[NNB];
};

// One column window of one heavy row.
struct WinItem {
    int32_t row;
    int32_t ch_lo;      // first chunk (inclusive)
    int32_t ch_hi;      // last chunk (exclusive)
    int32_t count;      // output entries in the window (from the symbolic bitmap)
    int64_t out_pos;    // absolute position in cols_C / vals_C
    int32_t a0, a1;     // the row's entries of A: [a0, a1)
    int32_t slot;       // the row's index within the bitmap bin
    int32_t pad;
};

// Stored symbolic bitmaps of the bitmap-bin rows (one bit per column of C,
// whole chunks per row) are kept when they take at most this many bytes.
constexpr unsigned long long BM_STORE_MAX = 64ull << 30;

// A row of a numeric hash or heap bin list: its entries of A [a0, a1), and
// out_n = (position of the row in C) << 16 | nnz(c_i) (those bins hold rows
// of at most WIN_CAP < 2^16 entries).
struct alignas(16) NumRow {
    int32_t a0, a1;
    uint64_t out_n;
};
static_assert(WIN_CAP < (1 << 16), "nnz(c_i) of a listed row fits 16 bits");

struct HeavyRow {
    int32_t row;
    int32_t slot;       // index of the row within the bitmap bin (chunk-count slot)
};



constexpr int PLAN_HDR_BYTES = 512;
constexpr int WS_HDR_BYTES = 1024;
static_assert(sizeof(PlanHdr) <= PLAN_HDR_BYTES, "plan header");
static_assert(sizeof(WsHdr) <= WS_HDR_BYTES, "ws header");

}  // namespace spg
