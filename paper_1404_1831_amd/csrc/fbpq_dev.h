// Internal definitions shared by the HIP kernels and the host side of libfbpq.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct fbpq_index;

namespace fbpq {

constexpr int kWave = 64;
constexpr int kKc = 256;
constexpr int kMaxPrefix = 16384;     // longest sorted half list the traversal tracks (row and column LUT slots,
                                      // fewer than 2 * kMaxPrefix, pack into the 16-bit halves of an int32)
constexpr int kMaxFastPrefix = 4096;  // longest one the LDS-resident traversal and layouts hold
constexpr int kMaxPopPrefix = 2048;  // longest one the one-cell-at-a-time traversal holds
constexpr int kMaxK = 1024;

// Per-query traversal status written by the traversal kernel.
// kStDefer: the one-cell-at-a-time kernel used up its pop budget and leaves
// the query to the threshold-stepping kernel (never seen by the host).
enum : int32_t { kStOk = 0, kStNeedPrefix = 1, kStNeedCells = 2, kStDefer = 3 };

// Per-query traversal summary (one record per workspace slot).
struct TravHdr {
    int32_t status;
    int32_t A;        // rows of the visited diagram (ranks a with w[a] > 0)
    int32_t B;        // columns (= w[0])
    int32_t cut_a;    // rank pair of the last visited cell
    int32_t cut_b;
    int32_t nne;      // nonempty visited cells (set by the layout kernel)
    int32_t a_ne;     // rows holding a nonempty cell (layout kernel)
    int32_t b_ne;     // columns holding a nonempty cell (layout kernel)
    int32_t n_items;  // blocks of kItem candidates (0: scanned by a two-pass kernel)
    int32_t gscan;    // 1: two-pass scan with partial sums in HBM (many candidates in sparse cells)
    int64_t ncells;   // visited cells (= sum of w)
    int64_t ncand;    // candidates (= min(L, N))
    int64_t cut_take; // points taken from the last visited cell
};

// Path counters (slots of FBPQ_STAT_*), incremented when the pointer is set.
constexpr int kStatCellScan = 0, kStatFused = 1, kStatTwoPass = 2, kStatPrefixWave = 3, kStatPrefixWG = 4;
constexpr int kStatWide = 7, kStatWideBands = 8, kStatWideEvals = 9, kStatWideLoads = 10;
constexpr int kStatCandCell = 11, kStatCandTwoPass = 12, kStatCandWide = 13;  // candidates each scan scored
constexpr int kStatFusedRescan = 14, kStatWinAdmitted = 15, kStatWinLost = 16;
constexpr int kNumStatSlots = 20;

// Candidate block of the cell scan: up to kItem candidates of one nonempty cell.
constexpr int kItem = 2048;
constexpr int kItemMinAvg = 128;   // mean points per nonempty cell for the item scan
constexpr int kWideChunk = 2048;   // candidates of one task of the HBM two-pass scan
constexpr int kScanWideMin = 8192; // candidates above which a query with sparse cells (fewer than
                                   // kItemMinAvg points per nonempty cell) keeps its sums in HBM

// Device view of an index and its tables.
struct DevIndex {
    int32_t D, T, M, Kc;
    int64_t N;
    const float *C1, *C2, *R;
    const int64_t *offsets;
    const uint8_t *codesA;  // [N][M/2] bytes of subspaces 0..M/2-1
    const uint8_t *codesB;  // [N][M/2] bytes of subspaces M/2..M-1
    const uint32_t *ids;
    const float *CR1, *CR2, *nR, *nC1, *nC2;  // CR1/CR2 hold CQ1/CQ2 with local codebooks
    float cmax1, cmax2;  // largest squared half-centroid norm of each half
    const float *QL, *SL;  // local codebooks [T][M/2][Kc][D/M] (HBPQ), or null
    const float *Rot;      // OPQ rotation [D][D] row-major, or null
    int32_t local;         // 1: local codebooks
    int32_t od;            // 1: candidates scored by explicit O(D) reconstruction (Multi-D-ADC baseline)
    // Half-centroids scaled by csc (a power of two) and split into two FP16
    // parts, hi = fp16(c csc) and lo = fp16(c csc - hi), row c at [c][2 D/2]
    // (hi then lo); null when the approximate keys use FP32 products only.
    const _Float16 *Cs1, *Cs2;
    float csc1, csc2;
    // e(q) = ecoef 2^-23 (||q_h|| + max ||c||)^2 bounds the error of every
    // approximate key (FP32 products, or the split FP16 ones)
    float ecoef;
};

// Launchers (each defined next to its kernel).
hipError_t launch_tables(const DevIndex &ix, float *CR1, float *CR2, float *nR, float *nC1,
                         float *nC2, hipStream_t st);

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st);
// Device budgets L[n], k[n] into Lo, ko clamped to [1, L_max], [1, k_max]; *nclamped counts the changed entries.
hipError_t launch_sanitize(const int64_t *L, const int32_t *k, int64_t n, int64_t L_max, int32_t k_max, int64_t *Lo,
                           int32_t *ko, int32_t *nclamped, hipStream_t st);
hipError_t launch_copy_i32(const int32_t *src, int32_t *dst, hipStream_t st);  // *dst = *src on the stream

// out[c][0, h) = fp16(C[c] scale), out[c][h, 2h) = fp16(C[c] scale - hi) for T rows of h floats
hipError_t launch_split_centroids(const float *C, int64_t T, int h, float scale, _Float16 *out, hipStream_t st);

hipError_t launch_split_codes(const uint8_t *src, int64_t n, int M, uint8_t *a, uint8_t *b,
                              hipStream_t st);

// Approximate half keys ||q||^2 + ||c||^2 - 2 <q, c> into ka [slot][2][T]
// (slot s holds query qlist[s], or s when qlist is null).
// q' = Rot q for nq queries of dimension D (OPQ), FP64 chains rounded to FP32
hipError_t launch_rotate(const float *q, int64_t nq, int D, const float *Rot, float *out, hipStream_t st);
// kmin (optional) [slot][2][ceil(T/16)]: the smallest approximate key of each
// block of 16 consecutive centroids.
hipError_t launch_half_approx(const DevIndex &ix, const float *q, const int32_t *qlist, int64_t nslots,
                              float *ka, float *kmin, hipStream_t st);

constexpr int kWaveS = 512;  // survivors a wavefront select ranks

// Sorted prefix of each half list from the key array ka [slot][2][T]. The
// wave select handles the (slot, half) pairs it can and records in pstat
// [nslots][2] (0 done, 1 left over) which remain; the workgroup kernel then
// takes the pairs left over (every pair when pstat is null), from ka, or by
// an exact radix select alone when ka is null.
bool prefix_wave_ok(const DevIndex &ix, int32_t P);
// The wave select can take its samples from the block minima (and read only
// the blocks that can hold survivors) at this geometry.
bool prefix_blocks_ok(const DevIndex &ix, int32_t P);
hipError_t launch_prefix_wave(const DevIndex &ix, const float *q, const float *ka, const float *kmin,
                              int64_t nslots, const int32_t *qlist, int32_t P, double *lkey, int32_t *lidx,
                              int32_t *pstat, unsigned long long *stats, hipStream_t st);
hipError_t launch_prefix_block(const DevIndex &ix, const float *q, const float *ka, int64_t nslots,
                               const int32_t *qlist, int32_t P, double *lkey, int32_t *lidx,
                               const int32_t *pstat, unsigned long long *stats, unsigned char *gsort,
                               hipStream_t st);
// Bytes per (slot, half) of the HBM sort buffer gsort that the workgroup
// select needs at prefix length P (0: its sort buffer fits in LDS).
size_t prefix_sort_bytes(const DevIndex &ix, int32_t P);

struct TravArgs {
    DevIndex ix;
    const double *lkey;    // [slot][2][P]
    const int32_t *lidx;   // [slot][2][P]
    int32_t P;
    const int32_t *qlist;  // slot -> query (null: identity)
    const int64_t *L;      // [query]
    int64_t max_cells;
    TravHdr *hdr;          // [slot]
    int32_t *w;            // [slot][P] final row widths
    int32_t *fail_count;   // number of slots whose status is not kStOk
    int32_t *fail_list;    // their query ids
    int32_t *dbg_ab;       // optional [slot][max_cells][2] visited (a, b) in order
    int64_t *dbg_take;     // optional [slot][max_cells] points taken
    int64_t *dbg_beg;      // optional [slot][max_cells] storage begin of the cell
    int32_t pop_budget;    // pops before a query is left to the threshold kernel (0: none)
    int32_t wide_all;      // threshold kernel: take every slot, not only deferred ones
    unsigned long long *stats;  // optional path counters
    int32_t *big;          // long prefixes: [slot][big_trav_ints(P)] per-row state in HBM
};
hipError_t launch_traverse(const TravArgs &a, int64_t nslots, hipStream_t st);
hipError_t launch_traverse_wide(const TravArgs &a, int64_t nslots, hipStream_t st);
size_t wide_lds_bytes(int P);
// Traversal for prefixes longer than kMaxFastPrefix: the same visited cells
// and cut, with its per-row state in HBM (args.big).
hipError_t launch_traverse_big(const TravArgs &a, int64_t nslots, hipStream_t st);
__host__ __device__ inline int64_t big_trav_ints(int P) { return 4 * (int64_t)P + 4; }

struct LayoutArgs {
    DevIndex ix;
    const double *lkey;    // [slot][2][P]
    const int32_t *lidx;   // [slot][2][P]
    int32_t P;
    TravHdr *hdr;
    const int32_t *w;      // [slot][P]
    int64_t max_cells;
    int32_t *row_ne;       // [slot][P+1] first compacted cell of each row
    int32_t *row_cand;     // [slot][P+1] first candidate of each row
    int32_t *col_ne;       // [slot][P+1] first column-list entry of each column
    int32_t *col_tot;      // [slot][P] candidates in each column
    int32_t *ne_cs;        // [slot][max_cells] first candidate of each nonempty cell
    int32_t *ne_cnt;       // points taken
    int64_t *ne_beg;       // storage begin
    float *ne_cst;         // fl32(d1[i] + d2[j])
    int32_t *cm_cell;      // [slot][max_cells] column lists: compacted cell index
    int32_t *cm_pre;       // candidates before it in its column
    int32_t *ne_slot;      // [slot][max_cells] LUT slots of the cell: row slot | (col slot << 16)
    int32_t *slot_ij;      // [slot][2P] centroid of each LUT slot: rows, then columns
    int32_t allow_items;   // 0: every query goes to the two-pass scan
    unsigned char *gscr;   // long prefixes: [slot][layout_rank_bytes(P)] per-rank arrays in HBM, else null (LDS)
};
// Bytes of the layouts' per-rank arrays (column cursors, row and column
// starts, LUT slots) at prefix length P, rounded to 16.
__host__ __device__ inline size_t layout_rank_bytes(int P)
{
    return (((size_t)P * 8 + (size_t)3 * (P + 1) * 4 + (size_t)2 * P * 4) + 15) & ~(size_t)15;
}
hipError_t launch_layout(const LayoutArgs &a, int64_t nslots, hipStream_t st);
hipError_t launch_layout_wide(const LayoutArgs &a, int64_t nslots, hipStream_t st);
constexpr int64_t kLayoutWaveMax = 4096;  // visited cells above which the workgroup layout runs

struct ScanArgs {
    DevIndex ix;
    const float *q;        // [query][D]
    const int32_t *qlist;
    const int32_t *k;      // [query]
    int32_t k_max;         // output row stride
    const int32_t *lidx;
    int32_t P;
    const TravHdr *hdr;
    int64_t max_cells;
    const int32_t *row_ne, *row_cand, *col_ne, *col_tot;
    const int32_t *ne_cs, *ne_cnt;
    const int64_t *ne_beg;
    const float *ne_cst;
    const int32_t *cm_cell, *cm_pre;
    const int32_t *ne_slot, *slot_ij;
    int32_t chunk;         // candidates per LDS chunk
    const float *lq;       // [slot][M][Kc] query tables (wide scan)
    float *dist;           // [slot][lcap] partial and final distances (wide scan)
    int64_t lcap;
    int32_t *sel_done;     // [slot] 1: the wide scan selected the top-k itself
    int32_t od_group;      // O(D) scan: subspaces whose codebooks are staged per group (set by the launcher)
    int64_t *out_ids;      // [query][k_max]
    float *out_d;
    int64_t *dbg_pos;      // optional [slot][dbg_cap]
    float *dbg_d;
    int64_t dbg_cap;
    unsigned long long *stats;  // optional path counters
};
hipError_t launch_scan(const ScanArgs &a, int64_t nslots, hipStream_t st);
hipError_t launch_scan_wide(const ScanArgs &a, int64_t nslots, hipStream_t st);
// reads the static LDS of every k_scan_wide form for M subspaces (once per process)
void scan_wide_prepare(int M);

size_t scan_lds_bytes(int D, int M, int chunk, int k_max, int P);
constexpr int kScanCellsLds = 256;  // nonempty cells whose tables the scan keeps in LDS

struct ItemArgs {
    DevIndex ix;
    const float *q;        // [query][D]
    const int32_t *qlist;
    const int32_t *k;      // [query]
    int32_t k_max;
    int32_t P;
    int64_t nslots;
    const TravHdr *hdr;
    int64_t max_cells;
    const int32_t *ne_cs, *ne_cnt;
    const int64_t *ne_beg;
    const float *ne_cst;
    const int32_t *ne_slot, *slot_ij;
    float *lq;             // [slot][M][Kc] query tables
    float *dist;           // [slot][lcap] FP32 distance of every candidate (row-major index)
    int64_t lcap;
    int32_t wcap;
    int32_t *sel_done;     // [slot] 1: top-k written by the cell scan itself
    int64_t *out_ids;      // [query][k_max]
    float *out_d;
    int64_t *dbg_pos;
    float *dbg_d;
    int64_t dbg_cap;
    unsigned long long *stats;  // optional path counters
};
hipError_t launch_items_prep(const ItemArgs &a, hipStream_t st);   // LQ tables
hipError_t launch_items_scan(const ItemArgs &a, hipStream_t st);   // query-major cell scan
hipError_t launch_items_merge(const ItemArgs &a, hipStream_t st);  // per-query top-k

// Persistent form of the cell scan: a device queue of (query, cell range)
// items of at least `tile` candidates, largest queries first, taken by
// resident workgroups of `waves` wavefronts; the workgroup finishing a
// query's last item selects its top-k (else k_select_dist does).
struct PersistArgs {
    int32_t *items;  // [cap][3]: slot, first cell, end cell
    int32_t *ctl;    // [2 + 2 * 32]: queue head, item count, per-class counts and cursors
    int32_t *qnit;   // [slot] items of the query
    int32_t *qdone;  // [slot] items finished
    int32_t tile;
};
int64_t persist_items_cap(int64_t nslots, int64_t lcap, int32_t tile);
hipError_t launch_items_persist(const ItemArgs &a, const PersistArgs &p, int waves, hipStream_t st);
int items_wcap(int k_max);
size_t select_dist_lds(int k_max);

// Serving lanes (api.hip): handles over another handle's index arrays.
int lane_create(fbpq_index *src, fbpq_index **out);
int lane_device(const fbpq_index *ix);
int lane_dim(const fbpq_index *ix);
int64_t lane_points(const fbpq_index *ix);
// Workspace bytes one query of budget L and k may need in a search on ix (a
// fixed part per query plus bytes per candidate and per visited cell, from the
// buffer sizes of the search pipeline, with room for its retry round).
int64_t search_ws_estimate(const fbpq_index *ix, int64_t L, int32_t k);

}  // namespace fbpq
