// Multi-sequence traversal of the inverted multi-index (Section 2.3.3): visit
// cells (i, j) in ascending d1[i] + d2[j] until the visited cells hold L points.
//
// Cells are addressed by rank pairs (a, b) into the two sorted half lists
// (u, v). One wavefront serves one query. The visited set is always a Young
// diagram in rank space (row a holds b < w[a], w non-increasing), because a
// cell's key is not smaller than the keys of the cells left of and above it.
// So the frontier is one candidate cell per row: (a, w[a]), available when
// a == 0 or w[a-1] > w[a]. Each lane owns rows a = lane + 64*r in registers
// (width, width of the row above, key of its next cell); a pop is a wave-wide
// argmin over (key, a) and touches at most two rows. Pops are taken in
// batches (16, then 64 at a time); a batch's point counts are then read from
// the offsets array in one vector load and prefix-summed, and the batch is cut
// at the cell that completes min(L, N) points (that cell is truncated in
// storage order, pops after it are undone).
//
// A query still unfinished after pop_budget cells is marked kStDefer and left
// to the threshold-stepping kernel, which starts it again from the first cell.
//
// Only the first P ranks of each half list are known. A cell outside the
// P x P window has key >= min(k1[P-1] + k2[0], k1[0] + k2[P-1]); the query is
// flagged for a longer prefix when the next pop reaches that bound.
#include "fbpq_dev.h"

#include <type_traits>

namespace fbpq {

// Wave-wide minimum of (key, a), ties to the smaller a; every lane gets it.
// Keys are non-negative doubles or +inf, so their bit patterns order as the
// values do. Within each row of 16 lanes the pairs are exchanged with DPP moves
// (lane xor 1, xor 2, then the mirrors of 8 and of 16 lanes: each step pairs
// every lane with one holding a disjoint set), and the four rows are combined
// through lanes 0, 16, 32 and 48. The minimum of a total order does not depend
// on the order of combination, so the result is the same as any other reduction.
__device__ __forceinline__ void wave_argmin(double &key, int &a)
{
    uint64_t kb = (uint64_t)__double_as_longlong(key);
    int ab = a;
    auto step = [&](auto ctrl) __attribute__((always_inline)) {
        constexpr int c = decltype(ctrl)::value;
        const uint32_t lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)kb, c, 0xf, 0xf, false);
        const uint32_t hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(kb >> 32), c, 0xf, 0xf, false);
        const int oa = __builtin_amdgcn_update_dpp(0, ab, c, 0xf, 0xf, false);
        const uint64_t ok = ((uint64_t)hi << 32) | lo;
        if (ok < kb || (ok == kb && oa < ab)) {
            kb = ok;
            ab = oa;
        }
    };
    step(std::integral_constant<int, 0xb1>{});   // quad_perm [1,0,3,2]: lane xor 1
    step(std::integral_constant<int, 0x4e>{});   // quad_perm [2,3,0,1]: lane xor 2
    step(std::integral_constant<int, 0x141>{});  // row_half_mirror: 7 - lane within 8
    step(std::integral_constant<int, 0x140>{});  // row_mirror: 15 - lane within 16
    uint64_t best = ~0ull;
    int besta = 0x7fffffff;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)kb, 16 * r);
        const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(kb >> 32), 16 * r);
        const int ra = __builtin_amdgcn_readlane(ab, 16 * r);
        const uint64_t rk = ((uint64_t)hi << 32) | lo;
        if (rk < best || (rk == best && ra < besta)) {
            best = rk;
            besta = ra;
        }
    }
    key = __longlong_as_double((long long)best);
    a = besta;
}

template <int RPL>
__global__ __launch_bounds__(64) void k_traverse(TravArgs args)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int P = args.P;
    double *k2s = reinterpret_cast<double *>(smem);            // [P]
    int *wl = reinterpret_cast<int *>(k2s + P);                 // [P]
    const int slot = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t qs = args.qlist ? args.qlist[slot] : slot;
    const int T = args.ix.T;
    const double *k1 = args.lkey + (int64_t)slot * 2 * P;
    const double *k2 = k1 + P;
    const int32_t *u = args.lidx + (int64_t)slot * 2 * P;
    const int32_t *v = u + P;
    const int64_t *off = args.ix.offsets;
    for (int i = lane; i < P; i += 64) k2s[i] = k2[i];
    __syncthreads();

    const int64_t L = args.L[qs];
    const int64_t Leff = L < args.ix.N ? L : args.ix.N;
    const bool full = P >= T;
    const double INF = __builtin_huge_val();
    const double kbound = full ? INF : fmin(k1[P - 1] + k2s[0], k1[0] + k2s[P - 1]);

    int w[RPL], wp[RPL];
    double nk[RPL], k1r[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int a = lane + 64 * r;
        k1r[r] = a < P ? k1[a] : INF;
        w[r] = 0;
        wp[r] = a == 0 ? 0x7fffffff : 0;
        nk[r] = (a < P && (a == 0)) ? k1r[r] + k2s[0] : INF;
    }

    int status = kStOk;
    int64_t total = 0, ncells = 0;
    int cut_a = -1, cut_b = -1;
    int64_t cut_take = 0;
    int jc = -1, nb_last = 0, pa = -1, pb = -1;
    bool done = Leff <= 0;
    int bsz = 16;  // pops per batch: 16 first (most queries end there), then 64
    while (!done) {
        if (args.pop_budget > 0 && ncells >= args.pop_budget) {
            status = kStDefer;  // large visited set: the threshold kernel takes over
            break;
        }
        pa = -1;
        pb = -1;
        int nb = 0;
        bool exhausted = false;
        for (int j = 0; j < bsz; ++j) {
            double bk = INF;
            int ba = 0x7fffffff;
#pragma unroll
            for (int r = 0; r < RPL; ++r)
                if (nk[r] < bk) {
                    bk = nk[r];
                    ba = lane + 64 * r;
                }
            wave_argmin(bk, ba);
            if (bk == INF) {
                exhausted = true;
                break;
            }
            if (bk >= kbound) {
                status = kStNeedPrefix;
                break;
            }
            const int ro = ba >> 6, lo = ba & 63;
            int wsel = 0;
#pragma unroll
            for (int r = 0; r < RPL; ++r)
                if (r == ro) wsel = w[r];
            const int bb = __builtin_amdgcn_readlane(wsel, lo);  // lo is the same on every lane
            if (lane == j) {
                pa = ba;
                pb = bb;
            }
            ++nb;
            if (lane == lo) {
#pragma unroll
                for (int r = 0; r < RPL; ++r)
                    if (r == ro) {
                        w[r] = bb + 1;
                        nk[r] = (w[r] < P && (ba == 0 || wp[r] > w[r])) ? k1r[r] + k2s[w[r]] : INF;
                    }
            }
            const int an = ba + 1;
            if (an < P && lane == (an & 63)) {
#pragma unroll
                for (int r = 0; r < RPL; ++r)
                    if (r == (an >> 6)) {
                        wp[r] = bb + 1;
                        nk[r] = (w[r] < P && wp[r] > w[r]) ? k1r[r] + k2s[w[r]] : INF;
                    }
            }
        }
        if (status != kStOk) break;
        if (nb == 0) {
            // every tracked cell is visited and fewer than min(L, N) points were found
            status = full ? kStOk : kStNeedPrefix;
            done = true;
            break;
        }
        int64_t beg = 0, cnt = 0;
        if (lane < nb) {
            const int64_t c = (int64_t)u[pa] * T + v[pb];
            beg = off[c];
            cnt = off[c + 1] - beg;
        }
        int64_t x = cnt;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        const int64_t incl = total + x, excl = incl - cnt;
        const uint64_t m = __ballot(lane < nb && incl >= Leff);
        jc = m ? __ffsll((long long)m) - 1 : -1;
        const int nkeep = jc >= 0 ? jc + 1 : nb;
        if (ncells + nkeep > args.max_cells) {
            status = kStNeedCells;
            break;
        }
        if (args.dbg_ab && lane < nkeep) {
            const int64_t o = (int64_t)slot * args.max_cells + ncells + lane;
            args.dbg_ab[2 * o] = pa;
            args.dbg_ab[2 * o + 1] = pb;
            args.dbg_take[o] = lane == jc ? Leff - excl : cnt;
            args.dbg_beg[o] = beg;
        }
        const int last = nkeep - 1;
        cut_a = __shfl(pa, last);
        cut_b = __shfl(pb, last);
        const int64_t last_excl = __shfl(excl, last);
        const int64_t last_cnt = __shfl(cnt, last);
        ncells += nkeep;
        nb_last = nb;
        bsz = 64;
        if (jc >= 0) {
            cut_take = Leff - last_excl;
            total = Leff;
            done = true;
        } else {
            cut_take = last_cnt;
            total = last_excl + last_cnt;
            if (exhausted) {
                status = full ? kStOk : kStNeedPrefix;
                done = true;
            }
        }
    }

    // final row widths: the register state minus the pops after the cut
    for (int r = 0; r < RPL; ++r) {
        const int a = lane + 64 * r;
        if (a < P) wl[a] = w[r];
    }
    __syncthreads();
    if (status == kStOk && jc >= 0 && lane > jc && lane < nb_last) atomicSub(&wl[pa], 1);
    __syncthreads();
    int myA = 0;
    for (int a = lane; a < P; a += 64) {
        const int wa = wl[a];
        args.w[(int64_t)slot * P + a] = wa;
        myA += wa > 0;
    }
    for (int o = 32; o > 0; o >>= 1) myA += __shfl_xor(myA, o);
    if (lane == 0) {
        TravHdr h;
        h.status = status;
        h.A = myA;
        h.B = P > 0 ? wl[0] : 0;
        h.cut_a = cut_a;
        h.cut_b = cut_b;
        h.nne = 0;
        h.a_ne = 0;
        h.b_ne = 0;
        h.n_items = 0;
        h.gscan = 0;
        h.ncells = ncells;
        h.ncand = total;
        h.cut_take = cut_take;
        if (Leff <= 0) {
            h.A = 0;
            h.B = 0;
            h.ncells = 0;
            h.ncand = 0;
        }
        args.hdr[slot] = h;
        if (status != kStOk && status != kStDefer) args.fail_list[atomicAdd(args.fail_count, 1)] = (int32_t)qs;
    }
}

hipError_t launch_traverse(const TravArgs &a, int64_t nslots, hipStream_t st)
{
    if (nslots == 0) return hipSuccess;
    const size_t lds = (size_t)a.P * (sizeof(double) + sizeof(int));
    const dim3 g((unsigned)nslots), b(64);
    const int rpl = (a.P + 63) / 64;
    if (rpl <= 1) hipLaunchKernelGGL(k_traverse<1>, g, b, lds, st, a);
    else if (rpl <= 2) hipLaunchKernelGGL(k_traverse<2>, g, b, lds, st, a);
    else if (rpl <= 4) hipLaunchKernelGGL(k_traverse<4>, g, b, lds, st, a);
    else if (rpl <= 8) hipLaunchKernelGGL(k_traverse<8>, g, b, lds, st, a);
    else if (rpl <= 16) hipLaunchKernelGGL(k_traverse<16>, g, b, lds, st, a);
    else if (rpl <= 32) hipLaunchKernelGGL(k_traverse<32>, g, b, lds, st, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// ---- compacted layout of the visited diagram --------------------------------
// The scan walks candidates row by row (fixed i, first half of the code) and
// column by column (fixed j, second half). Only nonempty cells matter, so the
// visited cells are compacted: row-major (a, then b) entries with storage
// begin, points taken, first candidate index (candidates numbered in row-major
// order) and the cell constant fl32(d1[i] + d2[j]); each row gets its first
// entry and first candidate, each column the list of its entries (in arbitrary
// order) with a running candidate prefix inside the column.
__global__ __launch_bounds__(64) void k_layout(LayoutArgs args)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const int P = args.P;
    // per-rank arrays in LDS, or (long prefixes) in this slot's slice of HBM
    unsigned char *smem = args.gscr ? args.gscr + (size_t)blockIdx.x * layout_rank_bytes(P) : lds;
    unsigned long long *colcur = reinterpret_cast<unsigned long long *>(smem);  // [P] cells | candidates
    int *rc = reinterpret_cast<int *>(colcur + P);      // [P + 1] first diagram cell of each row
    int *rowcnt = rc + (P + 1);                         // [P + 1] nonempty cells per row
    int *colcnt = rowcnt + (P + 1);                     // [P + 1] nonempty cells per column
    int *rslot = colcnt + (P + 1);                      // [2P] LUT slot of each row, then column
    const int slot = blockIdx.x;
    const int lane = threadIdx.x;
    TravHdr h = args.hdr[slot];
    if (h.status != kStOk || h.ncells > kLayoutWaveMax) return;
    const int A = h.A, B = h.B;
    const int T = args.ix.T;
    const int32_t *w = args.w + (int64_t)slot * P;
    const double *k1 = args.lkey + (int64_t)slot * 2 * P;
    const double *k2 = k1 + P;
    const int32_t *u = args.lidx + (int64_t)slot * 2 * P;
    const int32_t *v = u + P;
    const int64_t *off = args.ix.offsets;
    const int64_t mc = args.max_cells;
    int32_t *row_ne = args.row_ne + (int64_t)slot * (P + 1);
    int32_t *row_cand = args.row_cand + (int64_t)slot * (P + 1);
    int32_t *col_ne = args.col_ne + (int64_t)slot * (P + 1);
    int32_t *col_tot = args.col_tot + (int64_t)slot * P;
    int32_t *ne_cs = args.ne_cs + (int64_t)slot * mc;
    int32_t *ne_cnt = args.ne_cnt + (int64_t)slot * mc;
    int64_t *ne_beg = args.ne_beg + (int64_t)slot * mc;
    float *ne_cst = args.ne_cst + (int64_t)slot * mc;
    int32_t *cm_cell = args.cm_cell + (int64_t)slot * mc;
    int32_t *cm_pre = args.cm_pre + (int64_t)slot * mc;

    int run = 0;
    for (int a0 = 0; a0 < A; a0 += 64) {
        const int a = a0 + lane;
        const int wa = a < A ? w[a] : 0;
        int x = wa;
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (a < A) rc[a] = run + x - wa;
        run += __shfl(x, 63);
    }
    if (lane == 0) rc[A] = run;
    for (int a = lane; a <= P; a += 64) {
        rowcnt[a] = 0;
        colcnt[a] = 0;
    }
    int32_t *ne_slot = args.ne_slot + (int64_t)slot * mc;
    int32_t *slot_ij = args.slot_ij + (int64_t)slot * 2 * P;
    for (int b = lane; b < P; b += 64) colcur[b] = 0ull;
    __syncthreads();
    const int64_t ncells = run;
    if (ncells > mc) return;

    // pass 1: nonempty cells per row and per column
    for (int64_t x0 = 0; x0 < ncells; x0 += 64) {
        const int64_t xi = x0 + lane;
        if (xi < ncells) {
            int lo = 0, hi = A;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (rc[mid] <= xi) lo = mid;
                else hi = mid - 1;
            }
            const int a = lo, b = (int)(xi - rc[a]);
            const int64_t c = (int64_t)u[a] * T + v[b];
            const int64_t beg = off[c];
            const int64_t cnt = (a == h.cut_a && b == h.cut_b) ? h.cut_take : off[c + 1] - beg;
            if (cnt > 0) {
                atomicAdd(&rowcnt[a], 1);
                atomicAdd(&colcnt[b], 1);
            }
        }
    }
    __syncthreads();
    // exclusive scans: first compacted entry of each row and of each column
    {
        int r1 = 0, r2 = 0;
        for (int a0 = 0; a0 <= P; a0 += 64) {
            const int a = a0 + lane;
            const int x1 = a <= A ? rowcnt[a] : 0;
            const int x2 = a <= B ? colcnt[a] : 0;
            int s1 = x1, s2 = x2;
            for (int o = 1; o < 64; o <<= 1) {
                const int y1 = __shfl_up(s1, o), y2 = __shfl_up(s2, o);
                if (lane >= o) {
                    s1 += y1;
                    s2 += y2;
                }
            }
            __syncthreads();
            if (a <= A) {
                rowcnt[a] = r1 + s1 - x1;
                row_ne[a] = r1 + s1 - x1;
            }
            if (a <= B) {
                colcnt[a] = r2 + s2 - x2;
                col_ne[a] = r2 + s2 - x2;
            }
            r1 += __shfl(s1, 63);
            r2 += __shfl(s2, 63);
            __syncthreads();
        }
    }
    __syncthreads();
    // LUT slots: rank of each row (column) among rows (columns) that hold a nonempty cell
    int nr = 0, ncol = 0;
    for (int a0 = 0; a0 < P; a0 += 64) {
        const int a = a0 + lane;
        const bool rne = a < A && rowcnt[a + 1] > rowcnt[a];
        const bool cne = a < B && colcnt[a + 1] > colcnt[a];
        const uint64_t mr = __ballot(rne), mcl = __ballot(cne);
        const uint64_t below = (1ull << lane) - 1ull;
        if (rne) {
            rslot[a] = nr + __popcll(mr & below);
            slot_ij[nr + __popcll(mr & below)] = u[a];
        }
        if (cne) {
            rslot[P + a] = ncol + __popcll(mcl & below);
        }
        nr += __popcll(mr);
        ncol += __popcll(mcl);
    }
    __syncthreads();
    for (int b = lane; b < B; b += 64)
        if (colcnt[b + 1] > colcnt[b]) slot_ij[nr + rslot[P + b]] = v[b];
    if (lane == 0) {
        args.hdr[slot].a_ne = nr;
        args.hdr[slot].b_ne = ncol;
    }
    __syncthreads();
    // pass 2: write the compacted entries
    int64_t crun = 0;
    int nerun = 0, itrun = 0;
    for (int64_t x0 = 0; x0 < ncells; x0 += 64) {
        const int64_t xi = x0 + lane;
        int64_t cnt = 0, beg = 0;
        int a = 0, b = 0;
        if (xi < ncells) {
            int lo = 0, hi = A;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (rc[mid] <= xi) lo = mid;
                else hi = mid - 1;
            }
            a = lo;
            b = (int)(xi - rc[a]);
            const int64_t c = (int64_t)u[a] * T + v[b];
            beg = off[c];
            cnt = (a == h.cut_a && b == h.cut_b) ? h.cut_take : off[c + 1] - beg;
        }
        int64_t s = cnt;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(s, o);
            if (lane >= o) s += y;
        }
        const uint64_t nem = __ballot(cnt > 0);
        const int nit = (int)((cnt + kItem - 1) / kItem);
        int is = nit;
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(is, o);
            if (lane >= o) is += y;
        }
        itrun += __shfl(is, 63);
        if (xi < ncells) {
            const int64_t cs = crun + s - cnt;
            if (b == 0) row_cand[a] = (int32_t)cs;
            if (cnt > 0) {
                const int e = nerun + __popcll(nem & ((1ull << lane) - 1ull));
                ne_cs[e] = (int32_t)cs;
                ne_cnt[e] = (int32_t)cnt;
                ne_beg[e] = beg;
                ne_cst[e] = (float)(k1[a] + k2[b]);
                ne_slot[e] = rslot[a] | ((nr + rslot[P + b]) << 16);
                const unsigned long long old = atomicAdd(&colcur[b], (1ull << 40) + (unsigned long long)cnt);
                const int slotc = colcnt[b] + (int)(old >> 40);
                cm_cell[slotc] = e;
                cm_pre[slotc] = (int32_t)(old & ((1ull << 40) - 1ull));
            }
        }
        nerun += __popcll(nem);
        crun += __shfl(s, 63);
    }
    __syncthreads();
    if (lane == 0) row_cand[A] = (int32_t)crun;
    for (int b = lane; b < B; b += 64) col_tot[b] = (int32_t)(colcur[b] & ((1ull << 40) - 1ull));
    if (lane == 0) {
        args.hdr[slot].nne = nerun;
        const bool dense = nerun > 0 && crun >= (int64_t)kItemMinAvg * nerun;
        const bool items = args.allow_items && dense && !args.ix.local && !args.ix.od;
        args.hdr[slot].n_items = items ? itrun : 0;
        args.hdr[slot].gscan = args.ix.local || args.ix.od || (!dense && crun > kScanWideMin) ? 1 : 0;
    }
}

hipError_t launch_layout(const LayoutArgs &a, int64_t nslots, hipStream_t st)
{
    if (nslots == 0) return hipSuccess;
    const size_t lds = a.gscr ? 0 : layout_rank_bytes(a.P);
    if (lds > 144 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_layout, dim3((unsigned)nslots), dim3(64), lds, st, a);
    return hipGetLastError();
}

}  // namespace fbpq
