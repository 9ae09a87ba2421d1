// Candidate scoring with the FBPQ distance (Section 3.1) fused with the
// per-query lookup table and the top-k rerank (Section 2.3.3).
//
// For a candidate with code bytes b_0..b_{M-1} in cell (i, j), equations
// (distance) and (decomposition) give
//   ||q - x||^2 ~ ||q1 - c1_i||^2 + ||q2 - c2_j||^2
//               + sum_{k<M}   (||R_k(b_k)||^2 - 2 <q|k, R_k(b_k)>)     [LQ]
//               + sum_{k<M/2}  2 <c1_i|k, R_k(b_k)>                     [CR1]
//               + sum_{k<M/2}  2 <c2_j|k, R_{M/2+k}(b_{M/2+k})>         [CR2]
// -- O(M) work per candidate. The two half distances come from the first
// layer (FP64 keys, added in FP64 and rounded once to FP32: the cell constant).
// The LQ and CR terms of a half are folded into one table per row i
// (LUT1_i = LQ[k<M/2] + CR1[i]) or column j (LUT2_j = LQ[k>=M/2] + CR2[j]), so
// a candidate costs M lookups, and each CR row is read once per query.
//
// This kernel takes the queries the item scan leaves (visited cells holding
// few points on average, or more work items than it tracks): two passes over
// an LDS array of partial sums, rows then columns, with each row's and
// column's folded table built once. It keeps the k smallest (distance, id)
// with select_k after every chunk of candidates.
#include "codes.h"
#include "fbpq_dev.h"
#include "select_k.h"

namespace fbpq {

namespace {

constexpr int kTieCap = 512;

__device__ __forceinline__ uint64_t wave_or64(uint64_t v)
{
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
    return v;
}

template <int MH>
__device__ __forceinline__ float lut_sum(const float *lut, const uint8_t *__restrict__ codes, int64_t p)
{
    return lsum<MH>(lut, load_c<MH>(codes, p));
}

// last index x in [lo, hi) with v[x] <= t (v ascending over the range, v[lo] <= t)
template <typename P>
__device__ __forceinline__ int last_le(P v, int lo, int hi, int64_t t)
{
    hi -= 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)v[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

}  // namespace

// ============================ two-pass scan ===================================
template <int MH, bool TAB_LDS>
__global__ __launch_bounds__(512) void k_scan2(ScanArgs a)
{
    constexpr int NT = 512;
    constexpr int NW = NT / 64;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ SelShared sh;
    __shared__ int s_alo, s_ahi;

    constexpr int M = 2 * MH;
    const int slot = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t qs = a.qlist ? a.qlist[slot] : slot;
    const TravHdr h = a.hdr[slot];
    if (h.status != kStOk || h.n_items != 0 || h.gscan) return;
    if (TAB_LDS != (h.nne <= kScanCellsLds)) return;
    if (a.stats && tid == 0) {
        atomicAdd(&a.stats[kStatTwoPass], 1ull);
        atomicAdd(&a.stats[kStatCandTwoPass], (unsigned long long)h.ncand);
    }
    const int D = a.ix.D, ds = D / M, P = a.P;
    const int kq = a.k[qs];
    int KP = 1;
    while (KP < a.k_max) KP <<= 1;
    const int WCAP = KP * 2 < 256 ? 256 : KP * 2;

    float *qv = reinterpret_cast<float *>(smem);
    float *LQ = qv + ((D + 3) & ~3);
    float *LUT = LQ + M * kKc;
    float *part = LUT + MH * kKc;
    unsigned char *after = reinterpret_cast<unsigned char *>(part + ((a.chunk + 3) & ~3));
    uint64_t *win = reinterpret_cast<uint64_t *>(after);
    uint64_t *run = win + WCAP;
    uint32_t *tie = reinterpret_cast<uint32_t *>(run + KP);
    int64_t *lbeg = reinterpret_cast<int64_t *>(tie + kTieCap);
    int32_t *lcs = reinterpret_cast<int32_t *>(lbeg + kScanCellsLds);
    float *lcst = reinterpret_cast<float *>(lcs + kScanCellsLds);
    int32_t *lcmc = reinterpret_cast<int32_t *>(lcst + kScanCellsLds);
    int32_t *lcmp = lcmc + kScanCellsLds;

    const int64_t mc = a.max_cells;
    const int nne = h.nne;
    const int32_t *g_cs = a.ne_cs + slot * mc;
    const int64_t *g_beg = a.ne_beg + slot * mc;
    const float *g_cst = a.ne_cst + slot * mc;
    const int32_t *g_cmc = a.cm_cell + slot * mc;
    const int32_t *g_cmp = a.cm_pre + slot * mc;
    if (TAB_LDS) {
        for (int e = tid; e < nne; e += NT) {
            lcs[e] = g_cs[e];
            lbeg[e] = g_beg[e];
            lcst[e] = g_cst[e];
            lcmc[e] = g_cmc[e];
            lcmp[e] = g_cmp[e];
        }
    }
    const int32_t *t_cs = TAB_LDS ? lcs : g_cs;
    const int64_t *t_beg = TAB_LDS ? lbeg : g_beg;
    const float *t_cst = TAB_LDS ? lcst : g_cst;
    const int32_t *t_cmc = TAB_LDS ? lcmc : g_cmc;
    const int32_t *t_cmp = TAB_LDS ? lcmp : g_cmp;

    for (int t = tid; t < D; t += NT) qv[t] = a.q[qs * D + t];
    __syncthreads();
    // LQ[k][r] = ||R_k(r)||^2 - 2 <q|k, R_k(r)>   (the query part of the ADC table, Section 2.1)
    for (int e = tid; e < M * kKc; e += NT) {
        const int k = e / kKc;
        const float *rw = a.ix.R + (int64_t)e * ds;
        float acc = 0.f;
        for (int t = 0; t < ds; ++t) acc = fmaf(qv[k * ds + t], rw[t], acc);
        LQ[e] = a.ix.nR[e] - 2.f * acc;
    }

    const int32_t *u = a.lidx + (int64_t)slot * 2 * P;
    const int32_t *v = u + P;
    const int32_t *row_ne = a.row_ne + (int64_t)slot * (P + 1);
    const int32_t *row_cand = a.row_cand + (int64_t)slot * (P + 1);
    const int32_t *col_ne = a.col_ne + (int64_t)slot * (P + 1);
    const int32_t *col_tot = a.col_tot + (int64_t)slot * P;
    const int64_t ncand = h.ncand;
    const int A = h.A, B = h.B;
    const uint64_t below_lane = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);

    int nrun = 0;
    for (int64_t c0 = 0; c0 < ncand; c0 += a.chunk) {
        const int64_t c1 = c0 + a.chunk < ncand ? c0 + a.chunk : ncand;
        const int n = (int)(c1 - c0);
        if (tid == 0) {
            s_alo = last_le(row_cand, 0, A, c0);
            s_ahi = last_le(row_cand, 0, A, c1 - 1);
        }
        __syncthreads();
        const int alo = s_alo, ahi = s_ahi;

        // pass 1: rows, first half of the code, plus the cell constant
        for (int ar = alo; ar <= ahi; ++ar) {
            const int64_t rs = row_cand[ar] > c0 ? row_cand[ar] : c0;
            const int64_t re = row_cand[ar + 1] < c1 ? row_cand[ar + 1] : c1;
            if (rs >= re) continue;
            __syncthreads();
            const float *cr = a.ix.CR1 + (int64_t)u[ar] * MH * kKc;
            for (int e = tid; e < MH * kKc; e += NT) LUT[e] = LQ[e] + cr[e];
            __syncthreads();
            const int xb = row_ne[ar], xe = row_ne[ar + 1];
            for (int64_t t0 = rs + 64 * wv; t0 < re; t0 += 64 * NW) {
                const int x0 = last_le(t_cs, xb, xe, t0);
                const int x = x0 + lane;
                int32_t cs = 0;
                int64_t beg = 0;
                float cst = 0.f;
                bool vc = false;
                if (x < xe) {
                    cs = t_cs[x];
                    vc = cs < t0 + 64;
                    beg = t_beg[x];
                    cst = t_cst[x];
                }
                const int sr = cs > t0 ? (int)(cs - t0) : 0;
                const uint64_t mask = wave_or64(vc ? (1ull << sr) : 0ull);
                const int owner = __popcll(mask & below_lane) - 1;
                const int32_t cso = __shfl(cs, owner);
                const int64_t bego = __shfl(beg, owner);
                const float csto = __shfl(cst, owner);
                const int64_t t = t0 + lane;
                if (t < re) part[t - c0] = lut_sum<MH>(LUT, a.ix.codesA, bego + (t - cso)) + csto;
            }
        }
        // pass 2: columns, second half of the code
        for (int b = 0; b < B; ++b) {
            const int yb = col_ne[b], ye = col_ne[b + 1];
            if (yb >= ye) continue;
            const int U = col_tot[b];
            __syncthreads();
            const float *cr = a.ix.CR2 + (int64_t)v[b] * MH * kKc;
            for (int e = tid; e < MH * kKc; e += NT) LUT[e] = LQ[MH * kKc + e] + cr[e];
            __syncthreads();
            for (int u0 = 64 * wv; u0 < U; u0 += 64 * NW) {
                const int y0 = last_le(t_cmp, yb, ye, u0);
                const int y = y0 + lane;
                int32_t pre = 0, cs = 0;
                int64_t beg = 0;
                bool vc = false;
                if (y < ye) {
                    pre = t_cmp[y];
                    vc = pre < u0 + 64;
                    const int e = t_cmc[y];
                    cs = t_cs[e];
                    beg = t_beg[e];
                }
                const int sr = pre > u0 ? pre - u0 : 0;
                const uint64_t mask = wave_or64(vc ? (1ull << sr) : 0ull);
                const int owner = __popcll(mask & below_lane) - 1;
                const int32_t preo = __shfl(pre, owner);
                const int32_t cso = __shfl(cs, owner);
                const int64_t bego = __shfl(beg, owner);
                const int uu = u0 + lane;
                if (uu < U) {
                    const int64_t t = cso + (uu - preo);
                    if (t >= c0 && t < c1) {
                        const int64_t p = bego + (t - cso);
                        const float d = part[t - c0] + lut_sum<MH>(LUT, a.ix.codesB, p);
                        part[t - c0] = d;
                        if (a.dbg_pos) {
                            a.dbg_pos[(int64_t)slot * a.dbg_cap + t] = p;
                            a.dbg_d[(int64_t)slot * a.dbg_cap + t] = d;
                        }
                    }
                }
            }
        }
        __syncthreads();
        const int nr = nrun;
        auto visit = [&](auto &&f) __attribute__((always_inline)) {
            for (int e = tid; e < n; e += NT)
                f(fkey(part[e]), [&]() __attribute__((always_inline)) {
                    const int64_t t = c0 + e;
                    const int x = last_le(t_cs, 0, nne, t);
                    return a.ix.ids[t_beg[x] + (t - t_cs[x])];
                });
            for (int e = tid; e < nr; e += NT) f((uint32_t)(run[e] >> 32), [&]() __attribute__((always_inline)) { return (uint32_t)run[e]; });
        };
        nrun = select_k<NT>(visit, n + nr, kq, win, WCAP, tie, kTieCap, sh, true, run);
    }

    int64_t *oid = a.out_ids + qs * a.k_max;
    float *od = a.out_d + qs * a.k_max;
    for (int r = tid; r < a.k_max; r += NT) {
        if (r < nrun && r < kq) {
            oid[r] = (int64_t)(uint32_t)run[r];
            od[r] = unfkey((uint32_t)(run[r] >> 32));
        } else {
            oid[r] = -1;
            od[r] = __builtin_huge_valf();
        }
    }
}

// ============================ wide two-pass scan ==============================
// Queries with more than kScanWideMin candidates in sparse cells, and every
// query of an index with local codebooks. The partial sums live in the
// query's HBM distance row (index = row-major candidate number), so each row
// table LUT1_i and column table LUT2_j is folded once per task. The rows
// (then the columns) are cut into tasks of at most kWideChunk candidates;
// wavefront w takes tasks w, w + NW, ... and folds each task's table in its
// own LDS region, without workgroup barriers. The k smallest are selected
// afterwards from the row.
//
// Folded tables: with the global codebooks LUT1_i = LQ[k<M/2] + CR1[i]; with
// local codebooks (HBPQ, Section 3.2) LUT1_i = CQ1[i] - 2 <q1|k, Q^i_k(r)>,
// the query part computed here from the row's own codebooks (and likewise for
// the columns with S^j).
// Wavefronts per query: as many as 64 KB of folded tables allow, up to 16.
// Scan modes: the FBPQ tables of the global codebooks, the tables of local
// codebooks, or (the Multi-D-ADC baseline) the explicit O(D) reconstruction.
enum : int { kWideFbpq = 0, kWideLocal = 1, kWideOD = 2 };
template <int MH, int MODE>
constexpr int wide_waves() { return MODE != kWideFbpq && MH <= 8 ? 16 : (MH <= 4 ? 16 : (MH == 8 ? 8 : 4)); }
// With local codebooks, a query with at most this many distinct row and column
// tables folds each of them once into LDS, shared by all its tasks.
template <int MH>
constexpr int wide_tables() { return MH <= 8 ? 16 : 8; }
template <int MH, int MODE>
constexpr int wide_regions()
{
    return MODE == kWideLocal && wide_tables<MH>() > wide_waves<MH, MODE>() ? wide_tables<MH>()
                                                                            : wide_waves<MH, MODE>();
}
// floats before the task prefix: folded tables, or (O(D) mode) the codebooks of
// `group` subspaces of the current half [group][Kc][D/M] and each wavefront's
// q - c of its task. A half whose codebooks do not fit in LDS at once (large D)
// is scanned in several groups of subspaces; group 0 reads them from memory.
template <int MH, int MODE>
__host__ __device__ constexpr int64_t wide_region_floats(int D, int group = MH)
{
    return MODE == kWideOD ? (int64_t)group * kKc * (D / (2 * MH)) + (int64_t)wide_waves<MH, MODE>() * (D / 2)
                           : (int64_t)wide_regions<MH, MODE>() * MH * kKc;
}
// task prefix entries: one per rank of the longer half list (at most P) plus the
// total, so P + 1 of them; sized at launch from the prefix length
__host__ __device__ constexpr int64_t wide_ranks(int P) { return (int64_t)P + 1; }
constexpr int kWideU = 4;         // 64-candidate chunks a wavefront has in flight
constexpr int kWideKeep = 6;      // (distance, candidate) pairs each lane keeps for the selection
constexpr int kWideWin = 512;     // candidates the fused selection can rank

// the last lane o < n whose start v (held by lane o, ascending over lanes) is <= x
__device__ __forceinline__ int lane_owner(int32_t v, int n, int32_t x)
{
    int lo = 0, hi = n - 1;
    for (int it = 0; it < 6; ++it) {
        const int mid = (lo + hi + 1) >> 1;
        const bool le = __shfl(v, mid) <= x;
        lo = lo < hi && le ? mid : lo;
        hi = lo < hi && !le ? mid - 1 : hi;
    }
    return lo;
}

// exclusive prefix of x[0..n) in place, n <= wide_ranks(P); every thread calls it
template <int NT>
__device__ void wide_scan(int *x, int n, int *wtot)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int per = (n + NT - 1) / NT;
    const int i0 = tid * per, i1 = i0 + per < n ? i0 + per : n;
    int s = 0;
    for (int i = i0; i < i1; ++i) s += x[i];
    int v = s;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(v, o);
        if (lane >= o) v += y;
    }
    __syncthreads();
    if (lane == 63) wtot[wv] = v;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wv; ++w) before += wtot[w];
    int run = before + v - s;
    for (int i = i0; i < i1; ++i) {
        const int t = x[i];
        x[i] = run;
        run += t;
    }
    __syncthreads();
}

template <int MH, int MODE>
__global__ __launch_bounds__((64 * wide_waves<MH, MODE>())) void k_scan_wide(ScanArgs a)
{
    constexpr bool LOCAL = MODE == kWideLocal;
    constexpr bool OD = MODE == kWideOD;
    constexpr int NW = wide_waves<MH, MODE>();
    constexpr int NT = 64 * NW;
    constexpr int TL = MH * kKc;  // floats of one folded half table
    // the regions (wide_regions of them: folded tables, or the O(D) codebooks and
    // q - c), then the task prefix [wide_ranks(P)], then q [D]
    extern __shared__ __align__(16) float wlut[];
    __shared__ int wtot[NW];
    const int slot = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const TravHdr h = a.hdr[slot];
    if (h.status != kStOk || !h.gscan) return;
    if (tid == 0) {
        a.sel_done[slot] = 0;
        if (a.stats) {
            atomicAdd(&a.stats[kStatTwoPass], 1ull);
            atomicAdd(&a.stats[kStatCandWide], (unsigned long long)h.ncand);
        }
    }
    // this lane's kWideKeep smallest (distance key, candidate) pairs, ascending,
    // and the smallest key it did not keep (for the fused selection)
    uint64_t kp[kWideKeep];
#pragma unroll
    for (int q = 0; q < kWideKeep; ++q) kp[q] = ~0ull;
    uint32_t dmin = 0xffffffffu;
    auto keep = [&](float d, int64_t t) __attribute__((always_inline)) {
        const uint64_t kv = ((uint64_t)fkey(d) << 32) | (uint32_t)t;
        if (kv < kp[kWideKeep - 1]) {
            const uint32_t out = (uint32_t)(kp[kWideKeep - 1] >> 32);
            dmin = out < dmin ? out : dmin;
            kp[kWideKeep - 1] = kv;
#pragma unroll
            for (int q = kWideKeep - 1; q > 0; --q) {
                if (kp[q] < kp[q - 1]) {
                    const uint64_t x = kp[q - 1];
                    kp[q - 1] = kp[q];
                    kp[q] = x;
                }
            }
        } else {
            const uint32_t kk = (uint32_t)(kv >> 32);
            dmin = kk < dmin ? kk : dmin;
        }
    };
    float *lut = wlut + wv * TL;
    const int og = OD ? a.od_group : MH;  // O(D): subspaces staged per group (0: none, read from memory)
    int *tpre = reinterpret_cast<int *>(wlut + wide_region_floats<MH, MODE>(a.ix.D, og));
    const float *cbh = wlut;  // O(D): codebooks of subspaces [k0, k1) of the pass (LDS or memory)
    int k0 = 0, k1 = MH;
    float *qcw = wlut + (int64_t)og * kKc * (a.ix.D / (2 * MH)) + wv * (a.ix.D / 2);  // O(D): q - c
    float *qs = reinterpret_cast<float *>(tpre + wide_ranks(a.P));
    const int P = a.P;
    const int D = a.ix.D, ds = D / (2 * MH);
    const int64_t mc = a.max_cells;
    const int32_t *t_cs = a.ne_cs + slot * mc;
    const int64_t *t_beg = a.ne_beg + slot * mc;
    const float *t_cst = a.ne_cst + slot * mc;
    const int32_t *t_cmc = a.cm_cell + slot * mc;
    const int32_t *t_cmp = a.cm_pre + slot * mc;
    const int32_t *u = a.lidx + (int64_t)slot * 2 * P;
    const int32_t *v = u + P;
    const int32_t *row_ne = a.row_ne + (int64_t)slot * (P + 1);
    const int32_t *row_cand = a.row_cand + (int64_t)slot * (P + 1);
    const int32_t *col_ne = a.col_ne + (int64_t)slot * (P + 1);
    const int32_t *col_tot = a.col_tot + (int64_t)slot * P;
    const float *lq = a.lq + (int64_t)slot * 2 * TL;
    float *dist = a.dist + (int64_t)slot * a.lcap;
    const uint64_t below_lane = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    const int A = h.A, B = h.B;
    if (LOCAL || OD) {
        const int64_t qsl = a.qlist ? a.qlist[slot] : slot;
        for (int t = tid; t < D; t += NT) qs[t] = a.q[qsl * D + t];
    }
    // O(D): the codebooks of group g of the half (subspaces [k0, k1) of the
    // half's M/2), staged in LDS, or all of them in memory when og is 0
    const int ng = OD && og > 0 ? (MH + og - 1) / og : 1;
    auto stage_half = [&](int half, int g) __attribute__((always_inline)) {
        if (!OD) return;
        const float *src = a.ix.R + (int64_t)half * TL * ds;
        if (og == 0) {
            cbh = src;
            k0 = 0;
            k1 = MH;
            return;
        }
        k0 = g * og;
        k1 = k0 + og < MH ? k0 + og : MH;
        const int64_t n = (int64_t)(k1 - k0) * kKc * ds;
        src += (int64_t)k0 * kKc * ds;
        for (int64_t e = tid; e < n; e += NT) wlut[e] = src[e];
        cbh = wlut;
    };
    // O(D): this wavefront's q_h - c for its current task
    auto set_qc = [&](int half, int cent) __attribute__((always_inline)) {
        const float *c = (half ? a.ix.C2 : a.ix.C1) + (int64_t)cent * (D / 2);
        __builtin_amdgcn_wave_barrier();
        for (int t = lane; t < D / 2; t += 64) qcw[t] = qs[half * (D / 2) + t] - c[t];
        __builtin_amdgcn_wave_barrier();
    };
    // O(D): sum over the half's subspaces of ||(q - c)|k - R_k(b_k)||^2
    auto od_sum = [&](typename CodeU<MH>::T code) __attribute__((always_inline)) {
        uint8_t bytes[MH];
        __builtin_memcpy(bytes, &code, MH);
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < MH; ++k) {
            if (k < k0 || k >= k1) continue;
            const float *w = cbh + ((int64_t)(k - k0) * kKc + bytes[k]) * ds;
            const float *qk = qcw + k * ds;
            if ((ds & 3) == 0) {
                // 16-byte reads of the codeword and of q - c (both 16-byte aligned)
                for (int t = 0; t < ds; t += 4) {
                    const float4 wv4 = *reinterpret_cast<const float4 *>(w + t);
                    const float4 qv4 = *reinterpret_cast<const float4 *>(qk + t);
                    const float e0 = qv4.x - wv4.x, e1 = qv4.y - wv4.y, e2 = qv4.z - wv4.z, e3 = qv4.w - wv4.w;
                    acc = fmaf(e0, e0, acc);
                    acc = fmaf(e1, e1, acc);
                    acc = fmaf(e2, e2, acc);
                    acc = fmaf(e3, e3, acc);
                }
            } else {
                for (int t = 0; t < ds; ++t) {
                    const float e = qk[t] - w[t];
                    acc = fmaf(e, e, acc);
                }
            }
        }
        return acc;
    };

    constexpr int TQ = TL / 4 / 64;  // float4 of a table per lane
    float4 nxt[TQ];
    // the global-codebook fold reads the CR row prefetched into nxt
    auto fetch = [&](const float *crrow) __attribute__((always_inline)) {
        if (LOCAL || OD) return;
        const float4 *cr = reinterpret_cast<const float4 *>(crrow);
#pragma unroll
        for (int e = 0; e < TQ; ++e) nxt[e] = cr[lane + 64 * e];
    };
    auto fold = [&](int half, int cent, float *lut) __attribute__((always_inline)) {
        __builtin_amdgcn_wave_barrier();  // the previous table's lookups are done
        if (LOCAL) {
            // CQ[cent] - 2 <q|k, Q_k(r)> with the codebooks of this centroid
            const float *cq = (half ? a.ix.CR2 : a.ix.CR1) + (int64_t)cent * TL;
            const float *cb = (half ? a.ix.SL : a.ix.QL) + (int64_t)cent * TL * ds;
            const float *qh = qs + half * (D / 2);
            for (int f = lane; f < TL; f += 64) {
                const int k = f >> 8;
                const float *w = cb + (int64_t)f * ds;
                const float *qk = qh + k * ds;
                float acc = 0.f;
                for (int t = 0; t < ds; ++t) acc = fmaf(qk[t], w[t], acc);
                lut[f] = cq[f] - 2.f * acc;
            }
        } else {
            const float4 *lq4 = reinterpret_cast<const float4 *>(lq + half * TL);
#pragma unroll
            for (int e = 0; e < TQ; ++e) {
                const int f = lane + 64 * e;
                const float4 x = lq4[f], y = nxt[e];
                reinterpret_cast<float4 *>(lut)[f] = make_float4(x.x + y.x, x.y + y.y, x.z + y.z, x.w + y.w);
            }
        }
        __builtin_amdgcn_wave_barrier();
    };

    // Local codebooks and few distinct tables: fold each table once, shared.
    // Table s < a_ne belongs to row centroid slot_ij[s], the others to columns;
    // a cell's ne_slot holds its row table | (its column table << 16).
    const int nsl = h.a_ne + h.b_ne;
    const bool shared_tab = LOCAL && nsl <= wide_tables<MH>();
    const int32_t *sij = a.slot_ij + (int64_t)slot * 2 * P;
    const int32_t *t_nsl = a.ne_slot + slot * mc;
    if (shared_tab) {
        __syncthreads();  // the query vector is staged
        for (int sidx = wv; sidx < nsl; sidx += NW) fold(sidx < h.a_ne ? 0 : 1, sij[sidx], wlut + sidx * TL);
    }

    // ---- pass 1: row tasks, first half of the code plus the cell constant ----
    stage_half(0, 0);
    for (int ar = tid; ar <= A; ar += NT)
        tpre[ar] = ar < A ? (row_cand[ar + 1] - row_cand[ar] + kWideChunk - 1) / kWideChunk : 0;
    __syncthreads();
    wide_scan<NT>(tpre, A + 1, wtot);
    for (int g = 0; g < ng; ++g) {
        if (g > 0) {
            __syncthreads();  // every wavefront is done with the previous group's codebooks
            stage_half(0, g);
            __syncthreads();
        }
        const int ntask = tpre[A];
        auto task_row = [&](int tk) __attribute__((always_inline)) {
            int lo = 0, hi = A - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (tpre[mid] <= tk) lo = mid;
                else hi = mid - 1;
            }
            return lo;
        };
        int tk = wv;
        int ar = tk < ntask ? task_row(tk) : 0;
        if (tk < ntask) fetch(a.ix.CR1 + (int64_t)u[ar] * TL);
        while (tk < ntask) {
            const int ch = tk - tpre[ar];
            if (OD) set_qc(0, u[ar]);
            else if (shared_tab) lut = wlut + (t_nsl[row_ne[ar]] & 0xffff) * TL;
            else fold(0, u[ar], lut);
            const int tn = tk + NW;
            const int an = tn < ntask ? task_row(tn) : 0;
            if (tn < ntask) fetch(a.ix.CR1 + (int64_t)u[an] * TL);
            const int64_t rs = row_cand[ar] + (int64_t)ch * kWideChunk;
            const int64_t re0 = row_cand[ar + 1];
            const int64_t re = rs + kWideChunk < re0 ? rs + kWideChunk : re0;
            const int xe = row_ne[ar + 1];
            if (xe - row_ne[ar] <= 64) {
                // the row's cells sit one per lane; a candidate's cell is found
                // by a binary search over the lanes, kWideU chunks in flight
                const int xb = row_ne[ar], ncell = xe - xb;
                int32_t ccs = 0x7fffffff;
                int64_t cbeg = 0;
                float ccst = 0.f;
                if (lane < ncell) {
                    ccs = t_cs[xb + lane];
                    cbeg = t_beg[xb + lane];
                    ccst = t_cst[xb + lane];
                }
                for (int64_t t0 = rs; t0 < re; t0 += 64 * kWideU) {
                    typename CodeU<MH>::T cv[kWideU];
                    float cst_[kWideU];
#pragma unroll
                    for (int j = 0; j < kWideU; ++j) {
                        const int64_t t = t0 + 64 * j + lane;
                        const int o = lane_owner(ccs, ncell, (int32_t)(t < re ? t : re - 1));
                        const int32_t cso = __shfl(ccs, o);
                        const int64_t bego = __shfl(cbeg, o);
                        cst_[j] = __shfl(ccst, o);
                        if (t < re) cv[j] = load_c<MH>(a.ix.codesA, bego + (t - cso));
                    }
#pragma unroll
                    for (int j = 0; j < kWideU; ++j) {
                        const int64_t t = t0 + 64 * j + lane;
                        if (t < re)
                            dist[t] = OD ? (g == 0 ? 0.f : dist[t]) + od_sum(cv[j])
                                         : lsum<MH>(lut, cv[j]) + cst_[j];
                    }
                }
                tk = tn;
                ar = an;
                continue;
            }
            int x0 = ch == 0 ? row_ne[ar] : last_le(t_cs, row_ne[ar], xe, rs);
            for (int64_t t0 = rs; t0 < re; t0 += 64) {
                const int x = x0 + lane;
                int32_t cs = 0;
                int64_t beg = 0;
                float cst = 0.f;
                bool vc = false;
                if (x < xe) {
                    cs = t_cs[x];
                    vc = cs < t0 + 64;
                    beg = t_beg[x];
                    cst = t_cst[x];
                }
                const int sr = cs > t0 ? (int)(cs - t0) : 0;
                const uint64_t mask = wave_or64(vc ? (1ull << sr) : 0ull);
                const int owner = __popcll(mask & below_lane) - 1;
                const int32_t cso = __shfl(cs, owner);
                const int64_t bego = __shfl(beg, owner);
                const float csto = __shfl(cst, owner);
                const int64_t t = t0 + lane;
                if (t < re) {
                    const auto code = load_c<MH>(a.ix.codesA, bego + (t - cso));
                    dist[t] = OD ? (g == 0 ? 0.f : dist[t]) + od_sum(code) : lsum<MH>(lut, code) + csto;
                }
                // cell of candidate t0 + 64: that of lane 63's candidate, or the next
                const int o63 = __shfl(owner, 63);
                int xn = x0 + o63;
                const int csn = __shfl(cs, (o63 + 1) & 63);
                if (o63 < 63 && xn + 1 < xe && csn <= t0 + 64) ++xn;
                else if (o63 == 63 && xn + 1 < xe && t_cs[xn + 1] <= t0 + 64) ++xn;
                x0 = xn;
            }
            tk = tn;
            ar = an;
        }
    }
    __syncthreads();  // every partial sum of the query is stored; tpre is free

    // ---- pass 2: column tasks, second half of the code ----
    stage_half(1, 0);
    for (int b = tid; b <= B; b += NT)
        tpre[b] = b < B ? (col_tot[b] + kWideChunk - 1) / kWideChunk : 0;
    __syncthreads();
    wide_scan<NT>(tpre, B + 1, wtot);
    for (int g = 0; g < ng; ++g) {
        if (g > 0) {
            __syncthreads();  // every wavefront is done with the previous group's codebooks
            stage_half(1, g);
            __syncthreads();
        }
        const bool last = g == ng - 1;  // the distances are complete: keep them for the selection
        const int ntask = tpre[B];
        auto task_col = [&](int tk) __attribute__((always_inline)) {
            int lo = 0, hi = B - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (tpre[mid] <= tk) lo = mid;
                else hi = mid - 1;
            }
            return lo;
        };
        int tk = wv;
        int b = tk < ntask ? task_col(tk) : 0;
        if (tk < ntask) fetch(a.ix.CR2 + (int64_t)v[b] * TL);
        while (tk < ntask) {
            const int ch = tk - tpre[b];
            if (OD) set_qc(1, v[b]);
            else if (shared_tab) lut = wlut + (t_nsl[t_cmc[col_ne[b]]] >> 16) * TL;
            else fold(1, v[b], lut);
            const int tn = tk + NW;
            const int bn = tn < ntask ? task_col(tn) : 0;
            if (tn < ntask) fetch(a.ix.CR2 + (int64_t)v[bn] * TL);
            const int yb = col_ne[b], ye = col_ne[b + 1];
            const int U = col_tot[b];
            const int us = ch * kWideChunk;
            const int ue = us + kWideChunk < U ? us + kWideChunk : U;
            if (ye - yb <= 64) {
                const int ny = ye - yb;
                int32_t cpre = 0x7fffffff, ccs = 0;
                int64_t cbeg = 0;
                if (lane < ny) {
                    cpre = t_cmp[yb + lane];
                    const int e = t_cmc[yb + lane];
                    ccs = t_cs[e];
                    cbeg = t_beg[e];
                }
                for (int u0 = us; u0 < ue; u0 += 64 * kWideU) {
                    typename CodeU<MH>::T cv[kWideU];
                    int64_t tt[kWideU], pp[kWideU];
#pragma unroll
                    for (int j = 0; j < kWideU; ++j) {
                        const int uu = u0 + 64 * j + lane;
                        const int o = lane_owner(cpre, ny, uu < ue ? uu : ue - 1);
                        const int32_t preo = __shfl(cpre, o);
                        const int32_t cso = __shfl(ccs, o);
                        const int64_t bego = __shfl(cbeg, o);
                        tt[j] = cso + (uu - preo);
                        pp[j] = bego + (uu - preo);
                        if (uu < ue) cv[j] = load_c<MH>(a.ix.codesB, pp[j]);
                    }
#pragma unroll
                    for (int j = 0; j < kWideU; ++j) {
                        const int uu = u0 + 64 * j + lane;
                        if (uu < ue) {
                            const float d = dist[tt[j]] + (OD ? od_sum(cv[j]) : lsum<MH>(lut, cv[j]));
                            dist[tt[j]] = d;
                            if (!last) continue;
                            keep(d, tt[j]);
                            if (a.dbg_pos) {
                                a.dbg_pos[(int64_t)slot * a.dbg_cap + tt[j]] = pp[j];
                                a.dbg_d[(int64_t)slot * a.dbg_cap + tt[j]] = d;
                            }
                        }
                    }
                }
                tk = tn;
                b = bn;
                continue;
            }
            int y0 = ch == 0 ? yb : last_le(t_cmp, yb, ye, us);
            for (int u0 = us; u0 < ue; u0 += 64) {
                const int y = y0 + lane;
                int32_t pre = 0, cs = 0;
                int64_t beg = 0;
                bool vc = false;
                if (y < ye) {
                    pre = t_cmp[y];
                    vc = pre < u0 + 64;
                    const int e = t_cmc[y];
                    cs = t_cs[e];
                    beg = t_beg[e];
                }
                const int sr = pre > u0 ? pre - u0 : 0;
                const uint64_t mask = wave_or64(vc ? (1ull << sr) : 0ull);
                const int owner = __popcll(mask & below_lane) - 1;
                const int32_t preo = __shfl(pre, owner);
                const int32_t cso = __shfl(cs, owner);
                const int64_t bego = __shfl(beg, owner);
                const int uu = u0 + lane;
                if (uu < ue) {
                    const int64_t t = cso + (uu - preo);
                    const int64_t p = bego + (t - cso);
                    const auto code = load_c<MH>(a.ix.codesB, p);
                    const float d = dist[t] + (OD ? od_sum(code) : lsum<MH>(lut, code));
                    dist[t] = d;
                    if (last) keep(d, t);
                    if (last && a.dbg_pos) {
                        a.dbg_pos[(int64_t)slot * a.dbg_cap + t] = p;
                        a.dbg_d[(int64_t)slot * a.dbg_cap + t] = d;
                    }
                }
                const int o63 = __shfl(owner, 63);
                int yn = y0 + o63;
                const int pren = __shfl(pre, (o63 + 1) & 63);
                if (o63 < 63 && yn + 1 < ye && pren <= u0 + 64) ++yn;
                else if (o63 == 63 && yn + 1 < ye && t_cmp[yn + 1] <= u0 + 64) ++yn;
                y0 = yn;
            }
            tk = tn;
            b = bn;
        }
    }

    // Fused selection of the kq smallest (distance, id) from the kept pairs.
    // Each wavefront finds the ceil(kq/NW)-th smallest of its kept keys; the
    // largest of these bounds tau has kq distinct candidates at or below it.
    // The kept pairs at or below tau are all the candidates at or below it
    // unless some lane dropped a key <= tau: then (or with too many keys at or
    // below tau) the query is left to k_select_dist, which reads the row.
    __shared__ uint64_t s_win[kWideWin];
    __shared__ uint32_t s_hist[256];
    __shared__ uint32_t s_tau, s_digit;
    __shared__ int s_nwin, s_unsafe, s_need, s_total;
    const int64_t qry = a.qlist ? a.qlist[slot] : slot;
    const int kq = a.k[qry];
    const int nne = h.nne;
    if (tid == 0) {
        s_nwin = 0;
        s_unsafe = 0;
        s_total = 0;
    }
    __syncthreads();
    {
        int nv = 0;
#pragma unroll
        for (int q = 0; q < kWideKeep; ++q) nv += kp[q] != ~0ull;
        for (int o = 32; o > 0; o >>= 1) nv += __shfl_xor(nv, o);
        if (lane == 0) atomicAdd(&s_total, nv);
    }
    // tau: the kq-th smallest kept key, 8 bits at a time (every key when
    // fewer than kq are kept)
    uint32_t pre = 0;
    int need = kq;
    for (int sh8 = 24; sh8 >= 0; sh8 -= 8) {
        for (int b = tid; b < 256; b += NT) s_hist[b] = 0;
        __syncthreads();
        const uint32_t hm = sh8 == 24 ? 0u : (0xffffffffu << (sh8 + 8));
#pragma unroll
        for (int q = 0; q < kWideKeep; ++q) {
            const uint32_t kk = (uint32_t)(kp[q] >> 32);
            if (kp[q] != ~0ull && (kk & hm) == (pre & hm)) atomicAdd(&s_hist[(kk >> sh8) & 255u], 1u);
        }
        __syncthreads();
        if (wv == 0) {
            uint32_t c[4], sum = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                c[q] = s_hist[lane * 4 + q];
                sum += c[q];
            }
            uint32_t x = sum;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(x, o);
                if (lane >= o) x += y;
            }
            uint32_t before = x - sum;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (before < (uint32_t)need && before + c[q] >= (uint32_t)need) {
                    s_digit = lane * 4 + q;
                    s_need = need - (int)before;
                }
                before += c[q];
            }
        }
        __syncthreads();
        pre |= s_digit << sh8;
        need = s_need;
        __syncthreads();
    }
    if (tid == 0) s_tau = s_total >= kq ? pre : 0xffffffffu;
    __syncthreads();
    const uint32_t tau = s_tau;
    if (dmin <= tau) s_unsafe = 1;  // a dropped candidate lies at or below tau
    __syncthreads();
    auto append = [&](bool pred, uint64_t kk) __attribute__((always_inline)) {
        const uint64_t m = __ballot(pred);
        if (m) {
            int base = 0;
            if (lane == 0) base = atomicAdd(&s_nwin, (int)__popcll(m));
            base = __shfl(base, 0);
            if (pred) {
                const int wi = base + (int)__popcll(m & ((1ull << lane) - 1ull));
                if (wi < kWideWin) s_win[wi] = kk;
            }
        }
    };
    if (!s_unsafe) {
        // the kept pairs at or below tau are all the candidates at or below it
#pragma unroll
        for (int q = 0; q < kWideKeep; ++q)
            append(kp[q] != ~0ull && (uint32_t)(kp[q] >> 32) <= tau, kp[q]);
    } else {
        // a lane dropped a key <= tau (equal distances): read the whole row
        const int64_t ncand = h.ncand;
        for (int64_t t0 = 0; t0 < ncand; t0 += NT) {
            const int64_t t = t0 + tid;
            const uint32_t kk = t < ncand ? fkey(dist[t]) : 0xffffffffu;
            append(t < ncand && kk <= tau, ((uint64_t)kk << 32) | (uint32_t)t);
        }
    }
    __syncthreads();
    const int nwin = s_nwin;
    if (nwin > kWideWin) return;  // many equal distances at the bound: k_select_dist
    for (int i = tid; i < nwin; i += NT) {
        const uint64_t x = s_win[i];
        const int64_t t = (uint32_t)x;
        const int e = last_le(t_cs, 0, nne, t);
        s_win[i] = (x & 0xffffffff00000000ull) | a.ix.ids[t_beg[e] + (t - t_cs[e])];
    }
    __syncthreads();
    int64_t *oid = a.out_ids + qry * a.k_max;
    float *od = a.out_d + qry * a.k_max;
    const int nk = nwin < kq ? nwin : kq;
    for (int i = tid; i < nwin; i += NT) {
        const uint64_t x = s_win[i];
        int rank = 0;
        for (int j = 0; j < nwin; ++j) rank += s_win[j] < x;
        if (rank < nk) {
            oid[rank] = (int64_t)(uint32_t)x;
            od[rank] = unfkey((uint32_t)(x >> 32));
        }
    }
    for (int r = nk + tid; r < a.k_max; r += NT) {
        oid[r] = -1;
        od[r] = __builtin_huge_valf();
    }
    if (tid == 0) {
        a.sel_done[slot] = 1;
        if (a.stats) atomicAdd(&a.stats[kStatFused], 1ull);
    }
}

// ============================ host side =======================================
static size_t sel_bytes(int k_max)
{
    int KP = 1;
    while (KP < k_max) KP <<= 1;
    const int WCAP = KP * 2 < 256 ? 256 : KP * 2;
    return (size_t)(WCAP + KP) * 8 + (size_t)kTieCap * 4;
}

size_t scan_lds_bytes(int D, int M, int chunk, int k_max, int P)
{
    (void)P;
    const size_t f = (size_t)((D + 3) & ~3) + (size_t)M * kKc + (size_t)(M / 2) * kKc +
                     (size_t)((chunk + 3) & ~3);
    return f * 4 + sel_bytes(k_max) + (size_t)kScanCellsLds * (8 + 4 * 4);
}

template <bool TL>
static hipError_t launch_scan2(const ScanArgs &a, int64_t nslots, hipStream_t st)
{
    const size_t lds = scan_lds_bytes(a.ix.D, a.ix.M, a.chunk, a.k_max, a.P);
    const dim3 g((unsigned)nslots), b(512);
    switch (a.ix.M / 2) {
    case 1: hipLaunchKernelGGL((k_scan2<1, TL>), g, b, lds, st, a); break;
    case 2: hipLaunchKernelGGL((k_scan2<2, TL>), g, b, lds, st, a); break;
    case 4: hipLaunchKernelGGL((k_scan2<4, TL>), g, b, lds, st, a); break;
    case 8: hipLaunchKernelGGL((k_scan2<8, TL>), g, b, lds, st, a); break;
    case 16: hipLaunchKernelGGL((k_scan2<16, TL>), g, b, lds, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_scan(const ScanArgs &a, int64_t nslots, hipStream_t st)
{
    if (nslots == 0) return hipSuccess;
    hipError_t e = launch_scan2<true>(a, nslots, st);
    if (e != hipSuccess) return e;
    return launch_scan2<false>(a, nslots, st);
}

// LDS a workgroup of `kernel` holds before its dynamic part (its __shared__
// arrays); a dispatch asks for that plus the dynamic bytes, within 160 KiB
static size_t static_lds(const void *kernel)
{
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, kernel) != hipSuccess) {
        (void)hipGetLastError();
        return 16 * 1024;  // unknown: keep a wide margin
    }
    return fa.sharedSizeBytes;
}

// LDS left for the dynamic part of a k_scan_wide<MH, MODE> workgroup
template <int MH, int MODE>
static size_t wide_budget()
{
    static const size_t b = 160 * 1024 - static_lds(reinterpret_cast<const void *>(&k_scan_wide<MH, MODE>));
    return b;
}

void scan_wide_prepare(int M)
{
    switch (M / 2) {
#define FBPQ_WIDE_PREP(MH)                    \
    case MH:                                  \
        (void)wide_budget<MH, kWideFbpq>();   \
        (void)wide_budget<MH, kWideLocal>();  \
        (void)wide_budget<MH, kWideOD>();     \
        break;
        FBPQ_WIDE_PREP(1)
        FBPQ_WIDE_PREP(2)
        FBPQ_WIDE_PREP(4)
        FBPQ_WIDE_PREP(8)
        FBPQ_WIDE_PREP(16)
#undef FBPQ_WIDE_PREP
    default: break;
    }
}

hipError_t launch_scan_wide(const ScanArgs &a, int64_t nslots, hipStream_t st)
{
    if (nslots == 0) return hipSuccess;
    const dim3 g((unsigned)nslots);
    // rows (pass 1) and columns (pass 2) of a diagram are at most P each
    const size_t extra = (size_t)wide_ranks(a.P) * sizeof(int) + (size_t)a.ix.D * sizeof(float);
    const int mode = a.ix.od ? kWideOD : (a.ix.local ? kWideLocal : kWideFbpq);
#define FBPQ_WIDE_MODE(MH, MODE)                                                                  \
    {                                                                                             \
        constexpr int nt = 64 * wide_waves<MH, MODE>();                                           \
        const size_t budget = wide_budget<MH, MODE>();                                            \
        ScanArgs b = a;                                                                           \
        b.od_group = MH; /* O(D): the most subspaces whose codebooks fit in LDS at once */        \
        while (b.od_group > 0 &&                                                                  \
               (size_t)wide_region_floats<MH, MODE>(a.ix.D, b.od_group) * sizeof(float) + extra > \
                   budget)                                                                        \
            --b.od_group;                                                                         \
        const size_t lds =                                                                        \
            (size_t)wide_region_floats<MH, MODE>(a.ix.D, b.od_group) * sizeof(float) + extra;     \
        if (lds > budget) return hipErrorInvalidValue;                                            \
        hipLaunchKernelGGL((k_scan_wide<MH, MODE>), g, dim3(nt), lds, st, b);                     \
    }
#define FBPQ_WIDE_CASE(MH)                                                                        \
    case MH:                                                                                      \
        if (mode == kWideOD) FBPQ_WIDE_MODE(MH, kWideOD)                                          \
        else if (mode == kWideLocal) FBPQ_WIDE_MODE(MH, kWideLocal)                               \
        else FBPQ_WIDE_MODE(MH, kWideFbpq)                                                        \
        break;
    switch (a.ix.M / 2) {
        FBPQ_WIDE_CASE(1)
        FBPQ_WIDE_CASE(2)
        FBPQ_WIDE_CASE(4)
        FBPQ_WIDE_CASE(8)
        FBPQ_WIDE_CASE(16)
    default: return hipErrorInvalidValue;
    }
#undef FBPQ_WIDE_CASE
#undef FBPQ_WIDE_MODE
    return hipGetLastError();
}

}  // namespace fbpq
