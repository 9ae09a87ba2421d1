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
//
// One workgroup (8 wavefronts) per query. LQ (M x 256 floats) is built in LDS.
// The visited cells form a Young diagram in rank space, so candidates are
// scored in two passes over an LDS array of partial sums: pass 1 walks the
// rows (fixed i) with LUT1 = LQ[k<M/2] + CR1[i] folded in LDS and reads the
// first M/2 code bytes; pass 2 walks the columns (fixed j) with LUT2 =
// LQ[k>=M/2] + CR2[j] and reads the last M/2 bytes (codes are stored as two
// half planes, so each pass reads only its bytes). Each CR row is read once per
// query rather than once per cell, and a candidate costs M LDS lookups.
//
// Within a row (or column) the candidates of its nonempty cells are numbered
// contiguously; a wavefront takes 64 consecutive candidates, and each lane finds
// its cell from a 64-bit mask of the cell starts inside the window.
// Candidates are processed in chunks of `chunk`; after each chunk the k smallest
// (distance, id) are kept: value bins narrow down to a boundary bin, everything
// up to it is sorted by (distance, id).
#include "fbpq_dev.h"

namespace fbpq {

namespace {

constexpr int kScanThreads = 512;
constexpr int kNW = kScanThreads / 64;
constexpr int kSelBins = 1024;
constexpr int kTieCap = 512;

__device__ __forceinline__ uint32_t fkey(float f)
{
    const uint32_t b = __float_as_uint(f);
    return b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u);
}

__device__ __forceinline__ float unfkey(uint32_t k)
{
    const uint32_t b = (k & 0x80000000u) ? (k ^ 0x80000000u) : ~k;
    return __uint_as_float(b);
}

__device__ __forceinline__ uint64_t wave_or64(uint64_t v)
{
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
    return v;
}

template <int MH>
__device__ __forceinline__ float lut_sum(const float *lut, const uint8_t *__restrict__ codes, int64_t p)
{
    float s = 0.f;
    if constexpr (MH == 4) {
        const uint32_t c = *reinterpret_cast<const uint32_t *>(codes + p * 4);
#pragma unroll
        for (int k = 0; k < 4; ++k) s += lut[k * kKc + ((c >> (8 * k)) & 255)];
    } else if constexpr (MH == 8) {
        const uint2 c = *reinterpret_cast<const uint2 *>(codes + p * 8);
#pragma unroll
        for (int k = 0; k < 4; ++k) s += lut[k * kKc + ((c.x >> (8 * k)) & 255)];
#pragma unroll
        for (int k = 0; k < 4; ++k) s += lut[(k + 4) * kKc + ((c.y >> (8 * k)) & 255)];
    } else if constexpr (MH == 16) {
        const uint4 c = *reinterpret_cast<const uint4 *>(codes + p * 16);
        const uint32_t cw[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int k = 0; k < 4; ++k) s += lut[(q * 4 + k) * kKc + ((cw[q] >> (8 * k)) & 255)];
    } else {
#pragma unroll
        for (int k = 0; k < MH; ++k) s += lut[k * kKc + codes[p * MH + k]];
    }
    return s;
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

template <int MH, bool TAB_LDS>
__global__ __launch_bounds__(kScanThreads) void k_scan(ScanArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t hist[kSelBins];
    __shared__ uint32_t red32[kNW];
    __shared__ int redi[kNW];
    __shared__ int s_bin, s_nwin, s_nties, s_alo, s_ahi;
    __shared__ uint32_t s_before, s_cnt;

    constexpr int M = 2 * MH;
    const int slot = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t qs = a.qlist ? a.qlist[slot] : slot;
    const TravHdr h = a.hdr[slot];
    if (h.status != kStOk) return;
    if (TAB_LDS != (h.nne <= kScanCellsLds)) return;
    const int D = a.ix.D, ds = D / M, P = a.P;
    const int kq = a.k[qs];
    int KP = 1;
    while (KP < a.k_max) KP <<= 1;
    const int WCAP = KP * 2 < 256 ? 256 : KP * 2;

    // ---- LDS carve-up (see scan_lds_bytes)
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
        for (int e = tid; e < nne; e += kScanThreads) {
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

    const float *qg = a.q + qs * D;
    for (int t = tid; t < D; t += kScanThreads) qv[t] = qg[t];
    __syncthreads();
    // LQ[k][r] = ||R_k(r)||^2 - 2 <q|k, R_k(r)>   (the query part of the ADC table, Section 2.1)
    for (int e = tid; e < M * kKc; e += kScanThreads) {
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

        // ---- pass 1: rows, first half of the code, plus the cell constant
        for (int ar = alo; ar <= ahi; ++ar) {
            const int64_t rs = row_cand[ar] > c0 ? row_cand[ar] : c0;
            const int64_t re = row_cand[ar + 1] < c1 ? row_cand[ar + 1] : c1;
            if (rs >= re) continue;
            __syncthreads();
            const float *cr = a.ix.CR1 + (int64_t)u[ar] * MH * kKc;
            for (int e = tid; e < MH * kKc; e += kScanThreads) LUT[e] = LQ[e] + cr[e];
            __syncthreads();
            const int xb = row_ne[ar], xe = row_ne[ar + 1];
            for (int64_t t0 = rs + 64 * wv; t0 < re; t0 += 64 * kNW) {
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
        // ---- pass 2: columns, second half of the code
        for (int b = 0; b < B; ++b) {
            const int yb = col_ne[b], ye = col_ne[b + 1];
            if (yb >= ye) continue;
            const int U = col_tot[b];
            __syncthreads();
            const float *cr = a.ix.CR2 + (int64_t)v[b] * MH * kKc;
            for (int e = tid; e < MH * kKc; e += kScanThreads) LUT[e] = LQ[MH * kKc + e] + cr[e];
            __syncthreads();
            for (int u0 = 64 * wv; u0 < U; u0 += 64 * kNW) {
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

        // ---- keep the kq smallest (distance, id) of part[0..n) and run[0..nrun)
        const int ntot = n + nrun;
        auto key_of = [&](int e) -> uint32_t {
            return e < n ? fkey(part[e]) : (uint32_t)(run[e - n] >> 32);
        };
        auto id_of = [&](int e) -> uint32_t {
            if (e >= n) return (uint32_t)run[e - n];
            const int64_t t = c0 + e;
            const int x = last_le(t_cs, 0, nne, t);
            return a.ix.ids[t_beg[x] + (t - t_cs[x])];
        };
        if (tid == 0) {
            s_nwin = 0;
            s_nties = 0;
        }
        __syncthreads();
        if (ntot <= kq) {
            for (int e = tid; e < ntot; e += kScanThreads) {
                const int wi = atomicAdd(&s_nwin, 1);
                if (wi < WCAP) win[wi] = ((uint64_t)key_of(e) << 32) | id_of(e);
            }
        } else {
            uint32_t mn = 0xffffffffu, mx = 0;
            for (int e = tid; e < ntot; e += kScanThreads) {
                const uint32_t k = key_of(e);
                mn = k < mn ? k : mn;
                mx = k > mx ? k : mx;
            }
            for (int o = 32; o > 0; o >>= 1) {
                const uint32_t x1 = __shfl_xor(mn, o), x2 = __shfl_xor(mx, o);
                mn = x1 < mn ? x1 : mn;
                mx = x2 > mx ? x2 : mx;
            }
            if (lane == 0) red32[wv] = mn;
            __syncthreads();
            uint32_t lo = red32[0];
            for (int i = 1; i < kNW; ++i) lo = red32[i] < lo ? red32[i] : lo;
            __syncthreads();
            if (lane == 0) red32[wv] = mx;
            __syncthreads();
            uint32_t hi = red32[0];
            for (int i = 1; i < kNW; ++i) hi = red32[i] > hi ? red32[i] : hi;
            int need = kq;  // winners still to find among keys in [lo, hi]
            bool collected = false;
            for (int level = 0; level < 8 && hi > lo; ++level) {
                const uint64_t width = (uint64_t)(hi - lo) + 1ull;
                __syncthreads();
                for (int bb = tid; bb < kSelBins; bb += kScanThreads) hist[bb] = 0;
                __syncthreads();
                for (int e = tid; e < ntot; e += kScanThreads) {
                    const uint32_t k = key_of(e);
                    if (k >= lo && k <= hi) atomicAdd(&hist[(uint32_t)(((uint64_t)(k - lo) * kSelBins) / width)], 1u);
                }
                __syncthreads();
                if (tid < 64) {
                    constexpr int per = kSelBins / 64;
                    uint32_t c[per], sum = 0;
                    for (int j = 0; j < per; ++j) {
                        c[j] = hist[tid * per + j];
                        sum += c[j];
                    }
                    uint32_t x = sum;
                    for (int o = 1; o < 64; o <<= 1) {
                        const uint32_t y = __shfl_up(x, o);
                        if (tid >= o) x += y;
                    }
                    uint32_t before = x - sum;
                    for (int j = 0; j < per; ++j) {
                        if (before < (uint32_t)need && before + c[j] >= (uint32_t)need) {
                            s_bin = tid * per + j;
                            s_before = before;
                            s_cnt = c[j];
                        }
                        before += c[j];
                    }
                }
                __syncthreads();
                const uint32_t bstar = (uint32_t)s_bin;
                const int before = (int)s_before, cntb = (int)s_cnt;
                // key range of the boundary bin
                uint32_t bmn = 0xffffffffu, bmx = 0;
                for (int e = tid; e < ntot; e += kScanThreads) {
                    const uint32_t k = key_of(e);
                    if (k >= lo && k <= hi && (uint32_t)(((uint64_t)(k - lo) * kSelBins) / width) == bstar) {
                        bmn = k < bmn ? k : bmn;
                        bmx = k > bmx ? k : bmx;
                    }
                }
                for (int o = 32; o > 0; o >>= 1) {
                    const uint32_t x1 = __shfl_xor(bmn, o), x2 = __shfl_xor(bmx, o);
                    bmn = x1 < bmn ? x1 : bmn;
                    bmx = x2 > bmx ? x2 : bmx;
                }
                __syncthreads();
                if (lane == 0) red32[wv] = bmn;
                __syncthreads();
                uint32_t nlo = red32[0];
                for (int i = 1; i < kNW; ++i) nlo = red32[i] < nlo ? red32[i] : nlo;
                __syncthreads();
                if (lane == 0) red32[wv] = bmx;
                __syncthreads();
                uint32_t nhi = red32[0];
                for (int i = 1; i < kNW; ++i) nhi = red32[i] > nhi ? red32[i] : nhi;
                const int total = (kq - need) + before + cntb;  // keys <= nhi
                if (total <= WCAP) {
                    for (int e = tid; e < ntot; e += kScanThreads) {
                        const uint32_t k = key_of(e);
                        if (k <= nhi) {
                            const int wi = atomicAdd(&s_nwin, 1);
                            if (wi < WCAP) win[wi] = ((uint64_t)k << 32) | id_of(e);
                        }
                    }
                    collected = true;
                    break;
                }
                need -= before;
                lo = nlo;
                hi = nhi;
            }
            if (!collected) {
                // all remaining candidates share the key lo: keys below lo are in,
                // then the `need` smallest ids among the ties
                int my_eq = 0;
                for (int e = tid; e < ntot; e += kScanThreads) {
                    const uint32_t k = key_of(e);
                    if (k < lo) {
                        const int wi = atomicAdd(&s_nwin, 1);
                        if (wi < WCAP) win[wi] = ((uint64_t)k << 32) | id_of(e);
                    } else if (k == lo) {
                        ++my_eq;
                    }
                }
                for (int o = 32; o > 0; o >>= 1) my_eq += __shfl_xor(my_eq, o);
                __syncthreads();
                if (lane == 0) redi[wv] = my_eq;
                __syncthreads();
                int n_eq = 0;
                for (int i = 0; i < kNW; ++i) n_eq += redi[i];
                const bool buffered = n_eq <= kTieCap;
                if (buffered) {
                    for (int e = tid; e < ntot; e += kScanThreads)
                        if (key_of(e) == lo) {
                            const int ti = atomicAdd(&s_nties, 1);
                            if (ti < kTieCap) tie[ti] = id_of(e);
                        }
                }
                __syncthreads();
                uint32_t last = 0;
                for (int r = 0; r < need; ++r) {
                    uint32_t m = 0xffffffffu;
                    if (buffered) {
                        for (int e = tid; e < n_eq; e += kScanThreads) {
                            const uint32_t id = tie[e];
                            if ((r == 0 || id > last) && id < m) m = id;
                        }
                    } else {
                        for (int e = tid; e < ntot; e += kScanThreads) {
                            if (key_of(e) != lo) continue;
                            const uint32_t id = id_of(e);
                            if ((r == 0 || id > last) && id < m) m = id;
                        }
                    }
                    for (int o = 32; o > 0; o >>= 1) {
                        const uint32_t x1 = __shfl_xor(m, o);
                        m = x1 < m ? x1 : m;
                    }
                    __syncthreads();
                    if (lane == 0) red32[wv] = m;
                    __syncthreads();
                    uint32_t mm = red32[0];
                    for (int i = 1; i < kNW; ++i) mm = red32[i] < mm ? red32[i] : mm;
                    if (tid == 0) {
                        const int wi = atomicAdd(&s_nwin, 1);
                        if (wi < WCAP) win[wi] = ((uint64_t)lo << 32) | mm;
                    }
                    last = mm;
                }
            }
        }
        __syncthreads();
        // sort the collected (distance key, id) pairs; the first kq are the new running list
        const int nwin = s_nwin < WCAP ? s_nwin : WCAP;
        int S = 1;
        while (S < nwin) S <<= 1;
        for (int e = nwin + tid; e < S; e += kScanThreads) win[e] = ~0ull;
        __syncthreads();
        for (int size = 2; size <= S; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int t = tid; t < S / 2; t += kScanThreads) {
                    const int lo2 = 2 * t - (t & (stride - 1));
                    const int hi2 = lo2 + stride;
                    const bool up = (lo2 & size) == 0;
                    const uint64_t x0 = win[lo2], x1 = win[hi2];
                    if ((x0 > x1) == up) {
                        win[lo2] = x1;
                        win[hi2] = x0;
                    }
                }
                __syncthreads();
            }
        }
        const int nkeep = nwin < kq ? nwin : kq;
        for (int e = tid; e < nkeep; e += kScanThreads) run[e] = win[e];
        nrun = nkeep;
        __syncthreads();
    }

    int64_t *oid = a.out_ids + qs * a.k_max;
    float *od = a.out_d + qs * a.k_max;
    for (int r = tid; r < a.k_max; r += kScanThreads) {
        if (r < nrun && r < kq) {
            oid[r] = (int64_t)(uint32_t)run[r];
            od[r] = unfkey((uint32_t)(run[r] >> 32));
        } else {
            oid[r] = -1;
            od[r] = __builtin_huge_valf();
        }
    }
}

size_t scan_lds_bytes(int D, int M, int chunk, int k_max, int P)
{
    (void)P;
    int KP = 1;
    while (KP < k_max) KP <<= 1;
    const int WCAP = KP * 2 < 256 ? 256 : KP * 2;
    const size_t f = (size_t)((D + 3) & ~3) + (size_t)M * kKc + (size_t)(M / 2) * kKc +
                     (size_t)((chunk + 3) & ~3);
    return f * 4 + (size_t)(WCAP + KP) * 8 + (size_t)kTieCap * 4 + (size_t)kScanCellsLds * (8 + 4 * 4);
}

template <bool TL>
static hipError_t launch_scan_t(const ScanArgs &a, int64_t nslots, hipStream_t st)
{
    const size_t lds = scan_lds_bytes(a.ix.D, a.ix.M, a.chunk, a.k_max, a.P);
    const dim3 g((unsigned)nslots), b(kScanThreads);
    switch (a.ix.M / 2) {
    case 1: hipLaunchKernelGGL((k_scan<1, TL>), g, b, lds, st, a); break;
    case 2: hipLaunchKernelGGL((k_scan<2, TL>), g, b, lds, st, a); break;
    case 4: hipLaunchKernelGGL((k_scan<4, TL>), g, b, lds, st, a); break;
    case 8: hipLaunchKernelGGL((k_scan<8, TL>), g, b, lds, st, a); break;
    case 16: hipLaunchKernelGGL((k_scan<16, TL>), g, b, lds, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_scan(const ScanArgs &a, int64_t nslots, hipStream_t st)
{
    if (nslots == 0) return hipSuccess;
    // queries whose nonempty-cell tables fit in LDS, then the others
    hipError_t e = launch_scan_t<true>(a, nslots, st);
    if (e != hipSuccess) return e;
    return launch_scan_t<false>(a, nslots, st);
}

}  // namespace fbpq
