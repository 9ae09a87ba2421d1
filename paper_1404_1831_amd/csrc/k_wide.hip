// Threshold-stepping form of the multi-sequence traversal (Section 2.3.3), for
// queries whose visited set is too large to pop one cell at a time.
//
// Cells are visited in ascending (key, a, b), key = fl64(k1[a] + k2[b]) over
// the rank pairs of the two sorted half lists. For a threshold t, the cells
// with key <= t form a Young diagram: row a holds the first w_t(a) cells,
// found by one binary search per row because keys grow along every row and
// column. The visited prefix is therefore grown in bands: pick t_new > t, load
// the point counts of the cells with t < key <= t_new in parallel, and accept
// the band while the running total stays below min(L, N). The band that
// reaches min(L, N) is sorted by (key, a, b) and cut at the cell that
// completes the count. This gives exactly the cells, order and truncated last
// cell of the one-at-a-time traversal.
//
// Band sizes. A first band of a few hundred cells measures the points per
// cell. Later bands aim at part of the cells still expected, and only their
// counts are summed. The band expected to hold the cut has at most kWCap
// cells, so that it fits in LDS for the sort. A summed band that overshoots
// is dropped and a smaller one is taken. A band whose cells all share one key
// (t and t_new adjacent doubles) is already in (a, b) order; it is walked in
// chunks of kWCap cells.
//
// One workgroup per query; thread t owns rows a = t + NT r (r < kWRows).
// Queries whose visited set exceeds the cell capacity keep counting (without
// writing cells) so that the header reports the capacity they need.
#include "fbpq_dev.h"

namespace fbpq {

constexpr int kWRows = 8;      // rows per thread: P <= NT * kWRows
constexpr int kWCap = 2048;    // cells of a band held in LDS
constexpr int kWPos = 8;       // band positions per thread per pass
constexpr int64_t kWHardCells = (int64_t)1 << 26;  // counting past the capacity stops here

// order-preserving map of doubles to unsigned integers, and its inverse
__device__ __forceinline__ uint64_t dord(double x)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ double dunord(uint64_t o)
{
    const uint64_t b = (o >> 63) ? (o & 0x7fffffffffffffffull) : ~o;
    return __longlong_as_double((long long)b);
}

template <int NT>
__device__ __forceinline__ int64_t wg_sum(int64_t v, int64_t *red)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int64_t r = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) r += red[i];
    return r;
}

template <int NT>
__device__ __forceinline__ int64_t wg_min(int64_t v, int64_t *red)
{
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t x = __shfl_xor(v, o);
        v = x < v ? x : v;
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int64_t r = red[0];
#pragma unroll
    for (int i = 1; i < NT / 64; ++i) r = red[i] < r ? red[i] : r;
    return r;
}

// exclusive prefix of v over the workgroup in thread order; *total gets the sum
template <int NT>
__device__ __forceinline__ int64_t wg_scan(int64_t v, int64_t *red, int64_t *total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int64_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == 63) red[wv] = x;
    __syncthreads();
    int64_t before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        const int64_t t = red[i];
        before += i < wv ? t : 0;
        tot += t;
    }
    *total = tot;
    return before + x - v;
}

// Row widths at threshold t: out[r] = first b in [lo[r], hi[r]) with
// k1r[r] + k2s[b] > t (hi[r] if none). All rows step together.
__device__ __forceinline__ void widths_at(double t, const double *k1r, const int *lo0, const int *hi0, int *out,
                                          const double *k2s)
{
    int lo[kWRows], hi[kWRows];
#pragma unroll
    for (int r = 0; r < kWRows; ++r) {
        lo[r] = lo0[r];
        hi[r] = hi0[r];
    }
    bool any = true;
    while (any) {
        any = false;
#pragma unroll
        for (int r = 0; r < kWRows; ++r) {
            if (lo[r] < hi[r]) {
                const int mid = (lo[r] + hi[r]) >> 1;
                if (k1r[r] + k2s[mid] <= t) lo[r] = mid + 1;
                else hi[r] = mid;
                any |= lo[r] < hi[r];
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kWRows; ++r) out[r] = lo[r];
}

// (a, b) of band positions xs[e] (rowpre: exclusive prefix of the row lengths,
// wsh: first band column of each row). Positions must be < rowpre[P].
__device__ __forceinline__ void locate(const int *xs, int n, const int *rowpre, const int *wsh, int P, int *as,
                                       int *bs)
{
    int lo[kWPos], hi[kWPos];
#pragma unroll
    for (int e = 0; e < kWPos; ++e) {
        lo[e] = 0;
        hi[e] = e < n ? P - 1 : 0;
    }
    bool any = true;
    while (any) {
        any = false;
#pragma unroll
        for (int e = 0; e < kWPos; ++e) {
            if (lo[e] < hi[e]) {
                const int mid = (lo[e] + hi[e] + 1) >> 1;
                if (rowpre[mid] <= xs[e]) lo[e] = mid;
                else hi[e] = mid - 1;
                any |= lo[e] < hi[e];
            }
        }
    }
#pragma unroll
    for (int e = 0; e < kWPos; ++e) {
        as[e] = lo[e];
        bs[e] = e < n ? wsh[lo[e]] + (xs[e] - rowpre[lo[e]]) : 0;
    }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_traverse_wide(TravArgs args)
{
    constexpr int R = kWRows;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int64_t red[NT / 64];
    __shared__ int64_t s_cut[4];
    const int P = args.P;
    const int slot = blockIdx.x;
    const int tid = threadIdx.x;
    if (!args.wide_all && args.hdr[slot].status != kStDefer) return;
    double *k2s = reinterpret_cast<double *>(smem);                 // [P]
    double *bkey = k2s + P;                                         // [kWCap]
    int64_t *bcnt = reinterpret_cast<int64_t *>(bkey + kWCap);      // [kWCap]
    int *wsh = reinterpret_cast<int *>(bcnt + kWCap);               // [P]
    int *rowpre = wsh + P;                                          // [P + 1]
    uint32_t *bab = reinterpret_cast<uint32_t *>(rowpre + P + 1);   // [kWCap]

    const int64_t qs = args.qlist ? args.qlist[slot] : slot;
    const int T = args.ix.T;
    const double *k1 = args.lkey + (int64_t)slot * 2 * P;
    const double *k2 = k1 + P;
    const int32_t *u = args.lidx + (int64_t)slot * 2 * P;
    const int32_t *v = u + P;
    const int64_t *off = args.ix.offsets;
    for (int i = tid; i < P; i += NT) k2s[i] = k2[i];
    if (args.stats && tid == 0) atomicAdd(&args.stats[kStatWide], 1ull);
    __syncthreads();

    const int64_t L = args.L[qs];
    const int64_t Leff = L < args.ix.N ? L : args.ix.N;
    const bool full = P >= T;
    const double INF = __builtin_huge_val();
    const double DMAX = 1.7976931348623157e308;
    // every visited cell has key <= tmax: below the smallest key outside the
    // P x P window, or the largest key when the lists are complete
    double tmax;
    if (full) {
        tmax = k1[P - 1] + k2s[P - 1];
    } else {
        const double kb = fmin(k1[P - 1] + k2s[0], k1[0] + k2s[P - 1]);
        tmax = dunord(dord(kb) - 1);
    }
    if (!(tmax < INF)) tmax = DMAX;

    double k1r[R];
    int w[R], wmax[R], wn[R];
    {
        int zero[R], top[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int a = tid + NT * r;
            k1r[r] = a < P ? k1[a] : INF;
            w[r] = 0;
            zero[r] = 0;
            top[r] = a < P ? P : 0;
        }
        widths_at(tmax, k1r, zero, top, wmax, k2s);
    }
    int64_t my = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) my += wmax[r];
    const int64_t navail = wg_sum<NT>(my, red);

    int64_t tot = 0, nc = 0;
    double tcur = dunord(dord(k1[0] + k2s[0]) - 1);  // below every key: nothing visited
    double rho = -1.0;                               // points per cell of the last band
    int status = kStOk;
    bool done = Leff <= 0;
    bool over = false;  // visited cells exceed the capacity: count only
    int cut_a = -1, cut_b = -1;
    int64_t cut_take = 0;
    const bool dbg = args.dbg_ab != nullptr;
    int64_t n_bands = 0, n_evals = 1, n_loads = 0;  // path counters (thread 0's copies)

    while (!done) {
        const int64_t need = Leff - tot;
        const int64_t rem = navail - nc;
        if (rem <= 0) {
            status = kStNeedPrefix;
            break;
        }
        if (nc > kWHardCells) break;  // over the capacity by far: report what was counted
        // band size window [lo_t, hi_t]
        const double est = rho > 0.0 ? (double)need / rho : 384.0;
        const double e125 = est * 1.25 + 32.0;
        int64_t lo_t, hi_t;
        if (dbg || e125 <= (double)kWCap) {
            lo_t = (int64_t)fmin(e125, 0.75 * kWCap);
            hi_t = lo_t * 2 < kWCap ? lo_t * 2 : kWCap;
        } else {
            const double e = fmin(est, 4.0e15);
            lo_t = (int64_t)(0.5 * e);
            hi_t = (int64_t)(0.9 * e);
        }
        if (!over) {
            const int64_t room = args.max_cells - nc + 1;  // a band this large fails the capacity
            if (room >= 1 && hi_t > room) hi_t = room;
        }
        if (lo_t > hi_t) lo_t = hi_t;
        if (lo_t < 1) lo_t = 1;
        if (hi_t < 1) hi_t = 1;

        // choose the band (tcur, tnew]
        ++n_bands;
        double tnew;
        int64_t nb;
        bool tie = false;
        if (rem <= hi_t) {
            tnew = tmax;
#pragma unroll
            for (int r = 0; r < R; ++r) wn[r] = wmax[r];
            nb = rem;
        } else {
            double tl = tcur, th = tmax;
            int64_t cl = 0, ch = rem;
            int wl[R], wh[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                wl[r] = w[r];
                wh[r] = wmax[r];
            }
            // The cell count grows about like a power of (t - tmin): interpolate
            // log(count) against log(t - tmin) between the bracket ends; every
            // fourth step bisects the bit range, so that tl and th meet within
            // 256 steps
            const double tmin = k1[0] + k2s[0];
            const double ytg = log((double)nc + sqrt((double)lo_t * (double)hi_t));
            bool found = false;
            for (int it = 0; it < 260; ++it) {
                const uint64_t ol = dord(tl), oh = dord(th);
                if (oh - ol <= 1) break;
                double tm = 0.0;
                bool bis = (it & 3) == 3 || !(th > tmin);
                if (!bis) {
                    const double xh = log(th - tmin), yh = log((double)(nc + ch));
                    double x;
                    if (tl > tmin) {  // count at tl >= 1
                        const double xl = log(tl - tmin), yl = log((double)(nc + cl));
                        x = yh > yl ? xl + (ytg - yl) * (xh - xl) / (yh - yl) : 0.5 * (xl + xh);
                    } else {
                        x = xh + (ytg - yh) * 0.125;
                    }
                    tm = tmin + exp(x);
                    bis = !(tm > tl) || !(tm < th);
                }
                if (bis) tm = dunord(ol + (oh - ol) / 2);
                ++n_evals;
                int wm[R];
                widths_at(tm, k1r, wl, wh, wm, k2s);
                int64_t m2 = 0;
#pragma unroll
                for (int r = 0; r < R; ++r) m2 += wm[r] - w[r];
                const int64_t cm = wg_sum<NT>(m2, red);
                if (cm < lo_t) {
                    tl = tm;
                    cl = cm;
#pragma unroll
                    for (int r = 0; r < R; ++r) wl[r] = wm[r];
                } else if (cm > hi_t) {
                    th = tm;
                    ch = cm;
#pragma unroll
                    for (int r = 0; r < R; ++r) wh[r] = wm[r];
                } else {
                    tnew = tm;
#pragma unroll
                    for (int r = 0; r < R; ++r) wn[r] = wm[r];
                    nb = cm;
                    found = true;
                    break;
                }
            }
            if (!found) {
                if (cl > 0) {
                    tnew = tl;
#pragma unroll
                    for (int r = 0; r < R; ++r) wn[r] = wl[r];
                    nb = cl;
                } else {
                    tnew = th;
#pragma unroll
                    for (int r = 0; r < R; ++r) wn[r] = wh[r];
                    nb = ch;
                    tie = dord(th) - dord(tl) <= 1;  // every band cell has key th
                }
            }
        }

        // band layout: row a holds columns [wsh[a], wsh[a] + len(a)); rowpre is
        // the exclusive prefix of the lengths
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int a = tid + NT * r;
            if (a < P) {
                wsh[a] = w[r];
                rowpre[a] = wn[r] - w[r];
            }
        }
        __syncthreads();
        {
            int loc[R];
            int64_t s = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int a = tid * R + r;
                loc[r] = a < P ? rowpre[a] : 0;
                s += loc[r];
            }
            int64_t tl;
            int64_t run = wg_scan<NT>(s, red, &tl);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int a = tid * R + r;
                if (a < P) rowpre[a] = (int)run;
                run += loc[r];
            }
            if (tid == 0) rowpre[P] = (int)tl;
        }
        __syncthreads();

        n_loads += nb;
        if (nb > kWCap && !tie) {
            // Summed band, split into kSub sub-bands by threshold (th_[i], th_[i+1]]
            // with points and cells counted per sub-band. If the band completes
            // min(L, N), the sub-bands before the one that does are kept and
            // the search goes on inside that one.
            constexpr int kSub = 8;
            double th_[kSub + 1];
            th_[0] = tcur;
            th_[kSub] = tnew;
#pragma unroll
            for (int i = 1; i < kSub; ++i) {
                const double t = tcur + (tnew - tcur) * ((double)i / kSub);
                th_[i] = t > th_[i - 1] ? (t < tnew ? t : tnew) : th_[i - 1];
            }
            int64_t sub[kSub];  // (points << 25) | cells, this thread's share
#pragma unroll
            for (int i = 0; i < kSub; ++i) sub[i] = 0;
            for (int64_t x0 = 0; x0 < nb; x0 += (int64_t)NT * kWPos) {
                int xs[kWPos], as[kWPos], bs[kWPos];
                int n = 0;
#pragma unroll
                for (int e = 0; e < kWPos; ++e) {
                    const int64_t x = x0 + tid + (int64_t)NT * e;
                    xs[e] = (int)x;
                    n += x < nb;
                }
                locate(xs, n, rowpre, wsh, P, as, bs);
#pragma unroll
                for (int e = 0; e < kWPos; ++e) {
                    if (e < n) {
                        const int64_t c = (int64_t)u[as[e]] * T + v[bs[e]];
                        const int64_t cnt = off[c + 1] - off[c];
                        const double key = k1[as[e]] + k2s[bs[e]];
                        int js = 0;
#pragma unroll
                        for (int i = 1; i < kSub; ++i) js += key > th_[i];
                        const int64_t add = (cnt << 25) | 1;
#pragma unroll
                        for (int i = 0; i < kSub; ++i) sub[i] += js == i ? add : 0;
                    }
                }
            }
            int64_t spts[kSub], scel[kSub];
#pragma unroll
            for (int i = 0; i < kSub; ++i) {
                const int64_t v2 = wg_sum<NT>(sub[i], red);
                spts[i] = v2 >> 25;
                scel[i] = v2 & ((1ll << 25) - 1);
            }
            int jcut = -1;
            int64_t pbefore = 0, cbefore = 0;
#pragma unroll
            for (int i = 0; i < kSub; ++i) {
                if (jcut < 0) {
                    if (tot + pbefore + spts[i] >= Leff) jcut = i;
                    else {
                        pbefore += spts[i];
                        cbefore += scel[i];
                    }
                }
            }
            if (jcut < 0) {
                tot += pbefore;
                nc += nb;
                tcur = tnew;
#pragma unroll
                for (int r = 0; r < R; ++r) w[r] = wn[r];
                rho = fmax((double)pbefore, 0.5) / (double)nb;
            } else {
                double tj = th_[0];
#pragma unroll
                for (int i = 1; i < kSub; ++i)
                    if (i == jcut) tj = th_[i];
                if (jcut > 0) {
                    // keep the sub-bands below jcut: cells with key <= tj
                    int wa[R];
                    widths_at(tj, k1r, w, wn, wa, k2s);
                    ++n_evals;
                    tot += pbefore;
                    nc += cbefore;
                    tcur = tj;
#pragma unroll
                    for (int r = 0; r < R; ++r) w[r] = wa[r];
                }
                int64_t pj = 0, cj = 1;
#pragma unroll
                for (int i = 0; i < kSub; ++i)
                    if (i == jcut) {
                        pj = spts[i];
                        cj = scel[i] > 0 ? scel[i] : 1;
                    }
                rho = fmax((double)pj, 0.5) / (double)cj;
            }
            if (nc > args.max_cells) over = true;
            continue;
        }

        // stored band (nb <= kWCap), or an equal-key band in (a, b) order
        const int64_t nc0 = nc;
        int64_t bsum = 0;
        for (int64_t x0 = 0; x0 < nb && !done; x0 += kWCap) {
            const int n = (int)(nb - x0 < kWCap ? nb - x0 : kWCap);
            int npad = 64;
            while (npad < n) npad <<= 1;
            int64_t s = 0;
            for (int i0 = 0; i0 < npad; i0 += NT * kWPos) {
                int xs[kWPos], as[kWPos], bs[kWPos];
                int nv = 0;
#pragma unroll
                for (int e = 0; e < kWPos; ++e) {
                    const int i = i0 + tid + NT * e;
                    xs[e] = (int)(x0 + i);
                    nv += i < n;
                }
                locate(xs, nv, rowpre, wsh, P, as, bs);
#pragma unroll
                for (int e = 0; e < kWPos; ++e) {
                    const int i = i0 + tid + NT * e;
                    if (i < n) {
                        const int64_t c = (int64_t)u[as[e]] * T + v[bs[e]];
                        const int64_t cnt = off[c + 1] - off[c];
                        bkey[i] = k1[as[e]] + k2s[bs[e]];
                        bab[i] = ((uint32_t)as[e] << 16) | (uint32_t)bs[e];
                        bcnt[i] = cnt;
                        s += cnt;
                    } else if (i < npad) {
                        bkey[i] = INF;
                        bab[i] = 0xffffffffu;
                        bcnt[i] = 0;
                    }
                }
            }
            s = wg_sum<NT>(s, red);  // its barriers also publish the LDS writes
            const bool hit = tot + s >= Leff;
            if (hit || dbg) {
                if (!tie) {
                    // bitonic sort of [0, npad) by (key, a, b)
                    for (int kk = 2; kk <= npad; kk <<= 1) {
                        for (int j = kk >> 1; j > 0; j >>= 1) {
                            for (int i = tid; i < npad / 2; i += NT) {
                                const int lo = ((i & ~(j - 1)) << 1) | (i & (j - 1));
                                const int hi = lo + j;
                                const double ka = bkey[lo], kb = bkey[hi];
                                const uint32_t aa = bab[lo], ab = bab[hi];
                                const bool gt = ka > kb || (ka == kb && aa > ab);
                                if (gt == ((lo & kk) == 0)) {
                                    bkey[lo] = kb;
                                    bkey[hi] = ka;
                                    bab[lo] = ab;
                                    bab[hi] = aa;
                                    const int64_t t = bcnt[lo];
                                    bcnt[lo] = bcnt[hi];
                                    bcnt[hi] = t;
                                }
                            }
                            __syncthreads();
                        }
                    }
                }
                // running totals in sorted order; first entry that reaches min(L, N)
                const int EP = (npad + NT - 1) / NT;
                const int i0 = tid * EP, i1 = i0 + EP < n ? i0 + EP : n;
                int64_t ls = 0;
                for (int i = i0; i < i1; ++i) ls += bcnt[i];
                int64_t ctot;
                const int64_t ex = wg_scan<NT>(ls, red, &ctot);
                int64_t run = tot + ex;
                int64_t jmine = INT64_MAX, take_mine = 0;
                for (int i = i0; i < i1; ++i) {
                    const int64_t c = bcnt[i];
                    if (hit && jmine == INT64_MAX && run + c >= Leff) {
                        jmine = i;
                        take_mine = Leff - run;  // points taken if this is the cut cell
                    }
                    run += c;
                }
                const int64_t j = hit ? wg_min<NT>(jmine, red) : INT64_MAX;
                if (hit && jmine == j) s_cut[1] = take_mine;  // one thread owns entry j
                const int nkeep = hit ? (int)j + 1 : n;
                if (dbg && !over) {
                    int64_t r2 = tot + ex;
                    for (int i = i0; i < i1 && i < nkeep; ++i) {
                        const int64_t o = nc0 + x0 + i;
                        const int64_t c = bcnt[i];
                        if (o < args.max_cells) {
                            const int a = (int)(bab[i] >> 16), b = (int)(bab[i] & 0xffffu);
                            const int64_t cell = (int64_t)u[a] * T + v[b];
                            const int64_t so = (int64_t)slot * args.max_cells + o;
                            args.dbg_ab[2 * so] = a;
                            args.dbg_ab[2 * so + 1] = b;
                            args.dbg_take[so] = i == j ? Leff - r2 : c;
                            args.dbg_beg[so] = off[cell];
                        }
                        r2 += c;
                    }
                }
                if (hit) {
                    __syncthreads();
                    const uint32_t abj = bab[j];
                    cut_a = (int)(abj >> 16);
                    cut_b = (int)(abj & 0xffffu);
                    cut_take = s_cut[1];
                    // widths: cells of earlier chunks (row-major positions < x0),
                    // then the kept entries of this chunk, counted per row
                    int base[R];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int a = tid + NT * r;
                        base[r] = 0;
                        if (a < P) {
                            const int64_t f = x0 - rowpre[a];
                            const int len = wn[r] - w[r];
                            base[r] = f <= 0 ? 0 : (f >= len ? len : (int)f);
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int a = tid + NT * r;
                        if (a < P) rowpre[a] = 0;
                    }
                    __syncthreads();
                    for (int i = tid; i <= (int)j; i += NT) atomicAdd(&rowpre[bab[i] >> 16], 1);
                    __syncthreads();
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int a = tid + NT * r;
                        if (a < P) w[r] += base[r] + rowpre[a];
                    }
                    nc = nc0 + x0 + nkeep;
                    tot = Leff;
                    if (nc > args.max_cells) over = true;
                    done = true;
                }
            }
            if (!done) {
                tot += s;
                bsum += s;
            }
            __syncthreads();
        }
        if (!done) {
            nc = nc0 + nb;
            tcur = tnew;
#pragma unroll
            for (int r = 0; r < R; ++r) w[r] = wn[r];
            rho = fmax((double)bsum, 0.5) / (double)nb;
            if (nc > args.max_cells) over = true;
        }
    }
    if (status == kStOk && (over || !done)) status = kStNeedCells;

    // outputs, as the one-at-a-time kernel writes them
    int myA = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int a = tid + NT * r;
        if (a < P) {
            args.w[(int64_t)slot * P + a] = w[r];
            myA += w[r] > 0;
        }
    }
    const int64_t A = wg_sum<NT>(myA, red);
    if (tid == 0) {
        TravHdr h;
        h.status = status;
        h.A = (int32_t)A;
        h.B = w[0];
        h.cut_a = cut_a;
        h.cut_b = cut_b;
        h.nne = 0;
        h.a_ne = 0;
        h.b_ne = 0;
        h.n_items = 0;
        h.gscan = 0;
        h.ncells = nc;
        h.ncand = tot;
        h.cut_take = cut_take;
        if (Leff <= 0) {
            h.A = 0;
            h.B = 0;
            h.ncells = 0;
            h.ncand = 0;
        }
        args.hdr[slot] = h;
        if (status != kStOk) args.fail_list[atomicAdd(args.fail_count, 1)] = (int32_t)qs;
        if (args.stats) {
            atomicAdd(&args.stats[kStatWideBands], (unsigned long long)n_bands);
            atomicAdd(&args.stats[kStatWideEvals], (unsigned long long)n_evals);
            atomicAdd(&args.stats[kStatWideLoads], (unsigned long long)n_loads);
        }
    }
}

size_t wide_lds_bytes(int P)
{
    return (size_t)P * 8 + (size_t)kWCap * (8 + 8) + (size_t)P * 4 + (size_t)(P + 1) * 4 + (size_t)kWCap * 4;
}

hipError_t launch_traverse_wide(const TravArgs &a, int64_t nslots, hipStream_t st)
{
    if (nslots == 0) return hipSuccess;
    const size_t lds = wide_lds_bytes(a.P);
    const dim3 g((unsigned)nslots);
    if (a.P <= 256 * kWRows) hipLaunchKernelGGL(k_traverse_wide<256>, g, dim3(256), lds, st, a);
    else if (a.P <= 512 * kWRows) hipLaunchKernelGGL(k_traverse_wide<512>, g, dim3(512), lds, st, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// ---- traversal for long prefixes (P > kMaxFastPrefix) -----------------------
// The same visited cells, order and cut as the kernels above, for prefixes
// whose per-rank arrays do not fit in LDS. Per-row state lives in this slot's
// slice of HBM (args.big): wlo, the row widths of the cells with key <= lo
// (the visited part so far); whi, the widths at hi; wm, the widths at a probe
// threshold t; pre, the exclusive prefix over rows of a band's lengths.
//
// Invariants: the cells with key <= lo hold C_lo < min(L, N) points; once
// hi_ok is set, the cells with key <= hi hold at least min(L, N). A step takes
// a threshold t in (lo, hi]: before hi_ok the largest whose band (lo, t] has at
// most kBigBand cells (searched on cell counts, which need no loads), after it
// the midpoint of (lo, hi) in the order of doubles. The band's point counts
// are loaded and summed: below the target the band is accepted (lo = t),
// otherwise hi = t. When t is the next double after lo, every cell of the band
// has key t and the band is walked in (a, b) order, chunk by chunk, up to the
// cell that completes min(L, N). Each step after hi_ok halves the range of
// doubles, so at most 64 follow.
constexpr int kBigNT = 1024;
constexpr int64_t kBigBand = 1 << 16;  // cells of a band searched by threshold
constexpr int kBigPos = 4;             // band positions per thread per step

// first b in [lo, hi) with k1a + k2[b] > t, hi if none
__device__ __forceinline__ int width_at(double t, double k1a, const double *k2, int lo, int hi)
{
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (k1a + k2[mid] <= t) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// largest a in [0, P) with pre[a] <= x (x < pre[P])
__device__ __forceinline__ int row_of(const int32_t *pre, int P, int64_t x)
{
    int lo = 0, hi = P - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int NT>
__global__ __launch_bounds__(NT) void k_traverse_big(TravArgs args)
{
    __shared__ int64_t red[NT / 64];
    __shared__ int64_t s_take;
    const int P = args.P;
    const int slot = blockIdx.x;
    const int tid = threadIdx.x;
    if (!args.wide_all && args.hdr[slot].status != kStDefer) return;
    int32_t *wlo = args.big + (int64_t)slot * big_trav_ints(P);
    int32_t *whi = wlo + P;
    int32_t *wm = whi + P;
    int32_t *pre = wm + P;  // [P + 1]

    const int64_t qs = args.qlist ? args.qlist[slot] : slot;
    const int T = args.ix.T;
    const double *k1 = args.lkey + (int64_t)slot * 2 * P;
    const double *k2 = k1 + P;
    const int32_t *u = args.lidx + (int64_t)slot * 2 * P;
    const int32_t *v = u + P;
    const int64_t *off = args.ix.offsets;
    if (args.stats && tid == 0) atomicAdd(&args.stats[kStatWide], 1ull);

    const int64_t L = args.L[qs];
    const int64_t Leff = L < args.ix.N ? L : args.ix.N;
    const double INF = __builtin_huge_val();
    const double DMAX = 1.7976931348623157e308;
    // every visited cell has key <= tmax (as in the kernels above)
    double tmax;
    if (P >= T) {
        tmax = k1[P - 1] + k2[P - 1];
    } else {
        const double kb = fmin(k1[P - 1] + k2[0], k1[0] + k2[P - 1]);
        tmax = dunord(dord(kb) - 1);
    }
    if (!(tmax < INF)) tmax = DMAX;
    for (int a = tid; a < P; a += NT) {
        wlo[a] = 0;
        whi[a] = width_at(tmax, k1[a], k2, 0, P);
    }
    __syncthreads();

    double lo = dunord(dord(k1[0] + k2[0]) - 1);  // below every key: nothing visited
    double hi = tmax;
    bool hi_ok = false;
    int64_t C_lo = 0;
    int status = kStOk;
    int cut_a = -1, cut_b = -1;
    int64_t cut_take = 0;
    bool found = Leff <= 0;
    int64_t n_bands = 0, n_evals = 1, n_loads = 0;
    const int RP = (P + NT - 1) / NT;  // rows per thread in the prefix over rows

    // band lengths wm - wlo: their exclusive prefix over rows into pre, returns the total
    auto band_prefix = [&]() -> int64_t {
        const int a0 = tid * RP, a1 = a0 + RP < P ? a0 + RP : P;
        int64_t s = 0;
        for (int a = a0; a < a1; ++a) s += wm[a] - wlo[a];
        int64_t tot;
        int64_t run = wg_scan<NT>(s, red, &tot);
        for (int a = a0; a < a1; ++a) {
            pre[a] = (int32_t)run;
            run += wm[a] - wlo[a];
        }
        if (tid == 0) pre[P] = (int32_t)tot;
        __syncthreads();
        return tot;
    };
    // widths at t into wm (rows searched between wlo and whi); returns the band's cell count
    auto widths = [&](double t) -> int64_t {
        int64_t s = 0;
        for (int a = tid; a < P; a += NT) {
            const int w = width_at(t, k1[a], k2, wlo[a], whi[a]);
            wm[a] = w;
            s += w - wlo[a];
        }
        ++n_evals;
        return wg_sum<NT>(s, red);
    };
    auto count_at = [&](int64_t x) -> int64_t {
        const int a = row_of(pre, P, x);
        const int b = wlo[a] + (int)(x - pre[a]);
        const int64_t c = (int64_t)u[a] * T + v[b];
        return off[c + 1] - off[c];
    };

    while (!found && status == kStOk) {
        const uint64_t ol = dord(lo), oh = dord(hi);
        double t;
        int64_t nb;
        ++n_bands;
        if (hi_ok) {
            if (oh - ol <= 1) {
                t = hi;
                for (int a = tid; a < P; a += NT) wm[a] = whi[a];
                __syncthreads();
                nb = -1;
            } else {
                t = dunord(ol + (oh - ol) / 2);
                nb = widths(t);
            }
        } else {
            for (int a = tid; a < P; a += NT) wm[a] = whi[a];
            int64_t s = 0;
            for (int a = tid; a < P; a += NT) s += whi[a] - wlo[a];
            nb = wg_sum<NT>(s, red);
            t = hi;
            if (nb > kBigBand) {
                // the largest t with a band of at most kBigBand cells, bisecting the doubles
                uint64_t tl = ol, th = oh;
                int64_t nl = 0;
                while (th - tl > 1) {
                    const uint64_t tm = tl + (th - tl) / 2;
                    const int64_t nm = widths(dunord(tm));
                    if (nm <= kBigBand) {
                        tl = tm;
                        nl = nm;
                        if (nm >= kBigBand / 4) break;
                    } else {
                        th = tm;
                    }
                }
                if (tl > ol) {
                    t = dunord(tl);
                    if (nl >= 0) nb = widths(t);
                } else {
                    t = dunord(th);  // the next double: one key, more than kBigBand cells
                    nb = widths(t);
                }
            }
        }
        const bool tie = dord(t) - ol <= 1;
        nb = band_prefix();
        n_loads += nb;
        if (tie) {
            // one key value: walk the band in (a, b) order up to the cell that completes min(L, N)
            int64_t run = C_lo;
            for (int64_t x0 = 0; x0 < nb && !found; x0 += (int64_t)NT * kBigPos) {
                int64_t c[kBigPos];
                int64_t s = 0;
#pragma unroll
                for (int e = 0; e < kBigPos; ++e) {
                    const int64_t x = x0 + (int64_t)tid * kBigPos + e;
                    c[e] = x < nb ? count_at(x) : 0;
                    s += c[e];
                }
                int64_t tot;
                const int64_t ex = wg_scan<NT>(s, red, &tot);
                int64_t r = run + ex, xmine = INT64_MAX, take = 0;
#pragma unroll
                for (int e = 0; e < kBigPos; ++e) {
                    const int64_t x = x0 + (int64_t)tid * kBigPos + e;
                    if (xmine == INT64_MAX && x < nb && r + c[e] >= Leff) {
                        xmine = x;
                        take = Leff - r;
                    }
                    r += c[e];
                }
                const int64_t xcut = wg_min<NT>(xmine, red);
                if (xcut != INT64_MAX) {
                    if (xmine == xcut) s_take = take;
                    __syncthreads();
                    cut_a = row_of(pre, P, xcut);
                    cut_b = wlo[cut_a] + (int)(xcut - pre[cut_a]);
                    cut_take = s_take;
                    found = true;
                } else {
                    run += tot;
                }
            }
            if (found) {
                // rows before the cut row take their whole band, the cut row up to the cut
                for (int a = tid; a < P; a += NT) {
                    if (a < cut_a) wlo[a] = wm[a];
                    else if (a == cut_a) wlo[a] = cut_b + 1;
                }
                __syncthreads();
                C_lo = Leff;
            } else {
                C_lo = run;
                lo = t;
                for (int a = tid; a < P; a += NT) wlo[a] = wm[a];
                __syncthreads();
                if (t == hi) status = kStNeedPrefix;  // every cell up to tmax taken, min(L, N) not reached
            }
            continue;
        }
        // sum the band's points
        int64_t s = 0;
        for (int64_t x = tid; x < nb; x += NT) s += count_at(x);
        const int64_t S = wg_sum<NT>(s, red);
        if (C_lo + S < Leff) {
            C_lo += S;
            lo = t;
            for (int a = tid; a < P; a += NT) wlo[a] = wm[a];
            __syncthreads();
            if (t == hi) status = kStNeedPrefix;
        } else {
            hi = t;
            hi_ok = true;
            for (int a = tid; a < P; a += NT) whi[a] = wm[a];
            __syncthreads();
        }
    }

    // outputs: final widths (wlo), as the kernels above write them
    int64_t myc = 0;
    int myA = 0;
    for (int a = tid; a < P; a += NT) {
        const int w = wlo[a];
        args.w[(int64_t)slot * P + a] = w;
        myc += w;
        myA += w > 0;
    }
    const int64_t nc = wg_sum<NT>(myc, red);
    const int64_t A = wg_sum<NT>(myA, red);
    if (status == kStOk && Leff > 0 && nc > args.max_cells) status = kStNeedCells;
    if (args.dbg_ab && status == kStOk && Leff > 0) {
        // visited cells in row-major order (the host orders them by (key, a, b))
        for (int a = tid; a < P; a += NT) pre[a] = wlo[a];
        __syncthreads();
        const int a0 = tid * RP, a1 = a0 + RP < P ? a0 + RP : P;
        int64_t s2 = 0;
        for (int a = a0; a < a1; ++a) s2 += pre[a];
        int64_t tot;
        int64_t o = wg_scan<NT>(s2, red, &tot);
        for (int a = a0; a < a1; ++a) {
            for (int b = 0; b < pre[a]; ++b, ++o) {
                const int64_t cell = (int64_t)u[a] * T + v[b];
                const int64_t so = (int64_t)slot * args.max_cells + o;
                args.dbg_ab[2 * so] = a;
                args.dbg_ab[2 * so + 1] = b;
                args.dbg_take[so] = (a == cut_a && b == cut_b) ? cut_take : off[cell + 1] - off[cell];
                args.dbg_beg[so] = off[cell];
            }
        }
    }
    if (tid == 0) {
        TravHdr h;
        h.status = status;
        h.A = (int32_t)A;
        h.B = args.w[(int64_t)slot * P];
        h.cut_a = cut_a;
        h.cut_b = cut_b;
        h.nne = 0;
        h.a_ne = 0;
        h.b_ne = 0;
        h.n_items = 0;
        h.gscan = 0;
        h.ncells = nc;
        h.ncand = status == kStOk ? Leff : C_lo;
        h.cut_take = cut_take;
        if (Leff <= 0) {
            h.A = 0;
            h.B = 0;
            h.ncells = 0;
            h.ncand = 0;
        }
        args.hdr[slot] = h;
        if (status != kStOk) args.fail_list[atomicAdd(args.fail_count, 1)] = (int32_t)qs;
        if (args.stats) {
            atomicAdd(&args.stats[kStatWideBands], (unsigned long long)n_bands);
            atomicAdd(&args.stats[kStatWideEvals], (unsigned long long)n_evals);
            atomicAdd(&args.stats[kStatWideLoads], (unsigned long long)n_loads);
        }
    }
}

hipError_t launch_traverse_big(const TravArgs &a, int64_t nslots, hipStream_t st)
{
    if (nslots == 0) return hipSuccess;
    if (!a.big || a.P > kMaxPrefix) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_traverse_big<kBigNT>, dim3((unsigned)nslots), dim3(kBigNT), 0, st, a);
    return hipGetLastError();
}

// ---- workgroup form of the row-major layout, for large visited sets ---------
// Same outputs as the one-wavefront layout kernel (compacted nonempty cells in
// row-major order, per-row and per-column starts, column lists, LUT slots),
// with 512 threads taking kLayE consecutive cells each per step, so that a
// query with 10^5 visited cells needs about fifty dependent steps (512
// threads keep every value in registers: no scratch memory for the dispatch).
constexpr int kLayNT = 512;
constexpr int kLayE = 4;

// exclusive prefix of x[0..n) in place (n <= kLayNT * per), returns the total
template <int NT>
__device__ __forceinline__ int64_t wg_scan_array(int *x, int n, int64_t *red)
{
    const int per = (n + NT - 1) / NT;
    const int i0 = threadIdx.x * per, i1 = i0 + per < n ? i0 + per : n;
    int64_t s = 0;
    for (int i = i0; i < i1; ++i) s += x[i];
    int64_t tot;
    int64_t run = wg_scan<NT>(s, red, &tot);
    for (int i = i0; i < i1; ++i) {
        const int v = x[i];
        x[i] = (int)run;
        run += v;
    }
    __syncthreads();
    return tot;
}

__global__ __launch_bounds__(kLayNT) void k_layout_wide(LayoutArgs args)
{
    constexpr int NT = kLayNT, E = kLayE;
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ int64_t red[NT / 64];
    const int P = args.P;
    // per-rank arrays in LDS, or (long prefixes) in this slot's slice of HBM
    unsigned char *smem = args.gscr ? args.gscr + (size_t)blockIdx.x * layout_rank_bytes(P) : lds;
    unsigned long long *colcur = reinterpret_cast<unsigned long long *>(smem);  // [P] cells | candidates
    int *rc = reinterpret_cast<int *>(colcur + P);      // [P + 1] first diagram cell of each row
    int *rowcnt = rc + (P + 1);                         // [P + 1] nonempty cells per row, then starts
    int *colcnt = rowcnt + (P + 1);                     // [P + 1] same per column
    int *rslot = colcnt + (P + 1);                      // [2P] LUT slot of each row, then column
    const int slot = blockIdx.x;
    const int tid = threadIdx.x;
    const TravHdr h = args.hdr[slot];
    if (h.status != kStOk || h.ncells <= kLayoutWaveMax) return;
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
    int32_t *ne_slot = args.ne_slot + (int64_t)slot * mc;
    int32_t *slot_ij = args.slot_ij + (int64_t)slot * 2 * P;

    // first diagram cell of each row (exclusive prefix of the widths)
    for (int a = tid; a <= P; a += NT) rc[a] = a < A ? w[a] : 0;
    __syncthreads();
    const int64_t ncells = wg_scan_array<NT>(rc, A + 1, red);
    if (ncells > mc) return;
    for (int a = tid; a <= P; a += NT) {
        rowcnt[a] = 0;
        colcnt[a] = 0;
    }
    for (int b = tid; b < P; b += NT) colcur[b] = 0ull;
    __syncthreads();

    // cell of diagram position xi: row by binary search over rc, then column
    auto cells = [&](int64_t x0, int (&as)[E], int (&bs)[E], int64_t (&begs)[E], int64_t (&cnts)[E]) __attribute__((always_inline)) {
        int lo[E], hi[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            lo[e] = 0;
            hi[e] = x0 + e < ncells ? A - 1 : 0;
        }
        bool any = true;
        while (any) {
            any = false;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (lo[e] < hi[e]) {
                    const int mid = (lo[e] + hi[e] + 1) >> 1;
                    if (rc[mid] <= x0 + e) lo[e] = mid;
                    else hi[e] = mid - 1;
                    any |= lo[e] < hi[e];
                }
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            as[e] = lo[e];
            bs[e] = (int)(x0 + e - rc[lo[e]]);
            begs[e] = 0;
            cnts[e] = 0;
            if (x0 + e < ncells) {
                const int64_t c = (int64_t)u[as[e]] * T + v[bs[e]];
                begs[e] = off[c];
                cnts[e] = (as[e] == h.cut_a && bs[e] == h.cut_b) ? h.cut_take : off[c + 1] - begs[e];
            }
        }
    };

    // pass 1: nonempty cells per row and per column
    for (int64_t xb = 0; xb < ncells; xb += (int64_t)NT * E) {
        int as[E], bs[E];
        int64_t begs[E], cnts[E];
        cells(xb + (int64_t)tid * E, as, bs, begs, cnts);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (cnts[e] > 0) {
                atomicAdd(&rowcnt[as[e]], 1);
                atomicAdd(&colcnt[bs[e]], 1);
            }
        }
    }
    __syncthreads();
    // rows and columns holding a nonempty cell get LUT slots in order
    for (int a = tid; a < P; a += NT) {
        rslot[a] = a < A && rowcnt[a] > 0;
        rslot[P + a] = a < B && colcnt[a] > 0;
    }
    __syncthreads();
    const int64_t tne = wg_scan_array<NT>(rowcnt, A + 1, red);
    (void)wg_scan_array<NT>(colcnt, B + 1, red);
    const int nr = (int)wg_scan_array<NT>(rslot, P, red);
    const int ncol = (int)wg_scan_array<NT>(rslot + P, P, red);
    for (int a = tid; a <= A; a += NT) row_ne[a] = rowcnt[a];
    for (int b = tid; b <= B; b += NT) col_ne[b] = colcnt[b];
    for (int a = tid; a < A; a += NT)
        if (rowcnt[a + 1] > rowcnt[a]) slot_ij[rslot[a]] = u[a];
    for (int b = tid; b < B; b += NT)
        if (colcnt[b + 1] > colcnt[b]) slot_ij[nr + rslot[P + b]] = v[b];
    if (tid == 0) {
        args.hdr[slot].a_ne = nr;
        args.hdr[slot].b_ne = ncol;
    }
    __syncthreads();

    // pass 2: compacted entries, candidates numbered in row-major order
    int64_t crun = 0, nerun = 0, itrun = 0;
    for (int64_t xb = 0; xb < ncells; xb += (int64_t)NT * E) {
        const int64_t x0 = xb + (int64_t)tid * E;
        int as[E], bs[E];
        int64_t begs[E], cnts[E];
        cells(x0, as, bs, begs, cnts);
        int64_t lc = 0, ln = 0, li = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            lc += cnts[e];
            ln += cnts[e] > 0;
            li += (cnts[e] + kItem - 1) / kItem;
        }
        int64_t tc, tn;
        const int64_t cb = wg_scan<NT>(lc, red, &tc);
        const int64_t nb = wg_scan<NT>(ln, red, &tn);
        const int64_t ti = wg_sum<NT>(li, red);
        int64_t cs = crun + cb, ne = nerun + nb;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (x0 + e < ncells) {
                const int a = as[e], b = bs[e];
                if (b == 0) row_cand[a] = (int32_t)cs;
                if (cnts[e] > 0) {
                    ne_cs[ne] = (int32_t)cs;
                    ne_cnt[ne] = (int32_t)cnts[e];
                    ne_beg[ne] = begs[e];
                    ne_cst[ne] = (float)(k1[a] + k2[b]);
                    ne_slot[ne] = rslot[a] | ((nr + rslot[P + b]) << 16);
                    const unsigned long long old =
                        atomicAdd(&colcur[b], (1ull << 40) + (unsigned long long)cnts[e]);
                    const int slotc = colcnt[b] + (int)(old >> 40);
                    cm_cell[slotc] = (int32_t)ne;
                    cm_pre[slotc] = (int32_t)(old & ((1ull << 40) - 1ull));
                    ++ne;
                }
                cs += cnts[e];
            }
        }
        crun += tc;
        nerun += tn;
        itrun += ti;
    }
    __syncthreads();
    if (tid == 0) row_cand[A] = (int32_t)crun;
    for (int b = tid; b < B; b += NT) col_tot[b] = (int32_t)(colcur[b] & ((1ull << 40) - 1ull));
    if (tid == 0) {
        args.hdr[slot].nne = (int32_t)nerun;
        const bool dense = nerun > 0 && crun >= (int64_t)kItemMinAvg * nerun;
        const bool items = args.allow_items && dense && !args.ix.local && !args.ix.od;
        args.hdr[slot].n_items = items ? (int32_t)itrun : 0;
        args.hdr[slot].gscan = args.ix.local || args.ix.od || (!dense && crun > kScanWideMin) ? 1 : 0;
    }
    (void)tne;
}

hipError_t launch_layout_wide(const LayoutArgs &a, int64_t nslots, hipStream_t st)
{
    if (nslots == 0) return hipSuccess;
    const size_t lds = a.gscr ? 0 : layout_rank_bytes(a.P);
    if (lds > 144 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_layout_wide, dim3((unsigned)nslots), dim3(kLayNT), lds, st, a);
    return hipGetLastError();
}

}  // namespace fbpq
