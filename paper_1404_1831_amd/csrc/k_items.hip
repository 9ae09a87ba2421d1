// Cell scan: the FBPQ distance (Section 3.1) of every candidate of a query.
//
// A candidate of nonempty visited cell (i, j) is scored with the folded pair
//   LUT1 = LQ[k < M/2] + CR1[i],   LUT2 = LQ[k >= M/2] + CR2[j]
// (LQ[k][r] = ||R_k(r)||^2 - 2 <q|k, R_k(r)>, the query part of the ADC table of
// Section 2.1; CR the centroid-by-codeword tables of equation decomposition),
// so it costs M lookups plus the cell constant fl32(d1[i] + d2[j]).
//
// Kernels, in launch order:
//  k_lq           per query, LQ into HBM;
//  k_score_query  one workgroup per query walks its nonempty cells in
//                 row-major order: LQ sits in LDS, LUT1 is rebuilt only when
//                 the row changes (the paper's per-row table reuse), LUT2 once
//                 per cell; the cell's first block of codes is requested before
//                 its table rows, and the FP32 distances stream to HBM;
//                 A query whose k fits is then selected in the same workgroup;
//  k_select_dist  per query left over, the k smallest (distance, id) of its
//                 distances.
#include "codes.h"
#include "fbpq_dev.h"
#include "select_k.h"

namespace fbpq {

namespace {

constexpr int kNT = 256;                // threads of the item scan and merge
constexpr int kCPT = kItem / kNT;       // candidates per thread of an item
constexpr int kTieCapI = 4096;  // equal keys at the bound the distance select buffers

}  // namespace

int items_wcap(int k_max)
{
    int KP = 1;
    while (KP < k_max) KP <<= 1;
    return KP * 2 < 512 ? 512 : KP * 2;
}

// LQ[k][r] = ||R_k(r)||^2 - 2 <q|k, R_k(r)> for kLqQ queries per workgroup:
// each thread reads one codeword R_k(r) and scores it against every query of
// the group, so the codebooks are read once per kLqQ queries. The M*Kc entries
// are split into chunks of kLqE over blockIdx.y, for enough workgroups.
constexpr int kLqQ = 16;
constexpr int kLqE = 1024;

// DS > 0: the subspace width, codeword held in registers; DS == 0: any width.
template <int DS>
__global__ __launch_bounds__(256) void k_lq(ItemArgs a)
{
    extern __shared__ __align__(16) float qv[];  // [kLqQ][D]
    __shared__ int64_t slots[kLqQ];
    __shared__ int nsel;
    const int D = a.ix.D, M = a.ix.M, ds = DS > 0 ? DS : D / M;
    const int tid = threadIdx.x;
    if (tid == 0) {
        int n = 0;
        for (int i = 0; i < kLqQ; ++i) {
            const int64_t slot = (int64_t)blockIdx.x * kLqQ + i;
            if (slot >= a.nslots) break;
            const TravHdr h = a.hdr[slot];
            if (h.status == kStOk && (h.n_items != 0 || h.gscan)) slots[n++] = slot;
        }
        nsel = n;
    }
    __syncthreads();
    const int n = nsel;
    if (n == 0) return;
    for (int e = tid; e < n * D; e += 256) {
        const int i = e / D, t = e - i * D;
        const int64_t slot = slots[i];
        const int64_t qs = a.qlist ? a.qlist[slot] : slot;
        qv[i * D + t] = a.q[qs * D + t];
    }
    __syncthreads();
    const int e1 = (int)(blockIdx.y + 1) * kLqE < M * kKc ? (int)(blockIdx.y + 1) * kLqE : M * kKc;
    for (int e = (int)blockIdx.y * kLqE + tid; e < e1; e += 256) {
        const int k = e / kKc;
        const float *rw = a.ix.R + (int64_t)e * ds;
        const float nr = a.ix.nR[e];
        if constexpr (DS > 0) {
            float r[DS];
#pragma unroll
            for (int t = 0; t < DS; ++t) r[t] = rw[t];
            for (int i = 0; i < n; ++i) {
                const float *qk = qv + i * D + k * DS;
                float acc = 0.f;
#pragma unroll
                for (int t = 0; t < DS; ++t) acc = fmaf(qk[t], r[t], acc);
                a.lq[slots[i] * M * kKc + e] = nr - 2.f * acc;
            }
        } else {
            // any width: the codeword passes through registers 16 floats at a
            // time, against every query of the group (same order of sums)
            float acc[kLqQ];
#pragma unroll
            for (int i = 0; i < kLqQ; ++i) acc[i] = 0.f;
            for (int t0 = 0; t0 < ds; t0 += 16) {
                float r[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) r[u] = t0 + u < ds ? rw[t0 + u] : 0.f;
                const int tn = ds - t0 < 16 ? ds - t0 : 16;
#pragma unroll
                for (int i = 0; i < kLqQ; ++i) {
                    if (i < n) {
                        const float *qk = qv + i * D + k * ds + t0;
                        for (int u = 0; u < tn; ++u) acc[i] = fmaf(qk[u], r[u], acc[i]);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < kLqQ; ++i)
                if (i < n) a.lq[slots[i] * M * kKc + e] = nr - 2.f * acc[i];
        }
    }
}

// Per-cell values staged in LDS for the first kMetaLds cells of a query.
constexpr int kMetaLds = 64;
constexpr int kFWin = 512;  // candidates the fused selection can rank
#ifndef QWAVES
#define QWAVES 4
#endif

template <int MH>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(QWAVES))) void k_score_query(ItemArgs a)
{
    constexpr int LW = MH * kKc;   // floats of one half table
    constexpr int PT = LW / kNT;   // table floats per thread
    using CodeT = typename CodeU<MH>::T;
    __shared__ __align__(16) float lut1[LW];
    __shared__ __align__(16) float lut2[LW];
    __shared__ int64_t m_p0[kMetaLds];
    __shared__ int32_t m_n[kMetaLds], m_t0[kMetaLds], m_rs[kMetaLds], m_i[kMetaLds], m_j[kMetaLds];
    __shared__ float m_cst[kMetaLds];
    __shared__ uint64_t s_win[kFWin];
    __shared__ uint32_t s_tau;
    __shared__ int s_nwin;
    const int slot = blockIdx.x;
    const TravHdr h = a.hdr[slot];
    if (h.status != kStOk || h.n_items == 0) return;
    const int tid = threadIdx.x, lane = tid & 63;
    if (tid == 0) {
        a.sel_done[slot] = 0;
        if (a.stats) {
            atomicAdd(&a.stats[kStatCellScan], 1ull);
            atomicAdd(&a.stats[kStatCandCell], (unsigned long long)h.ncand);
        }
    }
    const int64_t mc = a.max_cells;
    const int32_t *g_cs = a.ne_cs + slot * mc, *g_cnt = a.ne_cnt + slot * mc;
    const int32_t *g_sl = a.ne_slot + slot * mc;
    const int64_t *g_beg = a.ne_beg + slot * mc;
    const float *g_cst = a.ne_cst + slot * mc;
    const int32_t *sij = a.slot_ij + (int64_t)slot * 2 * a.P;
    const int nne = h.nne;
    for (int e = tid; e < nne && e < kMetaLds; e += kNT) {
        const int sl = g_sl[e];
        m_p0[e] = g_beg[e];
        m_n[e] = g_cnt[e];
        m_t0[e] = g_cs[e];
        m_rs[e] = sl & 0xffff;
        m_i[e] = sij[sl & 0xffff];
        m_j[e] = sij[sl >> 16];
        m_cst[e] = g_cst[e];
    }
    // each thread folds the same table positions for every cell: LQ in registers
    const float *lqg = a.lq + (int64_t)slot * 2 * LW;
    float lql[PT], lqh[PT];
#pragma unroll
    for (int u = 0; u < PT; ++u) {
        lql[u] = lqg[tid + kNT * u];
        lqh[u] = lqg[LW + tid + kNT * u];
    }
    __syncthreads();
    float *dst = a.dist + (int64_t)slot * a.lcap;
    float smin = __builtin_huge_valf();  // this thread's smallest distance: a selection sample
    bool scored = false;
    int cur_rs = -1;
    for (int e = 0; e < nne; ++e) {
        int64_t p0;
        int n, t0, rs, ci, cj;
        float cst;
        if (e < kMetaLds) {
            p0 = m_p0[e];
            n = m_n[e];
            t0 = m_t0[e];
            rs = m_rs[e];
            ci = m_i[e];
            cj = m_j[e];
            cst = m_cst[e];
        } else {
            const int sl = g_sl[e];
            p0 = g_beg[e];
            n = g_cnt[e];
            t0 = g_cs[e];
            rs = sl & 0xffff;
            ci = sij[sl & 0xffff];
            cj = sij[sl >> 16];
            cst = g_cst[e];
        }
        CodeT ca[kCPT], cb[kCPT];
#pragma unroll
        for (int j = 0; j < kCPT; ++j) {
            const int o = tid + kNT * j;
            if (o < n) {
                ca[j] = load_c<MH>(a.ix.codesA, p0 + o);
                cb[j] = load_c<MH>(a.ix.codesB, p0 + o);
            }
        }
        const bool newrow = rs != cur_rs;
        float c1[PT], c2[PT];
        const float *cr2 = a.ix.CR2 + (int64_t)cj * LW;
#pragma unroll
        for (int u = 0; u < PT; ++u) c2[u] = cr2[tid + kNT * u];
        if (newrow) {
            const float *cr1 = a.ix.CR1 + (int64_t)ci * LW;
#pragma unroll
            for (int u = 0; u < PT; ++u) c1[u] = cr1[tid + kNT * u];
        }
        __syncthreads();  // the previous cell's lookups are done
#pragma unroll
        for (int u = 0; u < PT; ++u) lut2[tid + kNT * u] = lqh[u] + c2[u];
        if (newrow) {
#pragma unroll
            for (int u = 0; u < PT; ++u) lut1[tid + kNT * u] = lql[u] + c1[u];
        }
        cur_rs = rs;
        __syncthreads();
        for (int o0 = 0; o0 < n; o0 += kItem) {
            if (o0 > 0) {
#pragma unroll
                for (int j = 0; j < kCPT; ++j) {
                    const int o = o0 + tid + kNT * j;
                    if (o < n) {
                        ca[j] = load_c<MH>(a.ix.codesA, p0 + o);
                        cb[j] = load_c<MH>(a.ix.codesB, p0 + o);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < kCPT; ++j) {
                const int o = o0 + tid + kNT * j;
                if (o < n) {
                    const float d = cst + lsum<MH>(lut1, ca[j]) + lsum<MH>(lut2, cb[j]);
                    dst[t0 + o] = d;
                    smin = d < smin ? d : smin;
                    scored = true;
                    if (a.dbg_pos) {
                        a.dbg_pos[(int64_t)slot * a.dbg_cap + t0 + o] = p0 + o;
                        a.dbg_d[(int64_t)slot * a.dbg_cap + t0 + o] = d;
                    }
                }
            }
        }
    }

    // Fused selection of the kq smallest (distance, id). Per-thread minima are
    // samples, each the distance of a distinct candidate, so any value with kq
    // samples at or below it bounds the kq-th smallest distance. The distances
    // are read back while they are still in the cache. Queries with kq above
    // the thread count, too few samples or too many candidates at or below the
    // bound are left to k_select_dist.
    const int64_t qs = a.qlist ? a.qlist[slot] : slot;
    const int kq = a.k[qs];
    const int64_t ncand = h.ncand;
    if (kq > kNT) return;
    // Each wavefront finds the ceil(kq/4)-th smallest of its own 64 samples;
    // the largest of the four has at least kq samples at or below it.
    __shared__ uint32_t s_wtau[kNT / 64];
    if (tid == 0) s_nwin = 0;
    {
        const uint32_t u = scored ? fkey(smin) : 0xffffffffu;
        const int kw = (kq + kNT / 64 - 1) / (kNT / 64);
        uint32_t pre = 0;
        int need = kw;
        for (int b = 31; b >= 0; --b) {
            const uint32_t hm = b == 31 ? 0u : (0xffffffffu << (b + 1));
            const int cnt = __popcll(__ballot(((u & hm) == pre) && !((u >> b) & 1u)));
            if (cnt < need) {
                pre |= 1u << b;
                need -= cnt;
            }
        }
        if (lane == 0) s_wtau[tid >> 6] = pre;
    }
    __syncthreads();  // the wavefront bounds, and every thread's distance stores
    if (tid == 0) {
        uint32_t m = 0;
        for (int w = 0; w < kNT / 64; ++w) m = s_wtau[w] > m ? s_wtau[w] : m;
        s_tau = ncand <= kq ? 0xffffffffu : m;
    }
    __syncthreads();
    const uint32_t tau = s_tau;
    if (tau == 0xffffffffu && ncand > kq) return;  // fewer than kq samples
    constexpr int kFB = 24;  // distances per thread loaded before they are tested
    for (int64_t b0 = 0; b0 < ncand; b0 += kNT * kFB) {
        float dv[kFB];
#pragma unroll
        for (int j = 0; j < kFB; ++j) {
            const int64_t t = b0 + tid + kNT * j;
            dv[j] = t < ncand ? dst[t] : 0.f;
        }
#pragma unroll
        for (int j = 0; j < kFB; ++j) {
            const int64_t t = b0 + tid + kNT * j;
            const uint32_t key = fkey(dv[j]);
            const bool pred = t < ncand && key <= tau;
            const uint64_t m = __ballot(pred);
            if (m) {
                int base = 0;
                if (lane == 0) base = atomicAdd(&s_nwin, (int)__popcll(m));
                base = __shfl(base, 0);
                if (pred) {
                    const int wi = base + (int)__popcll(m & ((1ull << lane) - 1ull));
                    if (wi < kFWin) s_win[wi] = ((uint64_t)key << 32) | (uint32_t)t;
                }
            }
        }
    }
    __syncthreads();
    const int nwin = s_nwin;
    if (nwin > kFWin) return;
    for (int i = tid; i < nwin; i += kNT) {
        const uint64_t x = s_win[i];
        const int64_t t = (uint32_t)x;
        int lo = 0, hi = nne - 1;
        int64_t p;
        if (nne <= kMetaLds) {
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (m_t0[mid] <= t) lo = mid;
                else hi = mid - 1;
            }
            p = m_p0[lo] + (t - m_t0[lo]);
        } else {
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (g_cs[mid] <= t) lo = mid;
                else hi = mid - 1;
            }
            p = g_beg[lo] + (t - g_cs[lo]);
        }
        s_win[i] = (x & 0xffffffff00000000ull) | a.ix.ids[p];
    }
    __syncthreads();
    int64_t *oid = a.out_ids + qs * a.k_max;
    float *od = a.out_d + qs * a.k_max;
    const int nk = nwin < kq ? nwin : kq;
    for (int i = tid; i < nwin; i += kNT) {
        const uint64_t x = s_win[i];
        int rank = 0;
        for (int j = 0; j < nwin; ++j) rank += s_win[j] < x;
        if (rank < nk) {
            oid[rank] = (int64_t)(uint32_t)x;
            od[rank] = unfkey((uint32_t)(x >> 32));
        }
    }
    for (int r = nk + tid; r < a.k_max; r += kNT) {
        oid[r] = -1;
        od[r] = __builtin_huge_valf();
    }
    if (tid == 0) {
        a.sel_done[slot] = 1;
        if (a.stats) atomicAdd(&a.stats[kStatFused], 1ull);
    }
}

// The k smallest (distance, id) of one query over its streamed distances.
// A pass holds kSelPT distances per thread in registers, plus the running
// list of the previous pass. Each thread's smallest key is a sample; the
// kq-th smallest sample bounds the kq-th smallest key from above (kq distinct
// elements lie at or below it), so the elements at or below it contain the
// answer. They are appended with one LDS atomic per wave and ranked by
// (key, id). When they do not fit the window (many equal keys), the general
// histogram selection runs over the pass instead.
constexpr int kSelNT = 256;
constexpr int kSelPT = 48;
constexpr int kSelChunk = kSelNT * kSelPT;
constexpr int kRunPT = 1024 / kSelNT;  // k_max is at most 1024
constexpr int kIdxLds = 512;  // cells whose start offsets are staged in LDS

size_t select_dist_lds(int k_max)
{
    int KP = 1;
    while (KP < k_max) KP <<= 1;
    const int wcap = items_wcap(k_max);
    return (size_t)(wcap + KP) * 8 + (size_t)kTieCapI * 4;
}

__global__ __launch_bounds__(kSelNT) void k_select_dist(ItemArgs a)
{
    __shared__ SelShared sh;
    __shared__ uint32_t smp[kSelNT];
    __shared__ int32_t s_cs[kIdxLds];
    __shared__ int64_t s_beg[kIdxLds];
    __shared__ uint32_t s_tau;
    extern __shared__ __align__(16) unsigned char smem[];
    const int slot = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63;
    const TravHdr h = a.hdr[slot];
    if (h.status != kStOk || (h.n_items == 0 && !h.gscan)) return;
    if (a.sel_done[slot]) return;  // selected inside the cell scan or the wide scan
    const int64_t qs = a.qlist ? a.qlist[slot] : slot;
    const int kq = a.k[qs];
    int KP = 1;
    while (KP < a.k_max) KP <<= 1;
    const int wcap = a.wcap;
    uint64_t *win = reinterpret_cast<uint64_t *>(smem);
    uint64_t *run = win + wcap;
    uint32_t *tie = reinterpret_cast<uint32_t *>(run + KP);
    const int64_t mc = a.max_cells;
    const int32_t *cs = a.ne_cs + slot * mc;
    const int64_t *beg = a.ne_beg + slot * mc;
    const int nne = h.nne;
    const bool idx_lds = nne <= kIdxLds;
    if (idx_lds) {
        for (int e = tid; e < nne; e += kSelNT) {
            s_cs[e] = cs[e];
            s_beg[e] = beg[e];
        }
    }
    // id of candidate t (row-major position in the query's candidate list)
    auto id_of = [&](int64_t t) __attribute__((always_inline)) -> uint32_t {
        int lo = 0, hi = nne - 1;
        int64_t p;
        if (idx_lds) {
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_cs[mid] <= t) lo = mid;
                else hi = mid - 1;
            }
            p = s_beg[lo] + (t - s_cs[lo]);
        } else {
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (cs[mid] <= t) lo = mid;
                else hi = mid - 1;
            }
            p = beg[lo] + (t - cs[lo]);
        }
        return a.ix.ids[p];
    };
    // appends (key, ref) for lanes with pred; the call is wave-uniform
    auto append = [&](bool pred, uint32_t key, uint32_t ref) __attribute__((always_inline)) {
        const uint64_t m = __ballot(pred);
        if (m == 0) return;
        int base = 0;
        if (lane == 0) base = atomicAdd(&sh.s_nwin, (int)__popcll(m));
        base = __shfl(base, 0);
        if (pred) {
            const int wi = base + (int)__popcll(m & ((1ull << lane) - 1ull));
            if (wi < wcap) win[wi] = ((uint64_t)key << 32) | ref;
        }
    };
    const float *src = a.dist + (int64_t)slot * a.lcap;
    const int64_t ncand = h.ncand;
    int nrun = 0;
    for (int64_t c0 = 0; c0 < ncand; c0 += kSelChunk) {
        const int n = (int)(ncand - c0 < kSelChunk ? ncand - c0 : kSelChunk);
        const int nr = nrun;
        // element 4 * (tid + kSelNT * j4) + c of the pass sits in v[4 * j4 + c]
        uint32_t v[kSelPT], rk[kRunPT];
        const float *sp = src + c0;
#pragma unroll
        for (int j4 = 0; j4 < kSelPT / 4; ++j4) {
            const int e = 4 * (tid + kSelNT * j4);
            if (e + 3 < n) {
                const float4 f = *reinterpret_cast<const float4 *>(sp + e);
                v[4 * j4] = fkey(f.x);
                v[4 * j4 + 1] = fkey(f.y);
                v[4 * j4 + 2] = fkey(f.z);
                v[4 * j4 + 3] = fkey(f.w);
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) v[4 * j4 + c] = e + c < n ? fkey(sp[e + c]) : 0xffffffffu;
            }
        }
#pragma unroll
        for (int r = 0; r < kRunPT; ++r) {
            const int e = tid + kSelNT * r;
            rk[r] = e < nr ? (uint32_t)(run[e] >> 32) : 0xffffffffu;
        }
        if (tid == 0) sh.s_nwin = 0;
        const int ntot = n + nr;
        const bool any = 4 * tid < n || tid < nr;
        const int n4 = (n + 3) / 4;  // threads that own pass elements
        const int nsamp = (n4 > nr ? n4 : nr) < kSelNT ? (n4 > nr ? n4 : nr) : kSelNT;
        bool done = false;
        if (ntot <= kq || nsamp >= kq) {
            uint32_t tau = 0xffffffffu;
            if (ntot > kq) {
                uint32_t mn = 0xffffffffu;
#pragma unroll
                for (int j = 0; j < kSelPT; ++j) mn = v[j] < mn ? v[j] : mn;
#pragma unroll
                for (int r = 0; r < kRunPT; ++r) mn = rk[r] < mn ? rk[r] : mn;
                smp[tid] = mn;
                __syncthreads();
                if (any) {
                    int rank = 0;
                    for (int u = 0; u < kSelNT; ++u) {
                        const uint32_t x = smp[u];
                        rank += (x < mn) | ((x == mn) & (u < tid));
                    }
                    if (rank == kq - 1) s_tau = mn;
                }
                __syncthreads();
                tau = s_tau;
            } else {
                __syncthreads();
            }
            // refs: position in the pass, or kSelChunk + index in the running list
#pragma unroll
            for (int j = 0; j < kSelPT; ++j) {
                const int e = 4 * (tid + kSelNT * (j / 4)) + (j % 4);
                append(e < n && v[j] <= tau, v[j], (uint32_t)e);
            }
#pragma unroll
            for (int r = 0; r < kRunPT; ++r) {
                const int e = tid + kSelNT * r;
                append(e < nr && rk[r] <= tau, rk[r], (uint32_t)(kSelChunk + e));
            }
            __syncthreads();
            const int nwin = sh.s_nwin;
            if (nwin <= wcap) {
                for (int i = tid; i < nwin; i += kSelNT) {
                    const uint64_t x = win[i];
                    const uint32_t ref = (uint32_t)x;
                    const uint32_t id = ref < (uint32_t)kSelChunk ? id_of(c0 + ref) : (uint32_t)run[ref - kSelChunk];
                    win[i] = (x & 0xffffffff00000000ull) | id;
                }
                __syncthreads();
                // the (key, id) pairs are distinct, so the ranks are too
                const int nk = nwin < kq ? nwin : kq;
                for (int i = tid; i < nwin; i += kSelNT) {
                    const uint64_t x = win[i];
                    int rank = 0;
                    for (int j = 0; j < nwin; ++j) rank += win[j] < x;
                    if (rank < nk) run[rank] = x;
                }
                nrun = nk;
                done = true;
            }
            __syncthreads();
        } else {
            __syncthreads();
        }
        if (done) continue;
        // general selection over the pass, read again from global memory and
        // from the running list (select_k writes run only after its last visit)
        auto visit = [&](auto &&f) __attribute__((always_inline)) {
#pragma unroll 1
            for (int e = tid; e < n; e += kSelNT)
                f(fkey(src[c0 + e]), [&]() __attribute__((always_inline)) { return id_of(c0 + e); });
#pragma unroll 1
            for (int e = tid; e < nr; e += kSelNT)
                f((uint32_t)(run[e] >> 32), [&]() __attribute__((always_inline)) { return (uint32_t)run[e]; });
        };
        nrun = select_k<kSelNT>(visit, ntot, kq, win, wcap, tie, kTieCapI, sh, true, run);
    }
    int64_t *oid = a.out_ids + qs * a.k_max;
    float *od = a.out_d + qs * a.k_max;
    for (int r = tid; r < a.k_max; r += kSelNT) {
        if (r < nrun && r < kq) {
            oid[r] = (int64_t)(uint32_t)run[r];
            od[r] = unfkey((uint32_t)(run[r] >> 32));
        } else {
            oid[r] = -1;
            od[r] = __builtin_huge_valf();
        }
    }
}


hipError_t launch_items_prep(const ItemArgs &a, hipStream_t st)
{
    if (a.nslots == 0) return hipSuccess;
    if (a.ix.D > 1024) return hipErrorInvalidValue;
    const dim3 g((unsigned)((a.nslots + kLqQ - 1) / kLqQ), (unsigned)((a.ix.M * kKc + kLqE - 1) / kLqE)), b(256);
    const size_t lds = (size_t)kLqQ * a.ix.D * sizeof(float);
    switch (a.ix.D / a.ix.M) {
    case 2: hipLaunchKernelGGL(k_lq<2>, g, b, lds, st, a); break;
    case 4: hipLaunchKernelGGL(k_lq<4>, g, b, lds, st, a); break;
    case 8: hipLaunchKernelGGL(k_lq<8>, g, b, lds, st, a); break;
    case 16: hipLaunchKernelGGL(k_lq<16>, g, b, lds, st, a); break;
    default: hipLaunchKernelGGL(k_lq<0>, g, b, lds, st, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_items_scan(const ItemArgs &a, hipStream_t st)
{
    if (a.nslots == 0) return hipSuccess;
    const dim3 g((unsigned)a.nslots), b(kNT);
    switch (a.ix.M / 2) {
    case 1: hipLaunchKernelGGL(k_score_query<1>, g, b, 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_score_query<2>, g, b, 0, st, a); break;
    case 4: hipLaunchKernelGGL(k_score_query<4>, g, b, 0, st, a); break;
    case 8: hipLaunchKernelGGL(k_score_query<8>, g, b, 0, st, a); break;
    case 16: hipLaunchKernelGGL(k_score_query<16>, g, b, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---- persistent form: a device work queue of (query, cell range) items ------
// A batch with budgets of very different sizes keeps every compute unit busy
// to the end when its scoring work is dealt out in items of bounded size,
// largest queries first, to workgroups that stay resident and take the next
// item as soon as they finish one. Items are built on the device after the
// layout: each query's nonempty cells are cut, in row-major order, into runs
// of at least `tile` candidates (the last run of a query may be shorter), and
// the items are ordered by the query's candidate count in power-of-two classes,
// largest class first. A workgroup scores an item's cells exactly as the
// per-query cell scan does (same tables, same FP32 order: the same distances);
// the workgroup that finishes a query's last item selects its top-k from the
// distance row.
constexpr int kPClasses = 32;  // power-of-two classes of candidate counts

// ctl: [0] queue head, [1] items, [2, 2 + kPClasses) items per class,
// [2 + kPClasses, 2 + 2 kPClasses) fill cursors per class
// Counts and positions are aggregated per workgroup in LDS, then one global
// atomic per class and workgroup: a batch whose queries share one class would
// otherwise serialize on a single counter.
__global__ __launch_bounds__(256) void k_pitems_count(ItemArgs a, PersistArgs p)
{
    __shared__ int cls[kPClasses];
    const int tid = threadIdx.x;
    if (tid < kPClasses) cls[tid] = 0;
    __syncthreads();
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + tid;
    if (slot < a.nslots) {
        const TravHdr h = a.hdr[slot];
        int nit = 0;
        if (h.status == kStOk && h.n_items != 0) {
            const int32_t *cnt = a.ne_cnt + slot * a.max_cells;
            int64_t acc = 0;
            for (int e = 0; e < h.nne; ++e) {
                acc += cnt[e];
                if (acc >= p.tile || e == h.nne - 1) {
                    ++nit;
                    acc = 0;
                }
            }
            const int c = 63 - __clzll((unsigned long long)(h.ncand > 0 ? h.ncand : 1));
            atomicAdd(&cls[c], nit);
            a.sel_done[slot] = 0;  // set again by the fused selection when it completes
            if (a.stats) {
                atomicAdd(&a.stats[kStatCellScan], 1ull);
                atomicAdd(&a.stats[kStatCandCell], (unsigned long long)h.ncand);
            }
        }
        p.qnit[slot] = nit;
        p.qdone[slot] = 0;
    }
    __syncthreads();
    if (tid < kPClasses && cls[tid]) atomicAdd(&p.ctl[2 + tid], cls[tid]);
}

__global__ __launch_bounds__(256) void k_pitems_fill(ItemArgs a, PersistArgs p)
{
    __shared__ int cls[kPClasses], bbase[kPClasses];
    const int tid = threadIdx.x;
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + tid;
    if (blockIdx.x == 0 && tid == 0) {
        int tot = 0;
        for (int c = 0; c < kPClasses; ++c) tot += p.ctl[2 + c];
        p.ctl[1] = tot;
    }
    if (tid < kPClasses) cls[tid] = 0;
    __syncthreads();
    int nit = 0, c = 0, mine = 0;
    TravHdr h{};
    if (slot < a.nslots) {
        nit = p.qnit[slot];
        if (nit) {
            h = a.hdr[slot];
            c = 63 - __clzll((unsigned long long)(h.ncand > 0 ? h.ncand : 1));
            mine = atomicAdd(&cls[c], nit);  // this query's place among the workgroup's items of its class
        }
    }
    __syncthreads();
    if (tid < kPClasses) {
        int base = 0;
        for (int c2 = kPClasses - 1; c2 > tid; --c2) base += p.ctl[2 + c2];  // larger classes first
        bbase[tid] = cls[tid] ? base + atomicAdd(&p.ctl[2 + kPClasses + tid], cls[tid]) : 0;
    }
    __syncthreads();
    if (nit == 0) return;
    int pos = bbase[c] + mine;
    const int32_t *cnt = a.ne_cnt + slot * a.max_cells;
    int64_t acc = 0;
    int e0 = 0;
    for (int e = 0; e < h.nne; ++e) {
        acc += cnt[e];
        if (acc >= p.tile || e == h.nne - 1) {
            p.items[3 * pos] = (int32_t)slot;
            p.items[3 * pos + 1] = e0;
            p.items[3 * pos + 2] = e + 1;
            ++pos;
            e0 = e + 1;
            acc = 0;
        }
    }
}

template <int MH, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(QWAVES))) void k_score_persist(ItemArgs a,
                                                                                                 PersistArgs p)
{
    constexpr int LW = MH * kKc;   // floats of one half table
    constexpr int PT = LW / NT;    // table floats per thread
    constexpr int CPT = kItem / NT;  // candidates per thread of a block of kItem
    using CodeT = typename CodeU<MH>::T;
    static_assert(PT >= 1 && LW % NT == 0, "table split");
    __shared__ __align__(16) float lut1[LW];
    __shared__ __align__(16) float lut2[LW];
    __shared__ int64_t m_p0[kMetaLds];
    __shared__ int32_t m_n[kMetaLds], m_t0[kMetaLds], m_rs[kMetaLds], m_i[kMetaLds], m_j[kMetaLds];
    __shared__ float m_cst[kMetaLds];
    __shared__ uint64_t s_win[kFWin];
    __shared__ uint32_t s_wtau[NT / 64];
    __shared__ uint32_t s_tau;
    __shared__ int s_nwin, s_item, s_last;
    __shared__ int4 s_desc;  // the item's slot, first cell, end cell
    const int tid = threadIdx.x, lane = tid & 63;
    int64_t cur_slot = -1;
    float lql[PT], lqh[PT];
    const int nitems = p.ctl[1];
    // thread 0 takes the next item (and reads its description) while the
    // workgroup works on the current one
    int next = 0;
    int4 ndesc{0, 0, 0, 0};
    if (tid == 0) {
        next = atomicAdd(&p.ctl[0], 1);
        if (next < nitems) ndesc = int4{p.items[3 * next], p.items[3 * next + 1], p.items[3 * next + 2], 0};
    }
    for (;;) {
        if (tid == 0) {
            s_item = next;
            s_desc = ndesc;
        }
        __syncthreads();
        const int item = s_item;
        if (item >= nitems) break;  // every workgroup reaches this: the queue only grows
        const int64_t slot = s_desc.x;
        const int e0 = s_desc.y, e1 = s_desc.z;
        if (tid == 0) {
            next = atomicAdd(&p.ctl[0], 1);
            if (next < nitems) ndesc = int4{p.items[3 * next], p.items[3 * next + 1], p.items[3 * next + 2], 0};
        }
        const TravHdr h = a.hdr[slot];
        const int64_t mc = a.max_cells;
        const int32_t *g_cs = a.ne_cs + slot * mc, *g_cnt = a.ne_cnt + slot * mc;
        const int32_t *g_sl = a.ne_slot + slot * mc;
        const int64_t *g_beg = a.ne_beg + slot * mc;
        const float *g_cst = a.ne_cst + slot * mc;
        const int32_t *sij = a.slot_ij + slot * 2 * a.P;
        if (slot != cur_slot) {
            const float *lqg = a.lq + slot * 2 * LW;
#pragma unroll
            for (int u = 0; u < PT; ++u) {
                lql[u] = lqg[tid + NT * u];
                lqh[u] = lqg[LW + tid + NT * u];
            }
            cur_slot = slot;
        }
        float *dst = a.dist + slot * a.lcap;
        float smin = __builtin_huge_valf();  // this thread's smallest distance of the item
        bool scored = false;
        int cur_rs = -1;
        // the item's first kMetaLds cells: their values in LDS, loaded at once
        for (int e = e0 + tid; e < e1 && e < e0 + kMetaLds; e += NT) {
            const int sl = g_sl[e], m = e - e0;
            m_p0[m] = g_beg[e];
            m_n[m] = g_cnt[e];
            m_t0[m] = g_cs[e];
            m_rs[m] = sl & 0xffff;
            m_i[m] = sij[sl & 0xffff];
            m_j[m] = sij[sl >> 16];
            m_cst[m] = g_cst[e];
        }
        __syncthreads();
        for (int e = e0; e < e1; ++e) {
            int64_t p0;
            int n, t0, rs, ci, cj;
            float cst;
            if (e - e0 < kMetaLds) {
                const int m = e - e0;
                p0 = m_p0[m];
                n = m_n[m];
                t0 = m_t0[m];
                rs = m_rs[m];
                ci = m_i[m];
                cj = m_j[m];
                cst = m_cst[m];
            } else {
                const int sl = g_sl[e];
                p0 = g_beg[e];
                n = g_cnt[e];
                t0 = g_cs[e];
                rs = sl & 0xffff;
                ci = sij[sl & 0xffff];
                cj = sij[sl >> 16];
                cst = g_cst[e];
            }
            CodeT ca[CPT], cb[CPT];
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const int o = tid + NT * j;
                if (o < n) {
                    ca[j] = load_c<MH>(a.ix.codesA, p0 + o);
                    cb[j] = load_c<MH>(a.ix.codesB, p0 + o);
                }
            }
            const bool newrow = rs != cur_rs;
            float c1[PT], c2[PT];
            const float *cr2 = a.ix.CR2 + (int64_t)cj * LW;
#pragma unroll
            for (int u = 0; u < PT; ++u) c2[u] = cr2[tid + NT * u];
            if (newrow) {
                const float *cr1 = a.ix.CR1 + (int64_t)ci * LW;
#pragma unroll
                for (int u = 0; u < PT; ++u) c1[u] = cr1[tid + NT * u];
            }
            __syncthreads();  // the previous cell's lookups are done
#pragma unroll
            for (int u = 0; u < PT; ++u) lut2[tid + NT * u] = lqh[u] + c2[u];
            if (newrow) {
#pragma unroll
                for (int u = 0; u < PT; ++u) lut1[tid + NT * u] = lql[u] + c1[u];
            }
            cur_rs = rs;
            __syncthreads();
            for (int o0 = 0; o0 < n; o0 += kItem) {
                if (o0 > 0) {
#pragma unroll
                    for (int j = 0; j < CPT; ++j) {
                        const int o = o0 + tid + NT * j;
                        if (o < n) {
                            ca[j] = load_c<MH>(a.ix.codesA, p0 + o);
                            cb[j] = load_c<MH>(a.ix.codesB, p0 + o);
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < CPT; ++j) {
                    const int o = o0 + tid + NT * j;
                    if (o < n) {
                        const float d = cst + lsum<MH>(lut1, ca[j]) + lsum<MH>(lut2, cb[j]);
                        dst[t0 + o] = d;
                        smin = d < smin ? d : smin;
                        scored = true;
                        if (a.dbg_pos) {
                            a.dbg_pos[slot * a.dbg_cap + t0 + o] = p0 + o;
                            a.dbg_d[slot * a.dbg_cap + t0 + o] = d;
                        }
                    }
                }
            }
        }
        // A query of one item is selected by the workgroup that scored it, from
        // its own per-thread minima. Otherwise the workgroup that completes the
        // query's last item does it (device-wide fences order the other
        // workgroups' distance stores before its reads) and takes the minima
        // from the distance row.
        const bool single = p.qnit[slot] == 1;
        if (!single) {
            __threadfence();
            __syncthreads();
            if (tid == 0) s_last = atomicAdd(&p.qdone[slot], 1) == p.qnit[slot] - 1;
            __syncthreads();
            if (!s_last) continue;
            __threadfence();
        }
        const int64_t qs = a.qlist ? a.qlist[slot] : slot;
        const int kq = a.k[qs];
        const int64_t ncand = h.ncand;
        if (kq > NT) continue;  // left to k_select_dist (sel_done stays 0)
        // per-thread minima are samples of distinct candidates: each
        // wavefront's ceil(kq / waves)-th smallest, the largest over the
        // wavefronts, bounds the kq-th smallest distance
        bool any = scored;
        if (!single) {
            smin = __builtin_huge_valf();
            any = false;
            for (int64_t t = tid; t < ncand; t += NT) {
                const float d = dst[t];
                smin = d < smin ? d : smin;
                any = true;
            }
        }
        __syncthreads();  // every thread's distance stores, before the read-back
        if (tid == 0) s_nwin = 0;
        {
            const uint32_t u = any ? fkey(smin) : 0xffffffffu;
            const int kw = (kq + NT / 64 - 1) / (NT / 64);
            uint32_t pre = 0;
            int need = kw;
            for (int b = 31; b >= 0; --b) {
                const uint32_t hm = b == 31 ? 0u : (0xffffffffu << (b + 1));
                const int cnt = __popcll(__ballot(((u & hm) == pre) && !((u >> b) & 1u)));
                if (cnt < need) {
                    pre |= 1u << b;
                    need -= cnt;
                }
            }
            if (lane == 0) s_wtau[tid >> 6] = pre;
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t m = 0;
            for (int w = 0; w < NT / 64; ++w) m = s_wtau[w] > m ? s_wtau[w] : m;
            s_tau = ncand <= kq ? 0xffffffffu : m;
        }
        __syncthreads();
        const uint32_t tau = s_tau;
        if (tau == 0xffffffffu && ncand > kq) continue;  // fewer than kq samples
        constexpr int kFB = 24;  // distances per thread loaded before they are tested
        for (int64_t b0 = 0; b0 < ncand; b0 += (int64_t)NT * kFB) {
            float dv[kFB];
#pragma unroll
            for (int j = 0; j < kFB; ++j) {
                const int64_t t = b0 + tid + (int64_t)NT * j;
                dv[j] = t < ncand ? dst[t] : 0.f;
            }
#pragma unroll
            for (int j = 0; j < kFB; ++j) {
                const int64_t t = b0 + tid + (int64_t)NT * j;
                const uint32_t key = fkey(dv[j]);
                const bool pred = t < ncand && key <= tau;
                const uint64_t m = __ballot(pred);
                if (m) {
                    int base = 0;
                    if (lane == 0) base = atomicAdd(&s_nwin, (int)__popcll(m));
                    base = __shfl(base, 0);
                    if (pred) {
                        const int wi = base + (int)__popcll(m & ((1ull << lane) - 1ull));
                        if (wi < kFWin) s_win[wi] = ((uint64_t)key << 32) | (uint32_t)t;
                    }
                }
            }
        }
        __syncthreads();
        const int nwin = s_nwin;
        if (nwin > kFWin) continue;  // many equal distances: left to k_select_dist
        const int nne = h.nne;
        // a query whose cells are all in this workgroup's LDS resolves ids there
        const bool meta = single && e0 == 0 && e1 == nne && nne <= kMetaLds;
        for (int i = tid; i < nwin; i += NT) {
            const uint64_t x = s_win[i];
            const int64_t t = (uint32_t)x;
            int lo = 0, hi = nne - 1;
            int64_t pos;
            if (meta) {
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (m_t0[mid] <= t) lo = mid;
                    else hi = mid - 1;
                }
                pos = m_p0[lo] + (t - m_t0[lo]);
            } else {
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (g_cs[mid] <= t) lo = mid;
                    else hi = mid - 1;
                }
                pos = g_beg[lo] + (t - g_cs[lo]);
            }
            s_win[i] = (x & 0xffffffff00000000ull) | a.ix.ids[pos];
        }
        __syncthreads();
        int64_t *oid = a.out_ids + qs * a.k_max;
        float *od = a.out_d + qs * a.k_max;
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
        __syncthreads();  // s_win is reused by the next item
    }
}

int64_t persist_items_cap(int64_t nslots, int64_t lcap, int32_t tile)
{
    return nslots * (lcap / (tile > 0 ? tile : 1) + 1);
}

hipError_t launch_items_persist(const ItemArgs &a, const PersistArgs &p, int waves, hipStream_t st)
{
    if (a.nslots == 0) return hipSuccess;
    if (p.tile < 1) return hipErrorInvalidValue;
    hipError_t e = launch_fill_i32(p.ctl, 0, 2 + 2 * kPClasses, st);
    if (e != hipSuccess) return e;
    const dim3 gs((unsigned)((a.nslots + 255) / 256)), bs(256);
    hipLaunchKernelGGL(k_pitems_count, gs, bs, 0, st, a, p);
    hipLaunchKernelGGL(k_pitems_fill, gs, bs, 0, st, a, p);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // one workgroup per resident slot of the device (more only exit at once)
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess)
        ncu = 256;
    auto go = [&](auto kern, int nt) {
        // at least as many workgroups as the device can hold at once (more
        // wait, then find the queue empty and leave)
        const int per = 16;
        const int64_t cap = persist_items_cap(a.nslots, a.lcap, p.tile);
        int64_t grid = (int64_t)ncu * per;
        grid = grid < cap ? grid : cap;
        hipLaunchKernelGGL(kern, dim3((unsigned)(grid > 1 ? grid : 1)), dim3(nt), 0, st, a, p);
    };
    // waves per workgroup: 2 only where the codes of 16 candidates per thread
    // fit in registers (M <= 8), 8 where a table has at least 512 entries
    switch (a.ix.M / 2) {
    case 1: go(k_score_persist<1, 256>, 256); break;
    case 2:
        if (waves == 2) go(k_score_persist<2, 128>, 128);
        else if (waves == 8) go(k_score_persist<2, 512>, 512);
        else go(k_score_persist<2, 256>, 256);
        break;
    case 4:
        if (waves == 2) go(k_score_persist<4, 128>, 128);
        else if (waves == 8) go(k_score_persist<4, 512>, 512);
        else go(k_score_persist<4, 256>, 256);
        break;
    case 8:
        if (waves == 8) go(k_score_persist<8, 512>, 512);
        else go(k_score_persist<8, 256>, 256);
        break;
    case 16:
        if (waves == 8) go(k_score_persist<16, 512>, 512);
        else go(k_score_persist<16, 256>, 256);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_items_merge(const ItemArgs &a, hipStream_t st)
{
    if (a.nslots == 0) return hipSuccess;
    hipLaunchKernelGGL(k_select_dist, dim3((unsigned)a.nslots), dim3(kSelNT),
                       select_dist_lds(a.k_max), st, a);
    return hipGetLastError();
}

}  // namespace fbpq
