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
//                 its table rows. A query whose k fits the workgroup keeps only
//                 the candidates under a running bound in an LDS window and is
//                 selected there; the others stream their FP32 distances to HBM;
//  k_select_dist  per query left over, the k smallest (distance, id) of its
//                 distances.
#include <type_traits>

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
    if (tid < 64) {
        // the group's headers read by kLqQ lanes at once, the selected slots
        // listed in ascending order
        const int64_t slot = (int64_t)blockIdx.x * kLqQ + tid;
        bool sel = false;
        if (tid < kLqQ && slot < a.nslots) {
            if (a.hdr) {
                const TravHdr h = a.hdr[slot];
                sel = h.status == kStOk && (h.n_items != 0 || h.gscan);
            } else {
                sel = true;  // every slot (launched before the traversal)
            }
        }
        const uint64_t m = __ballot(sel);
        if (sel) slots[__popcll(m & ((1ull << tid) - 1ull))] = slot;
        if (tid == 0) nsel = __popcll(m);
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
// The windowed scan synchronises its wavefronts' bounds on the blocks that
// start below this many candidates of the query.
constexpr int kSyncBelow = 4096;
constexpr int kFWin = 512;  // candidates the fused selection can rank
#ifndef QWAVES
#define QWAVES 4
#endif

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Largest kw-th smallest key of a wavefront's 64 lanes, resolved on the top
// (32 - LOW) bits and padded with ones below: at least kw of the keys lie at or
// below the result. LOW = 0 gives the exact key (kw <= 64).
template <int LOW>
__device__ __forceinline__ uint32_t wave_kth(uint32_t u, int kw)
{
    uint32_t pre = 0;
    int need = kw;
#pragma unroll
    for (int b = 31; b >= LOW; --b) {
        const uint32_t hm = b == 31 ? 0u : (0xffffffffu << (b + 1));
        const int cnt = __popcll(__ballot(((u & hm) == pre) && !((u >> b) & 1u)));
        if (cnt < need) {
            pre |= 1u << b;
            need -= cnt;
        }
    }
    return LOW == 0 ? pre : (pre | ((1u << LOW) - 1u));
}

// STREAM false: the windowed scan and selection of every query whose k fits
// the workgroup; STREAM true (launched after it): the streamed scan of the
// queries it left unselected (k above kNT, or an overflowed window).
template <int MH, bool STREAM>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(QWAVES))) void k_score_query(ItemArgs a)
{
    constexpr int LW = MH * kKc;   // floats of one half table
    constexpr int PT = LW / kNT;   // table floats per thread
    constexpr int WIN = MH >= 16 ? 512 : 1024;  // candidates the running bound admits
    using CodeT = typename CodeU<MH>::T;
    // LUT1 then LUT2; after the scan, the survivors of the final bound
    __shared__ __align__(16) float luts[2 * LW];
    float *const lut1 = luts, *const lut2 = luts + LW;
    __shared__ int64_t m_p0[kMetaLds];
    __shared__ int32_t m_n[kMetaLds], m_t0[kMetaLds], m_rs[kMetaLds], m_i[kMetaLds], m_j[kMetaLds];
    __shared__ float m_cst[kMetaLds];
    __shared__ uint64_t s_win[WIN];
    __shared__ uint32_t s_wb[kNT / 64];  // each wavefront's latest bound
    __shared__ int s_nwin, s_nsv, s_lost, s_admit;
    const int slot = blockIdx.x;
    const TravHdr h = a.hdr[slot];
    if (h.status != kStOk || h.n_items == 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t qs = a.qlist ? a.qlist[slot] : slot;
    const int kq = a.k[qs];
    if constexpr (STREAM) {
        if (a.sel_done[slot]) return;  // selected by the windowed scan
    } else if (kq > kNT) {
        if (tid == 0) {
            a.sel_done[slot] = 0;
            if (a.stats) {
                atomicAdd(&a.stats[kStatCellScan], 1ull);
                atomicAdd(&a.stats[kStatCandCell], (unsigned long long)h.ncand);
            }
        }
        return;
    }
    if (tid == 0 && !STREAM) {
        a.sel_done[slot] = 0;
        s_nwin = 0;
        s_nsv = 0;
        s_lost = 0;
        s_admit = 0;
        if (a.stats) {
            atomicAdd(&a.stats[kStatCellScan], 1ull);
            atomicAdd(&a.stats[kStatCandCell], (unsigned long long)h.ncand);
        }
    }
    if (tid < kNT / 64) s_wb[tid] = 0xffffffffu;
    const int64_t ncand = h.ncand;
    const int kw = (kq + kNT / 64 - 1) / (kNT / 64);
    const int64_t mc = a.max_cells;
    const int32_t *g_cs = a.ne_cs + slot * mc, *g_cnt = a.ne_cnt + slot * mc;
    const int32_t *g_sl = a.ne_slot + slot * mc;
    const int64_t *g_beg = a.ne_beg + slot * mc;
    const float *g_cst = a.ne_cst + slot * mc;
    const int32_t *sij = a.slot_ij + (int64_t)slot * 2 * a.P;
    const int nne = h.nne;
    // values of cells e0 .. e0 + kMetaLds - 1 into LDS (slot e mod kMetaLds)
    auto stage_meta = [&](int e0) {
        for (int e = e0 + tid; e < nne && e < e0 + kMetaLds; e += kNT) {
            const int sl = g_sl[e], em = e & (kMetaLds - 1);
            m_p0[em] = g_beg[e];
            m_n[em] = g_cnt[e];
            m_t0[em] = g_cs[e];
            m_rs[em] = sl & 0xffff;
            m_i[em] = sij[sl & 0xffff];
            m_j[em] = sij[sl >> 16];
            m_cst[em] = g_cst[e];
        }
    };
    stage_meta(0);
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

    // One pass over the query's cells. Streamed (WINDOW false): every distance
    // goes to HBM for k_select_dist. Windowed: each thread's minimum is a
    // sample (the distance of a distinct candidate), so a value with kq
    // samples at or below it bounds the kq-th smallest distance from above;
    // after each block of codes every wavefront publishes the bound of its own
    // samples (ceil(kq/4) of them), and the largest of the four published
    // bounds admits a candidate into the LDS window. Samples only decrease, so
    // a bound read before its wavefront's latest update is still a bound, and
    // every candidate of the final kq smallest is admitted. A window past half
    // full is compacted to the current bound at the next cell.
    // the largest published wavefront bound
    auto cur_bound = [&]() {
        uint32_t tau = 0;
#pragma unroll
        for (int w = 0; w < kNT / 64; ++w) {
            const uint32_t b = __hip_atomic_load(&s_wb[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            tau = b > tau ? b : tau;
        }
        return tau;
    };
    // wavefront-wide append of the lanes whose pred holds (one LDS atomic)
    auto append = [&](bool pred, uint64_t x, bool fresh) {
        const uint64_t m = __ballot(pred);
        if (m) {
            int base = 0;
            if (lane == 0) {
                base = atomicAdd(&s_nwin, (int)__popcll(m));
                if (fresh && a.stats) atomicAdd(&s_admit, (int)__popcll(m));
            }
            base = __shfl(base, 0);
            if (pred) {
                const int wi = base + (int)__popcll(m & ((1ull << lane) - 1ull));
                if (wi < WIN) s_win[wi] = x;
            }
        }
    };
    auto scan = [&](auto window) {
        constexpr bool WINDOW = decltype(window)::value;
        int cur_rs = -1, last_upd = 0;
        for (int e = 0; e < nne; ++e) {
            const int em = e & (kMetaLds - 1);
            if (em == 0 && e > 0) {
                // the next kMetaLds cells' values: every thread read the
                // previous ones before the last cell's barriers
                stage_meta(e);
                __syncthreads();
            }
            // the cell's values are the same in every lane: scalar registers
            const int64_t p0 = uni64(m_p0[em]);
            const int n = uni(m_n[em]), t0 = uni(m_t0[em]), rs = uni(m_rs[em]), ci = uni(m_i[em]), cj = uni(m_j[em]);
            const float cst = __int_as_float(uni(__float_as_int(m_cst[em])));
            // candidate t0 + o goes to thread (t0 + o) mod kNT, so that every
            // thread holds samples however small the cells are
            const int rot = (tid - t0) & (kNT - 1);
            const uint8_t *const ba = a.ix.codesA + p0 * MH, *const bb = a.ix.codesB + p0 * MH;
            CodeT ca[kCPT], cb[kCPT];
#pragma unroll
            for (int j = 0; j < kCPT; ++j) {
                const int o = rot + kNT * j;
                if (o < n) {
                    ca[j] = *reinterpret_cast<const CodeT *>(ba + (uint32_t)o * MH);
                    cb[j] = *reinterpret_cast<const CodeT *>(bb + (uint32_t)o * MH);
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
            __syncthreads();  // the previous cell's lookups and appends are done
            if constexpr (WINDOW) {
                // a window past half full keeps only what the current bound admits
                const int nw = s_nwin;
                if (nw > WIN / 2) {
                    const uint32_t tau = cur_bound();
                    uint64_t keep[WIN / kNT];
#pragma unroll
                    for (int u = 0; u < WIN / kNT; ++u) {
                        const int i = tid + kNT * u;
                        keep[u] = i < nw && i < WIN ? s_win[i] : ~0ull;
                    }
                    __syncthreads();
                    if (tid == 0) {
                        if (nw > WIN) s_lost = 1;
                        s_nwin = 0;
                    }
                    __syncthreads();
#pragma unroll
                    for (int u = 0; u < WIN / kNT; ++u) append((uint32_t)(keep[u] >> 32) <= tau && keep[u] != ~0ull, keep[u], false);
                }
            }
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
                        const int o = o0 + rot + kNT * j;
                        if (o < n) {
                            ca[j] = *reinterpret_cast<const CodeT *>(ba + (uint32_t)o * MH);
                            cb[j] = *reinterpret_cast<const CodeT *>(bb + (uint32_t)o * MH);
                        }
                    }
                }
                if constexpr (!WINDOW) {
                    // streamed: each distance stored as it is made
#pragma unroll
                    for (int j = 0; j < kCPT; ++j) {
                        const int o = o0 + rot + kNT * j;
                        if (o < n) {
                            const float d = cst + lsum<MH>(lut1, ca[j]) + lsum<MH>(lut2, cb[j]);
                            dst[t0 + o] = d;
                            if (a.dbg_pos) {
                                a.dbg_pos[(int64_t)slot * a.dbg_cap + t0 + o] = p0 + o;
                                a.dbg_d[(int64_t)slot * a.dbg_cap + t0 + o] = d;
                            }
                        }
                    }
                } else {
                    float dv[kCPT];
#pragma unroll
                    for (int j = 0; j < kCPT; ++j) {
                        const int o = o0 + rot + kNT * j;
                        if (o < n) {
                            const float d = cst + lsum<MH>(lut1, ca[j]) + lsum<MH>(lut2, cb[j]);
                            dv[j] = d;
                            smin = d < smin ? d : smin;
                            scored = true;
                        }
                    }
                    if (a.dbg_pos) {
#pragma unroll
                        for (int j = 0; j < kCPT; ++j) {
                            const int o = o0 + rot + kNT * j;
                            if (o < n) {
                                a.dbg_pos[(int64_t)slot * a.dbg_cap + t0 + o] = p0 + o;
                                a.dbg_d[(int64_t)slot * a.dbg_cap + t0 + o] = dv[j];
                            }
                        }
                    }
                    // the bounds are taken again on every block of the first
                    // kSyncBelow candidates, where they fall fastest (with every
                    // wavefront's bound of the block awaited), then each time the
                    // candidates seen have grown by a quarter since the last time
                    const int seen = t0 + o0;
                    if (seen < kSyncBelow || 4 * seen >= 5 * last_upd) {
                        const uint32_t wb = wave_kth<16>(scored ? fkey(smin) : 0xffffffffu, kw);
                        if (lane == 0) __hip_atomic_store(&s_wb[wave], wb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        last_upd = seen;
                    }
                    if (seen < kSyncBelow) __syncthreads();
                    const uint32_t tau = cur_bound();
#pragma unroll
                    for (int j = 0; j < kCPT; ++j) {
                        const int o = o0 + rot + kNT * j;
                        const uint32_t key = fkey(dv[j]);
                        append(o < n && key <= tau, ((uint64_t)key << 32) | (uint32_t)(t0 + o), true);
                    }
                }
            }
        }
    };

    if constexpr (STREAM) {
        scan(std::false_type{});
        return;
    } else {
        scan(std::true_type{});
    }

    // Fused selection of the kq smallest (distance, id): the exact bound of
    // the final samples keeps the window entries that can rank (all of them
    // when there are at most kq candidates).
    __syncthreads();  // every append and every table lookup is done
    if (tid == 0 && a.stats) {
        atomicAdd(&a.stats[kStatWinAdmitted], (unsigned long long)s_admit);
        if (s_lost || s_nwin > WIN) atomicAdd(&a.stats[kStatWinLost], 1ull);
    }
    const int nwin = s_lost ? WIN + 1 : s_nwin;
    if (nwin <= WIN) {
        const uint32_t wt = wave_kth<0>(scored ? fkey(smin) : 0xffffffffu, kw);
        if (lane == 0) s_wb[wave] = wt;
    }
    __syncthreads();
    uint64_t *sv = reinterpret_cast<uint64_t *>(luts);  // LW survivors fit
    if (nwin <= WIN) {
        uint32_t tau = 0;
#pragma unroll
        for (int w = 0; w < kNT / 64; ++w) tau = s_wb[w] > tau ? s_wb[w] : tau;
        if (ncand <= kq) tau = 0xffffffffu;
        for (int i0 = 0; i0 < nwin; i0 += kNT) {
            const int i = i0 + tid;
            const uint64_t x = i < nwin ? s_win[i] : 0;
            const bool pred = i < nwin && (uint32_t)(x >> 32) <= tau;
            const uint64_t m = __ballot(pred);
            if (m) {
                int base = 0;
                if (lane == 0) base = atomicAdd(&s_nsv, (int)__popcll(m));
                base = __shfl(base, 0);
                const int si = base + (int)__popcll(m & ((1ull << lane) - 1ull));
                if (pred && si < LW) sv[si] = x;
            }
        }
    }
    __syncthreads();
    const int nsv = s_nsv;
    if (nwin > WIN || nsv > LW) {
        // the window or the survivors overflowed (many candidates at the
        // bound): the streamed scan scores this query again
        if (tid == 0 && a.stats) atomicAdd(&a.stats[kStatFusedRescan], 1ull);
        return;
    }
    for (int i = tid; i < nsv; i += kNT) {
        const uint64_t x = sv[i];
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
        sv[i] = (x & 0xffffffff00000000ull) | a.ix.ids[p];
    }
    __syncthreads();
    int64_t *oid = a.out_ids + qs * a.k_max;
    float *od = a.out_d + qs * a.k_max;
    const int nk = nsv < kq ? nsv : kq;
    for (int i = tid; i < nsv; i += kNT) {
        const uint64_t x = sv[i];
        int rank = 0;
        for (int j = 0; j < nsv; ++j) rank += sv[j] < x;
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
    auto go = [&](auto win, auto str) {
        hipLaunchKernelGGL(win, g, b, 0, st, a);
        hipLaunchKernelGGL(str, g, b, 0, st, a);
    };
    switch (a.ix.M / 2) {
    case 1: go(k_score_query<1, false>, k_score_query<1, true>); break;
    case 2: go(k_score_query<2, false>, k_score_query<2, true>); break;
    case 4: go(k_score_query<4, false>, k_score_query<4, true>); break;
    case 8: go(k_score_query<8, false>, k_score_query<8, true>); break;
    case 16: go(k_score_query<16, false>, k_score_query<16, true>); break;
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
