// First layer of the search (Section 2.3.3): squared distances from each query
// half to all T half centroids (equations q1, q2) and the sorted prefix of the
// closest-centroid list of each half, the input of the multi-sequence
// traversal.
//
// The traversal order is decided by FP64 keys computed in one fixed order:
// key = sum over t = 0..D/2-1 of e_t^2, e_t = q[t] - c[t] in FP64, one fused
// multiply-add per coordinate in increasing t; lists are sorted by (key,
// centroid index). Computing that for all T centroids is FP64-ALU bound, so it
// is done in two steps:
//  1. an FP32 matrix-core product gives approximate keys
//     ka = ||q||^2 + ||c||^2 - 2 <q, c> for every centroid, with an error
//     below a bound e(q) that holds for any summation order;
//  2. per (query, half), with kP the P-th smallest approximate key, every
//     centroid with ka <= kP + 2e can be among the exact P smallest; those
//     survivors get their exact FP64 key and are sorted. kP is bounded from
//     above by a sample (the P-th smallest of the per-thread minima); value
//     bins bracket kP more tightly when that bound leaves too many survivors.
// A query whose survivor set is too large falls back to an exact radix select
// that recomputes FP64 keys for all centroids.
#include "fbpq_dev.h"

namespace fbpq {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));

// ---- OPQ: queries into the index's rotated space -----------------------------
// q' = Rot q (optimized product quantization, Section 2.1). Coordinate a is
// the FP64 fused multiply-add chain over b = 0..D-1 in that order, rounded
// once to FP32, so the rotated query is a single defined value whatever the
// launch shape. A workgroup stages kRotQ queries in LDS; a thread owns output
// coordinates a and runs the kRotQ chains of its row of Rot side by side.
constexpr int kRotQ = 8;    // queries per workgroup
constexpr int kRotNT = 128;  // threads per workgroup

__global__ __launch_bounds__(kRotNT) void k_rotate(const float *__restrict__ Q, int64_t nq, int D,
                                                   const float *__restrict__ Rot, float *__restrict__ out)
{
    extern __shared__ __align__(16) float qs[];  // [kRotQ][D]
    const int64_t q0 = (int64_t)blockIdx.x * kRotQ;
    const int nr = (int)(nq - q0 < kRotQ ? nq - q0 : kRotQ);
    for (int e = threadIdx.x; e < nr * D; e += kRotNT) qs[e] = Q[q0 * D + e];
    __syncthreads();
    const bool v4 = (D & 3) == 0;
    for (int a = threadIdx.x; a < D; a += kRotNT) {
        const float *row = Rot + (int64_t)a * D;
        double acc[kRotQ];
#pragma unroll
        for (int r = 0; r < kRotQ; ++r) acc[r] = 0.0;
        int b = 0;
        if (v4) {
            // 16-byte reads of the row, four terms at a time in increasing b
#pragma unroll 4
            for (; b < D; b += 4) {
                const float4 w4 = *reinterpret_cast<const float4 *>(row + b);
                const float w[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int r = 0; r < kRotQ; ++r)
                        if (r < nr) acc[r] = __builtin_fma((double)w[u], (double)qs[r * D + b + u], acc[r]);
            }
        }
        for (; b < D; ++b) {
            const double w = (double)row[b];
#pragma unroll
            for (int r = 0; r < kRotQ; ++r)
                if (r < nr) acc[r] = __builtin_fma(w, (double)qs[r * D + b], acc[r]);
        }
#pragma unroll
        for (int r = 0; r < kRotQ; ++r)
            if (r < nr) out[(q0 + r) * D + a] = (float)acc[r];
    }
}

hipError_t launch_rotate(const float *q, int64_t nq, int D, const float *Rot, float *out, hipStream_t st)
{
    if (nq == 0) return hipSuccess;
    const size_t lds = (size_t)kRotQ * D * sizeof(float);
    if (lds > 64 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rotate, dim3((unsigned)((nq + kRotQ - 1) / kRotQ)), dim3(kRotNT), lds, st, q, nq, D, Rot,
                       out);
    return hipGetLastError();
}

// ---- step 1: approximate keys on the matrix cores ---------------------------
// A workgroup takes a chunk of CT centroids of one half (256, or 512 when that
// still gives the chip enough wavefronts) for four groups of 16 kQT rows
// (query halves), one group per wavefront, which takes the chunk 16 centroids
// at a time. Workgroup b takes chunk b mod nchunk, so with a chunk count that
// is a multiple of the 8 XCDs each XCD's L2 serves a fixed eighth of the
// centroids. In the FP32 form the dot product runs over the D/2 coordinates in
// slabs of 64; inside a slab, coordinate 16k + s feeds step s of
// v_mfma_f32_16x16x4f32 from lane i + 16k (A: row i) and lane j + 16k (B:
// centroid j), so each lane reads 16 consecutive floats of its own row. The
// instruction leaves D[4*(lane/16) + r][lane % 16] in accumulator r. The
// summation order differs from a plain loop, which the error bound of step 2
// allows (it holds for any order). One tile holds only 64 bytes of each output
// row, so the keys of kFT tiles are staged in LDS and written as 128-byte runs
// of each row.
constexpr int kQT = 2;    // 16-row query tiles per wavefront
constexpr int kCT = 256;  // centroids per workgroup (a multiple of 64), or 2 kCT
constexpr int kFT = 2;    // tiles staged per key write-out
constexpr int kStgLd = 16 * kFT + 4;  // LDS row stride of the staged keys (floats)
constexpr int kPF = 4;    // shared centroid strips in flight per thread
static_assert(kPF < kCT / 16, "the prefetch ring is filled from the chunk's first strips");

// v[s] = row[t + s] for t + s < h, 0 beyond h or when the row is absent
__device__ __forceinline__ void load_strip(const float *__restrict__ row, bool ok, int t, int h, bool vec,
                                           float v[16])
{
    if (ok && vec && t + 16 <= h) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float4 x = *reinterpret_cast<const float4 *>(row + t + 4 * u);
            v[4 * u] = x.x;
            v[4 * u + 1] = x.y;
            v[4 * u + 2] = x.z;
            v[4 * u + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = (ok && t + u < h) ? row[t + u] : 0.f;
    }
}

// ONE: D/2 <= 64, so the query rows are loaded once and stay in registers.
// SPLIT: at D/2 = 64, workgroups whose four row groups and chunk are full take
// the split FP16 products (Cs1/Cs2 set); other row groups the FP32 ones.
template <bool ONE, bool SPLIT, int CT>
__global__ __launch_bounds__(256) void k_half_approx(const float *__restrict__ Q, int64_t nq, int D,
                                                     const int32_t *__restrict__ qlist,
                                                     const float *__restrict__ C1,
                                                     const float *__restrict__ C2,
                                                     const float *__restrict__ nC1,
                                                     const float *__restrict__ nC2, int T, int nchunk,
                                                     float *__restrict__ ka, float *__restrict__ kmin,
                                                     const _Float16 *__restrict__ Cs1,
                                                     const _Float16 *__restrict__ Cs2, float csc1, float csc2)
{
    // rows are slots 0..nq-1; slot s holds query qlist[s] (or s); ka is [slot][2][T]
    // and kmin (when set) [slot][2][ceil(T/16)]: the smallest key of each
    // block of 16 consecutive centroids, one per 16x16 tile column group
    __shared__ __align__(16) float stage[4][16 * kQT * kStgLd];  // per wavefront: 16 kQT rows x 16 kFT keys
    __shared__ __align__(16) float smin[4][16 * kQT][CT / 16];  // per wavefront: block minima of its chunk
    __shared__ __align__(16) half8 sstrip[2][256];  // shared split strips, piece-major (see below)
    __shared__ float snc[CT];                         // ||c||^2 of the chunk (shared form)
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    // the wavefront index, in a scalar register so that everything derived from
    // it (and every branch on it) is uniform
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t ngrp = (nq + 16 * kQT - 1) / (16 * kQT);
    const int64_t ngq = (ngrp + 3) / 4;  // groups of four row groups per half
    const int chunk = (int)(blockIdx.x % (unsigned)nchunk);
    const int64_t rest = blockIdx.x / (unsigned)nchunk;
    if (rest >= 2 * ngq) return;  // the whole workgroup
    const int half = (int)(rest / ngq);
    const int64_t quad = rest - (int64_t)half * ngq;
    const int64_t s0 = (quad * 4 + wv) * 16 * kQT;
    const int h = D / 2;
    const bool vec = ((h | D) & 3) == 0;
    const int cb = chunk * CT, ce = min(T, cb + CT);
    // The four wavefronts share the split centroid strips through LDS (with
    // barriers) when all four row groups and the chunk are full; every other
    // wavefront runs alone and may leave here.
    const bool shared = SPLIT && ONE && vec && h == 64 && (quad * 4 + 4) * 16 * kQT <= nq && ce - cb == CT;
    if (!shared && s0 >= nq) return;
    const float *C = half ? C2 : C1;
    const float *nC = half ? nC2 : nC1;
    const float *qrow[kQT];
    bool qok[kQT];
#pragma unroll
    for (int a = 0; a < kQT; ++a) {
        const int64_t slot = s0 + 16 * a + li;
        qok[a] = slot < nq;
        const int64_t qr = qok[a] ? (qlist ? qlist[slot] : slot) : 0;
        qrow[a] = Q + qr * D + (int64_t)half * h;
    }
    const int nsl = (h + 63) / 64;
    float av[kQT][16];
    float qn[kQT];  // ||q_h||^2 of row 16a + li
#pragma unroll
    for (int a = 0; a < kQT; ++a) {
        // ||q_h||^2 of row 16a + li: this lane's 16 coordinates of each slab,
        // then the four lanes of the row (any order suits the bound)
        float p = 0.f;
        for (int sl = 0; sl < (ONE ? 1 : nsl); ++sl) {
            load_strip(qrow[a], qok[a], 64 * sl + 16 * lk, h, vec, av[a]);
#pragma unroll
            for (int u = 0; u < 16; ++u) p = fmaf(av[a][u], av[a][u], p);
        }
        p += __shfl_xor(p, 16);
        p += __shfl_xor(p, 32);
        qn[a] = p;
    }
    float *kout = ka + (s0 * 2 + half) * (int64_t)T;  // row s0 + q of this half at kout[2 q T]
    // With 256-centroid chunks, full row groups outside a shared workgroup (at
    // most three per half) take the general loop below: without the register
    // form of the FP32 tiles the split kernel fits four wavefronts per SIMD.
    if (ONE && vec && h == 64 && s0 + 16 * kQT <= nq && ce - cb == CT && (shared || !SPLIT || CT != kCT)) {
        // every row and centroid present: the stores are unconditional, so
        // waiting for a prefetched centroid strip does not wait for them
        const int64_t ldq = 2 * (int64_t)T;
        float nq4[kQT][4];
#pragma unroll
        for (int a = 0; a < kQT; ++a)
#pragma unroll
            for (int r = 0; r < 4; ++r) nq4[a][r] = __shfl(qn[a], 4 * lk + r);
        // Split FP16 products (the index carries the two-part centroids): each
        // query row is scaled by a power of two to a largest magnitude below
        // 2^14 and split the same way, and <q, c> is taken as
        // q_hi c_hi + q_hi c_lo + q_lo c_hi, the three on the FP16 matrix
        // cores with FP32 sums (products of FP16 values are exact in FP32).
        // The dropped q_lo c_lo and the split remainders are below
        // 3 2^-22 |q| |c|, which the index's error coefficient covers.
        half8 qs[kQT][2][2];  // [tile][hi, lo][coordinates 0-7, 8-15 of the lane's 16]
        float inv4[kQT][4];   // 1 / (row scale x centroid scale) of each output row
        if (SPLIT && shared) {
            const float csc = half ? csc2 : csc1;
#pragma unroll
            for (int a = 0; a < kQT; ++a) {
                float mx = 0.f;
#pragma unroll
                for (int u = 0; u < 16; ++u) mx = fmaxf(mx, fabsf(av[a][u]));
                mx = fmaxf(mx, __shfl_xor(mx, 16));
                mx = fmaxf(mx, __shfl_xor(mx, 32));
                int ex;
                (void)frexpf(mx, &ex);  // mx < 2^ex
                const float sq = ldexpf(1.f, 14 - ex);
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const float x = av[a][u] * sq;
                    const _Float16 hi = (_Float16)x;
                    qs[a][0][u >> 3][u & 7] = hi;
                    qs[a][1][u >> 3][u & 7] = (_Float16)(x - (float)hi);
                }
                const float inv = 1.f / (sq * csc);  // a power of two
#pragma unroll
                for (int r = 0; r < 4; ++r) inv4[a][r] = __shfl(inv, 4 * lk + r);
            }
        }
        float *stg = stage[wv];
        float(*mn)[CT / 16] = smin[wv];
        auto tile_split = [&](const half8 (&hv)[2][2], float nc, int col) __attribute__((always_inline)) {
            floatx4 acc[kQT];
#pragma unroll
            for (int a = 0; a < kQT; ++a) acc[a] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int a = 0; a < kQT; ++a) {
                    acc[a] = __builtin_amdgcn_mfma_f32_16x16x32_f16(qs[a][0][p], hv[0][p], acc[a], 0, 0, 0);
                    acc[a] = __builtin_amdgcn_mfma_f32_16x16x32_f16(qs[a][0][p], hv[1][p], acc[a], 0, 0, 0);
                    acc[a] = __builtin_amdgcn_mfma_f32_16x16x32_f16(qs[a][1][p], hv[0][p], acc[a], 0, 0, 0);
                }
#pragma unroll
            for (int a = 0; a < kQT; ++a)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    stg[(16 * a + 4 * lk + r) * kStgLd + col + li] =
                        (nq4[a][r] + nc) - 2.f * (acc[a][r] * inv4[a][r]);
        };
        auto tile = [&](const float (&bv)[16], float nc, int col) __attribute__((always_inline)) {
            floatx4 acc[kQT];
#pragma unroll
            for (int a = 0; a < kQT; ++a) acc[a] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int u = 0; u < 16; ++u)
#pragma unroll
                for (int a = 0; a < kQT; ++a)
                    acc[a] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a][u], bv[u], acc[a], 0, 0, 0);
#pragma unroll
            for (int a = 0; a < kQT; ++a)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    stg[(16 * a + 4 * lk + r) * kStgLd + col + li] = (nq4[a][r] + nc) - 2.f * acc[a][r];
        };
        // LDS executes a wavefront's instructions in issue order: the staged
        // keys are visible to the other lanes once the writes have completed
        // (lgkmcnt 0, vector memory counters untouched); the empty asm keeps
        // the compiler from moving LDS accesses across
        auto lds_order = [&]() __attribute__((always_inline)) {
            __asm__ __volatile__("" ::: "memory");
            __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0) only
            __builtin_amdgcn_wave_barrier();
            __asm__ __volatile__("" ::: "memory");
        };
        // Block minima: a lane holds four consecutive keys of a row, four lanes
        // (a DPP quad) one block of 16; the quad's first lane stages its block
        // minimum for the chunk's write-out.
        auto flush = [&](int c0) __attribute__((always_inline)) {  // c0: first centroid of the staged tiles
            lds_order();
            constexpr int LPR = 4 * kFT;   // lanes per row, 16 bytes each
            constexpr int RPI = 64 / LPR;  // rows per instruction
#pragma unroll
            for (int i = 0; i < 16 * kQT / RPI; ++i) {
                const int row = RPI * i + lane / LPR, col = 4 * (lane % LPR);
                const float4 v = *reinterpret_cast<const float4 *>(stg + row * kStgLd + col);
                *reinterpret_cast<float4 *>(kout + row * ldq + c0 + col) = v;
                if (kmin) {
                    float m = fminf(fminf(v.x, v.y), fminf(v.z, v.w));
                    m = fminf(m, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(m), 0xb1, 0xf, 0xf,
                                                                            false)));  // quad lanes xor 1
                    m = fminf(m, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(m), 0x4e, 0xf, 0xf,
                                                                            false)));  // quad lanes xor 2
                    if ((lane & 3) == 0) mn[row][(c0 - cb) / 16 + (lane % LPR) / 4] = m;
                }
            }
            lds_order();
        };
        if (SPLIT && shared) {
            // The workgroup's four wavefronts score the same chunk for their own
            // rows, so each 16-centroid strip (16 rows of 64 hi then 64 lo FP16
            // values, sixteen 16-byte pieces per row) is fetched once per
            // workgroup: thread p loads piece p / 16 of centroid p % 16 kPF
            // strips ahead into a register and stores it at slot p of a
            // double-buffered LDS strip, piece-major, from which a lane reads
            // its four pieces (the hi and lo parts of its 16 coordinates) with
            // 16 lanes on 16 consecutive pieces. One barrier per tile (the LDS
            // counter only, no memory fence) keeps the prefetches in flight and
            // orders the slot writes against the reads of the tile before.
            constexpr int NT = CT / 16;
            const int p = threadIdx.x;
            const half8 *src = reinterpret_cast<const half8 *>((half ? Cs2 : Cs1) + (int64_t)(cb + (p & 15)) * 2 * h) + (p >> 4);
            constexpr int64_t kStripV = 16 * 16;  // half8 values per strip
            auto lds_barrier = [&]() __attribute__((always_inline)) {
                __asm__ __volatile__("" ::: "memory");
                __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0) only
                __asm__ __volatile__("" ::: "memory");
                __builtin_amdgcn_s_barrier();
                __asm__ __volatile__("" ::: "memory");
            };
            half8 pre[kPF];
#pragma unroll
            for (int i = 0; i < kPF; ++i) pre[i] = src[i * kStripV];
            for (int e = p; e < CT; e += 256) snc[e] = nC[cb + e];
            sstrip[0][p] = pre[0];
            pre[0] = src[kPF * kStripV];  // strip i is held in pre[i % kPF]
            lds_barrier();
#pragma unroll
            for (int t = 0; t < NT; ++t) {  // straight-line code: exact wait counts
                const int c0 = cb + 16 * t;
                if (t + 1 < NT) sstrip[(t + 1) & 1][p] = pre[(t + 1) % kPF];
                if (t + 1 + kPF < NT) pre[(t + 1) % kPF] = src[(t + 1 + kPF) * kStripV];
                const half8 *S = sstrip[t & 1];
                half8 hv[2][2];
                hv[0][0] = S[(2 * lk) * 16 + li];
                hv[0][1] = S[(2 * lk + 1) * 16 + li];
                hv[1][0] = S[(8 + 2 * lk) * 16 + li];
                hv[1][1] = S[(9 + 2 * lk) * 16 + li];
                tile_split(hv, snc[16 * t + li], 16 * (t % kFT));
                if (t % kFT == kFT - 1) flush(c0 - 16 * (kFT - 1));
                lds_barrier();
            }
        } else {
            // FP32 products; the next centroid strip is loaded before this
            // tile's products, alternating between two register sets
            float b0[16], b1[16];
            float n0, n1;
            load_strip(C + (int64_t)(cb + li) * h, true, 16 * lk, h, true, b0);
            n0 = nC[cb + li];
#pragma unroll
            for (int t = 0; t < CT / 16; ++t) {  // straight-line code: exact wait counts
                const int c0 = cb + 16 * t;
                if (t + 1 < CT / 16) {
                    if (t & 1) {
                        load_strip(C + (int64_t)(c0 + 16 + li) * h, true, 16 * lk, h, true, b0);
                        n0 = nC[c0 + 16 + li];
                    } else {
                        load_strip(C + (int64_t)(c0 + 16 + li) * h, true, 16 * lk, h, true, b1);
                        n1 = nC[c0 + 16 + li];
                    }
                }
                if (t & 1) tile(b1, n1, 16 * (t % kFT));
                else tile(b0, n0, 16 * (t % kFT));
                if (t % kFT == kFT - 1) flush(c0 - 16 * (kFT - 1));
            }
        }
        if (kmin) {
            // CT / 16 block minima per row of the chunk: contiguous in each row
            const int64_t G = (T + 15) / 16;
            float *mout = kmin + (s0 * 2 + half) * G + cb / 16;
            constexpr int NP = CT / 64;  // 16-byte parts per row
#pragma unroll
            for (int e0 = 0; e0 < 16 * kQT * NP; e0 += 64) {
                const int e = e0 + lane, row = e / NP, part = e - row * NP;
                const float4 v = *reinterpret_cast<const float4 *>(&mn[row][4 * part]);
                *reinterpret_cast<float4 *>(mout + row * 2 * G + 4 * part) = v;
            }
        }
        return;
    }
    for (int c0 = cb; c0 < ce; c0 += 16) {
        const int c = c0 + li;
        const bool cok = c < ce;
        const float *crow = C + (int64_t)(cok ? c : 0) * h;
        floatx4 acc[kQT];
#pragma unroll
        for (int a = 0; a < kQT; ++a) acc[a] = floatx4{0.f, 0.f, 0.f, 0.f};
        for (int sl = 0; sl < (ONE ? 1 : nsl); ++sl) {
            float bv[16];
            load_strip(crow, cok, 64 * sl + 16 * lk, h, vec, bv);
            if constexpr (!ONE) {
#pragma unroll
                for (int a = 0; a < kQT; ++a) load_strip(qrow[a], qok[a], 64 * sl + 16 * lk, h, vec, av[a]);
            }
#pragma unroll
            for (int u = 0; u < 16; ++u)
#pragma unroll
                for (int a = 0; a < kQT; ++a)
                    acc[a] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a][u], bv[u], acc[a], 0, 0, 0);
        }
        const float nc = cok ? nC[c] : 0.f;
#pragma unroll
        for (int a = 0; a < kQT; ++a)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t slot = s0 + 16 * a + 4 * lk + r;
                const float n = __shfl(qn[a], 4 * lk + r);  // the norm of this output's row
                const float key = (n + nc) - 2.f * acc[a][r];
                if (slot < nq && cok) ka[(slot * 2 + half) * (int64_t)T + c] = key;
                if (kmin) {
                    // block minimum over the tile's present columns (c0 is a multiple of 16)
                    float m = cok ? key : __builtin_huge_valf();
                    m = fminf(m, __shfl_xor(m, 1));
                    m = fminf(m, __shfl_xor(m, 2));
                    m = fminf(m, __shfl_xor(m, 4));
                    m = fminf(m, __shfl_xor(m, 8));
                    const int64_t G = (T + 15) / 16;
                    if (li == 0 && slot < nq) kmin[(slot * 2 + half) * G + c0 / 16] = m;
                }
            }
    }
}

hipError_t launch_half_approx(const DevIndex &ix, const float *q, const int32_t *qlist, int64_t nslots,
                              float *ka, float *kmin, hipStream_t st)
{
    if (nslots == 0) return hipSuccess;
    // wider chunks when the batch still gives at least 16384 wavefronts
    // (16 per SIMD): fewer query loads and splits per key
    const int64_t rows2 = 2 * ((nslots + 16 * kQT - 1) / (16 * kQT));
    const bool wide = rows2 * ((ix.T + 2 * kCT - 1) / (2 * kCT)) >= 16384;
    const int ct = wide ? 2 * kCT : kCT;
    const int nchunk = (ix.T + ct - 1) / ct;
    const int64_t ngq = (rows2 / 2 + 3) / 4;  // groups of four 16 kQT-row groups per half
    const dim3 grid((unsigned)(nchunk * 2 * ngq));
    const bool one = ix.D / 2 <= 64, split = one && ix.Cs1 && ix.Cs2;
    auto go = [&](auto kern, const _Float16 *c1, const _Float16 *c2) {
        hipLaunchKernelGGL(kern, grid, dim3(256), 0, st, q, nslots, ix.D, qlist, ix.C1, ix.C2, ix.nC1, ix.nC2, ix.T,
                           nchunk, ka, kmin, c1, c2, ix.csc1, ix.csc2);
    };
    if (split)
        wide ? go(k_half_approx<true, true, 2 * kCT>, ix.Cs1, ix.Cs2) : go(k_half_approx<true, true, kCT>, ix.Cs1, ix.Cs2);
    else if (one)
        wide ? go(k_half_approx<true, false, 2 * kCT>, nullptr, nullptr) : go(k_half_approx<true, false, kCT>, nullptr, nullptr);
    else
        wide ? go(k_half_approx<false, false, 2 * kCT>, nullptr, nullptr)
             : go(k_half_approx<false, false, kCT>, nullptr, nullptr);
    return hipGetLastError();
}

// ---- step 2: survivors, exact keys, sort -------------------------------------
constexpr int kSelThreads = 256;
constexpr int kBins = 1024;

__device__ __forceinline__ uint64_t dkey(double x) { return (uint64_t)__double_as_longlong(x); }

// Exact traversal key of centroid c: FP64, increasing t, one fma per coordinate.
// When h is a multiple of 4 the centroid row is fetched 64 floats at a time
// (sixteen 16-byte loads in flight); the arithmetic order is unchanged.
__device__ __forceinline__ double exact_key(const float *qh, const float *__restrict__ Crow, int h)
{
    double acc = 0.0;
    int t = 0;
    if ((h & 3) == 0) {
        for (; t + 64 <= h; t += 64) {
            float4 c[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) c[u] = *reinterpret_cast<const float4 *>(Crow + t + 4 * u);
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const float4 qv = *reinterpret_cast<const float4 *>(qh + t + 4 * u);
                const float qa[4] = {qv.x, qv.y, qv.z, qv.w};
                const float ca[4] = {c[u].x, c[u].y, c[u].z, c[u].w};
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const double e = (double)qa[v] - (double)ca[v];
                    acc = __builtin_fma(e, e, acc);
                }
            }
        }
        for (; t + 16 <= h; t += 16) {
            float4 c[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) c[u] = *reinterpret_cast<const float4 *>(Crow + t + 4 * u);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float4 qv = *reinterpret_cast<const float4 *>(qh + t + 4 * u);
                const float qa[4] = {qv.x, qv.y, qv.z, qv.w};
                const float ca[4] = {c[u].x, c[u].y, c[u].z, c[u].w};
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const double e = (double)qa[v] - (double)ca[v];
                    acc = __builtin_fma(e, e, acc);
                }
            }
        }
    }
    for (; t < h; ++t) {
        const double e = (double)qh[t] - (double)Crow[t];
        acc = __builtin_fma(e, e, acc);
    }
    return acc;
}

template <typename V>
__device__ V block_reduce(V v, V *red, bool is_min)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) {
        const V u = __shfl_xor(v, o);
        v = is_min ? (u < v ? u : v) : (u > v ? u : v);
    }
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    V r = red[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = is_min ? (red[i] < r ? red[i] : r) : (red[i] > r ? red[i] : r);
    return r;
}

__device__ int block_sum(int v, int *red)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    int r = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += red[i];
    return r;
}

// Exclusive block scan of one int per thread; *total gets the sum.
__device__ int block_excl_scan(int v, int *red, int *total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == 63) red[wv] = x;
    __syncthreads();
    int off = 0, tot = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
        if (i < wv) off += red[i];
        tot += red[i];
    }
    *total = tot;
    return off + x - v;
}

// Writes the first `keep` of n (key, idx) pairs in ascending (key, idx) order
// to ok/oi. Up to 512 pairs, each pair's rank is the number of pairs below it
// (pairs are distinct because indices are); beyond that the pairs are sorted
// in place by a bitonic network over the next power of two (<= cap, the
// buffers' length). Positions [n, keep), and entries whose index is not a
// centroid, get (+inf, 0): a key the traversal never visits. Every thread of
// the block calls it.
__device__ void rank_out(uint64_t *sk, int32_t *si, int n, int cap, int keep, int T,
                         double *__restrict__ ok, int32_t *__restrict__ oi)
{
    const int tid = threadIdx.x;
    if (n <= 512) {
        for (int i = tid; i < n; i += blockDim.x) {
            const uint64_t k = sk[i];
            const int x = si[i];
            int rank = 0;
            for (int j = 0; j < n; ++j) {
                const uint64_t kj = sk[j];
                rank += kj < k || (kj == k && si[j] < x);
            }
            if (rank < keep) {
                const bool valid = x >= 0 && x < T;
                ok[rank] = valid ? __longlong_as_double((long long)k) : __builtin_huge_val();
                oi[rank] = valid ? x : 0;
            }
        }
    } else {
        int np = 1;
        while (np < n) np <<= 1;
        if (np > cap) np = cap;  // n <= cap always; cap is a power of two
        for (int i = n + tid; i < np; i += blockDim.x) {
            sk[i] = ~0ull;
            si[i] = 0x7fffffff;
        }
        __syncthreads();
        for (int kk = 2; kk <= np; kk <<= 1) {
            for (int j = kk >> 1; j > 0; j >>= 1) {
                for (int i = tid; i < np / 2; i += blockDim.x) {
                    const int lo = ((i & ~(j - 1)) << 1) | (i & (j - 1));
                    const int hi = lo + j;
                    const uint64_t ka = sk[lo], kb = sk[hi];
                    const int xa = si[lo], xb = si[hi];
                    const bool gt = ka > kb || (ka == kb && xa > xb);
                    if (gt == ((lo & kk) == 0)) {
                        sk[lo] = kb;
                        sk[hi] = ka;
                        si[lo] = xb;
                        si[hi] = xa;
                    }
                }
                __syncthreads();
            }
        }
        const int m = n < keep ? n : keep;
        for (int i = tid; i < m; i += blockDim.x) {
            const int x = si[i];
            const bool valid = x >= 0 && x < T;
            ok[i] = valid ? __longlong_as_double((long long)sk[i]) : __builtin_huge_val();
            oi[i] = valid ? x : 0;
        }
    }
    for (int i = n + tid; i < keep; i += blockDim.x) {
        ok[i] = __builtin_huge_val();
        oi[i] = 0;
    }
}

// LDS: qh[h] floats | ka[T] floats (when staged) | sort keys u64[S] | sort idx i32[S]
constexpr int kApproxLds = 16384;

__global__ __launch_bounds__(kSelThreads) void k_select_prefix(
    const float *__restrict__ kapprox, const float *__restrict__ Q, int D,
    const float *__restrict__ C1, const float *__restrict__ C2, float cmax1, float cmax2, float ecoef, int T,
    const int32_t *qlist, int P, int S, int stage_ka, double *__restrict__ lkey, int32_t *__restrict__ lidx,
    const int32_t *__restrict__ pstat, unsigned long long *stats, unsigned char *__restrict__ gsort)
{
    if (pstat && pstat[(int64_t)blockIdx.x * 2 + blockIdx.y] == 0) return;  // done by the wave select
    if (stats && threadIdx.x == 0) atomicAdd(&stats[kStatPrefixWG], 1ull);
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t hist[kBins];
    __shared__ float redf[kSelThreads / 64];
    __shared__ int redi[kSelThreads / 64];
    __shared__ uint64_t red64[kSelThreads / 64];
    __shared__ int s_cnt, s_bin, s_need;
    __shared__ float smp[kSelThreads];
    __shared__ float s_tau;
    const int slot = blockIdx.x, half = blockIdx.y, tid = threadIdx.x;
    const int h = D / 2;
    const int64_t qs = qlist ? qlist[slot] : slot;
    const float *C = half ? C2 : C1;
    const float cmax = half ? cmax2 : cmax1;
    // kapprox null: no approximate keys, straight to the exact radix select
    const bool have_ka = kapprox != nullptr;
    const bool lds_ka = have_ka && stage_ka;  // key row staged in LDS (decided by the launcher)
    float *qh = reinterpret_cast<float *>(smem);
    const int hpad = (h + 3) & ~3;
    float *kal = qh + hpad;
    // sort buffer: in LDS, or (long prefixes) in this pair's slice of gsort
    uint64_t *sk = gsort ? reinterpret_cast<uint64_t *>(gsort + ((int64_t)slot * 2 + half) * (int64_t)S * 12)
                         : reinterpret_cast<uint64_t *>(kal + (lds_ka ? ((T + 1) & ~1) : 0));
    int32_t *si = reinterpret_cast<int32_t *>(sk + S);
    const float *kg = have_ka ? kapprox + ((int64_t)slot * 2 + half) * (int64_t)T : nullptr;

    for (int t = tid; t < h; t += kSelThreads) qh[t] = Q[qs * D + half * h + t];
    if (lds_ka)
        for (int i = tid; i < T; i += kSelThreads) kal[i] = kg[i];
    __syncthreads();
    const float *kv = lds_ka ? kal : kg;

    // error bound of the approximate keys (any summation order; the split
    // FP16 products too, through the index's coefficient)
    double qn = 0.0;  // each wave sums ||q_half||^2 on its own (any order suits a bound)
    for (int t = tid & 63; t < h; t += 64) qn += (double)qh[t] * (double)qh[t];
    for (int o = 32; o > 0; o >>= 1) qn += __shfl_xor(qn, o);
    const double rn = sqrt(qn) + sqrt((double)cmax) * (1.0 + 1e-6);
    const float err = (float)(ecoef * 0x1.0p-23 * rn * rn) + 1e-30f;

    bool done = false;
    double *ok = lkey + ((int64_t)slot * 2 + half) * P;
    int32_t *oi = lidx + ((int64_t)slot * 2 + half) * P;
    if (P >= T) {
        // every centroid: exact keys, ranked
        for (int i = tid; i < T; i += kSelThreads) {
            sk[i] = dkey(exact_key(qh, C + (int64_t)i * h, h));
            si[i] = i;
        }
        __syncthreads();
        rank_out(sk, si, T, S, P, T, ok, oi);
        done = true;
    }
    if (!done && have_ka && (T < kSelThreads ? T : kSelThreads) >= P) {
        // Each thread's smallest approximate key is a sample; P distinct
        // centroids lie at or below the P-th smallest sample, so it bounds kP
        // (the P-th smallest approximate key) from above.
        float mn = __builtin_huge_valf();
        for (int i = tid; i < T; i += kSelThreads) mn = kv[i] < mn ? kv[i] : mn;
        smp[tid] = mn;
        if (tid == 0) s_cnt = 0;
        __syncthreads();
        if (tid < T) {
            int rank = 0;
            for (int u = 0; u < kSelThreads; ++u) {
                const float x = smp[u];
                rank += (x < mn) | ((x == mn) & (u < tid));
            }
            if (rank == P - 1) s_tau = mn;
        }
        __syncthreads();
        const float thr = s_tau + 2.f * err;
        for (int i = tid; i < T; i += kSelThreads) {
            if (kv[i] <= thr) {
                const int w = atomicAdd(&s_cnt, 1);
                if (w < S) si[w] = i;
            }
        }
        __syncthreads();
        const int nsurv = s_cnt;
        if (nsurv <= S) {
            for (int w = tid; w < nsurv; w += kSelThreads)
                sk[w] = dkey(exact_key(qh, C + (int64_t)si[w] * h, h));
            __syncthreads();
            rank_out(sk, si, nsurv, S, P, T, ok, oi);
            done = true;
        }
        __syncthreads();
    }
    if (!done && have_ka) {
        // kP: the P-th smallest approximate key, bracketed by value bins
        float lo = 0.f;
        {
            float mn = __builtin_huge_valf(), mx = -__builtin_huge_valf();
            for (int i = tid; i < T; i += kSelThreads) {
                const float x = kv[i];
                mn = x < mn ? x : mn;
                mx = x > mx ? x : mx;
            }
            lo = block_reduce(mn, redf, true);
            float hi = block_reduce(mx, redf, false);
            int need = P;
            float kp = hi;
            int nsurv = T;
            for (int level = 0; level < 3 && hi > lo; ++level) {
                for (int b = tid; b < kBins; b += kSelThreads) hist[b] = 0;
                __syncthreads();
                const float scale = (float)kBins / (hi - lo);
                if (!(scale < 3.0e38f)) break;
                for (int i = tid; i < T; i += kSelThreads) {
                    const float x = kv[i];
                    if (x >= lo && x <= hi) {
                        int b = (int)((x - lo) * scale);
                        b = b < 0 ? 0 : (b >= kBins ? kBins - 1 : b);
                        atomicAdd(&hist[b], 1u);
                    }
                }
                __syncthreads();
                if (tid < 64) {
                    constexpr int per = kBins / 64;
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
                            s_need = need - (int)before;
                        }
                        before += c[j];
                    }
                }
                __syncthreads();
                const int bs = s_bin;
                need = s_need;
                // the keys of bin bs bound kP; narrow to that bin
                float bmn = __builtin_huge_valf(), bmx = -__builtin_huge_valf();
                for (int i = tid; i < T; i += kSelThreads) {
                    const float x = kv[i];
                    if (x >= lo && x <= hi) {
                        int b = (int)((x - lo) * scale);
                        b = b < 0 ? 0 : (b >= kBins ? kBins - 1 : b);
                        if (b == bs) {
                            bmn = x < bmn ? x : bmn;
                            bmx = x > bmx ? x : bmx;
                        }
                    }
                }
                const float nlo = block_reduce(bmn, redf, true);
                const float nhi = block_reduce(bmx, redf, false);
                kp = nhi;
                lo = nlo;
                hi = nhi;
                // stop as soon as the survivors of this bound fit the sort buffer
                const float thr = kp + 2.f * err;
                int mine = 0;
                for (int i = tid; i < T; i += kSelThreads) mine += kv[i] <= thr;
                nsurv = block_sum(mine, redi);
                if (nsurv <= S) break;
            }
            if (!(hi > lo)) {
                kp = hi;
                const float thr = kp + 2.f * err;
                int mine = 0;
                for (int i = tid; i < T; i += kSelThreads) mine += kv[i] <= thr;
                nsurv = block_sum(mine, redi);
            }
            // survivors: ka <= kp + 2 err (kp is >= the P-th smallest approximate key)
            const float thr = kp + 2.f * err;
            if (tid == 0) s_cnt = 0;
            __syncthreads();
            if (nsurv >= P && nsurv <= S) {
                for (int i = tid; i < T; i += kSelThreads) {
                    if (kv[i] <= thr) {
                        const int w = atomicAdd(&s_cnt, 1);
                        if (w < S) si[w] = i;
                    }
                }
                __syncthreads();
                const int ns = nsurv < S ? nsurv : S;
                for (int w = tid; w < ns; w += kSelThreads)
                    sk[w] = dkey(exact_key(qh, C + (int64_t)si[w] * h, h));
                __syncthreads();
                rank_out(sk, si, ns, S, P, T, ok, oi);
                done = true;
            }
        }
    }
    if (!done) {
        // exact radix select over recomputed FP64 keys (many near-equal keys)
        const int per = (T + kSelThreads - 1) / kSelThreads;
        const int i0 = tid * per, i1 = min(T, i0 + per);
        uint64_t kmin = ~0ull, kmax = 0;
        for (int i = i0; i < i1; ++i) {
            const uint64_t b = dkey(exact_key(qh, C + (int64_t)i * h, h));
            kmin = b < kmin ? b : kmin;
            kmax = b > kmax ? b : kmax;
        }
        kmin = block_reduce(kmin, red64, true);
        kmax = block_reduce(kmax, red64, false);
        uint64_t prefix = 0;
        int need = P;
        const uint64_t range = kmax - kmin;
        const int nb = range ? 64 - __clzll((long long)range) : 0;
        const int passes = (nb + 7) / 8;
        for (int p = 0; p < passes; ++p) {
            const int s = 8 * (passes - 1 - p);
            for (int b = tid; b < 256; b += kSelThreads) hist[b] = 0;
            __syncthreads();
            for (int i = i0; i < i1; ++i) {
                const uint64_t d = dkey(exact_key(qh, C + (int64_t)i * h, h)) - kmin;
                const uint64_t hi = (s + 8 >= 64) ? 0 : (d >> (s + 8));
                if (hi == prefix) atomicAdd(&hist[(d >> s) & 255], 1u);
            }
            __syncthreads();
            if (tid < 64) {
                uint32_t c[4], sum = 0;
                for (int j = 0; j < 4; ++j) {
                    c[j] = hist[tid * 4 + j];
                    sum += c[j];
                }
                uint32_t x = sum;
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t y = __shfl_up(x, o);
                    if (tid >= o) x += y;
                }
                uint32_t before = x - sum;
                for (int j = 0; j < 4; ++j) {
                    if (before < (uint32_t)need && before + c[j] >= (uint32_t)need) {
                        s_bin = tid * 4 + j;
                        s_need = need - (int)before;
                    }
                    before += c[j];
                }
            }
            __syncthreads();
            prefix = (prefix << 8) | (uint64_t)s_bin;
            need = s_need;
            __syncthreads();
        }
        const uint64_t kstar = kmin + prefix;
        if (tid == 0) s_cnt = 0;
        __syncthreads();
        int my_eq = 0;
        for (int i = i0; i < i1; ++i) {
            const uint64_t b = dkey(exact_key(qh, C + (int64_t)i * h, h));
            if (b < kstar) {
                const int w = atomicAdd(&s_cnt, 1);
                if (w < S) {
                    sk[w] = b;
                    si[w] = i;
                }
            } else if (b == kstar) {
                ++my_eq;
            }
        }
        int tot_eq;
        const int eq_before = block_excl_scan(my_eq, redi, &tot_eq);
        __syncthreads();
        int ord = eq_before;
        const int base = P - need;
        for (int i = i0; i < i1 && ord < need; ++i) {
            const uint64_t b = dkey(exact_key(qh, C + (int64_t)i * h, h));
            if (b == kstar && base + ord < S) {
                sk[base + ord] = b;
                si[base + ord] = i;
                ++ord;
            }
        }
        __syncthreads();
        rank_out(sk, si, P < S ? P : S, S, P, T, ok, oi);
    }
}

// ---- wave select: one wavefront per (query, half), no workgroup barriers ----
// Samples: the minimum approximate key of each of the G = 64 SPL centroid
// groups {c : c = g mod G} (SPL samples per lane, G >= 2P); the P-th smallest
// sample (found bit by bit with ballot counts) bounds kP from above, as P
// distinct centroids lie at or below it.
// Survivors (ka <= bound + 2e) are compacted with ballots, get their exact
// FP64 keys and are sorted by (key, index) inside the wave. When more than
// kWaveS survive, pstat keeps the pair for the workgroup kernel.
constexpr int kWPB = 4;  // wavefronts (query halves) per workgroup

__device__ __forceinline__ uint32_t okey(float f)
{
    const uint32_t b = __float_as_uint(f);
    return b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u);
}

__device__ __forceinline__ float unokey(uint32_t k)
{
    return __uint_as_float((k & 0x80000000u) ? (k ^ 0x80000000u) : ~k);
}

// Exact keys of the n survivors sidx[0..n) and their ranking by (key, centroid
// index): element i = 64 r + lane sits in register r of its lane, padded with
// (~0, INT_MAX) to 64 E elements, and a bitonic network sorts them (strides
// below 64 across lanes with shuffles, larger ones between registers). Position
// i of the sorted sequence is rank i; ranks below P are written.
template <int E>
__device__ __forceinline__ void rank_survivors(const float *qh, const float *__restrict__ C, int h,
                                               const int32_t *sidx, int n, int P, int lane,
                                               double *__restrict__ ok, int32_t *__restrict__ oi)
{
    uint64_t k[E];
    int32_t x[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int i = 64 * r + lane;
        if (i < n) {
            x[r] = sidx[i];
            k[r] = dkey(exact_key(qh, C + (int64_t)x[r] * h, h));
        } else {
            x[r] = 0x7fffffff;
            k[r] = ~0ull;
        }
    }
    constexpr int N = 64 * E;
#pragma unroll
    for (int kk = 2; kk <= N; kk <<= 1) {
#pragma unroll
        for (int j = kk >> 1; j > 0; j >>= 1) {
            if (j >= 64) {
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    const int rp = r ^ (j >> 6);
                    if (rp > r) {
                        const bool asc = ((64 * r + lane) & kk) == 0;
                        const bool gt = k[r] > k[rp] || (k[r] == k[rp] && x[r] > x[rp]);
                        if (gt == asc) {
                            const uint64_t tk = k[r];
                            k[r] = k[rp];
                            k[rp] = tk;
                            const int32_t tx = x[r];
                            x[r] = x[rp];
                            x[rp] = tx;
                        }
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    uint64_t ko;
                    int32_t xo;
                    if (j <= 2) {
                        // lane xor 1 / xor 2 inside each quad: DPP moves, no LDS
                        // (j is a constant once the loops are unrolled)
                        constexpr int kX1 = 0xb1, kX2 = 0x4e;  // quad_perm [1,0,3,2], [2,3,0,1]
                        const uint32_t lo = j == 1
                            ? __builtin_amdgcn_update_dpp(0, (int)(uint32_t)k[r], kX1, 0xf, 0xf, false)
                            : __builtin_amdgcn_update_dpp(0, (int)(uint32_t)k[r], kX2, 0xf, 0xf, false);
                        const uint32_t hi = j == 1
                            ? __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(k[r] >> 32), kX1, 0xf, 0xf, false)
                            : __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(k[r] >> 32), kX2, 0xf, 0xf, false);
                        xo = j == 1 ? __builtin_amdgcn_update_dpp(0, x[r], kX1, 0xf, 0xf, false)
                                    : __builtin_amdgcn_update_dpp(0, x[r], kX2, 0xf, 0xf, false);
                        ko = ((uint64_t)hi << 32) | lo;
                    } else {
                        ko = __shfl_xor(k[r], j);
                        xo = __shfl_xor(x[r], j);
                    }
                    const bool asc = ((64 * r + lane) & kk) == 0;
                    const bool lower = (lane & j) == 0;  // this element comes first in the pair
                    const bool olt = ko < k[r] || (ko == k[r] && xo < x[r]);
                    // the first of an ascending pair (or the second of a
                    // descending one) keeps the smaller element
                    if ((lower == asc) ? olt : !olt) {
                        k[r] = ko;
                        x[r] = xo;
                    }
                }
            }
        }
    }
    const int m = n < P ? n : P;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int i = 64 * r + lane;
        if (i < m) {
            ok[i] = __longlong_as_double((long long)k[r]);
            oi[i] = x[r];
        }
    }
}

// BLK: the samples are the block minima kmin [slot][2][T/16] of the key kernel
// (64 SPL of them per pair, SPL per lane), and only the blocks whose minimum
// is at or below the threshold are read for survivors. The P-th smallest
// block minimum bounds kP from above like any P-th smallest sample (the
// blocks are disjoint), and a centroid with ka <= thr lies in a block whose
// minimum is <= thr.
constexpr int kBlkCap = 512;  // blocks a wavefront reads for survivors

template <int SPL, bool BLK>
__global__ __launch_bounds__(kWPB * 64) __attribute__((amdgpu_waves_per_eu(4))) void k_prefix_wave(
    const float *__restrict__ kapprox, const float *__restrict__ kmin, const float *__restrict__ Q, int D,
    const float *__restrict__ C1, const float *__restrict__ C2, float cmax1, float cmax2, float ecoef, int T,
    const int32_t *qlist, int64_t nslots, int P, double *__restrict__ lkey, int32_t *__restrict__ lidx,
    int32_t *__restrict__ pstat, unsigned long long *stats)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t pair = (int64_t)blockIdx.x * kWPB + wv;
    if (pair >= nslots * 2) return;
    const int64_t slot = pair >> 1;
    const int half = (int)(pair & 1);
    const int h = D / 2, hpad = (h + 3) & ~3;
    float *qh = reinterpret_cast<float *>(smem) + (size_t)wv * hpad;
    int32_t *sidx = reinterpret_cast<int32_t *>(reinterpret_cast<float *>(smem) + (size_t)kWPB * hpad) +
                    (size_t)wv * kWaveS;
    uint32_t *hist = reinterpret_cast<uint32_t *>(reinterpret_cast<int32_t *>(reinterpret_cast<float *>(smem) +
                                                                              (size_t)kWPB * hpad) +
                                                  (size_t)kWPB * kWaveS) +
                     (size_t)wv * 256;
    const int64_t qs = qlist ? qlist[slot] : slot;
    const float *C = half ? C2 : C1;
    const float cmax = half ? cmax2 : cmax1;
    const float *kg = kapprox + (slot * 2 + half) * (int64_t)T;
    for (int t = lane; t < h; t += 64) qh[t] = Q[qs * D + half * h + t];

    // Keys are read 16 bytes per lane, kF4 loads per lane per chunk of
    // kChunk centroids; element c = cb + 4 (lane + 64 m) + j of chunk cb falls
    // in sample s = j + 4 (m mod SPL/4) of this lane (64 SPL disjoint groups).
    // A single chunk (T <= kChunk) stays in registers for the survivor pass.
    constexpr int kF4 = 16, kChunk = 64 * 4 * kF4;
    const bool v4 = (T & 3) == 0;
    float x[4 * kF4];
    auto load_chunk = [&](int cb) __attribute__((always_inline)) {
#pragma unroll
        for (int m = 0; m < kF4; ++m) {
            const int c = cb + 4 * (lane + 64 * m);
            if (v4 && c + 3 < T) {
                const float4 f = *reinterpret_cast<const float4 *>(kg + c);
                x[4 * m] = f.x;
                x[4 * m + 1] = f.y;
                x[4 * m + 2] = f.z;
                x[4 * m + 3] = f.w;
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) x[4 * m + j] = c + j < T ? kg[c + j] : __builtin_huge_valf();
            }
        }
    };
    float smp[SPL];
    const int nch = (T + kChunk - 1) / kChunk;
    if constexpr (BLK) {
        // this lane's SPL consecutive block minima (T = 1024 SPL)
        const float *mg = kmin + (slot * 2 + half) * (int64_t)(T / 16) + lane * SPL;
#pragma unroll
        for (int q = 0; q < SPL; q += 4) {
            const float4 f = *reinterpret_cast<const float4 *>(mg + q);
            smp[q] = f.x;
            smp[q + 1] = f.y;
            smp[q + 2] = f.z;
            smp[q + 3] = f.w;
        }
    } else {
#pragma unroll
        for (int q = 0; q < SPL; ++q) smp[q] = __builtin_huge_valf();
        for (int ch = 0; ch < nch; ++ch) {
            load_chunk(ch * kChunk);
#pragma unroll
            for (int m = 0; m < kF4; ++m)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int q = j + 4 * (m % (SPL / 4));
                    smp[q] = x[4 * m + j] < smp[q] ? x[4 * m + j] : smp[q];
                }
        }
    }
    uint32_t u[SPL];
#pragma unroll
    for (int q = 0; q < SPL; ++q) u[q] = okey(smp[q]);
    // The P-th smallest sample key, one byte at a time from its top three: a 256-bin
    // histogram of the samples that match the bytes found so far, a scan over
    // the lanes (four bins each), and the bin where the running count reaches
    // the rank still needed. LDS executes a wavefront's instructions in issue
    // order, so waiting for them (lgkmcnt 0) orders the clear, the atomic adds
    // and the reads; the empty asm keeps the compiler from moving them.
    auto lds_order = [&]() __attribute__((always_inline)) {
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0) only
        __builtin_amdgcn_wave_barrier();
        __asm__ __volatile__("" ::: "memory");
    };
    uint32_t pre = 0, hm = 0;
    int need = P;  // at most the 64 SPL samples, so a bin always reaches it
    for (int sh = 24; sh >= 8; sh -= 8) {
        reinterpret_cast<uint4 *>(hist)[lane] = uint4{0u, 0u, 0u, 0u};
        lds_order();
#pragma unroll
        for (int q = 0; q < SPL; ++q)
            if ((u[q] & hm) == pre) atomicAdd(&hist[(u[q] >> sh) & 255u], 1u);
        lds_order();
        const uint4 hb = reinterpret_cast<const uint4 *>(hist)[lane];  // bins 4 lane .. 4 lane + 3
        const uint32_t s4 = hb.x + hb.y + hb.z + hb.w;
        uint32_t inc = s4;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(inc, o);
            if (lane >= o) inc += t;
        }
        const uint32_t exc = inc - s4;
        const int L = __ffsll(__ballot(exc < (uint32_t)need && (uint32_t)need <= inc)) - 1;
        int bin = 0;
        uint32_t low = 0;
        if (lane == L) {
            // the first of the lane's four bins where the count reaches need
            // (no indexed array: the dispatch needs no scratch memory)
            uint32_t c = exc;
            int j = 0;
            if (c + hb.x < (uint32_t)need) {
                c += hb.x;
                j = 1;
                if (c + hb.y < (uint32_t)need) {
                    c += hb.y;
                    j = 2;
                    if (c + hb.z < (uint32_t)need) {
                        c += hb.z;
                        j = 3;
                    }
                }
            }
            bin = 4 * L + j;
            low = c;
        }
        bin = __shfl(bin, L);
        low = __shfl(low, L);
        pre |= (uint32_t)bin << sh;
        hm |= 255u << sh;
        need -= (int)low;
        lds_order();  // the reads are done before the next clear
    }
    // The largest key with those three bytes bounds the P-th smallest sample
    // from above (any value whose top 24 bits match is at most it); a bucket
    // that holds +inf keeps +inf, the rest of it being NaN patterns.
    pre = (pre >> 8) == 0xFF8000u ? 0xFF800000u : (pre | 0xFFu);
    // error bound of the approximate keys (any summation order; the split
    // FP16 products too, through the index's coefficient)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double qn = 0.0;
    for (int t = lane; t < h; t += 64) qn += (double)qh[t] * (double)qh[t];
    for (int o = 32; o > 0; o >>= 1) qn += __shfl_xor(qn, o);
    const double rn = sqrt(qn) + sqrt((double)cmax) * (1.0 + 1e-6);
    const float err = (float)(ecoef * 0x1.0p-23 * rn * rn) + 1e-30f;
    const float thr = unokey(pre) + 2.f * err;

    // survivors (ka <= thr), compacted with ballots
    const uint64_t below = (1ull << lane) - 1ull;
    int n = 0;
    if constexpr (BLK) {
        // the blocks that can hold a survivor, listed in LDS ...
        // (after the kWPB histograms: this wavefront's kBlkCap entries)
        int32_t *blk = reinterpret_cast<int32_t *>(hist - (size_t)wv * 256 + (size_t)kWPB * 256) + (size_t)wv * kBlkCap;
        int nb = 0;
#pragma unroll
        for (int q = 0; q < SPL; ++q) {
            const bool cand = smp[q] <= thr;
            const uint64_t bm = __ballot(cand);
            if (cand) {
                const int w = nb + __popcll(bm & below);
                if (w < kBlkCap) blk[w] = lane * SPL + q;
            }
            nb += __popcll(bm);
        }
        if (nb > kBlkCap) {
            if (lane == 0) pstat[pair] = 1;
            return;
        }
        lds_order();
        // ... then read them, four blocks (16 keys each) per step and kBlkU
        // steps' loads in flight at once
        constexpr int kBlkU = 8;
        for (int b0 = 0; b0 < nb; b0 += 4 * kBlkU) {
            int cc[kBlkU];
            float kv[kBlkU];
#pragma unroll
            for (int u = 0; u < kBlkU; ++u) {
                const int bi = b0 + 4 * u + (lane >> 4);
                cc[u] = bi < nb ? blk[bi] * 16 + (lane & 15) : T;
            }
#pragma unroll
            for (int u = 0; u < kBlkU; ++u) kv[u] = cc[u] < T ? kg[cc[u]] : __builtin_huge_valf();
#pragma unroll
            for (int u = 0; u < kBlkU; ++u) {
                const bool sv = cc[u] < T && kv[u] <= thr;
                const uint64_t bm = __ballot(sv);
                if (sv) {
                    const int w = n + __popcll(bm & below);
                    if (w < kWaveS) sidx[w] = cc[u];
                }
                n += __popcll(bm);
            }
        }
    } else {
        for (int ch = 0; ch < nch; ++ch) {
            if (nch > 1) load_chunk(ch * kChunk);
#pragma unroll
            for (int m = 0; m < kF4; ++m)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int c = ch * kChunk + 4 * (lane + 64 * m) + j;
                    const bool sv = c < T && x[4 * m + j] <= thr;
                    const uint64_t bm = __ballot(sv);
                    if (sv) {
                        const int w = n + __popcll(bm & below);
                        if (w < kWaveS) sidx[w] = c;
                    }
                    n += __popcll(bm);
                }
        }
    }
    if (n > kWaveS) {
        if (lane == 0) pstat[pair] = 1;
        return;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double *ok = lkey + (slot * 2 + half) * (int64_t)P;
    int32_t *oi = lidx + (slot * 2 + half) * (int64_t)P;
    if (n <= 64) rank_survivors<1>(qh, C, h, sidx, n, P, lane, ok, oi);
    else if (n <= 128) rank_survivors<2>(qh, C, h, sidx, n, P, lane, ok, oi);
    else if (n <= 256) rank_survivors<4>(qh, C, h, sidx, n, P, lane, ok, oi);
    else rank_survivors<8>(qh, C, h, sidx, n, P, lane, ok, oi);
    if (lane == 0) {
        pstat[pair] = 0;
        if (stats) atomicAdd(&stats[kStatPrefixWave], 1ull);
    }
}

int select_sort_size(int P, int T)
{
    int S = 1;
    // room for 4P survivors of the approximate threshold (2P beyond 2048 ranks,
    // so that the buffer stays within LDS); more survivors take the exact select
    const int want = P <= 2048 ? 4 * P : 2 * P;
    const int need = P >= T ? T : (want < T ? want : T);
    while (S < need) S <<= 1;
    return S < 64 ? 64 : S;
}

// Dynamic LDS of the workgroup select, with or without the staged key row
// and with or without the sort buffer.
size_t select_lds_bytes(int D, int T, int S, bool stage_ka, bool sort_in_lds = true)
{
    const int h = D / 2;
    const size_t f = (size_t)((h + 3) & ~3) + (stage_ka ? (size_t)((T + 1) & ~1) : 0);
    return f * 4 + (sort_in_lds ? (size_t)S * (sizeof(uint64_t) + sizeof(int32_t)) : 0);
}

constexpr size_t kSelLdsMax = 144 * 1024;  // static LDS of the kernel is about 6 KB of the 160 KB

size_t prefix_sort_bytes(const DevIndex &ix, int32_t P)
{
    const int S = select_sort_size(P, ix.T);
    if (select_lds_bytes(ix.D, ix.T, S, false) <= kSelLdsMax) return 0;
    return (size_t)S * (sizeof(uint64_t) + sizeof(int32_t));
}

bool prefix_wave_ok(const DevIndex &ix, int32_t P) { return ix.T >= 256 && P <= 256 && P < ix.T; }

bool prefix_blocks_ok(const DevIndex &ix, int32_t P)
{
    // 64 SPL block minima per pair, SPL a power of two from 4 to 64, at least 2P of them
    const int spl = ix.T / 1024;
    return prefix_wave_ok(ix, P) && ix.T % 1024 == 0 && spl >= 4 && spl <= 64 && (spl & (spl - 1)) == 0 &&
           ix.T / 16 >= 2 * P;
}

hipError_t launch_prefix_wave(const DevIndex &ix, const float *q, const float *ka, const float *kmin,
                              int64_t nslots, const int32_t *qlist, int32_t P, double *lkey, int32_t *lidx,
                              int32_t *pstat, unsigned long long *stats, hipStream_t st)
{
    if (nslots == 0) return hipSuccess;
    if (!prefix_wave_ok(ix, P) || !pstat) return hipErrorInvalidValue;
    const bool blk = kmin && prefix_blocks_ok(ix, P);
    const int hpad = (ix.D / 2 + 3) & ~3;
    const size_t lds = (size_t)kWPB * ((size_t)hpad * 4 + (size_t)kWaveS * 4 + 256 * 4 + (blk ? kBlkCap * 4 : 0));
    const int64_t pairs = nslots * 2;
    const dim3 g((unsigned)((pairs + kWPB - 1) / kWPB)), b(kWPB * 64);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, g, b, lds, st, ka, kmin, q, ix.D, ix.C1, ix.C2, ix.cmax1, ix.cmax2, ix.ecoef, ix.T, qlist,
                           nslots, P, lkey, lidx, pstat, stats);
    };
    if (blk) {
        switch (ix.T / 1024) {
        case 4: go(k_prefix_wave<4, true>); break;
        case 8: go(k_prefix_wave<8, true>); break;
        case 16: go(k_prefix_wave<16, true>); break;
        case 32: go(k_prefix_wave<32, true>); break;
        default: go(k_prefix_wave<64, true>); break;
        }
    } else if (P <= 128) {
        go(k_prefix_wave<4, false>);
    } else {
        go(k_prefix_wave<8, false>);
    }
    return hipGetLastError();
}

hipError_t launch_prefix_block(const DevIndex &ix, const float *q, const float *ka, int64_t nslots,
                               const int32_t *qlist, int32_t P, double *lkey, int32_t *lidx,
                               const int32_t *pstat, unsigned long long *stats, unsigned char *gsort,
                               hipStream_t st)
{
    if (nslots == 0) return hipSuccess;
    const int S = select_sort_size(P, ix.T);
    const bool glob = prefix_sort_bytes(ix, P) > 0;  // sort buffer in HBM (long prefixes)
    if (glob && !gsort) return hipErrorInvalidValue;
    // stage the key row in LDS when it and the sort buffer fit
    const bool stage = ka && ix.T <= kApproxLds && select_lds_bytes(ix.D, ix.T, S, true, !glob) <= kSelLdsMax;
    const size_t lds = select_lds_bytes(ix.D, ix.T, S, stage, !glob);
    if (lds > kSelLdsMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_select_prefix, dim3((unsigned)nslots, 2), dim3(kSelThreads), lds, st, ka,
                       q, ix.D, ix.C1, ix.C2, ix.cmax1, ix.cmax2, ix.ecoef, ix.T, qlist, P, S, stage ? 1 : 0, lkey, lidx,
                       pstat, stats, glob ? gsort : nullptr);
    return hipGetLastError();
}

}  // namespace fbpq
