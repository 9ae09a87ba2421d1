// Query-independent tables of the FBPQ distance (Section 3.1, equation
// decomposition; sizes in Section 3.3). Built once per index.
//
//   CR1[i][k][r] = 2 <c1_i|k, R_k(r)>          k < M/2
//   CR2[j][k][r] = 2 <c2_j|k, R_{M/2+k}(r)>    k < M/2
//   nR[k][r]     = ||R_k(r)||^2
//   nC1[i], nC2[j] = squared norms of the half centroids
//
// c|k is the k-th D/M slice of a half centroid. With local codebooks the
// CR tables hold the CQ tables below instead. Accumulation is FP64, storage
// FP32. One thread per table entry: the inner loop is D/M long, the whole
// build is T*Kc*D FMAs, a one-off cost next to any search.
#include "fbpq_dev.h"

namespace fbpq {

__global__ void k_cross_table(const float *__restrict__ C, const float *__restrict__ R, int T,
                              int h, int M, int ds, int sub0, float *__restrict__ CR)
{
    const int Mh = M / 2;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)T * Mh * kKc;
    if (e >= total) return;
    const int r = (int)(e % kKc);
    const int k = (int)((e / kKc) % Mh);
    const int64_t i = e / ((int64_t)kKc * Mh);
    const float *c = C + i * h + (int64_t)k * ds;
    const float *w = R + ((int64_t)(sub0 + k) * kKc + r) * ds;
    double acc = 0.0;
    for (int t = 0; t < ds; ++t) acc += (double)c[t] * (double)w[t];
    CR[e] = (float)(2.0 * acc);
}

__global__ void k_norms(const float *__restrict__ R, int M, int ds, const float *__restrict__ C1,
                        const float *__restrict__ C2, int T, int h, float *__restrict__ nR,
                        float *__restrict__ nC1, float *__restrict__ nC2)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nr = (int64_t)M * kKc;
    if (e < nr) {
        const float *w = R + e * ds;
        double acc = 0.0;
        for (int t = 0; t < ds; ++t) acc += (double)w[t] * (double)w[t];
        nR[e] = (float)acc;
    } else if (e < nr + 2 * (int64_t)T) {
        const int64_t i = e - nr;
        const float *c = i < T ? C1 + i * h : C2 + (i - T) * h;
        double acc = 0.0;
        for (int t = 0; t < h; ++t) acc += (double)c[t] * (double)c[t];
        (i < T ? nC1[i] : nC2[i - T]) = (float)acc;
    }
}

// Local codebooks (HBPQ, Section 3.2): the query-independent part of the
// folded table of row i,
//   CQ[i][k][r] = ||Q^i_k(r)||^2 + 2 <c_i|k, Q^i_k(r)>,
// so that the table of a visited row is CQ[i] - 2 <q|k, Q^i_k(r)> and the
// distance is d1[i] + d2[j] plus one lookup per subspace (the squared norm of
// a displacement reconstruction splits over the disjoint subspaces).
__global__ void k_local_table(const float *__restrict__ C, const float *__restrict__ QL, int T, int h,
                              int M, int ds, float *__restrict__ CQ)
{
    const int Mh = M / 2;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)T * Mh * kKc;
    if (e >= total) return;
    const int k = (int)((e / kKc) % Mh);
    const int64_t i = e / ((int64_t)kKc * Mh);
    const float *c = C + i * h + (int64_t)k * ds;
    const float *w = QL + e * ds;  // [T][M/2][Kc][ds]: entry e is codeword (i, k, r)
    double nn = 0.0, cr = 0.0;
    for (int t = 0; t < ds; ++t) {
        nn += (double)w[t] * (double)w[t];
        cr += (double)c[t] * (double)w[t];
    }
    CQ[e] = (float)(nn + 2.0 * cr);
}

// Two-part FP16 form of the half-centroids for the approximate keys: the
// scaled value x = c scale (a power of two, exact) is hi + lo + r with
// hi = fp16(x), lo = fp16(x - hi) (the difference is exact in FP32) and
// |r| <= 2^-22 |x| when lo is normal.
__global__ void k_split_centroids(const float *__restrict__ C, int64_t n, int h, float scale, _Float16 *__restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int64_t c = e / h, t = e - c * h;
    const float x = C[e] * scale;
    const _Float16 hi = (_Float16)x;
    out[c * 2 * h + t] = hi;
    out[c * 2 * h + h + t] = (_Float16)(x - (float)hi);
}

hipError_t launch_split_centroids(const float *C, int64_t T, int h, float scale, _Float16 *out, hipStream_t st)
{
    const int64_t n = T * h;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_split_centroids, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, C, n, h, scale, out);
    return hipGetLastError();
}

hipError_t launch_tables(const DevIndex &ix, float *CR1, float *CR2, float *nR, float *nC1,
                         float *nC2, hipStream_t st)
{
    const int h = ix.D / 2, ds = ix.D / ix.M;
    const int64_t total = (int64_t)ix.T * (ix.M / 2) * kKc;
    const int bs = 256;
    const unsigned grid = (unsigned)((total + bs - 1) / bs);
    if (ix.local) {
        hipLaunchKernelGGL(k_local_table, dim3(grid), dim3(bs), 0, st, ix.C1, ix.QL, ix.T, h, ix.M, ds, CR1);
        hipLaunchKernelGGL(k_local_table, dim3(grid), dim3(bs), 0, st, ix.C2, ix.SL, ix.T, h, ix.M, ds, CR2);
    } else {
        hipLaunchKernelGGL(k_cross_table, dim3(grid), dim3(bs), 0, st, ix.C1, ix.R, ix.T, h, ix.M, ds,
                           0, CR1);
        hipLaunchKernelGGL(k_cross_table, dim3(grid), dim3(bs), 0, st, ix.C2, ix.R, ix.T, h, ix.M, ds,
                           ix.M / 2, CR2);
    }
    const int64_t nn = (int64_t)ix.M * kKc + 2 * (int64_t)ix.T;
    hipLaunchKernelGGL(k_norms, dim3((unsigned)((nn + bs - 1) / bs)), dim3(bs), 0, st, ix.R, ix.M,
                       ds, ix.C1, ix.C2, ix.T, h, nR, nC1, nC2);
    return hipGetLastError();
}

}  // namespace fbpq

namespace fbpq {

// Split AoS codes [n][M] into the two half planes [n][M/2] used by the scan.
__global__ void k_split_codes(const uint8_t *__restrict__ src, int64_t n, int M,
                              uint8_t *__restrict__ a, uint8_t *__restrict__ b)
{
    const int Mh = M / 2;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * M) return;
    const int64_t p = e / M;
    const int k = (int)(e % M);
    if (k < Mh) a[p * Mh + k] = src[e];
    else b[p * Mh + (k - Mh)] = src[e];
}

// Fills n int32 with v (a kernel rather than a memset, so that it can sit in
// a captured graph).
__global__ void k_fill_i32(int32_t *__restrict__ p, int32_t v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

// Per-query budgets given on the device: copies L and k into the search's own
// arrays, clamped into [1, L_max] and [1, k_max], and counts the entries that
// were out of range in *nclamped.
__global__ void k_sanitize(const int64_t *__restrict__ L, const int32_t *__restrict__ k, int64_t n, int64_t L_max,
                           int32_t k_max, int64_t *__restrict__ Lo, int32_t *__restrict__ ko,
                           int32_t *__restrict__ nclamped)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t l = L[i];
    const int32_t kk = k[i];
    const int64_t lc = l < 1 ? 1 : (l > L_max ? L_max : l);
    const int32_t kc = kk < 1 ? 1 : (kk > k_max ? k_max : kk);
    Lo[i] = lc;
    ko[i] = kc;
    if (lc != l || kc != kk) atomicAdd(nclamped, 1);
}

hipError_t launch_sanitize(const int64_t *L, const int32_t *k, int64_t n, int64_t L_max, int32_t k_max, int64_t *Lo,
                           int32_t *ko, int32_t *nclamped, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sanitize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, L, k, n, L_max, k_max, Lo,
                       ko, nclamped);
    return hipGetLastError();
}

__global__ void k_copy_i32(const int32_t *__restrict__ src, int32_t *__restrict__ dst) { *dst = *src; }

hipError_t launch_copy_i32(const int32_t *src, int32_t *dst, hipStream_t st)
{
    hipLaunchKernelGGL(k_copy_i32, dim3(1), dim3(1), 0, st, src, dst);
    return hipGetLastError();
}

hipError_t launch_split_codes(const uint8_t *src, int64_t n, int M, uint8_t *a, uint8_t *b,
                              hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const int64_t total = n * M;
    hipLaunchKernelGGL(k_split_codes, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, src,
                       n, M, a, b);
    return hipGetLastError();
}

}  // namespace fbpq
