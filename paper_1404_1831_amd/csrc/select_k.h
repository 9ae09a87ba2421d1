// Block-level selection of the k smallest (distance, id) pairs, shared by the
// scan kernels. Elements are visited through a caller functor, so they can
// live in registers, in LDS or be computed on the fly.
//
// Keys are the order-preserving uint32 images of FP32 distances. Value bins
// over [lo, hi] locate the bin holding the k-th key; when the keys up to that
// bin number at most `wcap`, they are all collected and sorted by (key, id).
// Otherwise the range narrows to that bin and the histogram repeats. If the
// range collapses to a single key, the keys below it are taken and the ties
// are resolved by smallest id.
#pragma once

#include "fbpq_dev.h"

namespace fbpq {

constexpr int kSelBins = 1024;

struct SelShared {
    uint32_t hist[kSelBins];
    uint32_t red32[16];
    int redi[16];
    int s_bin, s_nwin, s_nties;
    uint32_t s_before, s_cnt;
};

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

template <int NT>
__device__ __forceinline__ uint32_t block_min_u32(uint32_t v, SelShared &sh)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t x = __shfl_xor(v, o);
        v = x < v ? x : v;
    }
    __syncthreads();
    if (lane == 0) sh.red32[wv] = v;
    __syncthreads();
    uint32_t r = sh.red32[0];
    for (int i = 1; i < NT / 64; ++i) r = sh.red32[i] < r ? sh.red32[i] : r;
    return r;
}

template <int NT>
__device__ __forceinline__ uint32_t block_max_u32(uint32_t v, SelShared &sh)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t x = __shfl_xor(v, o);
        v = x > v ? x : v;
    }
    __syncthreads();
    if (lane == 0) sh.red32[wv] = v;
    __syncthreads();
    uint32_t r = sh.red32[0];
    for (int i = 1; i < NT / 64; ++i) r = sh.red32[i] > r ? sh.red32[i] : r;
    return r;
}

template <int NT>
__device__ __forceinline__ int block_sum_i32(int v, SelShared &sh)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if (lane == 0) sh.redi[wv] = v;
    __syncthreads();
    int r = 0;
    for (int i = 0; i < NT / 64; ++i) r += sh.redi[i];
    return r;
}

// visit(f) calls f(key, getid) for every element this thread owns; getid()
// returns the element's id. Selects the kq smallest (key, id) of the `ntot`
// elements. win (wcap entries) is scratch for the collected candidates.
// sorted == true: writes the kq smallest, ascending, to out[0..n) and returns
// n = min(kq, ntot); out may be storage that visit reads (it is written only
// after the last visit). sorted == false: returns the collected set in
// win[0..n): every element whose key is below the kq-th smallest key plus
// possibly some at or above it (n <= wcap), unsorted. tie holds tcap entries.
template <int NT, typename Visit>
__device__ __forceinline__ int select_k(Visit &&visit, int ntot, int kq, uint64_t *win, int wcap,
                                        uint32_t *tie, int tcap, SelShared &sh, bool sorted,
                                        uint64_t *out)
{
    const int tid = threadIdx.x;
    if (tid == 0) {
        sh.s_nwin = 0;
        sh.s_nties = 0;
    }
    __syncthreads();
    auto put = [&](uint64_t val) __attribute__((always_inline)) {
        const int wi = atomicAdd(&sh.s_nwin, 1);
        if (wi < wcap) win[wi] = val;
    };
    if (ntot <= kq) {
        visit([&](uint32_t k, auto getid) __attribute__((always_inline)) { put(((uint64_t)k << 32) | getid()); });
    } else {
        uint32_t mn = 0xffffffffu, mx = 0;
        visit([&](uint32_t k, auto) __attribute__((always_inline)) {
            mn = k < mn ? k : mn;
            mx = k > mx ? k : mx;
        });
        uint32_t lo = block_min_u32<NT>(mn, sh);
        uint32_t hi = block_max_u32<NT>(mx, sh);
        int need = kq;
        bool collected = false;
        for (int level = 0; level < 8 && hi > lo; ++level) {
            // monotone bin map of [lo, hi] onto kSelBins bins (float scaling)
            const float scale = (float)kSelBins / ((float)(hi - lo) + 1.0f);
            auto bin_of = [&](uint32_t k) __attribute__((always_inline)) {
                const int b = (int)((float)(k - lo) * scale);
                return (uint32_t)(b < kSelBins ? b : kSelBins - 1);
            };
            for (int b = tid; b < kSelBins; b += NT) sh.hist[b] = 0;
            __syncthreads();
            visit([&](uint32_t k, auto) __attribute__((always_inline)) {
                if (k >= lo && k <= hi) atomicAdd(&sh.hist[bin_of(k)], 1u);
            });
            __syncthreads();
            if (tid < 64) {
                constexpr int per = kSelBins / 64;
                uint32_t c[per], sum = 0;
                for (int j = 0; j < per; ++j) {
                    c[j] = sh.hist[tid * per + j];
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
                        sh.s_bin = tid * per + j;
                        sh.s_before = before;
                        sh.s_cnt = c[j];
                    }
                    before += c[j];
                }
            }
            __syncthreads();
            const uint32_t bstar = (uint32_t)sh.s_bin;
            const int before = (int)sh.s_before, cntb = (int)sh.s_cnt;
            const int total = (kq - need) + before + cntb;  // keys below lo, plus bins <= bstar
            if (total <= wcap) {
                visit([&](uint32_t k, auto getid) __attribute__((always_inline)) {
                    if (k < lo || (k <= hi && bin_of(k) <= bstar))
                        put(((uint64_t)k << 32) | getid());
                });
                collected = true;
                break;
            }
            // narrow to the key range of the boundary bin
            uint32_t bmn = 0xffffffffu, bmx = 0;
            visit([&](uint32_t k, auto) __attribute__((always_inline)) {
                if (k >= lo && k <= hi && bin_of(k) == bstar) {
                    bmn = k < bmn ? k : bmn;
                    bmx = k > bmx ? k : bmx;
                }
            });
            const uint32_t nlo = block_min_u32<NT>(bmn, sh);
            const uint32_t nhi = block_max_u32<NT>(bmx, sh);
            need -= before;
            lo = nlo;
            hi = nhi;
            __syncthreads();
        }
        if (!collected) {
            // every remaining candidate has key lo: take the keys below it, then
            // the `need` smallest ids among the ties
            int my_eq = 0;
            visit([&](uint32_t k, auto getid) __attribute__((always_inline)) {
                if (k < lo) put(((uint64_t)k << 32) | getid());
                else if (k == lo) ++my_eq;
            });
            const int n_eq = block_sum_i32<NT>(my_eq, sh);
            const bool buffered = n_eq <= tcap;
            if (buffered) {
                visit([&](uint32_t k, auto getid) __attribute__((always_inline)) {
                    if (k == lo) {
                        const int ti = atomicAdd(&sh.s_nties, 1);
                        if (ti < tcap) tie[ti] = getid();
                    }
                });
            }
            __syncthreads();
            uint32_t last = 0;
            for (int r = 0; r < need; ++r) {
                uint32_t m = 0xffffffffu;
                if (buffered) {
                    for (int e = tid; e < n_eq; e += NT) {
                        const uint32_t id = tie[e];
                        if ((r == 0 || id > last) && id < m) m = id;
                    }
                } else {
                    visit([&](uint32_t k, auto getid) __attribute__((always_inline)) {
                        if (k != lo) return;
                        const uint32_t id = getid();
                        if ((r == 0 || id > last) && id < m) m = id;
                    });
                }
                const uint32_t mm = block_min_u32<NT>(m, sh);
                if (tid == 0) put(((uint64_t)lo << 32) | mm);
                last = mm;
            }
        }
    }
    __syncthreads();
    const int nwin = sh.s_nwin < wcap ? sh.s_nwin : wcap;
    if (!sorted) return nwin;
    // rank of each collected (key, id): the pairs are distinct, so ranks are too
    const int nk = nwin < kq ? nwin : kq;
    for (int i = tid; i < nwin; i += NT) {
        const uint64_t v = win[i];
        int rank = 0;
        for (int j = 0; j < nwin; ++j) rank += win[j] < v;
        if (rank < nk) out[rank] = v;
    }
    __syncthreads();
    return nk;
}

}  // namespace fbpq
