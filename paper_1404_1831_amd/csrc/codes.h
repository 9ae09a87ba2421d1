// PQ code words of one half (M/2 bytes of a stored point) and the sum of
// their lookups in a half table lut [M/2][Kc]: the FP32 accumulation order
// every scan uses, table k = 0, 1, ... in turn (Section 3.1, equation
// decomposition, one lookup per subspace).
#pragma once

#include "fbpq_dev.h"

namespace fbpq {

template <int MH>
struct CodeU;
template <> struct CodeU<1> { using T = uint8_t; };
template <> struct CodeU<2> { using T = uint16_t; };
template <> struct CodeU<4> { using T = uint32_t; };
template <> struct CodeU<8> { using T = uint2; };
template <> struct CodeU<16> { using T = uint4; };

template <int MH>
__device__ __forceinline__ typename CodeU<MH>::T load_c(const uint8_t *__restrict__ codes, int64_t p)
{
    return *reinterpret_cast<const typename CodeU<MH>::T *>(codes + p * MH);
}

template <int MH>
__device__ __forceinline__ float lsum(const float *lut, typename CodeU<MH>::T c)
{
    // the running sum starts at the first lookup (0 + x = x for every
    // nonzero x, and the tables hold no -0 that could matter to a sum)
    if constexpr (MH == 1) {
        return lut[c];
    } else if constexpr (MH == 2) {
        return lut[c & 255] + lut[kKc + (c >> 8)];
    } else if constexpr (MH == 4) {
        float s = lut[c & 255];
#pragma unroll
        for (int k = 1; k < 4; ++k) s += lut[k * kKc + ((c >> (8 * k)) & 255)];
        return s;
    } else if constexpr (MH == 8) {
        float s = lut[c.x & 255];
#pragma unroll
        for (int k = 1; k < 4; ++k) s += lut[k * kKc + ((c.x >> (8 * k)) & 255)];
#pragma unroll
        for (int k = 0; k < 4; ++k) s += lut[(k + 4) * kKc + ((c.y >> (8 * k)) & 255)];
        return s;
    } else {
        const uint32_t cw[4] = {c.x, c.y, c.z, c.w};
        float s = lut[cw[0] & 255];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (q > 0 || k > 0) s += lut[(q * 4 + k) * kKc + ((cw[q] >> (8 * k)) & 255)];
        return s;
    }
}

// Byte k of a code word (k < MH).
template <int MH>
__device__ __forceinline__ uint32_t code_byte(typename CodeU<MH>::T c, int k)
{
    if constexpr (MH <= 4) {
        return ((uint32_t)c >> (8 * k)) & 255u;
    } else if constexpr (MH == 8) {
        return ((k < 4 ? c.x : c.y) >> (8 * (k & 3))) & 255u;
    } else {
        const uint32_t w = k < 4 ? c.x : k < 8 ? c.y : k < 12 ? c.z : c.w;
        return (w >> (8 * (k & 3))) & 255u;
    }
}

// cst + lsum(lut1, ca) + lsum(lut2, cb), the same additions in the same
// order, with all 2 * MH lookups issued before the first addition, so a
// wavefront keeps them in flight together.
template <int MH>
__device__ __forceinline__ float dsum(const float *lut1, const float *lut2, typename CodeU<MH>::T ca,
                                      typename CodeU<MH>::T cb, float cst)
{
    float v1[MH], v2[MH];
#pragma unroll
    for (int k = 0; k < MH; ++k) v1[k] = lut1[k * kKc + code_byte<MH>(ca, k)];
#pragma unroll
    for (int k = 0; k < MH; ++k) v2[k] = lut2[k * kKc + code_byte<MH>(cb, k)];
    float s1 = v1[0], s2 = v2[0];
#pragma unroll
    for (int k = 1; k < MH; ++k) s1 += v1[k];
#pragma unroll
    for (int k = 1; k < MH; ++k) s2 += v2[k];
    return cst + s1 + s2;
}

}  // namespace fbpq
