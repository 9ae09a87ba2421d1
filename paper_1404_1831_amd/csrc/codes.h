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

}  // namespace fbpq
