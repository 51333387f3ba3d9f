// 3-D Morton (bit-interleaved) cell indices, up to 10 bits per axis.
// Bit k of x goes to bit 3k+2, of y to 3k+1, of z to 3k.  With this order the
// eight children of cell P are 8P + o, o = 4 ox + 2 oy + oz.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace fmm {

__host__ __device__ inline uint32_t spread3(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__host__ __device__ inline uint32_t compact3(uint32_t v) {
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030C30C3u;
    v = (v | (v >> 4)) & 0x0300F00Fu;
    v = (v | (v >> 8)) & 0x030000FFu;
    v = (v | (v >> 16)) & 0x000003FFu;
    return v;
}

__host__ __device__ inline uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
    return (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
}

__host__ __device__ inline void demorton3(uint32_t k, uint32_t &x, uint32_t &y, uint32_t &z) {
    x = compact3(k >> 2);
    y = compact3(k >> 1);
    z = compact3(k);
}

}  // namespace fmm
