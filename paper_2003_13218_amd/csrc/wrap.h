// Periodic wrap and leaf index with explicitly rounded FP64 operations (no
// FMA contraction), so every kernel that needs them reproduces the plain
// definitions  w = x - b floor(x / b)  (0 when rounding gives b)  and
// c = floor(w * (2^L / b)) clamped to [0, 2^L - 1]  bit for bit.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace fmm {

__device__ inline double wrap_coord(double x, double b) {
    double y = __dsub_rn(x, __dmul_rn(b, floor(__ddiv_rn(x, b))));
    if (y >= b) y = 0.0;
    if (y < 0.0) y = 0.0;
    return y;
}

__device__ inline uint32_t leaf_coord(double w, double scale, uint32_t nc) {
    double f = floor(__dmul_rn(w, scale));
    uint32_t c = f < 0.0 ? 0u : (uint32_t)f;
    return c > nc - 1 ? nc - 1 : c;
}

}  // namespace fmm
