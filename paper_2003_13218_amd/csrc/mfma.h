// Matrix-core operand traits shared by the M2L and tree-translation kernels.
// v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64: lane l holds A[l % 16][l / 16]
// and B[l / 16][l % 16]; the 16x16 result is spread over 4 registers per lane
// with column l % 16 and a row given by row() (the layouts differ between the
// FP32 and FP64 instructions).
#pragma once
#include <hip/hip_runtime.h>

namespace fmm {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<float> {
    using V = f32x4;
    static constexpr int CB = 2;  // column blocks of 16 target cells per workgroup
    __device__ static inline V mma(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // row of the 16x16 result held by (lane, register r); the column is lane % 16
    __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct Mfma<double> {
    using V = f64x4;
    static constexpr int CB = 1;
    __device__ static inline V mma(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // the f64 variant interleaves result rows across registers
    __device__ static inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};


}  // namespace fmm
