// Stages a4 (M2M) and a7 (L2L) on the matrix cores.
//
// Both are dense contractions with the 8 scale-invariant octant operators:
//   M2M  M~(P)      = sum_{o=0..7} A_o M~(8P + o)        (children -> parent)
//   L2L  L~(8P + o) += B_o L~(P)                         (parent -> child, merge)
// A workgroup of 8 wavefronts owns 16 consecutive parents P and one 16-row
// block of the output; wavefront o applies octant operator o.  M2M sums the
// 8 octant partials through LDS in FP64 (fixed order o = 0..7); L2L needs no
// reduction (each wavefront writes its own child octant).  One row block per
// wavefront keeps the dependent MFMA chain short (K/4 steps) and gives the
// small upper levels (1 to 512 parents) enough wavefronts to hide latency.
//
// Operators are stored in the lane order of v_mfma_*_16x16x4 (the same
// swizzle as the M2L operators) and stay L2-resident (16 matrices).  All
// row blocks of one parent block are placed on the same XCD (blockIdx mod 8)
// so the parents' / children's expansions are fetched into one L2 only.
// Compute type: FP64 when either side of the translation is stored in FP64
// (levels 0-3 in mixed mode, everything in FP64 mode), FP32 otherwise.
#include <type_traits>

#include "fmm_internal.h"
#include "mfma.h"

namespace fmm {

template <typename Tin, typename Tout> struct TreeCompute {
    using T = typename std::conditional<(sizeof(Tin) == 8 || sizeof(Tout) == 8), double, float>::type;
};

template <typename T, typename Tin>
__device__ inline typename Mfma<T>::V load_frag(const Tin *p) {
    using V = typename Mfma<T>::V;
    if constexpr (sizeof(Tin) == sizeof(T)) {
        return *reinterpret_cast<const V *>(p);
    } else {
        const f32x4 f = *reinterpret_cast<const f32x4 *>(p);  // float expansion, FP64 compute
        return V{(T)f[0], (T)f[1], (T)f[2], (T)f[3]};
    }
}

// blockIdx -> (parent block, row block): consecutive groups of 8 blocks hold
// 8 different parent blocks (one per XCD); a parent block's NB row blocks
// are 8 blocks apart, hence on the same XCD.
__device__ inline void tree_tile(int NB, int64_t &pblk, int &rb) {
    const int64_t g = (int64_t)blockIdx.x >> 3;
    pblk = (g / NB) * 8 + (blockIdx.x & 7);
    rb = (int)(g % NB);
}

template <typename Tin, typename Tout, bool M2M>
__global__ __launch_bounds__(512) void k_tree(const typename TreeCompute<Tin, Tout>::T *__restrict__ ops,
                                              const Tin *__restrict__ in, Tout *__restrict__ out, int64_t nparent,
                                              int NB, int Kp) {
    using T = typename TreeCompute<Tin, Tout>::T;
    using V = typename Mfma<T>::V;
    __shared__ double red[M2M ? 8 : 1][4][64];
    const int lane = threadIdx.x & 63;
    const int o = threadIdx.x >> 6;  // octant
    int64_t pblk;
    int rb;
    tree_tile(NB, pblk, rb);
    if (pblk * 16 >= nparent) return;  // whole workgroup, before any barrier
    const int64_t P = pblk * 16 + (lane & 15);
    const bool valid = P < nparent;
    const int64_t Pc = valid ? P : 0;

    const Tin *src = in + (size_t)(M2M ? 8 * Pc + o : Pc) * Kp + 4 * (lane >> 4);
    const T *ap = ops + (size_t)o * NB * NB * 256 + ((size_t)rb * 64 + lane) * 4;
    V acc = V{0, 0, 0, 0};
    for (int kc = 0; kc < NB; ++kc) {
        const V b = load_frag<T, Tin>(src + 16 * kc);
        const V a = *reinterpret_cast<const V *>(ap + (size_t)kc * NB * 256);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc = Mfma<T>::mma(a[j], b[j], acc);
    }
    if constexpr (M2M) {
#pragma unroll
        for (int r = 0; r < 4; ++r) red[o][r][lane] = (double)acc[r];
        __syncthreads();
        if (threadIdx.x >= 256) return;
        const int r = threadIdx.x >> 6;
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) v += red[k][r][lane];
        if (valid) out[P * Kp + 16 * rb + Mfma<T>::row(lane, r)] = (Tout)v;
    } else {
        if (!valid) return;
        Tout *dst = out + (8 * P + o) * Kp + 16 * rb;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Tout *d = dst + Mfma<T>::row(lane, r);
            *d = (Tout)((double)*d + (double)acc[r]);  // merge into the M2L result
        }
    }
}

template <typename Tin, typename Tout>
static hipError_t launch_tree(bool m2m, int64_t nparent, const Tin *in, Tout *out, const void *ops, int p, int Kp,
                              hipStream_t s) {
    using T = typename TreeCompute<Tin, Tout>::T;
    (void)p;
    if (nparent <= 0) return hipSuccess;
    const int NB = Kp / 16;
    const int64_t nblk = (nparent + 15) / 16;
    const int64_t grid = ((nblk + 7) / 8) * 8 * NB;
    if (m2m)
        hipLaunchKernelGGL((k_tree<Tin, Tout, true>), dim3((unsigned)grid), dim3(512), 0, s, (const T *)ops, in, out,
                           nparent, NB, Kp);
    else
        hipLaunchKernelGGL((k_tree<Tin, Tout, false>), dim3((unsigned)grid), dim3(512), 0, s, (const T *)ops, in,
                           out, nparent, NB, Kp);
    return hipGetLastError();
}

template <typename Tin, typename Tout>
hipError_t launch_m2m_mfma(int64_t nparent, const Tin *Mchild, Tout *Mparent, const void *ops, int p, int Kp,
                           hipStream_t s) {
    return launch_tree<Tin, Tout>(true, nparent, Mchild, Mparent, ops, p, Kp, s);
}
template <typename Tin, typename Tout>
hipError_t launch_l2l_mfma(int64_t nparent, const Tin *Lparent, Tout *Lchild, const void *ops, int p, int Kp,
                           hipStream_t s) {
    return launch_tree<Tin, Tout>(false, nparent, Lparent, Lchild, ops, p, Kp, s);
}

template hipError_t launch_m2m_mfma<float, float>(int64_t, const float *, float *, const void *, int, int, hipStream_t);
template hipError_t launch_m2m_mfma<float, double>(int64_t, const float *, double *, const void *, int, int,
                                                   hipStream_t);
template hipError_t launch_m2m_mfma<double, double>(int64_t, const double *, double *, const void *, int, int,
                                                    hipStream_t);
template hipError_t launch_l2l_mfma<float, float>(int64_t, const float *, float *, const void *, int, int, hipStream_t);
template hipError_t launch_l2l_mfma<double, float>(int64_t, const double *, float *, const void *, int, int,
                                                   hipStream_t);
template hipError_t launch_l2l_mfma<double, double>(int64_t, const double *, double *, const void *, int, int,
                                                    hipStream_t);

}  // namespace fmm
