// Stage a9: P2P near field (eq. EqNF): for every atom i in leaf c,
//   phi_i = sum_{t in [-2,2]^3} sum_{j in leaf (c + t) mod n} q_j / |r_i - r_j - s_t|
// where s_t is the image shift implied by the unwrapped offset t (so a
// wrapped leaf seen under two shifts at shallow levels is visited twice),
// and i == j is skipped only for t = 0.  field_i = -grad phi_i.
//
// Coordinates are leaf-local (atom minus leaf centre), so the source
// position relative to the target leaf centre is x_j + t h: all FP32
// arithmetic stays at the scale of a few leaf edges.
//
// One wavefront per leaf.  The 64 lanes are split into TS = 64/G target
// slots x G source groups: lane (a, g) takes target atom a of the current
// target chunk and the source atoms j = g, g+G, ... of every neighbour leaf.
// The G partial sums of a target are combined with cross-lane shuffles at the
// end.  G is chosen from the mean leaf occupancy so both the target chunk and
// the source stride stay nearly full.
#include "fmm_internal.h"
#include "morton.h"

namespace fmm {

template <typename T> __device__ inline T rsqrt_t(T x);
template <> __device__ inline float rsqrt_t<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ inline double rsqrt_t<double>(double x) { return 1.0 / sqrt(x); }

template <typename T, int G>
__global__ __launch_bounds__(256) void k_p2p(int64_t nleaf, int levels, const T *__restrict__ xq,
                                             const int32_t *__restrict__ start, T h,
                                             double *__restrict__ phi, T *__restrict__ field) {
    constexpr int TS = 64 / G;
    const int lane = threadIdx.x & 63;
    const int64_t leaf = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (leaf >= nleaf) return;  // whole wavefront; no block barriers below
    const int g = lane % G;
    const int a = lane / G;
    uint32_t cx, cy, cz;
    demorton3((uint32_t)leaf, cx, cy, cz);
    const uint32_t nmask = (1u << levels) - 1u;
    const int32_t s0 = start[leaf], s1 = start[leaf + 1];
    for (int32_t base = s0; base < s1; base += TS) {
        const int32_t si = base + a;
        const bool act = si < s1;
        T xi = 0, yi = 0, zi = 0;
        if (act) {
            xi = xq[4 * (int64_t)si + 0];
            yi = xq[4 * (int64_t)si + 1];
            zi = xq[4 * (int64_t)si + 2];
        }
        // the potential sums ~125 x (atoms per leaf) terms whose partial sums
        // are O(1): it is accumulated in FP64 (an FP64 add costs one VALU
        // slot, like an FP32 add); the field terms fall off as 1/r^2 and stay
        // in the mode's precision
        double ph = 0;
        T fx = 0, fy = 0, fz = 0;
        for (int dx = -kWS; dx <= kWS; ++dx)
            for (int dy = -kWS; dy <= kWS; ++dy)
                for (int dz = -kWS; dz <= kWS; ++dz) {
                    const uint32_t sc = morton3((cx + dx) & nmask, (cy + dy) & nmask, (cz + dz) & nmask);
                    const int32_t j0 = start[sc], j1 = start[sc + 1];
                    const T ox = xi - (T)dx * h, oy = yi - (T)dy * h, oz = zi - (T)dz * h;
                    const bool center = (dx == 0 && dy == 0 && dz == 0);
                    for (int32_t j = j0 + g; j < j1; j += G) {
                        const T *b = xq + 4 * (int64_t)j;
                        const T ddx = ox - b[0], ddy = oy - b[1], ddz = oz - b[2];
                        const bool self = center && (j == si);
                        const T qj = (self || !act) ? (T)0 : b[3];
                        T r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                        r2 = self ? (T)1 : r2;
                        const T rinv = rsqrt_t<T>(r2);
                        const T qr = qj * rinv;
                        const T qr3 = qr * rinv * rinv;
                        ph += (double)qr;
                        fx += qr3 * ddx;
                        fy += qr3 * ddy;
                        fz += qr3 * ddz;
                    }
                }
#pragma unroll
        for (int m = 1; m < G; m <<= 1) {
            ph += __shfl_xor(ph, m);
            fx += __shfl_xor(fx, m);
            fy += __shfl_xor(fy, m);
            fz += __shfl_xor(fz, m);
        }
        if (act && g == 0) {
            phi[si] = ph;
            field[3 * (int64_t)si + 0] = fx;
            field[3 * (int64_t)si + 1] = fy;
            field[3 * (int64_t)si + 2] = fz;
        }
    }
}

template <typename T>
hipError_t launch_p2p(int64_t nleaf, int levels, const void *xq, const int32_t *start, double h, double *phi,
                      T *field, int groups, hipStream_t s) {
    const int64_t grid = (nleaf + 3) / 4;
    const T *x = (const T *)xq;
    switch (groups) {
        case 1: hipLaunchKernelGGL((k_p2p<T, 1>), dim3((unsigned)grid), dim3(256), 0, s, nleaf, levels, x, start, (T)h, phi, field); break;
        case 2: hipLaunchKernelGGL((k_p2p<T, 2>), dim3((unsigned)grid), dim3(256), 0, s, nleaf, levels, x, start, (T)h, phi, field); break;
        case 4: hipLaunchKernelGGL((k_p2p<T, 4>), dim3((unsigned)grid), dim3(256), 0, s, nleaf, levels, x, start, (T)h, phi, field); break;
        case 8: hipLaunchKernelGGL((k_p2p<T, 8>), dim3((unsigned)grid), dim3(256), 0, s, nleaf, levels, x, start, (T)h, phi, field); break;
        case 16: hipLaunchKernelGGL((k_p2p<T, 16>), dim3((unsigned)grid), dim3(256), 0, s, nleaf, levels, x, start, (T)h, phi, field); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template hipError_t launch_p2p<float>(int64_t, int, const void *, const int32_t *, double, double *, float *,
                                      int, hipStream_t);
template hipError_t launch_p2p<double>(int64_t, int, const void *, const int32_t *, double, double *,
                                       double *, int, hipStream_t);

// Near-field solute-solvent pairs: out[s] = q_s sum_{j in NF(s), solvent} q_j / r
// for solute atoms s (0 for solvent).  One thread per sorted atom; FP64 sum
// of terms evaluated in the mode's precision.
template <typename T>
__global__ void k_p2p_uv(int64_t n, int levels, const T *__restrict__ xq, const int32_t *__restrict__ start,
                         const int32_t *__restrict__ perm, const uint8_t *__restrict__ mask, T h,
                         double *__restrict__ out) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x) {
        if (!mask[perm[s]]) { out[s] = 0.0; continue; }
        // locate the leaf of s: binary search in start[]
        const int64_t nleaf = (int64_t)1 << (3 * levels);
        int64_t lo = 0, hi = nleaf;  // start[lo] <= s < start[hi]
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (start[mid] <= s) lo = mid; else hi = mid;
        }
        uint32_t cx, cy, cz;
        demorton3((uint32_t)lo, cx, cy, cz);
        const uint32_t nmask = (1u << levels) - 1u;
        const T xi = xq[4 * s], yi = xq[4 * s + 1], zi = xq[4 * s + 2], qi = xq[4 * s + 3];
        double acc = 0.0;
        for (int dx = -kWS; dx <= kWS; ++dx)
            for (int dy = -kWS; dy <= kWS; ++dy)
                for (int dz = -kWS; dz <= kWS; ++dz) {
                    const uint32_t sc = morton3((cx + dx) & nmask, (cy + dy) & nmask, (cz + dz) & nmask);
                    for (int32_t j = start[sc]; j < start[sc + 1]; ++j) {
                        if (mask[perm[j]]) continue;
                        const T ddx = xi - ((T)dx * h + xq[4 * (int64_t)j]);
                        const T ddy = yi - ((T)dy * h + xq[4 * (int64_t)j + 1]);
                        const T ddz = zi - ((T)dz * h + xq[4 * (int64_t)j + 2]);
                        const T r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                        acc += (double)(xq[4 * (int64_t)j + 3] * rsqrt_t<T>(r2));
                    }
                }
        out[s] = (double)qi * acc;
    }
}

template <typename T>
hipError_t launch_p2p_uv(int64_t n, int levels, const void *xq, const int32_t *start, const int32_t *perm,
                         const uint8_t *mask, double h, double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t g = (n + 255) / 256;
    if (g > 65535) g = 65535;
    hipLaunchKernelGGL(k_p2p_uv<T>, dim3((unsigned)g), dim3(256), 0, s, n, levels, (const T *)xq, start, perm,
                       mask, (T)h, out);
    return hipGetLastError();
}
template hipError_t launch_p2p_uv<float>(int64_t, int, const void *, const int32_t *, const int32_t *,
                                         const uint8_t *, double, double *, hipStream_t);
template hipError_t launch_p2p_uv<double>(int64_t, int, const void *, const int32_t *, const int32_t *,
                                          const uint8_t *, double, double *, hipStream_t);

}  // namespace fmm
