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
// slots x G source groups: lane (a, g) = lane (a G + g) takes target atom a
// of the current target chunk and the source atoms j = g, g+G, ... of every
// neighbour leaf.  Sources come from the padded copy xqp, in which every
// leaf holds a multiple of G atoms (q = 0 padding far away), so all lanes
// run the same trip count and the loop has no per-lane bounds test.  Each
// lane sums a leaf's (about n/G) potential terms in the mode's precision
// and adds that partial to an FP64 total, so rounding never accumulates over
// the ~125 n terms of a potential; the field terms fall off as 1/r^2 and are
// summed in the mode's precision.  The G partial sums of a target are
// combined with cross-lane shuffles at the end.
#include "fmm_internal.h"
#include "morton.h"

namespace fmm {

template <typename T> __device__ inline T rsqrt_t(T x);
template <> __device__ inline float rsqrt_t<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ inline double rsqrt_t<double>(double x) { return 1.0 / sqrt(x); }

template <typename T> struct Vec4 { typedef T type __attribute__((ext_vector_type(4))); };

// Potential and field at (ox, oy, oz) from the nk sources bp[0], bp[G], ...
// SELF: the sources are the target's own leaf; skip the source at index self.
template <typename T, int G, bool SELF>
__device__ inline void p2p_leaf(const typename Vec4<T>::type *__restrict__ bp, int nk, T ox, T oy, T oz,
                                const typename Vec4<T>::type *selfp, double &ph, T &fx, T &fy, T &fz) {
    T pc = 0;
#pragma unroll 4
    for (int k = 0; k < nk; ++k) {
        const typename Vec4<T>::type b = bp[k * G];
        const T dx = ox - b.x, dy = oy - b.y, dz = oz - b.z;
        const T r2 = dx * dx + dy * dy + dz * dz;
        T rinv = rsqrt_t<T>(r2);
        if (SELF) rinv = (bp + k * G == selfp) ? (T)0 : rinv;
        const T qr = b.w * rinv;
        const T qr3 = qr * rinv * rinv;
        pc += qr;
        fx += qr3 * dx;
        fy += qr3 * dy;
        fz += qr3 * dz;
    }
    ph += (double)pc;
}

template <typename T, int G>
__global__ __launch_bounds__(256) void k_p2p(int64_t nleaf, int levels, const T *__restrict__ xqp,
                                             const int32_t *__restrict__ pstart, const int32_t *__restrict__ start,
                                             T h, double *__restrict__ phi, T *__restrict__ field, int nsplit) {
    using V4 = typename Vec4<T>::type;
    constexpr int TS = 64 / G;
    const int lane = threadIdx.x & 63;
    const int g = lane % G;
    const int a = lane / G;
    const uint32_t nmask = (1u << levels) - 1u;
    const V4 *X = reinterpret_cast<const V4 *>(xqp);
    // Work items (leaf, part), wavefront-uniform so that the neighbour walk
    // stays on the scalar unit: the target chunks of a leaf are dealt
    // round-robin to nsplit items so that small boxes still fill the chip.
    // The grid may be smaller than the item count (each wavefront then takes
    // every stride-th item).  Capping it so that the far-field kernels of the
    // other stream keep room on every CU was measured slower on the 1M-atom
    // box (2 workgroups per CU: P2P 19.7 ms, step 29.7 ms), so the callers
    // launch the full grid.
    const int64_t nitem = nleaf * nsplit;
    const int first = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    const int stride = gridDim.x * 4;
    for (int64_t wv = first; wv < nitem; wv += stride) {
        const int64_t leaf = wv / nsplit;
        const int part = (int)(wv % nsplit);
        uint32_t cx, cy, cz;
        demorton3((uint32_t)leaf, cx, cy, cz);
        const int32_t s0 = start[leaf], cnt = start[leaf + 1] - s0;
        const int32_t p0 = pstart[leaf], pcnt = pstart[leaf + 1] - p0;
        for (int32_t tb = part * TS; tb < cnt; tb += nsplit * TS) {
            const int32_t t = tb + a;
            const int32_t tl = min(t, pcnt - 1);  // lanes past the leaf redo its last slot, unstored
            const V4 ti = X[p0 + tl];
            double ph = 0;
            T fx = 0, fy = 0, fz = 0;
            p2p_leaf<T, G, true>(X + p0 + g, pcnt / G, ti.x, ti.y, ti.z, X + p0 + tl, ph, fx, fy, fz);
            for (int c = 0; c < 125; ++c) {
                if (c == 62) continue;  // offset (0, 0, 0): done above
                const int dx = c / 25 - kWS, dy = (c / 5) % 5 - kWS, dz = c % 5 - kWS;
                const uint32_t sc = morton3((cx + dx) & nmask, (cy + dy) & nmask, (cz + dz) & nmask);
                const int32_t j0 = pstart[sc];
                const int nk = (pstart[sc + 1] - j0) / G;
                p2p_leaf<T, G, false>(X + j0 + g, nk, ti.x - (T)dx * h, ti.y - (T)dy * h, ti.z - (T)dz * h,
                                      nullptr, ph, fx, fy, fz);
            }
#pragma unroll
            for (int m = 1; m < G; m <<= 1) {
                ph += __shfl_xor(ph, m);
                fx += __shfl_xor(fx, m);
                fy += __shfl_xor(fy, m);
                fz += __shfl_xor(fz, m);
            }
            if (t < cnt && g == 0) {
                const int64_t si = s0 + t;
                phi[si] = ph;
                field[3 * si + 0] = fx;
                field[3 * si + 1] = fy;
                field[3 * si + 2] = fz;
            }
        }
    }
}

// max_wg > 0 caps the grid (the kernel loops over the remaining items)
template <typename T>
hipError_t launch_p2p(int64_t nleaf, int levels, const void *xqp, const int32_t *pstart, const int32_t *start,
                      double h, double *phi, T *field, int groups, int nsplit, int max_wg, hipStream_t s) {
    if (nsplit < 1 || nsplit > 64) return hipErrorInvalidValue;
    int64_t grid = (nleaf * nsplit + 3) / 4;
    if (max_wg > 0 && grid > max_wg) grid = max_wg;
    const T *x = (const T *)xqp;
    switch (groups) {
#define FMM_P2P_CASE(G)                                                                                    \
    case G:                                                                                                \
        hipLaunchKernelGGL((k_p2p<T, G>), dim3((unsigned)grid), dim3(256), 0, s, nleaf, levels, x, pstart, \
                           start, (T)h, phi, field, nsplit);                                              \
        break;
        FMM_P2P_CASE(1) FMM_P2P_CASE(2) FMM_P2P_CASE(4) FMM_P2P_CASE(8) FMM_P2P_CASE(16)
#undef FMM_P2P_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template hipError_t launch_p2p<float>(int64_t, int, const void *, const int32_t *, const int32_t *, double,
                                      double *, float *, int, int, int, hipStream_t);
template hipError_t launch_p2p<double>(int64_t, int, const void *, const int32_t *, const int32_t *, double,
                                       double *, double *, int, int, int, hipStream_t);

// Near-field solute-solvent pairs: out[s] = q_s sum_{j in NF(s), solvent} q_j / r
// for solute atoms s (0 for solvent).  One wavefront per leaf: the lanes flag
// the leaf's solute atoms; for each of them (wave-uniform loop) the lanes
// split the solvent sources of the 125 neighbour leaves, each lane summing its
// terms in FP64, then a fixed shuffle tree adds the lane sums.  Leaves without
// solute atoms only write zeros.
template <typename T>
__global__ __launch_bounds__(256) void k_p2p_uv(int64_t nleaf, int levels, const T *__restrict__ xq,
                                                const int32_t *__restrict__ start,
                                                const int32_t *__restrict__ perm, const uint8_t *__restrict__ mask,
                                                T h, double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t leaf = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    if (leaf >= nleaf) return;  // whole wavefront; no block barriers below
    uint32_t cx, cy, cz;
    demorton3((uint32_t)leaf, cx, cy, cz);
    const uint32_t nmask = (1u << levels) - 1u;
    const int32_t s0 = start[leaf], s1 = start[leaf + 1];
    for (int32_t base = s0; base < s1; base += 64) {
        const int32_t i = base + lane;
        const bool is_u = i < s1 && mask[perm[i]] != 0;
        if (i < s1 && !is_u) out[i] = 0.0;
        uint64_t todo = __ballot(is_u);
        while (todo) {
            const int k = __builtin_ctzll(todo);
            todo &= todo - 1;
            const int32_t a = base + k;  // wave-uniform solute atom
            const T xi = xq[4 * (int64_t)a], yi = xq[4 * (int64_t)a + 1], zi = xq[4 * (int64_t)a + 2];
            double acc = 0.0;
            for (int dx = -kWS; dx <= kWS; ++dx)
                for (int dy = -kWS; dy <= kWS; ++dy)
                    for (int dz = -kWS; dz <= kWS; ++dz) {
                        const uint32_t sc = morton3((cx + dx) & nmask, (cy + dy) & nmask, (cz + dz) & nmask);
                        const T ox = xi - (T)dx * h, oy = yi - (T)dy * h, oz = zi - (T)dz * h;
                        for (int32_t j = start[sc] + lane; j < start[sc + 1]; j += 64) {
                            if (mask[perm[j]]) continue;
                            const T *bj = xq + 4 * (int64_t)j;
                            const T ddx = ox - bj[0], ddy = oy - bj[1], ddz = oz - bj[2];
                            const T r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                            acc += (double)(bj[3] * rsqrt_t<T>(r2));
                        }
                    }
#pragma unroll
            for (int m = 1; m < 64; m <<= 1) acc += __shfl_xor(acc, m);
            if (lane == 0) out[a] = (double)xq[4 * (int64_t)a + 3] * acc;
        }
    }
}

template <typename T>
hipError_t launch_p2p_uv(int64_t n, int levels, const void *xq, const int32_t *start, const int32_t *perm,
                         const uint8_t *mask, double h, double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t nleaf = (int64_t)1 << (3 * levels);
    hipLaunchKernelGGL(k_p2p_uv<T>, dim3((unsigned)((nleaf + 3) / 4)), dim3(256), 0, s, nleaf, levels,
                       (const T *)xq, start, perm, mask, (T)h, out);
    return hipGetLastError();
}
template hipError_t launch_p2p_uv<float>(int64_t, int, const void *, const int32_t *, const int32_t *,
                                         const uint8_t *, double, double *, hipStream_t);
template hipError_t launch_p2p_uv<double>(int64_t, int, const void *, const int32_t *, const int32_t *,
                                          const uint8_t *, double, double *, hipStream_t);

}  // namespace fmm
