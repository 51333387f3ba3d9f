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
#include <type_traits>

#include "fmm_internal.h"
#include "morton.h"

namespace fmm {

template <typename T> __device__ inline T rsqrt_t(T x);
template <> __device__ inline float rsqrt_t<float>(float x) { return __builtin_amdgcn_rsqf(x); }
// FP64: the hardware estimate y0 of 1/sqrt(x), refined once in the series
// 1/sqrt(x) = y0 (1 - e)^(-1/2) = y0 (1 + e/2 + 3 e^2/8 + ...), e = 1 - x y0^2
// (Newton's step for the reciprocal square root with its second-order term):
// the relative error falls from |e| to about 5|e|^3/16, below rounding for any
// estimate good to 2^-18.  A correctly rounded 1/sqrt(x) (a square root and a
// division) costs about three times as many instructions.
template <> __device__ inline double rsqrt_t<double>(double x) {
    const double y0 = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y0, y0, 1.0);
    return fma(y0 * e, fma(0.375, e, 0.5), y0);
}

template <typename T> struct Vec4 { typedef T type __attribute__((ext_vector_type(4))); };

// One source-target pair: potential and field terms of source b at
// (ox, oy, oz); SKIP drops the pair (the target itself, or a zero lane).
template <typename T>
__device__ inline void p2p_pair(const typename Vec4<T>::type &b, T ox, T oy, T oz, bool skip, T &pc, T &fx, T &fy,
                                T &fz) {
    const T dx = ox - b.x, dy = oy - b.y, dz = oz - b.z;
    const T r2 = dx * dx + dy * dy + dz * dz;
    T rinv = rsqrt_t<T>(r2);
    rinv = skip ? (T)0 : rinv;
    const T qr = b.w * rinv;
    const T qr3 = qr * rinv * rinv;
    pc += qr;
    fx += qr3 * dx;
    fy += qr3 * dy;
    fz += qr3 * dz;
}

// BUF: the sources of one leaf read through a raw buffer descriptor (base
// address, no stride, the leaf's bytes as its size; GFX9 data-format word):
// a load takes the lane's byte offset in a vector register and the
// wave-uniform position in the leaf in a scalar register, so stepping through
// the leaf is one scalar add and no lane computes a 64-bit address.  Taken for
// FP64 sources (1M-atom box, FP64 near field 8.8 -> 8.4 ms); FP32 sources stay
// on global loads, with which that kernel measured faster (2.55 against 2.73
// ms) although it issues more vector instructions.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ inline __amdgpu_buffer_rsrc_t leaf_rsrc(const void *base, uint32_t nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)nbytes, 0x00020000);
}
__device__ inline Vec4<double>::type load_src(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
    const u32x4 b = __builtin_amdgcn_raw_buffer_load_b128(r, (int)(voff + 16u), (int)soff, 0);
    auto d = [](unsigned lo, unsigned hi) {
        return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    };
    return Vec4<double>::type{d(a.x, a.y), d(a.z, a.w), d(b.x, b.y), d(b.z, b.w)};
}

// Potential and field at (ox, oy, oz) from the sources base[g], base[g + G],
// ... of a leaf holding n (padded) sources starting at base.  n is a multiple
// of G, or of G / 2 when HALF: then a last half group may remain, whose upper
// lanes (g >= G / 2) read the same group's lower half again and drop it.
// SELF: the sources are the target's own leaf; skip source index self_i.
template <typename T, int G, bool SELF, bool HALF, bool BUF>
__device__ inline void p2p_leaf(const typename Vec4<T>::type *__restrict__ base, int n, int g, T ox, T oy, T oz,
                                int self_i, double &ph, T &fx, T &fy, T &fz) {
    using V4 = typename Vec4<T>::type;
    T pc = 0;
    const int nk = n / G;
    if constexpr (BUF) {
        static_assert(std::is_same<T, double>::value, "buffer loads of FP64 sources");
        constexpr uint32_t SZ = sizeof(V4);
        const __amdgpu_buffer_rsrc_t r = leaf_rsrc(base, (uint32_t)n * SZ);
        const uint32_t voff = (uint32_t)g * SZ;
#pragma unroll 4
        for (int k = 0; k < nk; ++k)
            p2p_pair<T>(load_src(r, voff, (uint32_t)k * G * SZ), ox, oy, oz, SELF && k * G + g == self_i, pc, fx, fy,
                        fz);
        if (HALF && n != nk * G) {  // wave-uniform
            const bool in = g < G / 2;
            const int i = nk * G + g - (in ? 0 : G / 2);
            p2p_pair<T>(load_src(r, (uint32_t)i * SZ, 0u), ox, oy, oz, !in || (SELF && i == self_i), pc, fx, fy, fz);
        }
    } else {
        const V4 *bp = base + g;
#pragma unroll 4
        for (int k = 0; k < nk; ++k) p2p_pair<T>(bp[k * G], ox, oy, oz, SELF && k * G + g == self_i, pc, fx, fy, fz);
        if (HALF && n != nk * G) {  // wave-uniform
            const bool in = g < G / 2;
            const int i = nk * G + g - (in ? 0 : G / 2);
            p2p_pair<T>(base[i], ox, oy, oz, !in || (SELF && i == self_i), pc, fx, fy, fz);
        }
    }
    ph += (double)pc;
}

// One chunk of up to 64 / G targets of a leaf (first target tb) against its
// 125 near-field leaves, G source groups per target; results stored by the
// lanes of group 0.
template <typename T, int G, bool HALF, bool BUF>
__device__ inline void p2p_chunk(const typename Vec4<T>::type *__restrict__ X, const int32_t *__restrict__ pstart,
                                 uint32_t cx, uint32_t cy, uint32_t cz, uint32_t nmask, int32_t s0, int32_t cnt,
                                 int32_t p0, int32_t pcnt, int32_t tb, T h, int lane, double *__restrict__ phi,
                                 T *__restrict__ field) {
    using V4 = typename Vec4<T>::type;
    const int g = lane % G;
    const int a = lane / G;
    const int32_t t = tb + a;
    const int32_t tl = min(t, pcnt - 1);  // lanes past the leaf redo its last slot, unstored
    const V4 ti = X[p0 + tl];
    double ph = 0;
    T fx = 0, fy = 0, fz = 0;
    p2p_leaf<T, G, true, HALF, BUF>(X + p0, pcnt, g, ti.x, ti.y, ti.z, tl, ph, fx, fy, fz);
    // The 124 other leaves of the 5^3 block, x slowest.  The image shift of
    // an axis runs through -2h, -h, 0, h, 2h by adding h, and every one of
    // those sums is exact, so ti - shift is rounded once, as ti - d h is: the
    // innermost leaf costs an add and a subtract instead of three conversions
    // and multiply-adds, and the compiler unrolls the five leaves of a z row
    // (1M-atom box, results bit-identical to one flat loop over the 125
    // offsets: FP32 near field 2.56 -> 2.45 ms, FP64 8.4 -> 5.8 ms).
    T xs = -(T)kWS * h;
    for (int dx = -kWS; dx <= kWS; ++dx, xs += h) {
        const T ox = ti.x - xs;
        T ys = -(T)kWS * h;
        for (int dy = -kWS; dy <= kWS; ++dy, ys += h) {
            const T oy = ti.y - ys;
            T zs = -(T)kWS * h;
            for (int dz = -kWS; dz <= kWS; ++dz, zs += h) {
                if (dx == 0 && dy == 0 && dz == 0) continue;  // the own leaf: done above
                const uint32_t sc = morton3((cx + dx) & nmask, (cy + dy) & nmask, (cz + dz) & nmask);
                const int32_t j0 = pstart[sc];
                p2p_leaf<T, G, false, HALF, BUF>(X + j0, pstart[sc + 1] - j0, g, ox, oy, ti.z - zs, -1, ph, fx, fy,
                                                 fz);
            }
        }
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

template <typename T, int G, bool BUF>
__global__ __launch_bounds__(256) void k_p2p(int64_t nleaf, int levels, const T *__restrict__ xqp,
                                             const int32_t *__restrict__ pstart, const int32_t *__restrict__ start,
                                             T h, double *__restrict__ phi, T *__restrict__ field, int nsplit) {
    using V4 = typename Vec4<T>::type;
    constexpr int TS = 64 / G;
    // a last chunk of at most TS / 2 targets runs with 2G source groups
    // (measured on the 1M-atom box: 7% fewer pair slots at G = 4)
    constexpr bool kHalfTail = G <= 8;
    const int lane = threadIdx.x & 63;
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
            if (kHalfTail && cnt - tb <= TS / 2)
                p2p_chunk<T, (kHalfTail ? 2 * G : G), true, BUF>(X, pstart, cx, cy, cz, nmask, s0, cnt, p0, pcnt, tb, h,
                                                            lane, phi, field);
            else
                p2p_chunk<T, G, false, BUF>(X, pstart, cx, cy, cz, nmask, s0, cnt, p0, pcnt, tb, h, lane, phi,
                                            field);
        }
    }
}

// max_wg > 0 caps the grid (the kernel loops over the remaining items);
// nsrc_max bounds the padded source count (buffer loads need every leaf's
// byte size and offsets below 2^31)
template <typename T>
hipError_t launch_p2p(int64_t nleaf, int levels, const void *xqp, const int32_t *pstart, const int32_t *start,
                      double h, double *phi, T *field, int groups, int nsplit, int max_wg, int64_t nsrc_max,
                      hipStream_t s) {
    if (nsplit < 1 || nsplit > 64) return hipErrorInvalidValue;
    int64_t grid = (nleaf * nsplit + 3) / 4;
    if (max_wg > 0 && grid > max_wg) grid = max_wg;
    const T *x = (const T *)xqp;
    const bool buf = std::is_same<T, double>::value && nsrc_max >= 0 &&
                     nsrc_max * (int64_t)sizeof(typename Vec4<T>::type) < ((int64_t)1 << 31);
    switch (groups) {
#define FMM_P2P_CASE(G)                                                                                        \
    case G:                                                                                                    \
        if constexpr (std::is_same<T, double>::value) {                                                        \
            if (buf) {                                                                                         \
                hipLaunchKernelGGL((k_p2p<T, G, true>), dim3((unsigned)grid), dim3(256), 0, s, nleaf, levels, x, \
                                   pstart, start, (T)h, phi, field, nsplit);                                   \
                break;                                                                                         \
            }                                                                                                  \
        }                                                                                                      \
        hipLaunchKernelGGL((k_p2p<T, G, false>), dim3((unsigned)grid), dim3(256), 0, s, nleaf, levels, x,      \
                           pstart, start, (T)h, phi, field, nsplit);                                           \
        break;
        FMM_P2P_CASE(1) FMM_P2P_CASE(2) FMM_P2P_CASE(4) FMM_P2P_CASE(8) FMM_P2P_CASE(16)
#undef FMM_P2P_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template hipError_t launch_p2p<float>(int64_t, int, const void *, const int32_t *, const int32_t *, double,
                                      double *, float *, int, int, int, int64_t, hipStream_t);
template hipError_t launch_p2p<double>(int64_t, int, const void *, const int32_t *, const int32_t *, double,
                                       double *, double *, int, int, int, int64_t, hipStream_t);

// Near-field solute-solvent pairs: nfuv[s] = q_s sum_{j in NF(s), solvent} q_j / r
// for the solute atoms s (ms[s] != 0; entries of solvent atoms are not
// written).  With a soft-core exponent set, also the soft-core sums of the
// lambda-coupled energy, in FP64: nfsc[s] = q_s sum q_j / s_ij and
// nfdl[s] = q_s sum q_j d(1/s_ij)/dlambda, s = (asc + r^c)^(1/c) with
// asc = alpha lambda sigma^c, and d(1/s)/dlambda = -kd s^(-c-1),
// kd = alpha sigma^c / c.
// One workgroup per leaf of every box.  The leaf's solute atoms are compacted (in order)
// into LDS; for each of them the 256 threads split the 125 neighbour leaves,
// two threads per leaf taking one half of its atoms each, sum their terms in
// FP64, and a fixed LDS tree adds the 256 partial sums.  Leaves without solute
// atoms read their mask bytes and return.
constexpr int kUvBlock = 256;

// r^c for a small positive integer c (r2 = r^2)
__device__ inline double pow_int_r(double r2, int c) {
    double x = (c & 1) ? sqrt(r2) : 1.0;
    for (int k = 0; k < c / 2; ++k) x *= r2;
    return x;
}

// blocks: one per leaf of every box (the box's leaf table)
template <typename T>
__global__ __launch_bounds__(kUvBlock) void k_uv_p2p(const UvBox *__restrict__ boxes, int nbox,
                                                     const int64_t *__restrict__ st) {
    __shared__ int32_t list[kUvBlock];
    __shared__ int wave_cnt[kUvBlock / 64];
    __shared__ double red[3][kUvBlock];
    const int w = box_of(st, nbox, blockIdx.x);
    const UvBox &b = boxes[w];
    const T *__restrict__ xq = reinterpret_cast<const T *>(b.xq);
    const int32_t *__restrict__ start = b.start;
    const uint8_t *__restrict__ ms = b.ms;
    const int levels = b.levels;
    const T h = (T)b.h;
    const bool soft = b.soft_c > 0;
    const int c = soft ? b.soft_c : 1;
    const double asc = b.asc, kd = b.kd;
    const double inv_c = 1.0 / (double)c;
    const uint32_t leaf = (uint32_t)(blockIdx.x - st[w]);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int32_t s0 = start[leaf], s1 = start[leaf + 1];
    bool ready = false;  // neighbour range of this thread set up
    int32_t j0 = 0, j1 = 0;
    T ox0 = 0, oy0 = 0, oz0 = 0;  // -(unwrapped offset) x h of this thread's neighbour leaf
    for (int32_t base = s0; base < s1; base += kUvBlock) {
        const int32_t i = base + tid;
        const bool is_u = i < s1 && ms[i] != 0;
        const uint64_t bal = __ballot(is_u);
        if (lane == 0) wave_cnt[wv] = __popcll(bal);
        __syncthreads();
        int off = 0, nu = 0;
        for (int k = 0; k < kUvBlock / 64; ++k) {
            if (k < wv) off += wave_cnt[k];
            nu += wave_cnt[k];
        }
        if (is_u) list[off + __popcll(bal & ((1ull << lane) - 1ull))] = i;
        __syncthreads();
        if (nu > 0 && !ready) {
            ready = true;
            const int cc = tid >> 1;
            if (cc < 125) {
                uint32_t cx, cy, cz;
                demorton3(leaf, cx, cy, cz);
                const uint32_t nmask = (1u << levels) - 1u;
                const int dx = cc / 25 - kWS, dy = (cc / 5) % 5 - kWS, dz = cc % 5 - kWS;
                const uint32_t sc = morton3((cx + dx) & nmask, (cy + dy) & nmask, (cz + dz) & nmask);
                const int32_t a0 = start[sc], a1 = start[sc + 1];
                const int32_t mid = a0 + (a1 - a0 + 1) / 2;
                j0 = (tid & 1) ? mid : a0;
                j1 = (tid & 1) ? a1 : mid;
                ox0 = -(T)dx * h;
                oy0 = -(T)dy * h;
                oz0 = -(T)dz * h;
            }
        }
        for (int k = 0; k < nu; ++k) {
            const int32_t a = list[k];
            const T xi = xq[4 * (int64_t)a] + ox0, yi = xq[4 * (int64_t)a + 1] + oy0,
                    zi = xq[4 * (int64_t)a + 2] + oz0;
            double acc = 0.0, asc_sum = 0.0, adl = 0.0;
            for (int32_t j = j0; j < j1; ++j) {
                if (ms[j]) continue;
                const T *bj = xq + 4 * (int64_t)j;
                const T ddx = xi - bj[0], ddy = yi - bj[1], ddz = zi - bj[2];
                const T r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                acc += (double)(bj[3] * rsqrt_t<T>(r2));
                if (soft) {
                    const double dx = (double)ddx, dy = (double)ddy, dz = (double)ddz;
                    const double x = asc + pow_int_r(dx * dx + dy * dy + dz * dz, c);
                    const double inv_s = pow(x, -inv_c);
                    asc_sum += (double)bj[3] * inv_s;
                    adl -= (double)bj[3] * kd * inv_s / x;
                }
            }
            red[0][tid] = acc;
            red[1][tid] = asc_sum;
            red[2][tid] = adl;
            __syncthreads();
            for (int sd = kUvBlock / 2; sd > 0; sd >>= 1) {
                if (tid < sd) {
                    red[0][tid] += red[0][tid + sd];
                    red[1][tid] += red[1][tid + sd];
                    red[2][tid] += red[2][tid + sd];
                }
                __syncthreads();
            }
            if (tid == 0) {
                const double qa = (double)xq[4 * (int64_t)a + 3];
                b.nfuv[a] = qa * red[0][0];
                if (soft) {
                    b.nfsc[a] = qa * red[1][0];
                    b.nfdl[a] = qa * red[2][0];
                }
            }
            __syncthreads();
        }
    }
}

template <typename T>
hipError_t launch_uv_p2p(const UvBox *b, int nbox, const int64_t *st_leaf, int64_t nb, hipStream_t s) {
    if (nb > 0) hipLaunchKernelGGL(k_uv_p2p<T>, dim3((unsigned)nb), dim3(kUvBlock), 0, s, b, nbox, st_leaf);
    return hipGetLastError();
}
template hipError_t launch_uv_p2p<float>(const UvBox *, int, const int64_t *, int64_t, hipStream_t);
template hipError_t launch_uv_p2p<double>(const UvBox *, int, const int64_t *, int64_t, hipStream_t);

}  // namespace fmm
