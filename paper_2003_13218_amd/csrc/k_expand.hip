// Stages a3 (P2M), a5 (lattice operator at level 0) and a8 (L2P with
// gradient) of the far field (Appendix B: eqs. P2M, EqFF; the level-0
// image-lattice sum of eq. 12).  M2M and L2L run on the matrix cores
// (k_tree.hip).
//
// Storage and scaling conventions are those of fmm_internal.h: real storage
// of the normalised harmonics, expansions at each level scaled by the cell
// edge so that every operator is level- and box-independent.
#include <algorithm>
#include <cmath>

#include "fmm_internal.h"
#include "morton.h"

namespace fmm {

constexpr int kTri = (kMaxP + 1) * (kMaxP + 2) / 2;
__constant__ double c_ra_d[kTri];
__constant__ double c_rb_d[kTri];
__constant__ double c_rc_d[kMaxP + 1];
__constant__ double c_rd_d[kMaxP + 1];
__constant__ float c_ra_f[kTri];
__constant__ float c_rb_f[kTri];
__constant__ float c_rc_f[kMaxP + 1];
__constant__ float c_rd_f[kMaxP + 1];

hipError_t upload_rec_tables(const RecTables &t) {
    float af[kTri], bf[kTri], cf[kMaxP + 1], df[kMaxP + 1];
    for (int i = 0; i < kTri; ++i) { af[i] = (float)t.a[i]; bf[i] = (float)t.b[i]; }
    for (int i = 0; i <= kMaxP; ++i) { cf[i] = (float)t.c[i]; df[i] = (float)t.d[i]; }
    hipError_t e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_ra_d), t.a, sizeof(t.a))) != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_rb_d), t.b, sizeof(t.b))) != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_rc_d), t.c, sizeof(t.c))) != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_rd_d), t.d, sizeof(t.d))) != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_ra_f), af, sizeof(af))) != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_rb_f), bf, sizeof(bf))) != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_rc_f), cf, sizeof(cf))) != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_rd_f), df, sizeof(df))) != hipSuccess) return e;
    return hipSuccess;
}

template <typename T> struct Rec;
template <> struct Rec<double> {
    __device__ static double a(int i) { return c_ra_d[i]; }
    __device__ static double b(int i) { return c_rb_d[i]; }
    __device__ static double c(int m) { return c_rc_d[m]; }
    __device__ static double d(int m) { return c_rd_d[m]; }
};
template <> struct Rec<float> {
    __device__ static float a(int i) { return c_ra_f[i]; }
    __device__ static float b(int i) { return c_rb_f[i]; }
    __device__ static float c(int m) { return c_rc_f[m]; }
    __device__ static float d(int m) { return c_rd_f[m]; }
};

// Calls f(n, m, re, im) with the normalised regular harmonic R^_n^m(x,y,z) for
// every 0 <= m <= n <= p (m outer, n inner), by the three-term recurrences
//   R^_m^m     = -c_m (x + i y) R^_{m-1}^{m-1}
//   R^_{m+1}^m = d_m z R^_m^m
//   R^_n^m     = a_nm z R^_{n-1}^m - b_nm r^2 R^_{n-2}^m.
template <typename T, typename F>
__device__ inline void regular_hat_foreach(T x, T y, T z, int p, F &&f) {
    const T r2 = x * x + y * y + z * z;
    T mre = 1, mim = 0;
    for (int m = 0; m <= p; ++m) {
        if (m > 0) {
            const T c = -Rec<T>::c(m);
            const T nre = c * (x * mre - y * mim);
            const T nim = c * (x * mim + y * mre);
            mre = nre;
            mim = nim;
        }
        f(m, m, mre, mim);
        if (m + 1 > p) continue;
        T p2re = mre, p2im = mim;
        const T dm = Rec<T>::d(m) * z;
        T p1re = dm * mre, p1im = dm * mim;
        f(m + 1, m, p1re, p1im);
        int ti = (m + 2) * (m + 3) / 2 + m;
        for (int n = m + 2; n <= p; ++n) {
            const T a = Rec<T>::a(ti) * z, b = Rec<T>::b(ti) * r2;
            const T cre = a * p1re - b * p2re;
            const T cim = a * p1im - b * p2im;
            f(n, m, cre, cim);
            p2re = p1re; p2im = p1im;
            p1re = cre; p1im = cim;
            ti += n + 1;
        }
    }
}

// The same recurrences for a compile-time order P, fully unrolled: every
// coefficient index is then a constant, and so is every recurrence constant,
// written here as the formula of build_rec_tables (harmonics_host.cpp) in FP64
// and rounded once to T, i.e. the value of the uploaded tables, which the
// compiler folds into the instructions instead of loading it.
template <typename T>
__device__ __forceinline__ T rec_a(int n, int m) {
    return (T)((double)(2 * n - 1) / __builtin_sqrt((double)((n + m) * (n - m))));
}
template <typename T>
__device__ __forceinline__ T rec_b(int n, int m) {
    return (T)__builtin_sqrt((double)((n + m - 1) * (n - m - 1)) / (double)((n + m) * (n - m)));
}
template <typename T>
__device__ __forceinline__ T rec_c(int m) {
    return (T)__builtin_sqrt((double)(2 * m - 1) / (double)(2 * m));
}
template <typename T>
__device__ __forceinline__ T rec_d(int m) {
    return (T)__builtin_sqrt((double)(2 * m + 1));
}
template <typename T, int P, typename F>
__device__ __forceinline__ void regular_hat_unrolled(T x, T y, T z, F &&f) {
    const T r2 = x * x + y * y + z * z;
    T mre = 1, mim = 0;
#pragma unroll
    for (int m = 0; m <= P; ++m) {
        if (m > 0) {
            const T c = -rec_c<T>(m);
            const T nre = c * (x * mre - y * mim);
            const T nim = c * (x * mim + y * mre);
            mre = nre;
            mim = nim;
        }
        f(m, m, mre, mim);
        if (m + 1 <= P) {
            T p2re = mre, p2im = mim;
            const T dm = rec_d<T>(m) * z;
            T p1re = dm * mre, p1im = dm * mim;
            f(m + 1, m, p1re, p1im);
#pragma unroll
            for (int n = m + 2; n <= P; ++n) {
                const T a = rec_a<T>(n, m) * z, b = rec_b<T>(n, m) * r2;
                const T cre = a * p1re - b * p2re;
                const T cim = a * p1im - b * p2im;
                f(n, m, cre, cim);
                p2re = p1re; p2im = p1im;
                p1re = cre; p1im = cim;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// P2M (eq. P2M): M~_n^m(leaf) = sum_j q_j conj(R^_n^m((r_j - c)/h)).
// One thread per (leaf, pair of orders {m, P - m}): the two columns n >= m of
// the pair hold P + 2 coefficients together whatever m is, so every thread
// does the same work per atom -- the two sectoral values (P steps of their
// recurrence) and P + 2 steps of the three-term recurrence in n, down column m
// and then down column P - m.  The middle column m = P/2 (P even) is a thread
// of its own.  Each thread walks its leaf's atoms in sorted order and keeps
// its P + 2 complex sums in FP64 registers (rounded once on store): no LDS,
// no cross-lane reduction, and every leaf (empty ones too) is written.
// ---------------------------------------------------------------------------
template <int P> constexpr int p2m_threads() { return P / 2 + 1; }

template <typename T, int P>
__global__ __launch_bounds__(256) void k_p2m(int64_t nleaf, const T *__restrict__ xq,
                                             const int32_t *__restrict__ start, T *__restrict__ M, int Kp,
                                             T inv_h) {
    constexpr int NT = p2m_threads<P>();  // threads per leaf
    constexpr int NS = P + 2;             // coefficients of a column pair
    constexpr int K = (P + 1) * (P + 1);
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t leaf = gid / NT;
    if (leaf >= nleaf) return;
    const int mA = (int)(gid - leaf * NT), mB = P - mA;
    const int nA = P + 1 - mA;             // steps down column mA (n = mA .. P)
    const int ns = mB != mA ? NS : nA;     // steps of this thread
    // per step: its order m, degree n and recurrence weights (z and r^2)
    T ca[NS], cb[NS];
#pragma unroll
    for (int st = 0; st < NS; ++st) {
        const int m = st < nA ? mA : mB;
        const int n = st < nA ? mA + st : mB + (st - nA);
        const int o = n - m;
        ca[st] = o == 1 ? Rec<T>::d(m) : (o >= 2 ? Rec<T>::a(n * (n + 1) / 2 + m) : (T)0);
        cb[st] = o >= 2 ? Rec<T>::b(n * (n + 1) / 2 + m) : (T)0;
    }
    double are[NS], aim[NS];
#pragma unroll
    for (int st = 0; st < NS; ++st) are[st] = aim[st] = 0.0;
    const int32_t s0 = start[leaf], s1 = start[leaf + 1];
    for (int32_t s = s0; s < s1; ++s) {
        const T *a = xq + 4 * (int64_t)s;
        const T x = a[0] * inv_h, y = a[1] * inv_h, z = a[2] * inv_h, q = a[3];
        const T r2 = x * x + y * y + z * z;
        // sectoral values R^_mA^mA and R^_mB^mB (mA <= mB)
        T sre = 1, sim = 0, Are = 1, Aim = 0;
#pragma unroll
        for (int k = 1; k <= P; ++k) {
            const T c = -Rec<T>::c(k);
            const T nre = c * (x * sre - y * sim);
            const T nim = c * (x * sim + y * sre);
            // past mB the value is kept (the same P steps for every thread)
            sre = k <= mB ? nre : sre;
            sim = k <= mB ? nim : sim;
            if (k == mA) { Are = sre; Aim = sim; }
        }
        T p1re = 0, p1im = 0, p2re = 0, p2im = 0;
#pragma unroll
        for (int st = 0; st < NS; ++st) {
            const bool first = st == 0 || st == nA;
            T vre = ca[st] * z * p1re - cb[st] * r2 * p2re;
            T vim = ca[st] * z * p1im - cb[st] * r2 * p2im;
            if (first) {
                vre = st == 0 ? Are : sre;
                vim = st == 0 ? Aim : sim;
            }
            p2re = first ? (T)0 : p1re;
            p2im = first ? (T)0 : p1im;
            p1re = vre;
            p1im = vim;
            are[st] += (double)(q * vre);
            aim[st] += (double)(q * vim);
        }
    }
    T *Ml = M + leaf * Kp;
#pragma unroll
    for (int st = 0; st < NS; ++st) {
        const int m = st < nA ? mA : mB;
        const int n = st < nA ? mA + st : mB + (st - nA);
        if (st < ns) {
            if (m == 0) {
                Ml[n * n] = (T)are[st];
            } else {
                Ml[n * n + 2 * m - 1] = (T)are[st];
                Ml[n * n + 2 * m] = (T)(-aim[st]);
            }
        }
    }
    if (mA == 0)
        for (int k = K; k < Kp; ++k) Ml[k] = (T)0;
}

template <typename T, int P>
static hipError_t launch_p2m_p(int64_t nleaf, const void *xq, const int32_t *start, T *M, int Kp, double inv_h,
                               hipStream_t s) {
    const int64_t nthreads = nleaf * p2m_threads<P>();
    const int64_t g = (nthreads + 255) / 256;
    hipLaunchKernelGGL((k_p2m<T, P>), dim3((unsigned)g), dim3(256), 0, s, nleaf, (const T *)xq, start, M, Kp,
                       (T)inv_h);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_p2m(int64_t nleaf, const void *xq, const int32_t *start, T *M, int p, int Kp,
                      double inv_h, hipStream_t s) {
    if (nleaf * (p / 2 + 1) > ((int64_t)0xffffffff) * 256) return hipErrorInvalidValue;
    switch (p) {
#define FMM_P2M_CASE(P) \
    case P: return launch_p2m_p<T, P>(nleaf, xq, start, M, Kp, inv_h, s);
        FMM_P2M_CASE(0) FMM_P2M_CASE(1) FMM_P2M_CASE(2) FMM_P2M_CASE(3) FMM_P2M_CASE(4) FMM_P2M_CASE(5)
        FMM_P2M_CASE(6) FMM_P2M_CASE(7) FMM_P2M_CASE(8) FMM_P2M_CASE(9) FMM_P2M_CASE(10) FMM_P2M_CASE(11)
        FMM_P2M_CASE(12) FMM_P2M_CASE(13) FMM_P2M_CASE(14) FMM_P2M_CASE(15) FMM_P2M_CASE(16) FMM_P2M_CASE(17)
        FMM_P2M_CASE(18) FMM_P2M_CASE(19) FMM_P2M_CASE(20)
#undef FMM_P2M_CASE
        default: return hipErrorInvalidValue;
    }
}
template hipError_t launch_p2m<float>(int64_t, const void *, const int32_t *, float *, int, int, double,
                                      hipStream_t);
template hipError_t launch_p2m<double>(int64_t, const void *, const int32_t *, double *, int, int, double,
                                       hipStream_t);

// ---------------------------------------------------------------------------
// Sparse solute pass (one-sided solute-solvent energy): P2M of the solute
// atoms of flagged leaves and L2P at solute atoms only, in FP64 from the FP64
// wrapped positions xs (measured from the box centre).
// ---------------------------------------------------------------------------

// R^_n^m for one order m and n = m..p, by the recurrences above (the sectoral
// value R^_m^m from m steps of its own recurrence).
template <typename T, typename F>
__device__ inline void regular_hat_column(T x, T y, T z, int m, int p, F &&f) {
    const T r2 = x * x + y * y + z * z;
    T mre = 1, mim = 0;
    for (int k = 1; k <= m; ++k) {
        const T c = -Rec<T>::c(k);
        const T nre = c * (x * mre - y * mim);
        const T nim = c * (x * mim + y * mre);
        mre = nre;
        mim = nim;
    }
    f(m, mre, mim);
    if (m + 1 > p) return;
    T p2re = mre, p2im = mim;
    const T dm = Rec<T>::d(m) * z;
    T p1re = dm * mre, p1im = dm * mim;
    f(m + 1, p1re, p1im);
    int ti = (m + 2) * (m + 3) / 2 + m;
    for (int n = m + 2; n <= p; ++n) {
        const T a = Rec<T>::a(ti) * z, b = Rec<T>::b(ti) * r2;
        const T cre = a * p1re - b * p2re;
        const T cim = a * p1im - b * p2im;
        f(n, cre, cim);
        p2re = p1re; p2im = p1im;
        p1re = cre; p1im = cim;
        ti += n + 1;
    }
}

// leaf-local FP64 coordinates (in units of the leaf edge) of sorted atom s
__device__ inline void leaf_local(const double *xs, int64_t s, uint32_t leaf, double box, double h, double &x,
                                  double &y, double &z) {
    uint32_t cx, cy, cz;
    demorton3(leaf, cx, cy, cz);
    const double hb = 0.5 * box;
    x = (xs[4 * s + 0] - (((double)cx + 0.5) * h - hb)) / h;
    y = (xs[4 * s + 1] - (((double)cy + 0.5) * h - hb)) / h;
    z = (xs[4 * s + 2] - (((double)cz + 0.5) * h - hb)) / h;
}

// cells of levels 1 .. l-1 (offset of level l in the concatenated level arrays)
__device__ inline int64_t cells_before(int l) { return l <= 1 ? 0 : (((int64_t)1 << (3 * l)) - 8) / 7; }

// One wavefront per leaf of every box (blocks of the box's leaf table);
// flagged leaves only.  Lane m accumulates the order-m coefficients of every
// solute atom of the leaf (each lane owns its entries).
__global__ __launch_bounds__(64) void k_uv_p2m(const UvBox *__restrict__ boxes, int nbox,
                                               const int64_t *__restrict__ st) {
    const int w = box_of(st, nbox, blockIdx.x);
    const UvBox &b = boxes[w];
    const int64_t leaf = blockIdx.x - st[w];
    const int L = b.levels, p = b.p, Kp = b.Kp;
    if (!b.flag[1 + cells_before(L) + leaf]) return;
    const int m = threadIdx.x;
    double *Ml = b.M + (cells_before(L) + leaf) * Kp;
    if (m <= p)
        for (int n = m; n <= p; ++n) {
            if (m == 0) Ml[n * n] = 0.0;
            else {
                Ml[n * n + 2 * m - 1] = 0.0;
                Ml[n * n + 2 * m] = 0.0;
            }
        }
    if (m == 0)
        for (int k = (p + 1) * (p + 1); k < Kp; ++k) Ml[k] = 0.0;
    if (m > p) return;
    for (int32_t s = b.start[leaf]; s < b.start[leaf + 1]; ++s) {
        if (!b.ms[s]) continue;
        double x, y, z;
        leaf_local(b.xs, s, (uint32_t)leaf, b.box, b.h, x, y, z);
        const double q = b.xs[4 * s + 3];
        regular_hat_column<double>(x, y, z, m, p, [&](int n, double re, double im) {
            if (m == 0) Ml[n * n] += q * re;
            else {
                Ml[n * n + 2 * m - 1] += q * re;
                Ml[n * n + 2 * m] -= q * im;
            }
        });
    }
}

hipError_t launch_uv_p2m(const UvBox *b, int nbox, const int64_t *st_leaf, int64_t nb, hipStream_t s) {
    if (nb > 0) hipLaunchKernelGGL(k_uv_p2m, dim3((unsigned)nb), dim3(64), 0, s, b, nbox, st_leaf);
    return hipGetLastError();
}

// Potential of the leaf's local expansion at every solute atom (0 elsewhere),
// one thread per sorted atom of every box (blocks of 256 of the box's atom table).
__global__ void k_uv_l2p(const UvBox *__restrict__ boxes, int nbox, const int64_t *__restrict__ st) {
    const int w = box_of(st, nbox, blockIdx.x);
    const UvBox &b = boxes[w];
    const int64_t s = (blockIdx.x - st[w]) * (int64_t)blockDim.x + threadIdx.x;
    if (s >= b.n) return;
    if (!b.ms[s]) {
        b.phi_u[s] = 0.0;
        return;
    }
    const uint32_t leaf = b.key[b.perm[s]];
    double x, y, z;
    leaf_local(b.xs, s, leaf, b.box, b.h, x, y, z);
    const double *Ll = b.L + (cells_before(b.levels) + leaf) * b.Kp;
    double acc = 0.0;
    regular_hat_foreach<double>(x, y, z, b.p, [&](int nn, int m, double re, double im) {
        if (m == 0) acc += re * Ll[nn * nn];
        else acc += re * Ll[nn * nn + 2 * m - 1] + im * Ll[nn * nn + 2 * m];
    });
    b.phi_u[s] = acc / b.h;
}

hipError_t launch_uv_l2p(const UvBox *b, int nbox, const int64_t *st_atoms, int64_t nb, hipStream_t s) {
    if (nb > 0) hipLaunchKernelGGL(k_uv_l2p, dim3((unsigned)nb), dim3(256), 0, s, b, nbox, st_atoms);
    return hipGetLastError();
}

// degree n of the real storage index idx (n^2 <= idx < (n+1)^2)
__device__ inline int degree_of(int idx) {
    int n = (int)sqrtf((float)idx);
    while ((n + 1) * (n + 1) <= idx) ++n;
    while (n * n > idx) --n;
    return n;
}

// ---------------------------------------------------------------------------
// Level 0 (eq. 12 applied through eq. Lcoeffdef): L~(0) = A_T M~(0), FP64.
// ---------------------------------------------------------------------------
// Rows in blocks of 64 (one per thread of a wavefront); the four wavefronts
// of a workgroup take interleaved quarters of the columns and their partial
// sums are added through LDS in a fixed order.  AT is stored transposed
// ([col][row]), so a wavefront reads 64 consecutive doubles per column.
__global__ __launch_bounds__(256) void k_lattice(const double *__restrict__ M0, double *__restrict__ L0,
                                                 const double *__restrict__ AT, int K, int Kp) {
    __shared__ double part[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int row = blockIdx.x * 64 + lane;
    double acc = 0.0;
    if (row < K)
        for (int c = w; c < K; c += 4) acc += AT[(size_t)c * K + row] * M0[c];
    part[w][lane] = acc;
    __syncthreads();
    if (w == 0 && row < Kp) L0[row] = row < K ? ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane] : 0.0;
}

// the same for every box of a solute-solvent stage table (ceil(Kp / 64)
// blocks per box)
__global__ __launch_bounds__(256) void k_uv_lattice(const UvBox *__restrict__ boxes, int nbox,
                                                   const int64_t *__restrict__ st) {
    __shared__ double part[4][64];
    const int w = box_of(st, nbox, blockIdx.x);
    const UvBox &b = boxes[w];
    const int K = b.K, Kp = b.Kp;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row = (int)(blockIdx.x - st[w]) * 64 + lane;
    double acc = 0.0;
    if (row < K)
        for (int c = wv; c < K; c += 4) acc += b.lat[(size_t)c * K + row] * b.M0[c];
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && row < Kp)
        b.L0[row] = row < K ? ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane] : 0.0;
}

hipError_t launch_uv_lattice(const UvBox *b, int nbox, const int64_t *st_one, int64_t nb, hipStream_t s) {
    if (nb > 0) hipLaunchKernelGGL(k_uv_lattice, dim3((unsigned)nb), dim3(256), 0, s, b, nbox, st_one);
    return hipGetLastError();
}

hipError_t launch_lattice(const double *M0, double *L0, const double *AT, int p, int Kp, hipStream_t s) {
    hipLaunchKernelGGL(k_lattice, dim3((unsigned)((Kp + 63) / 64)), dim3(256), 0, s, M0, L0, AT, num_coeffs(p), Kp);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// L2P (eq. EqFF) with gradient: phi(c + x) = (1/h) sum_k Rr_k(x/h) L~_k and
// grad phi = (1/h^2) sum_k Rr_k(x/h) G~_k, where G~ (degree <= p-1) follows
// from L~ by differentiating the regular harmonics:
//   dz R_n^m = R_{n-1}^m,  (dx + i dy) R_n^m = R_{n-1}^{m+1},
//   (dx - i dy) R_n^m = -R_{n-1}^{m-1}.
// A workgroup of 256 threads takes a group of consecutive leaves (chosen so
// that the group holds about 256 atoms): it stages their L~ in LDS, derives
// their G~ there, and every thread then evaluates one atom of the group (the
// group's atoms are contiguous in sorted order).
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline void get_local(const T *Ls, int n, int m, T &re, T &im) {
    const int am = m < 0 ? -m : m;
    if (am > n) { re = 0; im = 0; return; }
    if (am == 0) { re = Ls[n * n]; im = 0; return; }
    re = (T)0.5 * Ls[n * n + 2 * am - 1];
    im = (T)0.5 * Ls[n * n + 2 * am];
    if (m < 0) {  // L_n^{-m} = (-1)^m conj(L_n^m)
        const T s = (am & 1) ? (T)-1 : (T)1;
        re = s * re;
        im = -s * im;
    }
}

// FP64 at the middle orders: capped at three wavefronts per SIMD (left to
// itself the compiler keeps about 180 registers at p = 12, two wavefronts)
template <typename T, int P> constexpr int l2p_min_waves() {
    return (sizeof(T) == 8 && P >= 9 && P <= 12) ? 3 : 1;
}

template <typename T, int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(l2p_min_waves<T, P>()))) void k_l2p(
    int64_t nleaf, const T *__restrict__ xq,
                                             const int32_t *__restrict__ start, const T *__restrict__ L, int Kp,
                                             T inv_h, T inv_h2, double *__restrict__ phi, T *__restrict__ field,
                                             int gl) {
    constexpr int K = (P + 1) * (P + 1);
    constexpr int Kg = P * P;
    constexpr int per = K + 3 * Kg;  // per leaf: L~, then G~x, G~y, G~z
    extern __shared__ unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);
    int32_t *sst = reinterpret_cast<int32_t *>(smem_raw + (size_t)gl * per * sizeof(T));  // the group's leaf starts
    const int tid = threadIdx.x;
    const int64_t l0 = blockIdx.x * (int64_t)gl;
    const int nl = (int)min((int64_t)gl, nleaf - l0);
    const int32_t a0 = start[l0], a1 = start[l0 + nl];
    if (a1 <= a0) return;  // uniform per block
    for (int i = tid; i < nl * K; i += 256) {
        const int li = i / K, j = i - li * K;
        sm[li * per + j] = L[(l0 + li) * Kp + j];
    }
    if (tid <= nl) sst[tid] = start[l0 + tid];
    __syncthreads();
    for (int i = tid; i < nl * Kg; i += 256) {
        const int li = i / Kg, j = i - li * Kg;
        const T *Ls = sm + li * per;
        T *Gx = sm + li * per + K, *Gy = Gx + Kg, *Gz = Gy + Kg;
        const int n = degree_of(j);
        const int r = j - n * n;
        const int m = (r + 1) / 2;
        T are, aim, bre, bim, cre, cim;
        get_local(Ls, n + 1, m - 1, are, aim);
        get_local(Ls, n + 1, m + 1, bre, bim);
        get_local(Ls, n + 1, m, cre, cim);
        const T fa = sqrt((T)((n - m + 2) * (n - m + 1)));
        const T fb = sqrt((T)((n + m + 2) * (n + m + 1)));
        const T fc = sqrt((T)((n + 1 + m) * (n + 1 - m)));
        // complex G-hat values
        const T gxr = (T)0.5 * (fa * are - fb * bre), gxi = (T)0.5 * (fa * aim - fb * bim);
        // (i/2)(fa A + fb B)
        const T gyr = (T)-0.5 * (fa * aim + fb * bim), gyi = (T)0.5 * (fa * are + fb * bre);
        const T gzr = fc * cre, gzi = fc * cim;
        if (m == 0) {
            Gx[j] = gxr; Gy[j] = gyr; Gz[j] = gzr;
        } else if (r & 1) {  // real part slot, factor 2
            Gx[j] = 2 * gxr; Gy[j] = 2 * gyr; Gz[j] = 2 * gzr;
        } else {
            Gx[j] = 2 * gxi; Gy[j] = 2 * gyi; Gz[j] = 2 * gzi;
        }
    }
    __syncthreads();
    for (int32_t s = a0 + tid; s < a1; s += 256) {
        int li = 0;  // the atom's leaf within the group
        while (li + 1 < nl && sst[li + 1] <= s) ++li;
        const T *Ls = sm + li * per;
        const T *Gx = Ls + K, *Gy = Gx + Kg, *Gz = Gy + Kg;
        const T *a = xq + 4 * (int64_t)s;
        const T x = a[0] * inv_h, y = a[1] * inv_h, z = a[2] * inv_h;
        double ph = 0;  // potential accumulated in FP64 (see k_p2p)
        T gx = 0, gy = 0, gz = 0;
        // with P a compile-time constant every index below is one too: the
        // expansions are read from LDS at fixed offsets from the leaf's base
        regular_hat_unrolled<T, P>(x, y, z, [&](int n, int m, T re, T im) {
            if (m == 0) {
                const int k = n * n;
                ph += (double)(re * Ls[k]);
                if (n < P) { gx += re * Gx[k]; gy += re * Gy[k]; gz += re * Gz[k]; }
            } else {
                const int k = n * n + 2 * m - 1;
                ph += (double)(re * Ls[k] + im * Ls[k + 1]);
                if (n < P) {
                    gx += re * Gx[k] + im * Gx[k + 1];
                    gy += re * Gy[k] + im * Gy[k + 1];
                    gz += re * Gz[k] + im * Gz[k + 1];
                }
            }
        });
        phi[s] = ph * (double)inv_h;
        field[3 * (int64_t)s + 0] = -gx * inv_h2;
        field[3 * (int64_t)s + 1] = -gy * inv_h2;
        field[3 * (int64_t)s + 2] = -gz * inv_h2;
    }
}

// leaves per workgroup: about 256 atoms per group at the mean occupancy,
// within 48 KB of LDS
template <typename T, int P>
static hipError_t launch_l2p_p(int64_t nleaf, const void *xq, const int32_t *start, const T *L, int Kp, double h,
                               double *phi, T *field, hipStream_t s, int64_t natoms) {
    constexpr int K = (P + 1) * (P + 1);
    const size_t per = (size_t)(K + 3 * P * P) * sizeof(T);
    const double occ = nleaf > 0 ? (double)natoms / (double)nleaf : 1.0;
    int gl = (int)std::floor(256.0 / std::max(occ, 1.0));
    gl = std::max(1, std::min(gl, (int)((48 * 1024) / per)));
    gl = std::min(gl, 64);
    const int64_t g = (nleaf + gl - 1) / gl;
    const size_t lds = (size_t)gl * per + (size_t)(gl + 1) * sizeof(int32_t);
    hipLaunchKernelGGL((k_l2p<T, P>), dim3((unsigned)g), dim3(256), lds, s, nleaf, (const T *)xq, start, L, Kp,
                       (T)(1.0 / h), (T)(1.0 / (h * h)), phi, field, gl);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_l2p(int64_t nleaf, const void *xq, const int32_t *start, const T *L, int p, int Kp,
                      double h, double *phi, T *field, hipStream_t s, int64_t natoms) {
    switch (p) {
#define FMM_L2P_CASE(P) \
    case P: return launch_l2p_p<T, P>(nleaf, xq, start, L, Kp, h, phi, field, s, natoms);
        FMM_L2P_CASE(0) FMM_L2P_CASE(1) FMM_L2P_CASE(2) FMM_L2P_CASE(3) FMM_L2P_CASE(4) FMM_L2P_CASE(5)
        FMM_L2P_CASE(6) FMM_L2P_CASE(7) FMM_L2P_CASE(8) FMM_L2P_CASE(9) FMM_L2P_CASE(10) FMM_L2P_CASE(11)
        FMM_L2P_CASE(12) FMM_L2P_CASE(13) FMM_L2P_CASE(14) FMM_L2P_CASE(15) FMM_L2P_CASE(16) FMM_L2P_CASE(17)
        FMM_L2P_CASE(18) FMM_L2P_CASE(19) FMM_L2P_CASE(20)
#undef FMM_L2P_CASE
        default: return hipErrorInvalidValue;
    }
}
template hipError_t launch_l2p<float>(int64_t, const void *, const int32_t *, const float *, int, int,
                                      double, double *, float *, hipStream_t, int64_t);
template hipError_t launch_l2p<double>(int64_t, const void *, const int32_t *, const double *, int, int,
                                       double, double *, double *, hipStream_t, int64_t);

}  // namespace fmm
