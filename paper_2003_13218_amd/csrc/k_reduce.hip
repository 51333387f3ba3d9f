// Stages a10 (charged-system, quadrupole and dipole terms), a11 (energy
// reduction), a13 (scatter to the caller's order) and the reductions of the
// solute-solvent scheme.  All in FP64 with Neumaier-compensated, fixed-order
// (hence run-to-run deterministic) block reductions.
//
// With Q = sum q, mu = sum q r, S = sum q r^2 over wrapped positions measured
// from the box centre (the sum Q S - mu.mu does not depend on the origin):
//   E_corr = -pi Q^2 / (2 V kappa^2) + (2 pi / 3V)(Q S - mu.mu)      (eq. Velecfull)
//   phi_i += -pi Q / (V kappa^2) + (2 pi / 3V)(S + Q r_i^2 - 2 mu.r_i)   (= dE_corr/dq_i)
//   F_i   += -(4 pi / 3V) q_i (Q r_i - mu)                              (= -dE_corr/dr_i)
#include "fmm_internal.h"

namespace fmm {

constexpr int kRedBlock = 256;

struct NSum {
    double s, c;
    __device__ NSum() : s(0.0), c(0.0) {}
    __device__ inline void add(double x) {
        const double t = s + x;
        if (fabs(s) >= fabs(x)) c += (s - t) + x;
        else c += (x - t) + s;
        s = t;
    }
    __device__ inline void merge(double s2, double c2) {
        add(s2);
        c += c2;
    }
    __device__ inline double value() const { return s + c; }
};

// Block-level reduction of NV Neumaier pairs; thread 0 ends with the totals.
template <int NV>
__device__ inline void block_reduce(NSum (&v)[NV]) {
    __shared__ double sh_s[NV][kRedBlock];
    __shared__ double sh_c[NV][kRedBlock];
    for (int k = 0; k < NV; ++k) { sh_s[k][threadIdx.x] = v[k].s; sh_c[k][threadIdx.x] = v[k].c; }
    __syncthreads();
    for (int w = kRedBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < NV; ++k) {
                NSum a;
                a.s = sh_s[k][threadIdx.x];
                a.c = sh_c[k][threadIdx.x];
                a.merge(sh_s[k][threadIdx.x + w], sh_c[k][threadIdx.x + w]);
                sh_s[k][threadIdx.x] = a.s;
                sh_c[k][threadIdx.x] = a.c;
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < NV; ++k) { v[k].s = sh_s[k][0]; v[k].c = sh_c[k][0]; }
}

int moments_blocks(int64_t n) {
    int64_t b = (n + kRedBlock * 4 - 1) / (kRedBlock * 4);
    if (b < 1) b = 1;
    if (b > 1024) b = 1024;
    return (int)b;
}

// partial sums of (Q, mu_x, mu_y, mu_z, S) over sorted atoms s (xs: wrapped
// position from the box centre and charge), restricted to atoms whose flag
// mask[perm[s]] equals `want` when a mask is given
__global__ __launch_bounds__(kRedBlock) void k_moments(int64_t n, const double *__restrict__ xs,
                                                        const int32_t *__restrict__ perm,
                                                        const uint8_t *__restrict__ mask, int want,
                                                        double *__restrict__ partials) {
    NSum v[5];
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x) {
        if (mask && ((mask[perm[s]] != 0) != (want != 0))) continue;
        const double x = xs[4 * s], y = xs[4 * s + 1], z = xs[4 * s + 2];
        const double qi = xs[4 * s + 3];
        v[0].add(qi);
        v[1].add(qi * x);
        v[2].add(qi * y);
        v[3].add(qi * z);
        v[4].add(qi * (x * x + y * y + z * z));
    }
    block_reduce<5>(v);
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) {
            partials[(blockIdx.x * 5 + k) * 2] = v[k].s;
            partials[(blockIdx.x * 5 + k) * 2 + 1] = v[k].c;
        }
}

template <int NV>
__global__ __launch_bounds__(kRedBlock) void k_final_sum(const double *__restrict__ partials, int nblocks,
                                                          double *__restrict__ out) {
    NSum v[NV];
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
        for (int k = 0; k < NV; ++k) v[k].merge(partials[(b * NV + k) * 2], partials[(b * NV + k) * 2 + 1]);
    block_reduce<NV>(v);
    if (threadIdx.x == 0)
        for (int k = 0; k < NV; ++k) out[k] = v[k].value();
}

hipError_t launch_moments(int64_t n, const double *xs, const int32_t *perm, const uint8_t *mask, int want,
                          double *partials, int nblocks, double *out5, hipStream_t s) {
    hipLaunchKernelGGL(k_moments, dim3(nblocks), dim3(kRedBlock), 0, s, n, xs, perm, mask, want, partials);
    hipLaunchKernelGGL(k_final_sum<5>, dim3(1), dim3(kRedBlock), 0, s, partials, nblocks, out5);
    return hipGetLastError();
}

// Per sorted atom s (i = perm[s]): total potential and force in the caller's
// order, and the partial sums of E_pair = 1/2 sum q_i (phi_NF + phi_FF).
template <typename T>
__global__ __launch_bounds__(kRedBlock) void k_finalize(
    int64_t n, const int32_t *__restrict__ perm, const double *__restrict__ xs,
    double box, double kappa, double t00b, double mu_w, const double *__restrict__ mom,
    const double *__restrict__ m0, const double *__restrict__ phi_nf,
    const T *__restrict__ field_nf, const double *__restrict__ phi_ff, const T *__restrict__ field_ff,
    double *__restrict__ forces, double *__restrict__ phi_out, double *__restrict__ partials) {
    const double V = box * box * box;
    const double Q = mom[0], mux = mom[1], muy = mom[2], muz = mom[3], S = mom[4];
    // charged-system term (eq. 6) and the net-charge lattice constant
    // t00 Q_tree / b, with the tree's own level-0 monopole Q_tree = m0[0] (equal
    // to Q up to the rounding of the leaf multipoles), so that it cancels the
    // near-image monopole sums the tree itself computed
    const double c_bg = -M_PI * Q / (V * kappa * kappa) + t00b * m0[0];
    const double c23 = 2.0 * M_PI / (3.0 * V);
    const double c43 = 4.0 * M_PI / (3.0 * V);
    // under the vacuum boundary (mu_w = 0) the dipole surface term
    // (2 pi / 3V) mu.mu cancels the -mu.mu of the quadrupole/dipole terms
    const double wx = mu_w * mux, wy = mu_w * muy, wz = mu_w * muz;
    NSum e[1];
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = perm[s];
        const double qi = xs[4 * s + 3];
        const double ph = phi_nf[s] + phi_ff[s];
        e[0].add(0.5 * qi * ph);  // E_pair; the t00 part is added once below
        const double x = xs[4 * s], y = xs[4 * s + 1], z = xs[4 * s + 2];
        if (phi_out)
            phi_out[i] = ph + c_bg + c23 * (S + Q * (x * x + y * y + z * z) - 2.0 * (wx * x + wy * y + wz * z));
        if (forces) {
            const double ex = (double)field_nf[3 * s] + (double)field_ff[3 * s];
            const double ey = (double)field_nf[3 * s + 1] + (double)field_ff[3 * s + 1];
            const double ez = (double)field_nf[3 * s + 2] + (double)field_ff[3 * s + 2];
            forces[3 * i + 0] = qi * ex - c43 * qi * (Q * x - wx);
            forces[3 * i + 1] = qi * ey - c43 * qi * (Q * y - wy);
            forces[3 * i + 2] = qi * ez - c43 * qi * (Q * z - wz);
        }
    }
    block_reduce<1>(e);
    if (threadIdx.x == 0) {
        partials[blockIdx.x * 2] = e[0].s;
        partials[blockIdx.x * 2 + 1] = e[0].c;
    }
}

// E = E_pair + E_corr
__global__ __launch_bounds__(kRedBlock) void k_energy_final(const double *__restrict__ partials, int nblocks,
                                                             const double *__restrict__ mom, double box,
                                                             double kappa, double t00b, double mu_w,
                                                             const double *__restrict__ m0, double *__restrict__ out) {
    NSum v[1];
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) v[0].merge(partials[2 * b], partials[2 * b + 1]);
    block_reduce<1>(v);
    if (threadIdx.x == 0) {
        const double V = box * box * box;
        const double Q = mom[0], S = mom[4];
        const double mu2 = mom[1] * mom[1] + mom[2] * mom[2] + mom[3] * mom[3];
        NSum t;
        t.merge(v[0].s, v[0].c);
        t.add(-M_PI * Q * Q / (2.0 * V * kappa * kappa));
        t.add(0.5 * t00b * Q * m0[0]);
        t.add(2.0 * M_PI / (3.0 * V) * (Q * S - mu_w * mu2));
        out[0] = t.value();
        out[1] = v[0].value();
    }
}

template <typename T>
hipError_t launch_finalize(int64_t n, const int32_t *perm, const double *xs, double box, double kappa,
                           double t00b, double mu_w, const double *moments, const double *m0, const double *phi_nf,
                           const T *field_nf, const double *phi_ff, const T *field_ff, double *forces, double *phi,
                           double *partials, int nblocks, double *energy_out, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize<T>, dim3(nblocks), dim3(kRedBlock), 0, s, n, perm, xs, box, kappa, t00b, mu_w,
                       moments, m0, phi_nf, field_nf, phi_ff, field_ff, forces, phi, partials);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kRedBlock), 0, s, partials, nblocks, moments, box, kappa,
                       t00b, mu_w, m0, energy_out);
    return hipGetLastError();
}
template hipError_t launch_finalize<float>(int64_t, const int32_t *, const double *, double, double, double, double,
                                           const double *, const double *, const double *, const float *,
                                           const double *, const float *, double *, double *, double *, int, double *,
                                           hipStream_t);
template hipError_t launch_finalize<double>(int64_t, const int32_t *, const double *, double, double, double, double,
                                            const double *, const double *, const double *, const double *, const double *,
                                            const double *, double *, double *, double *, int, double *,
                                            hipStream_t);

// Sorted-order potential / field to the caller's order in FP64.
template <typename T>
__global__ void k_parts_out(int64_t n, const int32_t *__restrict__ perm, const double *__restrict__ phi_s,
                            const T *__restrict__ field_s, const double *__restrict__ m0, double cq,
                            double *__restrict__ phi, double *__restrict__ field) {
    const double c = cq * m0[0];
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = perm[s];
        if (phi) phi[i] = phi_s[s] + c;
        if (field) {
            field[3 * i] = (double)field_s[3 * s];
            field[3 * i + 1] = (double)field_s[3 * s + 1];
            field[3 * i + 2] = (double)field_s[3 * s + 2];
        }
    }
}

template <typename T>
hipError_t launch_parts_out(int64_t n, const int32_t *perm, const double *phi_s, const T *field_s, const double *mom,
                            double cq, double *phi, double *field, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t g = (n + 255) / 256;
    if (g > 65535) g = 65535;
    hipLaunchKernelGGL(k_parts_out<T>, dim3((unsigned)g), dim3(256), 0, s, n, perm, phi_s, field_s, mom, cq, phi,
                       field);
    return hipGetLastError();
}
template hipError_t launch_parts_out<float>(int64_t, const int32_t *, const double *, const float *, const double *,
                                            double, double *, double *, hipStream_t);
template hipError_t launch_parts_out<double>(int64_t, const int32_t *, const double *, const double *,
                                             const double *, double, double *, double *, hipStream_t);

// Solute-solvent sums of every box (sorted order s, solute flag ms[s]):
//   A = sum_u q phi_uv, B = sum_u q phi_u, C = sum_v q phi_u, D = sum_u nf_uv,
//   E = sum_u nf_sc, F = sum_u nf_dl (soft-core boxes), and the moments
//   (Q, mu, S) of u and of v.  Blocks: the box's reduction table; each block
// strides over the box's atoms and leaves 16 Neumaier pairs in the box's
// partials; one block per box then adds them in block order.
constexpr int kUvValues = 16;

__global__ __launch_bounds__(kRedBlock) void k_uv_reduce(const UvBox *__restrict__ boxes, int nbox,
                                                          const int64_t *__restrict__ st) {
    const int w = box_of(st, nbox, blockIdx.x);
    const UvBox &b = boxes[w];
    const int64_t bi = blockIdx.x - st[w], nb = st[w + 1] - st[w];
    const bool soft = b.soft_c > 0;
    NSum v[kUvValues];
    for (int64_t s = bi * kRedBlock + threadIdx.x; s < b.n; s += nb * kRedBlock) {
        const double x = b.xs[4 * s], y = b.xs[4 * s + 1], z = b.xs[4 * s + 2], qi = b.xs[4 * s + 3];
        const int o = b.ms[s] ? 6 : 11;  // moments of u at 6..10, of v at 11..15
        if (b.ms[s]) {
            v[0].add(qi * b.phi_uv[s]);
            v[1].add(qi * b.phi_u[s]);
            v[3].add(b.nfuv[s]);
            if (soft) {
                v[4].add(b.nfsc[s]);
                v[5].add(b.nfdl[s]);
            }
        } else {
            v[2].add(qi * b.phi_u[s]);
        }
        v[o].add(qi);
        v[o + 1].add(qi * x);
        v[o + 2].add(qi * y);
        v[o + 3].add(qi * z);
        v[o + 4].add(qi * (x * x + y * y + z * z));
    }
    // four passes of four values through the same LDS
    for (int g = 0; g < kUvValues; g += 4) {
        NSum part[4] = {v[g], v[g + 1], v[g + 2], v[g + 3]};
        block_reduce<4>(part);
        if (threadIdx.x == 0)
            for (int k = 0; k < 4; ++k) {
                b.partials[(bi * kUvValues + g + k) * 2] = part[k].s;
                b.partials[(bi * kUvValues + g + k) * 2 + 1] = part[k].c;
            }
    }
}

// one block per box: the box's partials in block order, then its scalar block
__global__ __launch_bounds__(kRedBlock) void k_uv_final(const UvBox *__restrict__ boxes, int nbox,
                                                         const int64_t *__restrict__ st_red,
                                                         const int64_t *__restrict__ st_one) {
    const int w = box_of(st_one, nbox, blockIdx.x);
    const UvBox &b = boxes[w];
    const int64_t nb = st_red[w + 1] - st_red[w];
    for (int g = 0; g < kUvValues; g += 4) {
        NSum v[4];
        for (int64_t k = threadIdx.x; k < nb; k += blockDim.x)
            for (int j = 0; j < 4; ++j)
                v[j].merge(b.partials[(k * kUvValues + g + j) * 2], b.partials[(k * kUvValues + g + j) * 2 + 1]);
        block_reduce<4>(v);
        if (threadIdx.x == 0)
            for (int j = 0; j < 4; ++j) {
                const int k = g + j;
                const double val = v[j].value();
                if (k < 6) b.sc[40 + k] = val;          // A, B, C, D, E, F
                else if (k < 11) b.sc[24 + k - 6] = val;  // Q_u, mu_u, S_u
                else b.sc[32 + k - 11] = val;             // Q_v, mu_v, S_v
            }
    }
    if (threadIdx.x == 0) b.sc[20] = b.M0[0];  // monopole of the solute-charge tree
}

hipError_t launch_uv_sums(const UvBox *b, int nbox, const int64_t *st_red, int64_t nb_red, const int64_t *st_one,
                          int64_t nb_one, hipStream_t s) {
    if (nb_red <= 0 || nb_one <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_uv_reduce, dim3((unsigned)nb_red), dim3(kRedBlock), 0, s, b, nbox, st_red);
    hipLaunchKernelGGL(k_uv_final, dim3((unsigned)nb_one), dim3(kRedBlock), 0, s, b, nbox, st_red, st_one);
    return hipGetLastError();
}

}  // namespace fmm
