// Sparse far field of the solute charges (one-sided solute-solvent energy).
//
// For W = sum_u q (Phi_uv - Phi_u) only Phi_u at the solute atoms is needed:
// the tree of the solute-only charges is non-zero only in the ancestors of the
// leaves holding solute atoms ("flagged" cells), and its potential is needed
// only there.  Every stage below runs the dense algorithm restricted to
// flagged cells -- M2M from flagged children, M2L from flagged sources of the
// interaction list into flagged targets, L2L down the flagged chain -- so the
// result equals the dense pass up to rounding order, at a cost proportional
// to the number of flagged cells.  Everything is FP64, with the FP64
// operators of the dense pass in their matrix-core swizzle.  One workgroup
// per cell of the level (unflagged ones return at once), which keeps the
// launch independent of the data (graph capture).
#include "fmm_internal.h"
#include "morton.h"

namespace fmm {

// flag[key[i]] = 1 for every solute atom i (plain stores of 1: races benign)
__global__ void k_flag_leaves(int64_t n, const uint8_t *__restrict__ mask, const uint32_t *__restrict__ key,
                              uint32_t *__restrict__ flag) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (mask[i]) flag[key[i]] = 1u;
}

// parent flags from child flags, one level
__global__ void k_flag_up(int64_t ncell, const uint32_t *__restrict__ child, uint32_t *__restrict__ parent) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncell;
         c += (int64_t)gridDim.x * blockDim.x) {
        uint32_t f = 0;
        for (int o = 0; o < 8; ++o) f |= child[8 * c + o];
        parent[c] = f ? 1u : 0u;
    }
}

hipError_t launch_flags(int64_t n, const uint8_t *mask, const uint32_t *key, int levels, uint32_t *const *flag,
                        hipStream_t s) {
    if (n > 0) {
        int64_t g = (n + 255) / 256;
        if (g > 65535) g = 65535;
        hipLaunchKernelGGL(k_flag_leaves, dim3((unsigned)g), dim3(256), 0, s, n, mask, key, flag[levels]);
    }
    for (int l = levels - 1; l >= 0; --l) {
        const int64_t nc = (int64_t)1 << (3 * l);
        hipLaunchKernelGGL(k_flag_up, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, nc, flag[l + 1], flag[l]);
    }
    return hipGetLastError();
}

// Element (row, col) of operator oid in the matrix-core swizzle
// [oid][col block (NKC)][row block (NBR)][lane][4] written by swizzle_ops and
// swizzle_m2l_ops: lanes hold rows 16 rb + lane % 16 and columns 16 kc +
// 4 (lane / 16) + j.  A thread per row walks the columns; for consecutive rows
// the elements sit 4 apart, so the four consecutive j of a column block share
// the lines it fetched.
__device__ inline size_t swz(int oid, int row, int col, int NKC, int NBR) {
    const int rb = row >> 4, kc = col >> 4;
    const int lane = (row & 15) + 16 * ((col & 15) >> 2);
    return ((((size_t)oid * NKC + kc) * NBR + rb) * 64 + lane) * 4 + (col & 3);
}

// acc + O_oid[row][:] . v[:] over the K columns (v: K doubles, uniform), row
// in the operator's own row order.  Two accumulators and an unrolled loop keep
// several loads in flight.
__device__ inline double swz_dot(const double *__restrict__ ops, int oid, int row, int NKC, int NBR, int K,
                                 const double *__restrict__ v, double acc) {
    const int k8 = K & ~7;
    double a1 = 0.0;
#pragma unroll 2
    for (int col = 0; col < k8; col += 8) {
        const double *o = ops + swz(oid, row, col, NKC, NBR);      // columns col .. col+3
        const double *o2 = ops + swz(oid, row, col + 4, NKC, NBR); // columns col+4 .. col+7
        acc += o[0] * v[col] + o[1] * v[col + 1] + o[2] * v[col + 2] + o[3] * v[col + 3];
        a1 += o2[0] * v[col + 4] + o2[1] * v[col + 5] + o2[2] * v[col + 6] + o2[3] * v[col + 7];
    }
    for (int col = k8; col < K; ++col) acc += ops[swz(oid, row, col, NKC, NBR)] * v[col];
    return acc + a1;
}

// M~(P) = sum over flagged children 8P + o of A_o M~(8P + o) with the swizzled
// FP64 octant operators (M2M block: ids 0..7).  all != 0: every parent is
// written (zero without flagged children), as the root must be whatever the
// mask.
__global__ __launch_bounds__(256) void k_m2m_sparse(const uint32_t *__restrict__ fparent,
                                                    const uint32_t *__restrict__ fchild,
                                                    const double *__restrict__ Mc, double *__restrict__ Mp,
                                                    const double *__restrict__ ops, int K, int Kp, int all) {
    const int64_t P = blockIdx.x;
    if (!all && !fparent[P]) return;
    const int NB = Kp / 16;
    for (int row = threadIdx.x; row < Kp; row += blockDim.x) {
        double acc = 0.0;
        if (row < K)
            for (int o = 0; o < 8; ++o)
                if (fchild[8 * P + o]) acc = swz_dot(ops, o, row, NB, NB, K, Mc + (8 * P + o) * Kp, acc);
        Mp[P * Kp + row] = acc;
    }
}

hipError_t launch_m2m_sparse(int64_t nparent, const uint32_t *fparent, const uint32_t *fchild, const double *Mc,
                             double *Mp, const void *ops, int K, int Kp, bool all, hipStream_t s) {
    hipLaunchKernelGGL(k_m2m_sparse, dim3((unsigned)nparent), dim3(256), 0, s, fparent, fchild, Mc, Mp,
                       (const double *)ops, K, Kp, all ? 1 : 0);
    return hipGetLastError();
}

constexpr int kSparseBlock = 256;

// L~(c) = sum over the list entries t of c whose source cell c + t is
// flagged of O_t M~(c + t), for the flagged targets c of a level with 2^l
// cells per axis.  The block first compacts the flagged entries of its list
// (in list order, so the sum order is fixed), then a thread per row sums
// their products.  rowpos: storage row -> operator row of the row-ordered
// full-list operators (NBR row blocks), or NULL for operators in storage
// order (the aliased levels).
__global__ __launch_bounds__(kSparseBlock) void k_m2l_sparse(int level, const uint32_t *__restrict__ flag,
                                                             const int32_t *__restrict__ il,
                                                             const int32_t *__restrict__ offs,
                                                             const double *__restrict__ ops,
                                                             const int32_t *__restrict__ rowpos, int NBR,
                                                             const double *__restrict__ M, double *__restrict__ L,
                                                             int K, int Kp, int nil) {
    __shared__ int32_t hit_oid[kILSize], hit_src[kILSize];
    __shared__ int wave_cnt[kSparseBlock / 64];
    const uint32_t c = blockIdx.x;
    if (!flag[c]) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int NB = Kp / 16;
    const uint32_t nmask = (1u << level) - 1u;
    uint32_t tx, ty, tz;
    demorton3(c, tx, ty, tz);
    const int32_t *ilp = il + (int)(c & 7u) * nil;
    int nhit = 0;
    for (int base = 0; base < nil; base += kSparseBlock) {
        const int t = base + tid;
        int oid = 0;
        uint32_t sc = 0;
        bool hit = false;
        if (t < nil) {
            oid = ilp[t];
            sc = morton3((tx + (uint32_t)offs[3 * oid]) & nmask, (ty + (uint32_t)offs[3 * oid + 1]) & nmask,
                         (tz + (uint32_t)offs[3 * oid + 2]) & nmask);
            hit = flag[sc] != 0;
        }
        const uint64_t b = __ballot(hit);
        if (lane == 0) wave_cnt[wv] = __popcll(b);
        __syncthreads();
        int off = nhit;
        for (int w = 0; w < wv; ++w) off += wave_cnt[w];
        if (hit) {
            const int k = off + __popcll(b & ((1ull << lane) - 1ull));
            hit_oid[k] = oid;
            hit_src[k] = (int32_t)sc;
        }
        for (int w = 0; w < kSparseBlock / 64; ++w) nhit += wave_cnt[w];
        __syncthreads();
    }
    const int nbr = rowpos ? NBR : NB;
    for (int row = tid; row < Kp; row += kSparseBlock) {
        double acc = 0.0;
        if (row < K) {
            const int orow = rowpos ? rowpos[row] : row;
            for (int h = 0; h < nhit; ++h)
                acc = swz_dot(ops, hit_oid[h], orow, NB, nbr, K, M + (size_t)hit_src[h] * Kp, acc);
        }
        L[(size_t)c * Kp + row] = acc;
    }
}

hipError_t launch_m2l_sparse(int level, const uint32_t *flag, const int32_t *il, const int32_t *offs,
                             const double *ops, const int32_t *rowpos, int nbr, const double *M, double *L, int K,
                             int Kp, int nil, hipStream_t s) {
    if (nil < 1 || nil > kILSize) return hipErrorInvalidValue;
    const int64_t nc = (int64_t)1 << (3 * level);
    hipLaunchKernelGGL(k_m2l_sparse, dim3((unsigned)nc), dim3(kSparseBlock), 0, s, level, flag, il, offs, ops, rowpos,
                       nbr, M, L, K, Kp, nil);
    return hipGetLastError();
}

// L~(c) += B_o L~(parent) for flagged cells c = 8P + o, with the swizzled FP64
// octant operators (L2L block: ids 8..15)
__global__ __launch_bounds__(256) void k_l2l_sparse(const uint32_t *__restrict__ flag,
                                                    const double *__restrict__ Lp, double *__restrict__ Lc,
                                                    const double *__restrict__ ops, int K, int Kp) {
    const int64_t c = blockIdx.x;
    if (!flag[c]) return;
    const int NB = Kp / 16;
    const int o = (int)(c & 7);
    const double *lp = Lp + (c >> 3) * Kp;
    for (int row = threadIdx.x; row < K; row += blockDim.x)
        Lc[c * Kp + row] += swz_dot(ops, 8 + o, row, NB, NB, K, lp, 0.0);
}

hipError_t launch_l2l_sparse(int64_t nchild, const uint32_t *flag, const double *Lp, double *Lc, const void *ops,
                             int K, int Kp, hipStream_t s) {
    hipLaunchKernelGGL(k_l2l_sparse, dim3((unsigned)nchild), dim3(256), 0, s, flag, Lp, Lc, (const double *)ops, K,
                       Kp);
    return hipGetLastError();
}

}  // namespace fmm
