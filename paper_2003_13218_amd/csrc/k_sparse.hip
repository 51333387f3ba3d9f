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
//
// Every stage runs for all boxes of a batch in one launch: block b belongs to
// the box w of the stage's block table (box_of), and takes that box's arrays
// from its UvBox entry.  A single-box plan is a batch of one.
#include "fmm_internal.h"
#include "morton.h"

namespace fmm {

// cells of levels 1 .. l-1 (offset of level l in the concatenated level arrays)
__device__ inline int64_t lvl_off(int l) { return l <= 1 ? 0 : (((int64_t)1 << (3 * l)) - 8) / 7; }
__device__ inline uint32_t *flags_at(const UvBox &b, int l) { return b.flag + (l == 0 ? 0 : 1 + lvl_off(l)); }

// Mask stage.  k_uv_fill clears every flag of the box (level 0 and levels
// 1 .. L); k_uv_mask writes the solute flag of every sorted atom and, for a
// solute atom, the flags of its leaf and of all the leaf's ancestors (plain
// stores of 1: concurrent writers store the same value).
__global__ void k_uv_fill(const UvBox *__restrict__ boxes, int nbox, const int64_t *__restrict__ st) {
    const int w = box_of(st, nbox, blockIdx.x);
    const UvBox &b = boxes[w];
    const int64_t nflag = 1 + lvl_off(b.levels + 1);
    const int64_t i = (blockIdx.x - st[w]) * (int64_t)blockDim.x + threadIdx.x;
    if (i < nflag) b.flag[i] = 0u;
}

__global__ void k_uv_mask(const UvBox *__restrict__ boxes, int nbox, const int64_t *__restrict__ st) {
    const int w = box_of(st, nbox, blockIdx.x);
    const UvBox &b = boxes[w];
    const int64_t s = (blockIdx.x - st[w]) * (int64_t)blockDim.x + threadIdx.x;
    if (s >= b.n) return;
    const int32_t i = b.perm[s];
    const bool u = (b.mask[i] != 0) != (b.invert != 0);
    b.ms[s] = u ? 1 : 0;
    if (!u) return;
    uint32_t c = b.key[i];
    for (int l = b.levels; l >= 0; --l, c >>= 3) flags_at(b, l)[c] = 1u;
}

hipError_t launch_uv_mask(const UvBox *b, int nbox, const int64_t *st_fill, int64_t nb_fill,
                          const int64_t *st_atoms, int64_t nb_atoms, hipStream_t s) {
    if (nb_fill > 0) hipLaunchKernelGGL(k_uv_fill, dim3((unsigned)nb_fill), dim3(256), 0, s, b, nbox, st_fill);
    if (nb_atoms > 0) hipLaunchKernelGGL(k_uv_mask, dim3((unsigned)nb_atoms), dim3(256), 0, s, b, nbox, st_atoms);
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
// FP64 octant operators (M2M block: ids 0..7), for the parents at level
// levels - step of every box.  Level 0 (the box's M0) is written whatever
// the flags, as the root must be whatever the mask.
__global__ __launch_bounds__(256) void k_uv_m2m(const UvBox *__restrict__ boxes, int nbox, int step,
                                                const int64_t *__restrict__ st, const double *__restrict__ ops) {
    const int w = box_of(st, nbox, blockIdx.x);
    const UvBox &b = boxes[w];
    const int l = b.levels - step;
    const int64_t P = blockIdx.x - st[w];
    const int K = b.K, Kp = b.Kp;
    if (l > 0 && !flags_at(b, l)[P]) return;
    const uint32_t *fchild = flags_at(b, l + 1);
    const double *Mc = b.M + lvl_off(l + 1) * Kp;
    double *Mp = l == 0 ? b.M0 : b.M + lvl_off(l) * Kp;
    const int NB = Kp / 16;
    for (int row = threadIdx.x; row < Kp; row += blockDim.x) {
        double acc = 0.0;
        if (row < K)
            for (int o = 0; o < 8; ++o)
                if (fchild[8 * P + o]) acc = swz_dot(ops, o, row, NB, NB, K, Mc + (8 * P + o) * Kp, acc);
        Mp[P * Kp + row] = acc;
    }
}

hipError_t launch_uv_m2m(const UvBox *b, int nbox, int step, const int64_t *st, int64_t nb, const void *ops,
                         hipStream_t s) {
    if (nb > 0)
        hipLaunchKernelGGL(k_uv_m2m, dim3((unsigned)nb), dim3(256), 0, s, b, nbox, step, st, (const double *)ops);
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
__global__ __launch_bounds__(kSparseBlock) void k_uv_m2l(const UvBox *__restrict__ boxes, int nbox, int level,
                                                         const int64_t *__restrict__ st,
                                                         const int32_t *__restrict__ il,
                                                         const int32_t *__restrict__ offs,
                                                         const double *__restrict__ ops,
                                                         const int32_t *__restrict__ rowpos, int NBR, int nil) {
    __shared__ int32_t hit_oid[kILSize], hit_src[kILSize];
    __shared__ int wave_cnt[kSparseBlock / 64];
    const int w = box_of(st, nbox, blockIdx.x);
    const UvBox &b = boxes[w];
    const uint32_t c = (uint32_t)(blockIdx.x - st[w]);
    const uint32_t *flag = flags_at(b, level);
    if (!flag[c]) return;
    const int K = b.K, Kp = b.Kp;
    const double *M = b.M + lvl_off(level) * Kp;
    double *L = b.L + lvl_off(level) * Kp;
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

hipError_t launch_uv_m2l(const UvBox *b, int nbox, int level, const int64_t *st, int64_t nb, const int32_t *il,
                         const int32_t *offs, const double *ops, const int32_t *rowpos, int nbr, int nil,
                         hipStream_t s) {
    if (nil < 1 || nil > kILSize) return hipErrorInvalidValue;
    if (nb > 0)
        hipLaunchKernelGGL(k_uv_m2l, dim3((unsigned)nb), dim3(kSparseBlock), 0, s, b, nbox, level, st, il, offs, ops,
                           rowpos, nbr, nil);
    return hipGetLastError();
}

// L~(c) += B_o L~(parent) for flagged cells c = 8P + o of level `level`, with
// the swizzled FP64 octant operators (L2L block: ids 8..15)
__global__ __launch_bounds__(256) void k_uv_l2l(const UvBox *__restrict__ boxes, int nbox, int level,
                                                const int64_t *__restrict__ st, const double *__restrict__ ops) {
    const int w = box_of(st, nbox, blockIdx.x);
    const UvBox &b = boxes[w];
    const int64_t c = blockIdx.x - st[w];
    if (!flags_at(b, level)[c]) return;
    const int K = b.K, Kp = b.Kp;
    const double *Lp = level == 1 ? b.L0 : b.L + lvl_off(level - 1) * Kp;
    double *Lc = b.L + lvl_off(level) * Kp;
    const int NB = Kp / 16;
    const int o = (int)(c & 7);
    const double *lp = Lp + (c >> 3) * Kp;
    for (int row = threadIdx.x; row < K; row += blockDim.x)
        Lc[c * Kp + row] += swz_dot(ops, 8 + o, row, NB, NB, K, lp, 0.0);
}

hipError_t launch_uv_l2l(const UvBox *b, int nbox, int level, const int64_t *st, int64_t nb, const void *ops,
                         hipStream_t s) {
    if (nb > 0)
        hipLaunchKernelGGL(k_uv_l2l, dim3((unsigned)nb), dim3(256), 0, s, b, nbox, level, st, (const double *)ops);
    return hipGetLastError();
}

}  // namespace fmm
