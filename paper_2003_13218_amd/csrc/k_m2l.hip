// Stage a6: M2L (eq. Lcoeffdef) on the matrix cores.
//
// At level l (n = 2^l cells per axis, periodic) every target cell c = 2P + pi
// of parity class pi receives  L~_c = sum_{t in IL(pi)} O_t M~_{(c + t) mod n},
// with the 875 offsets t of its interaction list and the scale-invariant
// K x K operators O_t (1206 distinct offsets over all parity classes).  The
// image shift of a wrapped source is implicit in t, so shallow levels where
// one wrapped cell appears under several shifts need no special case.
//
// For a fixed parity class this is one dense contraction
//   L_pi [K x n_pi] = [O_t1 | ... | O_t875] [K x 875K]  x  gather(M) [875K x n_pi],
// run here as an output-stationary tile GEMM:
//   * a workgroup owns 16*CB target cells of one parity class and all K rows;
//   * its 4 wavefronts split the rows into R groups and the offsets into
//     4/R slices, and reduce the slices through LDS at the end;
//   * operator fragments are pre-swizzled on the host into the exact lane
//     order of v_mfma_{f32,f64}_16x16x4 so each wavefront load is contiguous;
//   * multipole fragments are gathered as 4 consecutive coefficients per
//     lane (one 16/32-byte load), which fixes the order in which the K
//     dimension is walked -- the operator swizzle uses the same order;
//   * blockIdx mod 8 selects the parity class, so with the round-robin
//     dispatch of workgroups to the 8 XCDs every XCD streams one class's 875
//     operators through its own L2.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <vector>

#include "fmm_internal.h"
#include "mfma.h"
#include "morton.h"

namespace fmm {

constexpr int kRowBlocksPerWave = 11;  // 176 rows: K <= 169 (p <= 12) in one row group

// ---------------------------------------------------------------------------
// Row order of the M2L operators.  O_{-t} = D O_t D with D = diag((-1)^n) over
// the degree n of each coefficient (the irregular harmonics are odd or even in
// t with their degree), so for a target whose list holds both t and -t
//   O_t M_a + O_{-t} M_b = [rows of even n]  O_t (M_a + D M_b)
//                        + [rows of odd n]   O_t (M_a - D M_b):
// one operator product for the pair instead of two.  The operators are
// stored with the even-degree rows first and the odd-degree rows after, each
// group padded to whole 16-row blocks, so that every matrix-core row block
// belongs to one group; columns keep the storage order of the expansions.
// ---------------------------------------------------------------------------
static int even_degree_rows(int p) {
    int e = 0;
    for (int n = 0; n <= p; n += 2) e += 2 * n + 1;
    return e;
}
int m2l_even_blocks(int p) { return (even_degree_rows(p) + 15) / 16; }
int m2l_row_blocks(int p) {
    const int e = even_degree_rows(p), o = num_coeffs(p) - e;
    return (e + 15) / 16 + (o + 15) / 16;
}
// The padding rows K .. Kp-1 of the storage order take the first unused
// slots (their operator rows are zero), so the kernel writes every stored row.
void m2l_row_map(int p, int32_t *map) {
    const int nr = 16 * m2l_row_blocks(p), eb = 16 * m2l_even_blocks(p);
    for (int i = 0; i < nr; ++i) map[i] = -1;
    int ie = 0, io = eb;
    for (int n = 0; n <= p; ++n)
        for (int k = n * n; k < (n + 1) * (n + 1); ++k) map[(n & 1) ? io++ : ie++] = k;
    int pad = num_coeffs(p);
    for (int i = 0; i < nr && pad < padded_coeffs(p); ++i)
        if (map[i] < 0) map[i] = pad++;
}

// Interaction-list entries of the paired kernel: per parity class, every
// offset t whose negation is in the same list is paired with it (the entry
// (t, -t) appears once, at the first of the two in list order), the others
// stand alone (second id -1).  Within [-5, 4] or [-4, 5] per axis the pairs
// are the offsets inside [-4, 4]^3: 302 pairs and 271 single offsets.
void build_m2l_pairs(const int32_t *vec, const int32_t *il, int32_t *pairs) {
    for (int par = 0; par < 8; ++par) {
        const int32_t *l = il + par * kILSize;
        int32_t *out = pairs + (size_t)par * 2 * kM2LEntries;
        bool used[kNumOffsets] = {};
        int ne = 0;
        for (int i = 0; i < kILSize; ++i) {
            const int a = l[i];
            if (used[a]) continue;
            used[a] = true;
            int b = -1;
            for (int j = 0; j < kILSize; ++j) {
                const int c = l[j];
                if (vec[3 * c] == -vec[3 * a] && vec[3 * c + 1] == -vec[3 * a + 1] && vec[3 * c + 2] == -vec[3 * a + 2]) {
                    b = c;
                    break;
                }
            }
            if (b >= 0) used[b] = true;
            if (ne < kM2LEntries) {
                out[2 * ne] = a;
                out[2 * ne + 1] = b;
            }
            ++ne;
        }
        if (ne != kM2LEntries) {  // the list geometry guarantees 573
            for (int e = 0; e < 2 * kM2LEntries; ++e) out[e] = -1;
        }
    }
}

template <typename T>
size_t m2l_ops_elems(int p) {
    const size_t Kp = (size_t)padded_coeffs(p);
    return (size_t)kNumOffsets * (Kp / 16) * m2l_row_blocks(p) * 256;
}
template size_t m2l_ops_elems<float>(int);
template size_t m2l_ops_elems<double>(int);

// out[(((oid * NKC + kc) * NRB + rb) * 64 + lane) * 4 + j] =
//     O_oid[row = 16 rb + lane % 16][col = 16 kc + 4 (lane / 16) + j]
template <typename T>
void swizzle_ops(int p, int nops, const double *ops, T *out) {
    const int K = num_coeffs(p), Kp = padded_coeffs(p);
    const int NB = Kp / 16;
    for (int oid = 0; oid < nops; ++oid) {
        const double *A = ops + (size_t)oid * K * K;
        for (int kc = 0; kc < NB; ++kc)
            for (int rb = 0; rb < NB; ++rb)
                for (int lane = 0; lane < 64; ++lane)
                    for (int j = 0; j < 4; ++j) {
                        const int row = 16 * rb + (lane & 15);
                        const int col = 16 * kc + 4 * (lane >> 4) + j;
                        const double v = (row < K && col < K) ? A[(size_t)row * K + col] : 0.0;
                        out[((((size_t)oid * NB + kc) * NB + rb) * 64 + lane) * 4 + j] = (T)v;
                    }
    }
}
template void swizzle_ops<float>(int, int, const double *, float *);
template void swizzle_ops<double>(int, int, const double *, double *);

// The M2L operators with their rows in the order of m2l_row_map:
// out[(((oid * NKC + kc) * NBR + rb) * 64 + lane) * 4 + j] =
//     O_oid[map[16 rb + lane % 16]][16 kc + 4 (lane / 16) + j]
template <typename T>
void swizzle_m2l_ops(int p, const double *ops, T *out) {
    const int K = num_coeffs(p), NKC = padded_coeffs(p) / 16, NBR = m2l_row_blocks(p);
    std::vector<int32_t> map((size_t)16 * NBR);
    m2l_row_map(p, map.data());
    for (int oid = 0; oid < kNumOffsets; ++oid) {
        const double *A = ops + (size_t)oid * K * K;
        for (int kc = 0; kc < NKC; ++kc)
            for (int rb = 0; rb < NBR; ++rb)
                for (int lane = 0; lane < 64; ++lane)
                    for (int j = 0; j < 4; ++j) {
                        const int row = map[16 * rb + (lane & 15)];
                        const int col = 16 * kc + 4 * (lane >> 4) + j;
                        const double v = (row >= 0 && row < K && col < K) ? A[(size_t)row * K + col] : 0.0;
                        out[((((size_t)oid * NKC + kc) * NBR + rb) * 64 + lane) * 4 + j] = (T)v;
                    }
    }
}
template void swizzle_m2l_ops<float>(int, const double *, float *);
template void swizzle_m2l_ops<double>(int, const double *, double *);

template <typename T>
__global__ __launch_bounds__(256) void k_m2l(const T *__restrict__ ops, const int32_t *__restrict__ il,
                                             const int32_t *__restrict__ offs, const T *__restrict__ M,
                                             T *__restrict__ L, int nh_bits, int NB, int Kp, int R,
                                             int nslices, int nil) {
    constexpr int CB = Mfma<T>::CB;
    constexpr int NRW = kRowBlocksPerWave;
    using V = typename Mfma<T>::V;
    __shared__ T red[4][CB * 4][64];

    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const int parity = blockIdx.x & 7;
    const int tile = (blockIdx.x >> 3) / nslices;
    const int slice = (blockIdx.x >> 3) % nslices;
    const int rg = wid % R;
    const int ts = wid / R;
    const int nts = 4 / R;
    const int rb0 = rg * NRW;
    const int nrb = min(NRW, NB - rb0);
    const uint32_t ntarget = 1u << (3 * nh_bits);
    const uint32_t nmask = (2u << nh_bits) - 1u;
    const uint32_t px = (parity >> 2) & 1, py = (parity >> 1) & 1, pz = parity & 1;

    uint32_t tx[CB], ty[CB], tz[CB];
    uint32_t tcell[CB];
    bool valid[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const uint32_t P = (uint32_t)tile * (16 * CB) + cb * 16 + (lane & 15);
        valid[cb] = P < ntarget;
        uint32_t a, b, c;
        demorton3(valid[cb] ? P : 0u, a, b, c);
        tx[cb] = 2 * a + px;
        ty[cb] = 2 * b + py;
        tz[cb] = 2 * c + pz;
        tcell[cb] = 8 * P + (uint32_t)parity;
    }

    V acc[NRW][CB];
#pragma unroll
    for (int rb = 0; rb < NRW; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = V{0, 0, 0, 0};

    // offsets of this workgroup's slice, then of this wavefront's share of it
    const int s0 = slice * nil / nslices, s1 = (slice + 1) * nil / nslices;
    const int t0 = s0 + ts * (s1 - s0) / nts, t1 = s0 + (ts + 1) * (s1 - s0) / nts;
    const size_t op_stride = (size_t)NB * NB * 64 * 4;  // elements per offset
    if (nrb > 0) {
        for (int t = t0; t < t1; ++t) {
            const int oid = il[parity * nil + t];
            const int ox = offs[3 * oid], oy = offs[3 * oid + 1], oz = offs[3 * oid + 2];
            const T *bp[CB];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const uint32_t sx = (tx[cb] + (uint32_t)ox) & nmask;
                const uint32_t sy = (ty[cb] + (uint32_t)oy) & nmask;
                const uint32_t sz = (tz[cb] + (uint32_t)oz) & nmask;
                bp[cb] = M + (size_t)morton3(sx, sy, sz) * Kp + 4 * (lane >> 4);
            }
            const T *ap = ops + (size_t)oid * op_stride + ((size_t)rb0 * 64 + lane) * 4;
            for (int kc = 0; kc < NB; ++kc) {
                V b[CB];
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) b[cb] = *reinterpret_cast<const V *>(bp[cb] + 16 * kc);
                V a[NRW];
                const T *akc = ap + (size_t)kc * NB * 64 * 4;
#pragma unroll
                for (int rb = 0; rb < NRW; ++rb)
                    if (rb < nrb) a[rb] = *reinterpret_cast<const V *>(akc + (size_t)rb * 64 * 4);
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int rb = 0; rb < NRW; ++rb)
                        if (rb < nrb)
#pragma unroll
                            for (int cb = 0; cb < CB; ++cb)
                                acc[rb][cb] = Mfma<T>::mma(a[rb][j], b[cb][j], acc[rb][cb]);
            }
        }
    }

    // reduce the offset slices: waves with ts > 0 hand their partial sums to
    // the ts == 0 wave of the same row group, one row block at a time
    if (nts > 1) {
#pragma unroll
        for (int rb = 0; rb < NRW; ++rb) {
            if (ts > 0 && rb < nrb)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) red[wid][cb * 4 + r][lane] = acc[rb][cb][r];
            __syncthreads();
            if (ts == 0 && rb < nrb)
                for (int s = 1; s < nts; ++s) {
                    const int w2 = rg + s * R;
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc[rb][cb][r] += red[w2][cb * 4 + r][lane];
                }
            __syncthreads();
        }
    }

    if (ts == 0) {
        // split-K: slice k of the partial buffer holds this slice's sums
        T *out = L + (size_t)slice * ((size_t)8 << (3 * nh_bits)) * Kp;
#pragma unroll
        for (int rb = 0; rb < NRW; ++rb)
            if (rb < nrb)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
                    if (valid[cb])
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int row = 16 * (rb0 + rb) + Mfma<T>::row(lane, r);
                            out[(size_t)tcell[cb] * Kp + row] = acc[rb][cb][r];
                        }
    }
}

// ---------------------------------------------------------------------------
// M2L for levels with many cells: operator chunks shared through LDS.
//   * a workgroup owns 4 x 16 target cells (one parity class) and one group
//     of up to 11 row blocks; the four wavefronts walk the same offsets t and
//     coefficient chunks kc in lockstep, each on its own 16 targets;
//   * operator chunks (t, kc) -- nrb x 64 lanes x 4 values, already in MFMA
//     lane order -- are loaded once per workgroup, U chunks per stage, into a
//     double-buffered LDS stage while the previous stage feeds the matrix
//     cores; one barrier per stage;
//   * each wavefront prefetches the multipole fragments of the next stage;
//   * FP32: after each offset t the matrix-core accumulators are added into
//     FP64 accumulators, so every FP32 rounding chain is one offset long
//     (11 chunks x 4 steps) instead of 875 offsets.
// Split-K over offset slices is available as for k_m2l.
// ---------------------------------------------------------------------------
// Operand policies of the LDS-shared kernel.  A chunk is one (offset,
// KW-coefficient column block); its operator fragments are NRB row blocks x
// 64 lanes of 16-byte A operands.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <typename T> struct PolMfma {  // FP32 or FP64 operands, v_mfma_*_16x16x4
    using S = T;                          // storage type of M and L
    using A = typename Mfma<T>::V;        // 16-byte (FP32) / 32-byte (FP64) operator fragment
    using B = typename Mfma<T>::V;
    using Acc = typename Mfma<T>::V;
    using R = B;                          // multipole fragment as loaded
    static constexpr int KW = 16;
    static constexpr bool kFlush64 = sizeof(T) == 4;
    static constexpr bool kPaired = true;  // list of (t, -t) entries, row-ordered operators
    __device__ static R load_b(const S *p, bool in) {
        return in ? *reinterpret_cast<const R *>(p) : R{0, 0, 0, 0};
    }
    __device__ static B to_b(const R &r) { return r; }
    __device__ static Acc mma(const A &a, const B &b, Acc c) {
#pragma unroll
        for (int j = 0; j < 4; ++j) c = Mfma<T>::mma(a[j], b[j], c);
        return c;
    }
};
struct PolBf16 {  // BF16 operands, FP32 storage and accumulation, v_mfma_f32_16x16x32_bf16
    using S = float;
    using A = bf16x8;
    using B = bf16x8;
    using Acc = f32x4;
    typedef float R __attribute__((ext_vector_type(8)));  // loaded as FP32, rounded at use
    static constexpr int KW = 32;
    static constexpr bool kFlush64 = false;
    static constexpr bool kPaired = false;  // plain list, storage-ordered operators
    __device__ static R load_b(const S *p, bool in) {
        return in ? *reinterpret_cast<const R *>(p) : R{0, 0, 0, 0, 0, 0, 0, 0};
    }
    __device__ static B to_b(const R &r) {
        B b;
#pragma unroll
        for (int i = 0; i < 8; ++i) b[i] = (__bf16)r[i];
        return b;
    }
    __device__ static Acc mma(const A &a, const B &b, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

// Per-element choice between two fragments by an all-ones / zero mask (bit
// operations, so a run-time choice never becomes a branch).
__device__ inline float pick(float a, float b, uint32_t m) {
    return __uint_as_float((__float_as_uint(a) & m) | (__float_as_uint(b) & ~m));
}
__device__ inline double pick(double a, double b, uint32_t m) {
    const unsigned long long mm = ((unsigned long long)m << 32) | m;
    return __longlong_as_double((long long)(((unsigned long long)__double_as_longlong(a) & mm) |
                                            ((unsigned long long)__double_as_longlong(b) & ~mm)));
}

// Chunks per LDS stage: enough matrix-core work per barrier (about 40 FP32
// MFMA-equivalents) within 48 KB of double-buffered LDS and a few registers.
template <typename P, int NRB> constexpr int stage_chunks() {
    constexpr int bytes = (int)sizeof(typename P::A);                   // per lane and row block
    constexpr int cyc = std::is_same<P, PolBf16>::value ? 16 : (bytes == 16 ? 4 * 32 : 4 * 64);
    constexpr int want = (1280 + cyc * NRB - 1) / (cyc * NRB);
    constexpr int lds_cap = (48 * 1024) / (2 * NRB * 64 * bytes);
    constexpr int u = want < lds_cap ? want : lds_cap;
    return u < 1 ? 1 : (u > 6 ? 6 : u);
}

// ---------------------------------------------------------------------------
// M2L for levels with many cells: operator chunks shared through LDS.
//   * a workgroup owns 4 x 16 target cells (one parity class) and NRB row
//     blocks (rows 16 rb0 .. 16 (rb0 + NRB) - 1); its four wavefronts walk the
//     same chunks (offset t, column block kc) in lockstep, each on its own 16
//     targets;
//   * U chunks per stage are loaded once per workgroup -- already in MFMA lane
//     order -- into double-buffered LDS, prefetched into registers one stage
//     ahead together with the multipole fragments; one barrier per stage;
//   * NRB and U are compile-time constants so the stage is straight-line
//     code: a run-time row count turned every MFMA into a branch and made the
//     compiler wait for all outstanding loads before each stage's first MFMA;
//     past the end of the list the prefetch re-reads a valid chunk and its
//     multipole fragment is zero, so the extra products add nothing;
//   * FP32: after each offset the matrix-core accumulators are added into FP64
//     accumulators, so every FP32 rounding chain is one offset long;
//   * blockIdx mod 8 = parity class (one class's operators per XCD L2).
// SPLIT: split-K over offset slices (partials to a buffer, added in a fixed
// order by k_m2l_reduce), compiled separately so profiles tell levels apart.
// ---------------------------------------------------------------------------
// NE: the number of even-degree row blocks of this row group (the first NE
// blocks), fixed at compile time: the single group of p <= 12 holds both
// kinds, larger orders split their rows into groups of one kind (NE = NRB or
// 0).  Unused by the unpaired (BF16) policy.
template <typename P, bool SPLIT, int NRB, int U, int NE>
__global__ __launch_bounds__(256) void k_m2l_lds(const typename P::A *__restrict__ ops,
                                                 const int32_t *__restrict__ il, const int32_t *__restrict__ offs,
                                                 const int32_t *__restrict__ rowmap,
                                                 const typename P::S *__restrict__ M,
                                                 const typename P::S *__restrict__ Mneg,
                                                 typename P::S *__restrict__ L,
                                                 int nh_bits, int NB, int NKC, int Kp, int rb0, int nslices_arg) {
    using S = typename P::S;
    using A = typename P::A;
    using B = typename P::B;
    using Acc = typename P::Acc;
    using R = typename P::R;
    constexpr bool F64 = P::kFlush64;
    constexpr bool PAIR = P::kPaired;
    constexpr int NENT = PAIR ? kM2LEntries : kILSize;  // list entries per parity class
    constexpr int CHUNK = NRB * 64;             // fragments per chunk
    constexpr int PC = (CHUNK + 255) / 256;     // fragment loads per thread per chunk
    __shared__ A lds[2][U * CHUNK];
    const int nslices = SPLIT ? nslices_arg : 1;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const int parity = blockIdx.x & 7;
    const int rest = blockIdx.x >> 3;
    const int slice = rest % nslices;
    const int tile = rest / nslices;
    const uint32_t ntarget = 1u << (3 * nh_bits);
    const uint32_t nmask = (2u << nh_bits) - 1u;

    const uint32_t Pt = (uint32_t)tile * 64 + (uint32_t)wid * 16 + (lane & 15);
    const bool valid = Pt < ntarget;
    uint32_t tx, ty, tz;
    demorton3(valid ? Pt : 0u, tx, ty, tz);
    tx = 2 * tx + ((parity >> 2) & 1);
    ty = 2 * ty + ((parity >> 1) & 1);
    tz = 2 * tz + (parity & 1);
    const uint32_t tcell = 8 * Pt + (uint32_t)parity;

    const int t0 = slice * NENT / nslices, t1 = (slice + 1) * NENT / nslices;
    const int nchunk = (t1 - t0) * NKC;
    const int nstage = (nchunk + U - 1) / U;
    const size_t op_stride = (size_t)NKC * NB * 64;  // fragments per offset
    const int32_t *ilp = il + parity * NENT * (PAIR ? 2 : 1);
    const int kq = (P::KW / 4) * (lane >> 4);        // this lane's k offset inside a chunk

    // chunk cursor (t, kc); the operator id and the multipole rows of this
    // lane's source cells change only with t.  Paired entries have a second
    // source cell (offset -t), read from Mneg = D M (odd degrees negated); for
    // single offsets src2 repeats src and m2 = 0 zeroes its fragment.
    struct Cursor {
        int t, kc;
        size_t base;    // first fragment of the chunk
        const S *src;   // this lane's coefficients of the source multipole
        const S *src2;  // ... of the paired source (offset -t), sign-flipped
        uint32_t m2;    // all-ones if the entry is a pair, else 0
    };
    auto source = [&](const S *base, int oid) {
        const uint32_t sx = (tx + (uint32_t)offs[3 * oid]) & nmask;
        const uint32_t sy = (ty + (uint32_t)offs[3 * oid + 1]) & nmask;
        const uint32_t sz = (tz + (uint32_t)offs[3 * oid + 2]) & nmask;
        return base + (size_t)morton3(sx, sy, sz) * Kp + kq;
    };
    auto set_t = [&](Cursor &c, int t) {
        c.t = t;
        c.kc = 0;
        const int e = min(t, t1 - 1);  // past the end: stay on a valid chunk
        if constexpr (PAIR) {
            const int oid = ilp[2 * e], oid2 = ilp[2 * e + 1];
            c.src = source(M, oid);
            c.src2 = oid2 >= 0 ? source(Mneg, oid2) : c.src;
            c.m2 = oid2 >= 0 ? 0xffffffffu : 0u;
            c.base = (size_t)oid * op_stride + (size_t)rb0 * 64;
        } else {
            const int oid = ilp[e];
            c.src = source(M, oid);
            c.src2 = c.src;
            c.m2 = 0u;
            c.base = (size_t)oid * op_stride + (size_t)rb0 * 64;
        }
    };
    auto advance = [&](Cursor &c) {
        if (++c.kc == NKC) set_t(c, c.t + 1);
        else c.base += (size_t)NB * 64;
    };
    // the multipole fragment of the cursor's chunk: zero past the list (only
    // reachable inside a stage when U > 1) and past Kp (only for 32-wide
    // chunks, whose last one may stick out of the padded row)
    auto frag_b = [&](const Cursor &c, const S *src) -> R {
        bool in = true;
        if constexpr (U > 1) in = c.t < t1;
        if constexpr (P::KW > 16) in = in && P::KW * c.kc + kq < Kp;
        return P::load_b(src + P::KW * c.kc, in);
    };

    Acc acc[NRB];
    double hi[F64 ? NRB : 1][4];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) acc[rb] = Acc{0, 0, 0, 0};
    if constexpr (F64)
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) hi[rb][r] = 0.0;

    Cursor pc;  // prefetch cursor
    set_t(pc, t0);
    int kc = 0;  // compute side: column block of the next chunk
    const int e_last = min(tid + 256 * (PC - 1), CHUNK - 1);
    const bool last_in = tid + 256 * (PC - 1) < CHUNK;

    // prologue: stage 0 into LDS buffer 0
    R bcur[U], bcur2[PAIR ? U : 1];
    uint32_t mcur[PAIR ? U : 1];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int v = 0; v < PC - 1; ++v) lds[0][u * CHUNK + tid + 256 * v] = ops[pc.base + tid + 256 * v];
        const A x = ops[pc.base + e_last];
        if (last_in) lds[0][u * CHUNK + e_last] = x;
        bcur[u] = frag_b(pc, pc.src);
        if constexpr (PAIR) {
            bcur2[u] = frag_b(pc, pc.src2);
            mcur[u] = pc.m2;
        }
        advance(pc);
    }
    // drain every prologue load: otherwise the compiler's wait bookkeeping
    // carries them into the loop and waits on all loads before the MFMAs
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    for (int st = 0; st < nstage; ++st) {
        const int cur = st & 1;
        // prefetch the next stage (past the end: harmless re-reads)
        A pre[U][PC];
        R bnext[U], bnext2[PAIR ? U : 1];
        uint32_t mnext[PAIR ? U : 1];
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int v = 0; v < PC - 1; ++v) pre[u][v] = ops[pc.base + tid + 256 * v];
            pre[u][PC - 1] = ops[pc.base + e_last];
            bnext[u] = frag_b(pc, pc.src);
            if constexpr (PAIR) {
                bnext2[u] = frag_b(pc, pc.src2);
                mnext[u] = pc.m2;
            }
            // compiler-only barrier: keeps the loads above the cursor update
            // (otherwise they are sunk below its branch, towards their use)
            asm volatile("" ::: "memory");
            advance(pc);
        }
        // keep the prefetch loads ahead of the matrix-core work (the
        // scheduler would otherwise sink them towards their use at the end)
        if constexpr (sizeof(A) == 16) __builtin_amdgcn_sched_barrier(0);
        // this stage on the matrix cores
#pragma unroll
        for (int u = 0; u < U; ++u) {
            A a[NRB];
#pragma unroll
            for (int rb = 0; rb < NRB; ++rb) a[rb] = lds[cur][u * CHUNK + rb * 64 + lane];
            // all 16-byte fragment reads issued before the first MFMA (FP64
            // fragments are twice as large: there the compiler's interleaving
            // of reads and MFMAs is kept, measured faster)
            if constexpr (sizeof(A) == 16) __builtin_amdgcn_sched_barrier(0);
            if constexpr (PAIR) {
                // v1 = b + D b2 feeds the even-degree rows, v2 = b - D b2 the odd
                B v1, v2;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const S m = pick((S)bcur2[u][j], (S)0, mcur[u]);
                    v1[j] = bcur[u][j] + m;
                    v2[j] = bcur[u][j] - m;
                }
#pragma unroll
                for (int rb = 0; rb < NRB; ++rb) acc[rb] = P::mma(a[rb], rb < NE ? v1 : v2, acc[rb]);
            } else {
                const B b = P::to_b(bcur[u]);
#pragma unroll
                for (int rb = 0; rb < NRB; ++rb) acc[rb] = P::mma(a[rb], b, acc[rb]);
            }
            if (++kc == NKC) {
                kc = 0;
                if constexpr (F64) {
#pragma unroll
                    for (int rb = 0; rb < NRB; ++rb) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) hi[rb][r] += (double)acc[rb][r];
                        acc[rb] = Acc{0, 0, 0, 0};
                    }
                }
            }
        }
        // publish the prefetched stage: for 16-byte fragments after all of this
        // stage's MFMAs, so the waits for the prefetch loads come as late as
        // possible; FP64 stages are long enough that the compiler's placement
        // of the LDS writes among the MFMAs hides their latency (measured)
        if constexpr (sizeof(A) == 16) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int v = 0; v < PC - 1; ++v) lds[cur ^ 1][u * CHUNK + tid + 256 * v] = pre[u][v];
            if (last_in) lds[cur ^ 1][u * CHUNK + e_last] = pre[u][PC - 1];
            bcur[u] = bnext[u];
            if constexpr (PAIR) {
                bcur2[u] = bnext2[u];
                mcur[u] = mnext[u];
            }
        }
        __syncthreads();
    }

    if (!valid) return;
    S *out = L + (size_t)slice * ((size_t)8 << (3 * nh_bits)) * Kp;
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int prow = 16 * (rb0 + rb) + Mfma<S>::row(lane, r);
            const int row = PAIR ? rowmap[prow] : prow;
            if (row >= 0)
                out[(size_t)tcell * Kp + row] = F64 ? (S)(hi[rb][r] + (double)acc[rb][r]) : (S)acc[rb][r];
        }
}

// Even-degree row blocks of the single row group of order p <= 12 with NRB
// row blocks (NRB = m2l_row_blocks(p) determines it for those p; 0: none).
constexpr int single_group_even_blocks(int nrb) {
    constexpr int table[12] = {0, 1, 1, 1, 2, 2, 3, 3, 0, 5, 5, 6};
    return nrb >= 0 && nrb < 12 ? table[nrb] : 0;
}

// Launches the LDS-shared kernel for every row group (NRB, U and the group's
// even-degree block count fixed at compile time).  Row groups hold up to
// kRowBlocksPerWave blocks; with the paired list an order whose rows do not
// fit one group gets groups of even-degree blocks and groups of odd-degree
// blocks, so that no group mixes them at a position other than the one of
// single_group_even_blocks.
template <typename P>
static hipError_t launch_lds(const void *ops, const int32_t *il, const int32_t *offs, const int32_t *rowmap,
                             const typename P::S *M, const typename P::S *Mneg, typename P::S *out, int nh_bits,
                             int NB, int NKC, int Kp, int nslices, int ne_blocks, hipStream_t s) {
    using A = typename P::A;
    if (P::kPaired && NKC > 32) return hipErrorInvalidValue;  // column parity bits: two 64-bit words
    struct Group {
        int rb0, nrb, ne;
    };
    Group groups[16];
    int ng = 0;
    auto add = [&](int from, int to, bool even) {
        for (int r = from; r < to; r += kRowBlocksPerWave) {
            if (ng == 16) return false;
            const int n = std::min(kRowBlocksPerWave, to - r);
            groups[ng++] = Group{r, n, even ? n : 0};
        }
        return true;
    };
    if (!P::kPaired) {
        if (!add(0, NB, false)) return hipErrorInvalidValue;
    } else if (NB <= kRowBlocksPerWave) {
        if (ne_blocks != single_group_even_blocks(NB)) return hipErrorInvalidValue;
        groups[ng++] = Group{0, NB, ne_blocks};
    } else if (!add(0, ne_blocks, true) || !add(ne_blocks, NB, false)) {
        return hipErrorInvalidValue;
    }
    const int64_t ntile = (((int64_t)1 << (3 * nh_bits)) + 63) / 64;
    const int64_t grid = 8 * ntile * nslices;
    const A *o = reinterpret_cast<const A *>(ops);
    for (int gi = 0; gi < ng; ++gi) {
        const int rb0 = groups[gi].rb0, nrb = groups[gi].nrb, ne = groups[gi].ne;
        switch (nrb) {
#define FMM_M2L_LDS_LAUNCH(N, NE)                                                                              \
    if (nslices > 1)                                                                                           \
        hipLaunchKernelGGL((k_m2l_lds<P, true, N, stage_chunks<P, N>(), NE>), dim3((unsigned)grid), dim3(256), \
                           0, s, o, il, offs, rowmap, M, Mneg, out, nh_bits, NB, NKC, Kp, rb0, nslices);            \
    else                                                                                                       \
        hipLaunchKernelGGL((k_m2l_lds<P, false, N, stage_chunks<P, N>(), NE>), dim3((unsigned)grid),          \
                           dim3(256), 0, s, o, il, offs, rowmap, M, Mneg, out, nh_bits, NB, NKC, Kp, rb0, 1);
#define FMM_M2L_LDS_CASE(N)                                                                                    \
    case N:                                                                                                    \
        if (!P::kPaired || ne == 0) {                                                                          \
            FMM_M2L_LDS_LAUNCH(N, 0)                                                                           \
        } else if (ne == N) {                                                                                  \
            FMM_M2L_LDS_LAUNCH(N, N)                                                                           \
        } else if (ne == single_group_even_blocks(N)) {                                                        \
            FMM_M2L_LDS_LAUNCH(N, single_group_even_blocks(N))                                                 \
        } else {                                                                                               \
            return hipErrorInvalidValue;                                                                       \
        }                                                                                                      \
        break;
            FMM_M2L_LDS_CASE(1) FMM_M2L_LDS_CASE(2) FMM_M2L_LDS_CASE(3) FMM_M2L_LDS_CASE(4)
            FMM_M2L_LDS_CASE(5) FMM_M2L_LDS_CASE(6) FMM_M2L_LDS_CASE(7) FMM_M2L_LDS_CASE(8)
            FMM_M2L_LDS_CASE(9) FMM_M2L_LDS_CASE(10) FMM_M2L_LDS_CASE(11)
#undef FMM_M2L_LDS_CASE
#undef FMM_M2L_LDS_LAUNCH
            default: return hipErrorInvalidValue;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Sum of the split-K partial results in slice order (deterministic).
template <typename T>
__global__ void k_m2l_reduce(const T *__restrict__ partial, T *__restrict__ L, int nslices, int64_t elems) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < elems;
         i += (int64_t)gridDim.x * blockDim.x) {
        T acc = 0;
        for (int k = 0; k < nslices; ++k) acc += partial[(size_t)k * elems + i];
        L[i] = acc;
    }
}

// Slices per level: enough workgroups (>= ~512) to fill 256 CUs at two
// resident workgroups each; levels >= 5 have enough targets on their own.
int m2l_slices(int level) {
    static const int leaf = [] {
        const char *v = std::getenv("FMM_M2L_FINE_SLICES");
        const int k = v ? std::atoi(v) : 0;
        return (k == 1 || k == 2 || k == 4 || k == 8) ? k : 1;
    }();
    switch (level) {
        case 1: return 64;
        case 2: return 64;
        case 3: return 64;
        case 4: return 32;
        default: return leaf;
    }
}


// ---------------------------------------------------------------------------
// M2L with BF16 operands (precision mode FMM_MIXED_BF16_M2L): the same
// contraction L~_c += sum_t O_t M~_{c+t} on v_mfma_f32_16x16x32_bf16, which
// takes 8 consecutive k values per lane: lane l holds
//   A[l % 16][8 (l / 16) + i]  (operator rows, k)   and
//   B[8 (l / 16) + i][l % 16]  (k, target columns),  i = 0..7,
// and returns the 16x16 FP32 block with the layout of the FP32 instruction.
// K is walked in chunks of 32 (NKC = ceil(K / 32)); the FP32 multipoles are
// rounded to BF16 as they are loaded (coefficients past Kp read as 0).
// Workgroup layout, LDS staging (U chunks per stage, double buffered) and
// split-K are those of k_m2l_lds; accumulation stays in FP32 because the
// BF16 operand rounding (2^-9 relative) dominates the error.
// ---------------------------------------------------------------------------
static inline uint16_t bf16_round(double v) {
    const float f = (float)v;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}

static int bf16_chunks(int p) { return (num_coeffs(p) + 31) / 32; }

size_t m2l_bf16_ops_elems(int p) {
    return (size_t)kNumOffsets * bf16_chunks(p) * (padded_coeffs(p) / 16) * 64 * 8;
}

void swizzle_m2l_ops_bf16(int p, const double *ops, uint16_t *out) {
    const int K = num_coeffs(p), NB = padded_coeffs(p) / 16, NKC = bf16_chunks(p);
    for (int oid = 0; oid < kNumOffsets; ++oid) {
        const double *A = ops + (size_t)oid * K * K;
        for (int kc = 0; kc < NKC; ++kc)
            for (int rb = 0; rb < NB; ++rb)
                for (int lane = 0; lane < 64; ++lane)
                    for (int i = 0; i < 8; ++i) {
                        const int row = 16 * rb + (lane & 15);
                        const int col = 32 * kc + 8 * (lane >> 4) + i;
                        const double v = (row < K && col < K) ? A[(size_t)row * K + col] : 0.0;
                        out[((((size_t)oid * NKC + kc) * NB + rb) * 64 + lane) * 8 + i] = bf16_round(v);
                    }
    }
}

hipError_t launch_m2l_bf16(int level, const void *ops, const int32_t *il, const int32_t *offs, const float *M,
                           float *L, float *partial, int p, int Kp, hipStream_t s) {
    const int NB = Kp / 16;
    const int nh_bits = level - 1;
    const int nslices = partial ? m2l_slices(level) : 1;
    hipError_t e = launch_lds<PolBf16>(ops, il, offs, nullptr, M, M, nslices > 1 ? partial : L, nh_bits, NB,
                                       bf16_chunks(p), Kp, nslices, 0, s);
    if (e != hipSuccess || nslices == 1) return e;
    const int64_t elems = ((int64_t)8 << (3 * nh_bits)) * Kp;
    int64_t g = (elems + 255) / 256;
    if (g > 65535) g = 65535;
    hipLaunchKernelGGL(k_m2l_reduce<float>, dim3((unsigned)g), dim3(256), 0, s, partial, L, nslices, elems);
    return hipGetLastError();
}

// Mneg[c][k] = (-1)^n(k) M[c][k] (n(k) the degree of coefficient k): the
// multipoles as the paired kernel reads them for the offset -t of a pair.
template <typename T>
__global__ void k_m2l_flip(const T *__restrict__ M, T *__restrict__ Mneg, int64_t n, int Kp) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(i % Kp);
        int d = (int)sqrtf((float)k);
        if (d * d > k) --d;
        if ((d + 1) * (d + 1) <= k) ++d;
        Mneg[i] = (d & 1) ? -M[i] : M[i];
    }
}

// The full interaction list (nil == 875) runs on the LDS-shared kernel with
// the paired entries (Mneg: scratch for the level's sign-flipped multipoles,
// cells x Kp); the aliased lists of levels 1 and 2 (nil = 8 or 64 pre-summed
// operators) on the offset-split kernel.
template <typename T>
hipError_t launch_m2l(int level, const T *ops, const int32_t *list, const int32_t *offs, const int32_t *rowmap,
                      const T *M, T *Mneg, T *L, T *partial, int p, int Kp, hipStream_t s, int nil) {
    constexpr int CB = Mfma<T>::CB;
    const int NB = Kp / 16;
    const int nh_bits = level - 1;
    const int64_t ntarget = (int64_t)1 << (3 * nh_bits);
    const int nslices = partial ? std::min(m2l_slices(level), nil) : 1;
    if (nil == kILSize) {
        if (!rowmap || !Mneg) return hipErrorInvalidValue;
        const int64_t n = ((int64_t)8 << (3 * nh_bits)) * Kp;
        int64_t g = (n + 255) / 256;
        if (g > 65535) g = 65535;
        hipLaunchKernelGGL(k_m2l_flip<T>, dim3((unsigned)g), dim3(256), 0, s, M, Mneg, n, Kp);
        const hipError_t e = launch_lds<PolMfma<T>>(ops, list, offs, rowmap, M, Mneg, nslices > 1 ? partial : L,
                                                     nh_bits, m2l_row_blocks(p), NB, Kp, nslices, m2l_even_blocks(p),
                                                     s);
        if (e != hipSuccess) return e;
    } else {
        int R = 1;
        if (NB > kRowBlocksPerWave) R = 2;
        if (NB > 2 * kRowBlocksPerWave) R = 4;
        if (NB > 4 * kRowBlocksPerWave) return hipErrorInvalidValue;
        const int64_t ntile = (ntarget + 16 * CB - 1) / (16 * CB);
        const int64_t grid = 8 * ntile * nslices;
        hipLaunchKernelGGL(k_m2l<T>, dim3((unsigned)grid), dim3(256), 0, s, ops, list, offs, M,
                           nslices > 1 ? partial : L, nh_bits, NB, Kp, R, nslices, nil);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nslices == 1) return e;
    const int64_t elems = ((int64_t)8 << (3 * nh_bits)) * Kp;
    int64_t g = (elems + 255) / 256;
    if (g > 65535) g = 65535;
    hipLaunchKernelGGL(k_m2l_reduce<T>, dim3((unsigned)g), dim3(256), 0, s, partial, L, nslices, elems);
    return hipGetLastError();
}
template hipError_t launch_m2l<float>(int, const float *, const int32_t *, const int32_t *, const int32_t *,
                                      const float *, float *, float *, float *, int, int, hipStream_t, int);
template hipError_t launch_m2l<double>(int, const double *, const int32_t *, const int32_t *, const int32_t *,
                                       const double *, double *, double *, double *, int, int, hipStream_t, int);

}  // namespace fmm
