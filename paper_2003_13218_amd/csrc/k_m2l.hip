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
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <vector>

#include "fmm_internal.h"
#include "mfma.h"
#include "morton.h"

namespace fmm {

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
    static constexpr int kMaxNRB = 12;     // largest row group instantiated
    template <int SYM, int N, int NE> static constexpr bool allow() { return SYM != 0; }
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
    static constexpr int kMaxNRB = 11;
    template <int SYM, int N, int NE> static constexpr bool allow() { return SYM == 0; }
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

// Split FP16 operands (precision mode FMM_MIXED_SPLIT16_M2L): operator and
// multipole entries x are each written as x = hi + lo with hi = fp16(x) and
// lo = fp16(x - hi), and the product as hi*hi + hi*lo + lo*hi on
// v_mfma_f32_16x16x32_f16 with FP32 accumulation (the lo*lo term and the
// rounding of lo leave a relative error of about 2^-22 per product, against
// 2^-24 for FP32 operands).  FP16's range is kept by powers of two: column k
// of the operators is multiplied by 2^{b_k} and the multipoles divided by it
// (in a pre-pass over the level), row r by 2^{a_r} and the result divided by
// it on output, both exact.  Two kernels take them: k_m2l_lds with the policy
// below (folded orbit list, p = 11, 12) and k_m2l_f16rows (plain list).
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
struct F16Pair {
    f16x8 hi, lo;
};
__device__ inline f32x4 mma_split16(const F16Pair &a, const F16Pair &b, f32x4 c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_f16(a.lo, b.hi, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_f16(a.hi, b.lo, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a.hi, b.hi, c, 0, 0, 0);
}
// Folded orbit list with class-ordered operator rows (as the FP32 / FP64
// kernels), the four orbit classes of three blocks each in one launch: the
// class combinations of an entry's four sources are formed in FP32 and split
// into hi and lo inside the kernel.
struct PolF16x3F {
    using S = float;
    using A = F16Pair;
    using B = F16Pair;
    using Acc = f32x4;
    typedef float R __attribute__((ext_vector_type(8)));
    static constexpr int KW = 32;
    static constexpr bool kFlush64 = true;
    static constexpr bool kPaired = true;
    static constexpr int kMaxNRB = 12;
    template <int SYM, int N, int NE> static constexpr bool allow() { return SYM == 4 && N == 12 && NE == 3; }
    __device__ static R load_b(const S *p, bool in) {
        return in ? *reinterpret_cast<const R *>(p) : R{0, 0, 0, 0, 0, 0, 0, 0};
    }
    __device__ static B to_b(const R &r) {
        B b;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const _Float16 h = (_Float16)r[i];
            b.hi[i] = h;
            b.lo[i] = (_Float16)(r[i] - (float)h);
        }
        return b;
    }
    __device__ static Acc mma(const A &a, const B &b, Acc c) { return mma_split16(a, b, c); }
};
template <typename P> constexpr bool is_split16() { return std::is_same<P, PolF16x3F>::value; }

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

// Stages whose loads are in flight while one runs.  The folded split kernel
// runs one wavefront per SIMD, so no other wavefront covers the latency of a
// stage's gathers: it prefetches two stages ahead, one chunk per stage (1M-atom
// box, finest level: 5.98 ms against 6.22 ms one stage ahead).
template <typename P, int SYM> constexpr int prefetch_depth() { return (is_split16<P>() && SYM != 0) ? 2 : 1; }

// Chunks per LDS stage: enough matrix-core work per barrier (about 40 FP32
// MFMA-equivalents) within 48 KB of double-buffered LDS and a few registers
// (the folded split kernel: one, see prefetch_depth).
template <typename P, int NRB, int SYM> constexpr int stage_chunks() {
    constexpr int bytes = (int)sizeof(typename P::A);                   // per lane and row block
    constexpr int cyc = std::is_same<P, PolBf16>::value ? 16
                        : is_split16<P>() ? 3 * 16
                                                          : (bytes == 16 ? 4 * 32 : 4 * 64);
    constexpr int want = (1280 + cyc * NRB - 1) / (cyc * NRB);
    constexpr int lds_cap = (48 * 1024) / (2 * NRB * 64 * bytes);
    constexpr int reg_cap = is_split16<P>() ? 1 : 6;
    constexpr int u0 = want < lds_cap ? want : lds_cap;
    constexpr int u = u0 < reg_cap ? u0 : reg_cap;
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
// SYM: 0 plain list (one source per entry); 1 pairs (t, -t); 2 / 3 orbits of
// the two-axis flips, first / second half of the row classes; 4 orbits, all
// four row classes in one launch (NE blocks each).  For SYM 1-3 the first NE
// row blocks of the group take the first combination of the entry's sources,
// the others the second (compile-time constants).  Sources: M for the entry's
// first offset, the sign-flipped copies Mflip + f * fstride (D_s M of the
// group element s of slot f + 1) for the others, zeros for an absent image.
//
// Occupancy: left to itself the compiler gives the FP32 all-classes variant
// (12 row blocks: 48 FP32 accumulators, 96 FP64 ones, 48 operator fragment
// registers) 256 VGPRs plus a few AGPRs, i.e. one wavefront per SIMD, and the
// multipole gathers of a stage stall its matrix core.  Capped at 256 registers
// (237 once the operator fragment reads interleave with the MFMAs, below) two
// wavefronts per SIMD hide each other's waits: 8.2 -> 6.7 ms for the finest
// level of the 1M-atom box.  The FP64 half-class variants stay at two
// wavefronts: squeezed to three they spill inside the stage and lose.  The
// folded split kernel (all classes, 32-byte fragments, FP64 flush
// accumulators, two stages of prefetch) holds about 410 registers and runs one
// wavefront per SIMD.
template <typename P, int NRB, int SYM> constexpr int m2l_min_waves() {
    return (sizeof(typename P::S) == 4 && !is_split16<P>() && SYM == 4 && NRB == 12) ? 2 : 1;
}

template <typename P, bool SPLIT, int NRB, int U, int NE, int SYM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(m2l_min_waves<P, NRB, SYM>()))) void k_m2l_lds(
    const typename P::A *__restrict__ ops, const int32_t *__restrict__ il, const int32_t *__restrict__ offs,
    const int32_t *__restrict__ rowmap, const typename P::S *__restrict__ M, const typename P::S *__restrict__ Mflip,
    const typename P::S *__restrict__ zeros, int64_t fstride, typename P::S *__restrict__ L, double *__restrict__ L64,
    const float *__restrict__ rscale, int nh_bits, int NB, int NKC, int Kp, int rb0, int nslices_arg) {
    using S = typename P::S;
    using A = typename P::A;
    using B = typename P::B;
    using Acc = typename P::Acc;
    using R = typename P::R;
    constexpr bool F64 = P::kFlush64;
    constexpr int NSRC = SYM == 0 ? 1 : (SYM == 1 ? 2 : 4);       // sources per list entry
    constexpr int NRV = P::KW / 4;                                 // coefficients per lane and source
    constexpr int DB = prefetch_depth<P, SYM>();                   // stages in flight
    static_assert(SYM != 4 || NRB == 4 * NE, "all four classes: NE blocks each");
    constexpr int NENT = SYM == 0 ? kILSize : (SYM == 1 ? kM2LPairEntries : kM2LOrbitEntries);
    constexpr int CHUNK = NRB * 64;             // fragments per chunk
    constexpr int PC = (CHUNK + 255) / 256;     // fragment loads per thread per chunk
    // operator chunks in LDS.  The split-FP16 fragments (32 bytes: hi, lo) are
    // stored as two planes of 16-byte words, so each of the two 16-byte reads
    // of a fragment has its lanes 16 bytes apart, free of bank conflicts;
    // interleaved, lanes 32 bytes apart, every read conflicts two ways (1M-atom
    // box, finest level 6.04 -> 5.74 ms).  The FP64 fragments stay interleaved:
    // that kernel is bound by the FP64 matrix rate, and planes measured 1.7%
    // slower there.
    constexpr int NW = (int)(sizeof(A) / 16);
    static_assert(sizeof(A) % 16 == 0, "fragments of whole 16-byte words");
    constexpr bool PLANES = is_split16<P>();
    using LdsT = typename std::conditional<PLANES, uint4, A>::type;
    __shared__ LdsT lds[2][(PLANES ? NW : 1) * U * CHUNK];
    auto lds_put = [&](int buf, int idx, const A &x) __attribute__((always_inline)) {
        if constexpr (PLANES) {
            uint4 w[NW];
            __builtin_memcpy(w, &x, sizeof(A));
#pragma unroll
            for (int i = 0; i < NW; ++i) lds[buf][i * (U * CHUNK) + idx] = w[i];
        } else {
            lds[buf][idx] = x;
        }
    };
    auto lds_get = [&](int buf, int idx) __attribute__((always_inline)) -> A {
        if constexpr (PLANES) {
            uint4 w[NW];
#pragma unroll
            for (int i = 0; i < NW; ++i) w[i] = lds[buf][i * (U * CHUNK) + idx];
            A x;
            __builtin_memcpy(&x, w, sizeof(A));
            return x;
        } else {
            return lds[buf][idx];
        }
    };
    const int nslices = SPLIT ? nslices_arg : 1;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const int parity = blockIdx.x & 7;
    const int rest = blockIdx.x >> 3;
    const int slice = rest % nslices;
    const int tile = rest / nslices;
    const uint32_t ntarget = 1u << (3 * nh_bits);

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
    const int32_t *ilp = il + parity * NENT * NSRC;
    const int kq = (P::KW / 4) * (lane >> 4);        // this lane's k offset inside a chunk

    // chunk cursor (t, kc); the operator id and the multipole rows of this
    // lane's source cells change only with t
    struct Cursor {
        int t, kc;
        size_t base;         // first fragment of the chunk
        const S *src[NSRC];  // this lane's coefficients of each source multipole
    };
    // Source cells by dilated-integer addition: the target's Morton bits of
    // one axis with every other bit set, plus the spread (10-bit two's
    // complement) offset of that axis, carry through the other axes' bits; the
    // axis mask keeps the level's bits, i.e. the sum mod 2^l (periodic wrap).
    // The offsets are wave-uniform, so their spreading runs on the scalar unit.
    const uint32_t lvl = (8u << (3 * nh_bits)) - 1u;
    const uint32_t zm = 0x09249249u & lvl, ym = (0x09249249u << 1) & lvl, xm = (0x09249249u << 2) & lvl;
    const uint32_t tdx = (spread3(tx) << 2) | ~xm, tdy = (spread3(ty) << 1) | ~ym, tdz = spread3(tz) | ~zm;
    auto source = [&](const S *base, int oid) {
        const uint32_t cx = (tdx + (spread3((uint32_t)offs[3 * oid]) << 2)) & xm;
        const uint32_t cy = (tdy + (spread3((uint32_t)offs[3 * oid + 1]) << 1)) & ym;
        const uint32_t cz = (tdz + spread3((uint32_t)offs[3 * oid + 2])) & zm;
        return base + (size_t)(cx | cy | cz) * Kp + kq;
    };
    auto set_t = [&](Cursor &c, int t) {
        c.t = t;
        c.kc = 0;
        const int e = min(t, t1 - 1);  // past the end: stay on a valid chunk
        const int oid = ilp[NSRC * e];
        c.src[0] = source(M, oid);
#pragma unroll
        for (int f = 1; f < NSRC; ++f) {
            const int o2 = ilp[NSRC * e + f];
            c.src[f] = o2 >= 0 ? source(Mflip + (f - 1) * fstride, o2) : zeros + kq;
        }
        c.base = (size_t)oid * op_stride + (size_t)rb0 * 64;
    };
    auto advance = [&](Cursor &c) {
        if (++c.kc == NKC) set_t(c, c.t + 1);
        else c.base += (size_t)NB * 64;
    };
    // the multipole fragment of the cursor's chunk: zero past the list (only
    // reachable inside a stage when U > 1) and past Kp (only for 32-wide
    // chunks, whose last one may stick out of the padded row)
    // operator fragment i of the cursor's chunk: a wave-uniform chunk base
    // plus a small per-lane byte offset, so the load takes the scalar base +
    // 32-bit vector offset form and the chunk advance stays on the scalar unit
    // (the empty asm keeps the offset's widening inside the loop body, where
    // instruction selection can see it; hoisted, it became a 64-bit vector add
    // per load)
    auto op_frag = [&](const Cursor &c, int i) -> A {
        const char *chunk = reinterpret_cast<const char *>(ops + c.base);
        uint32_t off = (uint32_t)i * (uint32_t)sizeof(A);
        asm volatile("" : "+v"(off));
        return *reinterpret_cast<const A *>(chunk + off);
    };
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

    // prologue: stage 0 into LDS buffer 0 (and, two stages deep, stage 1's
    // operators into registers)
    R bcur[U][NSRC];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int v = 0; v < PC - 1; ++v) lds_put(0, u * CHUNK + tid + 256 * v, op_frag(pc, tid + 256 * v));
        const A x = op_frag(pc, e_last);
        if (last_in) lds_put(0, u * CHUNK + e_last, x);
#pragma unroll
        for (int f = 0; f < NSRC; ++f) bcur[u][f] = frag_b(pc, pc.src[f]);
        advance(pc);
    }

    // prefetch of a later stage: operators to registers (pre), multipole
    // fragments to bnext (past the end: harmless re-reads)
    auto issue = [&](A (&pre)[U][PC], R (&bnext)[U][NSRC]) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int v = 0; v < PC - 1; ++v) pre[u][v] = op_frag(pc, tid + 256 * v);
            pre[u][PC - 1] = op_frag(pc, e_last);
#pragma unroll
            for (int f = 0; f < NSRC; ++f) bnext[u][f] = frag_b(pc, pc.src[f]);
            // compiler-only barrier: keeps the loads above the cursor update
            // (otherwise they are sunk below its branch, towards their use)
            asm volatile("" ::: "memory");
            advance(pc);
        }
    };
    // one stage on the matrix cores from LDS buffer cur and bcur
    auto compute = [&](const int cur, R (&bcur)[U][NSRC]) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            A a[NRB];
#pragma unroll
            for (int rb = 0; rb < NRB; ++rb) a[rb] = lds_get(cur, u * CHUNK + rb * 64 + lane);
            // all 16-byte fragment reads issued before the first MFMA (FP64
            // fragments are twice as large: there the compiler's interleaving
            // of reads and MFMAs is kept, measured faster).  Not for the
            // all-classes variant: its 12 fragments held at once would push it
            // past 256 registers (spills), and at two wavefronts per SIMD the
            // interleaved reads are hidden (6.62 -> 6.38 ms, 1M-atom leaf level)
            if constexpr (sizeof(A) == 16 && SYM != 4) __builtin_amdgcn_sched_barrier(0);
            if constexpr (SYM == 0) {
                const B b = P::to_b(bcur[u][0]);
#pragma unroll
                for (int rb = 0; rb < NRB; ++rb) acc[rb] = P::mma(a[rb], b, acc[rb]);
            } else if constexpr (SYM == 4) {
                // all four classes of the orbit list (NE blocks each):
                // (w0 + w1) +- (w2 + w3), (w0 - w1) +- (w2 - w3)
                R w[4];
#pragma unroll
                for (int j = 0; j < NRV; ++j) {
                    const S xp = bcur[u][0][j] + bcur[u][1][j], xm = bcur[u][0][j] - bcur[u][1][j];
                    const S yp = bcur[u][2][j] + bcur[u][3][j], ym = bcur[u][2][j] - bcur[u][3][j];
                    w[0][j] = xp + yp;
                    w[1][j] = xp - yp;
                    w[2][j] = xm + ym;
                    w[3][j] = xm - ym;
                }
                const B v[4] = {P::to_b(w[0]), P::to_b(w[1]), P::to_b(w[2]), P::to_b(w[3])};
#pragma unroll
                for (int rb = 0; rb < NRB; ++rb) acc[rb] = P::mma(a[rb], v[rb / NE], acc[rb]);
                // 16-byte fragments: read one row-block pair ahead of the eight
                // MFMAs that use it, so the LDS latency hides behind the pair
                // before (left to itself the compiler issued each pair's reads
                // right after the previous pair's last MFMA and waited on them:
                // leaf level 6.04 -> 5.88 ms)
                if constexpr (sizeof(A) == 16) {
                    __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);  // LDS reads
#pragma unroll
                    for (int g = 0; g < NRB / 2; ++g) {
                        __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);  // MFMA
                        if (g + 2 < NRB / 2) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
                    }
                }
            } else {
                // the class combinations sum_s chi(s) D_s M_s of the entry:
                // pairs: w0 +- w1; orbits: (w0 +- w1) + (w2 +- w3) for the
                // first class of the half, (w0 +- w1) - (w2 +- w3) for the second
                R w1, w2;
#pragma unroll
                for (int j = 0; j < NRV; ++j) {
                    if constexpr (SYM == 1) {
                        w1[j] = bcur[u][0][j] + bcur[u][1][j];
                        w2[j] = bcur[u][0][j] - bcur[u][1][j];
                    } else {
                        const S x = SYM == 2 ? bcur[u][0][j] + bcur[u][1][j] : bcur[u][0][j] - bcur[u][1][j];
                        const S y = SYM == 2 ? bcur[u][2][j] + bcur[u][3][j] : bcur[u][2][j] - bcur[u][3][j];
                        w1[j] = x + y;
                        w2[j] = x - y;
                    }
                }
                const B v1 = P::to_b(w1), v2 = P::to_b(w2);
#pragma unroll
                for (int rb = 0; rb < NRB; ++rb) acc[rb] = P::mma(a[rb], rb < NE ? v1 : v2, acc[rb]);
                // FP64 orbit halves: each row block's 32-byte fragment (two
                // reads) issued two row blocks ahead of its four MFMAs (FP64
                // leaf level of the 1M-atom box 13.78 -> 13.56 ms)
                if constexpr (std::is_same<S, double>::value && SYM >= 2) {
                    __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);  // LDS reads
#pragma unroll
                    for (int g = 0; g < NRB; ++g) {
                        __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);  // MFMA
                        if (g + 2 < NRB) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
                    }
                }
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
    };
    // the prefetched operators of the next stage into LDS buffer nxt
    auto publish = [&](const int nxt, A (&pre)[U][PC]) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int v = 0; v < PC - 1; ++v) lds_put(nxt, u * CHUNK + tid + 256 * v, pre[u][v]);
            if (last_in) lds_put(nxt, u * CHUNK + e_last, pre[u][PC - 1]);
        }
    };

    if constexpr (DB == 1) {
        // drain every prologue load: otherwise the compiler's wait bookkeeping
        // carries them into the loop and waits on all loads before the MFMAs
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        // One stage: prefetch the next one, run this one, publish the
        // prefetched operators in LDS buffer cur ^ 1.  The loop below calls it
        // twice per iteration with the two fragment sets swapped, so no
        // register copy moves bnext into bcur.
        auto stage = [&](const int cur, R (&bcur)[U][NSRC], R (&bnext)[U][NSRC]) __attribute__((always_inline)) {
            A pre[U][PC];
            issue(pre, bnext);
            // keep the prefetch loads ahead of the matrix-core work (the
            // scheduler would otherwise sink them towards their use at the end)
            if constexpr (sizeof(A) == 16) __builtin_amdgcn_sched_barrier(0);
            compute(cur, bcur);
            // publish the prefetched stage: for 16-byte fragments after all of this
            // stage's MFMAs, so the waits for the prefetch loads come as late as
            // possible; FP64 stages are long enough that the compiler's placement
            // of the LDS writes among the MFMAs hides their latency (measured)
            if constexpr (sizeof(A) == 16) __builtin_amdgcn_sched_barrier(0);
            publish(cur ^ 1, pre);
            __syncthreads();
        };
        R bnext[U][NSRC];
        for (int st = 0; st < nstage; st += 2) {
            stage(0, bcur, bnext);
            if (st + 1 == nstage) break;
            stage(1, bnext, bcur);
        }
    } else {
        // Two stages deep: stage s + 2's loads are issued while stage s runs
        // and stage s + 1's are in flight, so a gather's latency may span two
        // stages.  Three multipole fragment sets rotate (b0, b1, b2) and two
        // operator register sets (p0, p1); six stages per loop iteration keep
        // every set's role a compile-time constant.
        A p0[U][PC], p1[U][PC];
        R b1[U][NSRC], b2[U][NSRC];
        issue(p1, b1);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        auto stage = [&](const int cur, R (&buse)[U][NSRC], R (&bissue)[U][NSRC], A (&pissue)[U][PC],
                         A (&pwrite)[U][PC]) __attribute__((always_inline)) {
            issue(pissue, bissue);
            __builtin_amdgcn_sched_barrier(0);
            compute(cur, buse);
            __builtin_amdgcn_sched_barrier(0);
            publish(cur ^ 1, pwrite);
            __syncthreads();
        };
        for (int st = 0; st < nstage; st += 6) {
            stage(0, bcur, b2, p0, p1);
            if (st + 1 == nstage) break;
            stage(1, b1, bcur, p1, p0);
            if (st + 2 == nstage) break;
            stage(0, b2, b1, p0, p1);
            if (st + 3 == nstage) break;
            stage(1, bcur, b2, p1, p0);
            if (st + 4 == nstage) break;
            stage(0, b1, bcur, p0, p1);
            if (st + 5 == nstage) break;
            stage(1, b2, b1, p1, p0);
        }
    }

    if (!valid) return;
    // FP32 operands with FP64 accumulators: split-K partials stay in FP64 (a
    // slice's sum rounded to FP32 before the slices cancel each other was
    // the largest FP32 error of the upper levels)
    constexpr bool OUT64 = SPLIT && F64;
    const size_t slice_off = (size_t)slice * ((size_t)8 << (3 * nh_bits)) * Kp;
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int prow = 16 * (rb0 + rb) + Mfma<S>::row(lane, r);
            const int row = SYM != 0 ? rowmap[prow] : prow;
            if (row < 0) continue;
            // split operands: undo the row's power-of-two scale (exact)
            const double rs = is_split16<P>() ? (double)rscale[row] : 1.0;
            if constexpr (OUT64)
                L64[slice_off + (size_t)tcell * Kp + row] = rs * (hi[rb][r] + (double)acc[rb][r]);
            else
                L[slice_off + (size_t)tcell * Kp + row] =
                    F64 ? (S)(rs * (hi[rb][r] + (double)acc[rb][r])) : (S)acc[rb][r];
        }
}

// Launches the LDS-shared kernel for every row group (NRB, U, NE and the
// variant fixed at compile time; combinations outside the instantiated set --
// all orders 0..20 of both schemes are covered -- give hipErrorInvalidValue).
template <typename P>
static hipError_t launch_lds(const void *ops, const int32_t *il, const int32_t *offs, const int32_t *rowmap,
                             const typename P::S *M, const typename P::S *Mflip, const typename P::S *zeros,
                             int64_t fstride, typename P::S *out, double *out64, int nh_bits, int NB, int NKC, int Kp,
                             int nslices, const RowGroup *groups, int ng, hipStream_t s,
                             const float *rscale = nullptr) {
    using A = typename P::A;
    const int64_t ntile = (((int64_t)1 << (3 * nh_bits)) + 63) / 64;
    const int64_t grid = 8 * ntile * nslices;
    const A *o = reinterpret_cast<const A *>(ops);
    for (int gi = 0; gi < ng; ++gi) {
        const int rb0 = groups[gi].rb0, nrb = groups[gi].nrb, ne = groups[gi].ne, sym = groups[gi].sym;
        if ((sym == 0) != !P::kPaired) return hipErrorInvalidValue;
        bool launched = false;
#define FMM_M2L_LDS_LAUNCH(SYM, N, NE)                                                                          \
    if (nslices > 1)                                                                                            \
        hipLaunchKernelGGL((k_m2l_lds<P, true, N, stage_chunks<P, N, SYM>(), NE, SYM>), dim3((unsigned)grid),       \
                           dim3(256), 0, s, o, il, offs, rowmap, M, Mflip, zeros, fstride, out, out64, rscale,    \
                           nh_bits, NB, NKC, Kp, rb0, nslices);                                                 \
    else                                                                                                        \
        hipLaunchKernelGGL((k_m2l_lds<P, false, N, stage_chunks<P, N, SYM>(), NE, SYM>), dim3((unsigned)grid),      \
                           dim3(256), 0, s, o, il, offs, rowmap, M, Mflip, zeros, fstride, out, out64, rscale,    \
                           nh_bits, NB, NKC, Kp, rb0, 1);
#define FMM_M2L_LDS_CASE(SYM, N, NE)                                                                            \
    if (!launched && sym == SYM && nrb == N && ne == NE && P::template allow<SYM, N, NE>()) {                \
        if constexpr (P::template allow<SYM, N, NE>()) {                                                        \
            FMM_M2L_LDS_LAUNCH(SYM, N, NE)                                                                      \
        }                                                                                                       \
        launched = true;                                                                                        \
    }
        FMM_M2L_LDS_CASE(0, 1, 0)
        FMM_M2L_LDS_CASE(0, 2, 0)
        FMM_M2L_LDS_CASE(0, 3, 0)
        FMM_M2L_LDS_CASE(0, 4, 0)
        FMM_M2L_LDS_CASE(0, 5, 0)
        FMM_M2L_LDS_CASE(0, 6, 0)
        FMM_M2L_LDS_CASE(0, 7, 0)
        FMM_M2L_LDS_CASE(0, 8, 0)
        FMM_M2L_LDS_CASE(0, 9, 0)
        FMM_M2L_LDS_CASE(0, 10, 0)
        FMM_M2L_LDS_CASE(0, 11, 0)
        FMM_M2L_LDS_CASE(1, 1, 1)
        FMM_M2L_LDS_CASE(1, 2, 1)
        FMM_M2L_LDS_CASE(1, 3, 1)
        FMM_M2L_LDS_CASE(1, 4, 2)
        FMM_M2L_LDS_CASE(1, 5, 2)
        FMM_M2L_LDS_CASE(1, 6, 3)
        FMM_M2L_LDS_CASE(1, 7, 3)
        FMM_M2L_LDS_CASE(1, 9, 5)
        FMM_M2L_LDS_CASE(1, 10, 5)
        FMM_M2L_LDS_CASE(1, 11, 6)
        FMM_M2L_LDS_CASE(4, 4, 1)
        FMM_M2L_LDS_CASE(4, 8, 2)
        FMM_M2L_LDS_CASE(4, 12, 3)
        FMM_M2L_LDS_CASE(2, 2, 1)
        FMM_M2L_LDS_CASE(2, 4, 2)
        FMM_M2L_LDS_CASE(2, 6, 3)
        FMM_M2L_LDS_CASE(2, 8, 4)
        FMM_M2L_LDS_CASE(2, 10, 5)
        FMM_M2L_LDS_CASE(2, 1, 1)
        FMM_M2L_LDS_CASE(2, 1, 0)
        FMM_M2L_LDS_CASE(2, 6, 6)
        FMM_M2L_LDS_CASE(2, 6, 0)
        FMM_M2L_LDS_CASE(2, 7, 7)
        FMM_M2L_LDS_CASE(2, 7, 0)
        FMM_M2L_LDS_CASE(3, 2, 1)
        FMM_M2L_LDS_CASE(3, 4, 2)
        FMM_M2L_LDS_CASE(3, 6, 3)
        FMM_M2L_LDS_CASE(3, 8, 4)
        FMM_M2L_LDS_CASE(3, 10, 5)
        FMM_M2L_LDS_CASE(3, 1, 1)
        FMM_M2L_LDS_CASE(3, 1, 0)
        FMM_M2L_LDS_CASE(3, 6, 6)
        FMM_M2L_LDS_CASE(3, 6, 0)
        FMM_M2L_LDS_CASE(3, 7, 7)
        FMM_M2L_LDS_CASE(3, 7, 0)
#undef FMM_M2L_LDS_CASE
#undef FMM_M2L_LDS_LAUNCH
        if (!launched) return hipErrorInvalidValue;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Sum of the split-K partial results in slice order (deterministic), in the
// partials' type, rounded once to the level's type.
template <typename P, typename T>
__global__ void k_m2l_reduce(const P *__restrict__ partial, T *__restrict__ L, int nslices, int64_t elems) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < elems;
         i += (int64_t)gridDim.x * blockDim.x) {
        P acc = 0;
#pragma unroll 8
        for (int k = 0; k < nslices; ++k) acc += partial[(size_t)k * elems + i];
        L[i] = (T)acc;
    }
}

// The level's multipoles scaled by cscale and split for the plain split-FP16
// kernel: x = M[c][k] cscale[k] as hi = fp16(x), lo = fp16(x - hi), one
// thread per group of 8 coefficients, written as 8 hi then 8 lo values in the
// group's 32 bytes (the layout k_m2l_f16rows loads).
__global__ void k_col_split(const float *__restrict__ M, float *__restrict__ Mc, const float *__restrict__ cscale,
                            int64_t ngroup, int Kp) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < ngroup;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i0 = 8 * g;
        const int k0 = (int)(i0 % Kp);
        F16Pair v;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float x = M[i0 + i] * cscale[k0 + i];
            const _Float16 h = (_Float16)x;
            v.hi[i] = h;
            v.lo[i] = (_Float16)(x - (float)h);
        }
        *reinterpret_cast<F16Pair *>(Mc + i0) = v;
    }
}

// ---------------------------------------------------------------------------
// Split-FP16 M2L on the plain list with the rows split over the wavefronts.
// With the split operands (32-byte fragments, three MFMAs per fragment pair)
// the LDS-shared kernel above makes every wavefront read the whole operator
// chunk from LDS for its own 16 targets: 22 of its 28 LDS instructions per
// stage.  Here a workgroup still owns 64 target cells of one parity class, but
// wavefront w owns RW row blocks, rows 16 (rb0 + RW w) .., for all 64 targets
// (four column blocks of 16):
//   * its operator fragments come from global memory (L2) straight into
//     registers, one stage ahead: no other wavefront reads them;
//   * the multipole fragments of the 64 targets are the operand shared
//     through LDS: wavefront w gathers the chunk's fragment of its 16 targets
//     (one 32-byte load per lane of the pairs written by k_col_split) into a
//     double-buffered LDS stage and every wavefront reads all four, one
//     barrier per stage;
//   * each operator fragment feeds 4 column blocks x 3 MFMAs.
// Accumulation as in k_m2l_lds: FP32 on the matrix cores over one offset's
// chunks, then into FP64.  Row blocks past the group (the last wavefront when
// the group is not a multiple of 4) run on a clamped fragment and are not
// stored, so every MFMA is unconditional.  SPLIT: split-K over offset slices
// into FP64 partials, as in k_m2l_lds.  What paces it (3M-atom box, p = 16):
// the operator fragments missing L2 (the 64 workgroups of an XCD walk the same
// chunks but drift apart), about 6.5 TB/s of reads, with the matrix cores busy
// 44% of the time.
// ---------------------------------------------------------------------------
template <bool SPLIT, int RW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_m2l_f16rows(
    const F16Pair *__restrict__ ops, const int32_t *__restrict__ il, const int32_t *__restrict__ offs,
    const float *__restrict__ Mc, float *__restrict__ L, double *__restrict__ L64, const float *__restrict__ rscale,
    int nh_bits, int NB, int NKC, int Kp, int rb0, int nrb, int nslices_arg) {
    __shared__ uint4 lds[2][2][256];  // [stage buffer][hi, lo plane][column block x 64 + lane]
    const int nslices = SPLIT ? nslices_arg : 1;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int parity = blockIdx.x & 7;
    const int rest = blockIdx.x >> 3;
    const int slice = rest % nslices;
    const int tile = rest / nslices;
    const uint32_t ntarget = 1u << (3 * nh_bits);

    // the target whose multipole fragments this lane gathers (column block wid)
    const uint32_t Pg = (uint32_t)tile * 64 + (uint32_t)wid * 16 + (lane & 15);
    uint32_t tx, ty, tz;
    demorton3(Pg < ntarget ? Pg : 0u, tx, ty, tz);
    tx = 2 * tx + ((parity >> 2) & 1);
    ty = 2 * ty + ((parity >> 1) & 1);
    tz = 2 * tz + (parity & 1);
    const int kq = 8 * (lane >> 4);
    // source cell by dilated-integer addition (as in k_m2l_lds)
    const uint32_t lvl = (8u << (3 * nh_bits)) - 1u;
    const uint32_t zm = 0x09249249u & lvl, ym = (0x09249249u << 1) & lvl, xm = (0x09249249u << 2) & lvl;
    const uint32_t tdx = (spread3(tx) << 2) | ~xm, tdy = (spread3(ty) << 1) | ~ym, tdz = spread3(tz) | ~zm;
    auto source = [&](int oid) {
        const uint32_t cx = (tdx + (spread3((uint32_t)offs[3 * oid]) << 2)) & xm;
        const uint32_t cy = (tdy + (spread3((uint32_t)offs[3 * oid + 1]) << 1)) & ym;
        const uint32_t cz = (tdz + spread3((uint32_t)offs[3 * oid + 2])) & zm;
        return Mc + (size_t)(cx | cy | cz) * Kp + kq;
    };

    // this wavefront's row blocks (fragment row block, clamped into the group)
    const int wr0 = RW * wid;
    int rbf[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) rbf[r] = rb0 + min(wr0 + r, nrb - 1);

    const int t0 = slice * kILSize / nslices, t1 = (slice + 1) * kILSize / nslices;
    const int nstage = (t1 - t0) * NKC;
    const int32_t *ilp = il + parity * kILSize;
    // prefetch cursor (offset t, column chunk kc); past the end of the list it
    // stays on the last offset and the multipole fragment is zero
    int pt = t0, pkc = 0;
    const float *psrc = Mc;
    size_t pbase = 0;
    auto set_t = [&](int t) {
        pt = t;
        pkc = 0;
        const int oid = ilp[min(t, t1 - 1)];
        psrc = source(oid);
        pbase = (size_t)oid * NKC * NB * 64 + lane;
    };
    auto advance = [&]() {
        if (++pkc == NKC) set_t(pt + 1);
        else pbase += (size_t)NB * 64;
    };
    auto load_a = [&](F16Pair (&a)[RW]) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < RW; ++r) a[r] = ops[pbase + (size_t)rbf[r] * 64];
    };
    auto load_b = [&]() __attribute__((always_inline)) -> F16Pair {
        F16Pair b;
        if (pt < t1 && 32 * pkc + kq < Kp) {
            b = *reinterpret_cast<const F16Pair *>(psrc + 32 * pkc);
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) b.hi[i] = b.lo[i] = (_Float16)0.0f;
        }
        return b;
    };
    auto put_b = [&](int buf, const F16Pair &b) __attribute__((always_inline)) {
        uint4 w[2];
        __builtin_memcpy(w, &b, sizeof(b));
        lds[buf][0][tid] = w[0];
        lds[buf][1][tid] = w[1];
    };

    f32x4 acc[RW][4];
    double hi[RW][4][4];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            acc[r][c] = f32x4{0, 0, 0, 0};
#pragma unroll
            for (int e = 0; e < 4; ++e) hi[r][c][e] = 0.0;
        }

    F16Pair a0[RW], a1[RW];
    set_t(t0);
    load_a(a0);
    {
        const F16Pair b = load_b();
        advance();
        put_b(0, b);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    int kc = 0;
    // one stage: prefetch the next chunk (operators to registers, this lane's
    // multipole fragment to bn), run this chunk from LDS buffer cur and acur,
    // publish bn in the other buffer
    auto stage = [&](const int cur, F16Pair (&acur)[RW], F16Pair (&anext)[RW]) __attribute__((always_inline)) {
        load_a(anext);
        const F16Pair bn = load_b();
        advance();
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            uint4 w[2] = {lds[cur][0][c * 64 + lane], lds[cur][1][c * 64 + lane]};
            F16Pair b;
            __builtin_memcpy(&b, w, sizeof(b));
#pragma unroll
            for (int r = 0; r < RW; ++r) acc[r][c] = mma_split16(acur[r], b, acc[r][c]);
        }
        if (++kc == NKC) {
            kc = 0;
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) hi[r][c][e] += (double)acc[r][c][e];
                    acc[r][c] = f32x4{0, 0, 0, 0};
                }
        }
        __builtin_amdgcn_sched_barrier(0);
        put_b(cur ^ 1, bn);
        __syncthreads();
    };
    for (int st = 0; st < nstage; st += 2) {
        stage(0, a0, a1);
        if (st + 1 == nstage) break;
        stage(1, a1, a0);
    }

    const size_t slice_off = (size_t)slice * ((size_t)8 << (3 * nh_bits)) * Kp;
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        if (wr0 + r >= nrb) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint32_t P = (uint32_t)tile * 64 + (uint32_t)c * 16 + (lane & 15);
            if (P >= ntarget) continue;
            const size_t tcell = 8 * (size_t)P + (size_t)parity;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = 16 * (rb0 + wr0 + r) + 4 * (lane >> 4) + e;
                const double v = (double)rscale[row] * (hi[r][c][e] + (double)acc[r][c][e]);
                if constexpr (SPLIT)
                    L64[slice_off + tcell * Kp + row] = v;
                else
                    L[tcell * Kp + row] = (float)v;
            }
        }
    }
}

// Launches k_m2l_f16rows for every row group (at most 12 blocks each: RW <= 3)
static hipError_t launch_f16rows(const void *ops, const int32_t *il, const int32_t *offs, const float *Mc, float *L,
                                 double *part, const float *rscale, int nh_bits, int NB, int NKC, int Kp, int nslices,
                                 const RowGroup *grp, int ng, hipStream_t s) {
    const int64_t ntile = (((int64_t)1 << (3 * nh_bits)) + 63) / 64;
    const int64_t grid = 8 * ntile * nslices;
    const F16Pair *o = reinterpret_cast<const F16Pair *>(ops);
    for (int gi = 0; gi < ng; ++gi) {
        const int rb0 = grp[gi].rb0, nrb = grp[gi].nrb;
        const int RW = (nrb + 3) / 4;
#define FMM_F16ROWS(R)                                                                                          \
    if (RW == R) {                                                                                              \
        if (nslices > 1)                                                                                        \
            hipLaunchKernelGGL((k_m2l_f16rows<true, R>), dim3((unsigned)grid), dim3(256), 0, s, o, il, offs, Mc,  \
                               L, part, rscale, nh_bits, NB, NKC, Kp, rb0, nrb, nslices);                        \
        else                                                                                                    \
            hipLaunchKernelGGL((k_m2l_f16rows<false, R>), dim3((unsigned)grid), dim3(256), 0, s, o, il, offs, Mc, \
                               L, part, rscale, nh_bits, NB, NKC, Kp, rb0, nrb, 1);                             \
    }
        if (RW < 1 || RW > 3) return hipErrorInvalidValue;
        FMM_F16ROWS(1)
        FMM_F16ROWS(2)
        FMM_F16ROWS(3)
#undef FMM_F16ROWS
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

static_assert(kSplit16RowBlocks == 12, "row groups of k_m2l_f16rows: at most 3 blocks per wavefront");

// Scaled and sign-flipped copies of the level's multipoles for the folded
// split kernel: Mc[0] = cscale M, Mc[1 + f] = D_f (cscale M) for the group
// elements of the scheme's list entries (the signs of k_m2l_flip)
__device__ inline int flip_sign(int scheme, int f, int k);
__global__ void k_m2l_flip_scaled(const float *__restrict__ M, float *__restrict__ Mc, const float *__restrict__ cscale,
                                  int64_t ncell, int Kp, int scheme, int ncopy) {
    const int k = threadIdx.x;
    if (k >= Kp) return;
    bool neg[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) neg[f] = f < ncopy && flip_sign(scheme, f, k) < 0;
    const float cs = cscale[k];
    const int64_t n = ncell * Kp;
    for (int64_t c = blockIdx.x; c < ncell; c += gridDim.x) {
        const int64_t i = c * Kp + k;
        const float v = M[i] * cs;
        Mc[i] = v;
#pragma unroll
        for (int f = 0; f < 3; ++f)
            if (f < ncopy) Mc[(size_t)(f + 1) * n + i] = neg[f] ? -v : v;
    }
}

hipError_t launch_m2l_split16(int level, const void *ops, const int32_t *list, const int32_t *offs,
                              const int32_t *rowmap, const float *M, float *Mc, size_t mc_cap, const float *cscale,
                              const float *rscale, const float *zeros, float *L, double *partial, size_t part_cap,
                              int p, int Kp, hipStream_t s) {
    const int nh_bits = level - 1;
    const int64_t ncell = (int64_t)8 << (3 * nh_bits);
    const int64_t n = ncell * Kp;
    const int nslices = partial ? m2l_slices(level) : 1;
    RowGroup grp[kMaxRowGroups];
    int ng = m2l_split16_fold_groups(p, grp);
    const bool fold = ng > 0;
    const int copies = fold ? 1 + m2l_flip_copies(p) : 1;
    if (mc_cap < (size_t)copies * n * sizeof(float)) return hipErrorInvalidValue;
    if (nslices > 1 && part_cap < m2l_partial_bytes(level, p, kILSize, sizeof(float))) return hipErrorInvalidValue;
    if (Kp > 1024) return hipErrorInvalidValue;
    hipError_t e;
    if (fold) {
        if (!rowmap || !zeros) return hipErrorInvalidValue;
        const int fb = (Kp + 63) / 64 * 64;
        const int64_t g = ncell < 16384 ? ncell : 16384;
        hipLaunchKernelGGL(k_m2l_flip_scaled, dim3((unsigned)g), dim3(fb), 0, s, M, Mc, cscale, ncell, Kp,
                           m2l_scheme(p), m2l_flip_copies(p));
        e = launch_lds<PolF16x3F>(ops, list, offs, rowmap, Mc, Mc + n, zeros, n, L, nslices > 1 ? partial : nullptr,
                                  nh_bits, m2l_row_blocks(p), m2l_k32_chunks(p), Kp, nslices, grp, ng, s, rscale);
    } else {
        int64_t g = (n / 8 + 255) / 256;
        if (g > 65535) g = 65535;
        hipLaunchKernelGGL(k_col_split, dim3((unsigned)g), dim3(256), 0, s, M, Mc, cscale, n / 8, Kp);
        const int NB = Kp / 16;
        ng = m2l_split16_plain_groups(NB, grp);
        e = launch_f16rows(ops, list, offs, Mc, L, nslices > 1 ? partial : nullptr, rscale, nh_bits, NB,
                           m2l_k32_chunks(p), Kp, nslices, grp, ng, s);
    }
    if (e != hipSuccess || nslices == 1) return e;
    int64_t g = (n + 255) / 256;
    if (g > 65535) g = 65535;
    hipLaunchKernelGGL((k_m2l_reduce<double, float>), dim3((unsigned)g), dim3(256), 0, s, partial, L, nslices, n);
    return hipGetLastError();
}

hipError_t launch_m2l_bf16(int level, const void *ops, const int32_t *il, const int32_t *offs, const float *M,
                           float *L, float *partial, size_t part_cap, int p, int Kp, hipStream_t s) {
    const int NB = Kp / 16;
    const int nh_bits = level - 1;
    const int nslices = partial ? m2l_slices(level) : 1;
    // the caller's split-K buffer must hold every slice (checked on the host)
    if (nslices > 1 && part_cap < (size_t)nslices * ((size_t)8 << (3 * nh_bits)) * (size_t)Kp * sizeof(float))
        return hipErrorInvalidValue;
    RowGroup grp[kMaxRowGroups];
    const int ng = m2l_row_groups(0, p, NB, false, grp);
    hipError_t e = launch_lds<PolBf16>(ops, il, offs, nullptr, M, M, M, 0, nslices > 1 ? partial : L, nullptr, nh_bits, NB,
                                       m2l_k32_chunks(p), Kp, nslices, grp, ng, s);
    if (e != hipSuccess || nslices == 1) return e;
    const int64_t elems = ((int64_t)8 << (3 * nh_bits)) * Kp;
    int64_t g = (elems + 255) / 256;
    if (g > 65535) g = 65535;
    hipLaunchKernelGGL((k_m2l_reduce<float, float>), dim3((unsigned)g), dim3(256), 0, s, partial, L, nslices, elems);
    return hipGetLastError();
}

// Sign-flipped copies of the level's multipoles, Mflip[f][c][k] =
// sigma(k) M[c][k] for the group elements of the scheme's list entries:
// scheme 1 one copy, (-1)^n (t -> -t); scheme 2 three copies, for the flips
// (-,-,+): (-1)^m, (-,+,-): (-1)^n (-1 for an imaginary part),
// (+,-,-): (-1)^(n+m) (-1 for an imaginary part).
__device__ inline int flip_sign(int scheme, int f, int k) {
    int n = (int)sqrtf((float)k);
    if (n * n > k) --n;
    if ((n + 1) * (n + 1) <= k) ++n;
    const int r = k - n * n, m = (r + 1) >> 1;
    const int im = (r > 0 && (r & 1) == 0) ? 1 : 0;
    if (scheme == 1) return (n & 1) ? -1 : 1;
    const int odd = f == 0 ? (m & 1) : (f == 1 ? ((n & 1) ^ im) : (((n + m) & 1) ^ im));
    return odd ? -1 : 1;
}

// A thread owns coefficient k of every cell its block visits (the block
// spans one padded row, blockDim >= Kp), so its signs are computed once.
template <typename T>
__global__ void k_m2l_flip(const T *__restrict__ M, T *__restrict__ Mflip, int64_t ncell, int Kp, int scheme,
                           int ncopy) {
    const int k = threadIdx.x;
    if (k >= Kp) return;
    bool neg[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) neg[f] = f < ncopy && flip_sign(scheme, f, k) < 0;
    const int64_t n = ncell * Kp;
    for (int64_t c = blockIdx.x; c < ncell; c += gridDim.x) {
        const int64_t i = c * Kp + k;
        const T v = M[i];
#pragma unroll
        for (int f = 0; f < 3; ++f)
            if (f < ncopy) Mflip[(size_t)f * n + i] = neg[f] ? -v : v;
    }
}

// The full interaction list (nil == 875) runs on the LDS-shared kernel with
// the symmetry-folded entries of m2l_scheme(p); the aliased lists of levels 1
// and 2 (nil = 8 or 64 pre-summed operators) on the offset-split kernel.
template <typename T>
hipError_t launch_m2l(int level, const T *ops, const int32_t *list, const int32_t *offs, const int32_t *rowmap,
                      const T *M, T *Mflip, size_t flip_cap, const T *zeros, T *L, T *partial, size_t part_cap, int p,
                      int Kp, hipStream_t s, int nil) {
    constexpr int CB = Mfma<T>::CB;
    const int NB = Kp / 16;
    const int nh_bits = level - 1;
    const int64_t ntarget = (int64_t)1 << (3 * nh_bits);
    const int nslices = partial ? std::min(m2l_slices(level), nil) : 1;
    // scratch capacities, checked on the host before anything is launched:
    // the split-K partials and the sign-flipped multipole copies of the level
    if (nslices > 1 && part_cap < m2l_partial_bytes(level, p, nil, sizeof(T))) return hipErrorInvalidValue;
    if (nil == kILSize && flip_cap < m2l_flip_bytes(level, p, sizeof(T))) return hipErrorInvalidValue;
    double *part64 = nullptr;
    if (nil == kILSize) {
        if (!rowmap || !Mflip || !zeros) return hipErrorInvalidValue;
        const int scheme = m2l_scheme(p);
        if (scheme == 1 && m2l_row_blocks(p) > kRowBlocksPerWave) return hipErrorInvalidValue;
        const int64_t ncell = (int64_t)8 << (3 * nh_bits);
        const int64_t n = ncell * Kp;
        if (Kp > 1024) return hipErrorInvalidValue;
        const int fb = (Kp + 63) / 64 * 64;
        const int64_t g = ncell < 16384 ? ncell : 16384;
        hipLaunchKernelGGL(k_m2l_flip<T>, dim3((unsigned)g), dim3(fb), 0, s, M, Mflip, ncell, Kp, scheme,
                           m2l_flip_copies(p));
        RowGroup grp[kMaxRowGroups];
        const int ng = m2l_row_groups(scheme, p, m2l_row_blocks(p), sizeof(T) == 8, grp);
        // FP32 operands: FP64 split-K partials (the buffer holds doubles)
        part64 = (sizeof(T) == 4 && nslices > 1) ? reinterpret_cast<double *>(partial) : nullptr;
        const hipError_t e = launch_lds<PolMfma<T>>(ops, list, offs, rowmap, M, Mflip, zeros, n,
                                                     nslices > 1 ? partial : L, part64, nh_bits, m2l_row_blocks(p), NB,
                                                     Kp, nslices, grp, ng, s);
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
    if (part64)
        hipLaunchKernelGGL((k_m2l_reduce<double, T>), dim3((unsigned)g), dim3(256), 0, s, part64, L, nslices, elems);
    else
        hipLaunchKernelGGL((k_m2l_reduce<T, T>), dim3((unsigned)g), dim3(256), 0, s, partial, L, nslices, elems);
    return hipGetLastError();
}
template hipError_t launch_m2l<float>(int, const float *, const int32_t *, const int32_t *, const int32_t *,
                                      const float *, float *, size_t, const float *, float *, float *, size_t, int, int,
                                      hipStream_t, int);
template hipError_t launch_m2l<double>(int, const double *, const int32_t *, const int32_t *, const int32_t *,
                                       const double *, double *, size_t, const double *, double *, double *, size_t,
                                       int, int, hipStream_t, int);

}  // namespace fmm
