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
#include <cstring>

#include "fmm_internal.h"
#include "mfma.h"
#include "morton.h"

namespace fmm {

constexpr int kRowBlocksPerWave = 11;  // 176 rows: K <= 169 (p <= 12) in one row group

template <typename T>
size_t m2l_ops_elems(int p) {
    const size_t Kp = (size_t)padded_coeffs(p);
    return (size_t)kNumOffsets * Kp * Kp;
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

template <typename T>
void swizzle_m2l_ops(int p, const double *ops, T *out) {
    swizzle_ops<T>(p, kNumOffsets, ops, out);
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
template <typename T> struct LdsTile;
template <> struct LdsTile<float> {
    static constexpr int U = 1;  // chunks per LDS stage
    static constexpr bool kFlush64 = true;
};
template <> struct LdsTile<double> {
    static constexpr int U = 1;
    static constexpr bool kFlush64 = false;
};

// SPLIT: compiled separately for split-K launches (offset slices written to a
// partial buffer) and whole launches, so profiles tell the finest level apart.
// NRB: row blocks of this launch (rows 16 rb0 .. 16 (rb0 + NRB) - 1), a
// compile-time constant so that the chunk loop is straight-line code (a
// run-time row count turned every MFMA into a branch and forced full
// memory waits inside the compute section).
template <typename T, bool SPLIT, int NRB>
__global__ __launch_bounds__(256) void k_m2l_lds(const T *__restrict__ ops, const int32_t *__restrict__ il,
                                                 const int32_t *__restrict__ offs, const T *__restrict__ M,
                                                 T *__restrict__ L, int nh_bits, int NB, int Kp, int rb0,
                                                 int nslices_arg) {
    const int nslices = SPLIT ? nslices_arg : 1;
    constexpr int CHUNK = NRB * 64;             // vec4 entries per operator chunk
    constexpr int PER_T = (CHUNK + 255) / 256;  // vec4 loads per thread per chunk
    constexpr bool F64 = LdsTile<T>::kFlush64;
    using V = typename Mfma<T>::V;
    __shared__ V lds[2][CHUNK];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const int parity = blockIdx.x & 7;
    const int rest = blockIdx.x >> 3;
    const int slice = rest % nslices;
    const int tile = rest / nslices;
    const uint32_t ntarget = 1u << (3 * nh_bits);
    const uint32_t nmask = (2u << nh_bits) - 1u;

    const uint32_t P = (uint32_t)tile * 64 + (uint32_t)wid * 16 + (lane & 15);
    const bool valid = P < ntarget;
    uint32_t tx, ty, tz;
    demorton3(valid ? P : 0u, tx, ty, tz);
    tx = 2 * tx + ((parity >> 2) & 1);
    ty = 2 * ty + ((parity >> 1) & 1);
    tz = 2 * tz + (parity & 1);
    const uint32_t tcell = 8 * P + (uint32_t)parity;

    const int t0 = slice * kILSize / nslices, t1 = (slice + 1) * kILSize / nslices;
    const int nstage = (t1 - t0) * NB;  // one (offset, 16-coefficient chunk) per stage
    const size_t op_stride = (size_t)NB * NB * 64;  // vec4 entries per offset
    const V *opsv = reinterpret_cast<const V *>(ops);
    const int32_t *ilp = il + parity * kILSize;
    // entries of a chunk this thread stages: tid + 256 v; only the last v can
    // fall past the chunk, and that load is clamped into it (stored only when
    // inside)
    const int e_last = min(tid + 256 * (PER_T - 1), CHUNK - 1);
    const bool last_in = tid + 256 * (PER_T - 1) < CHUNK;

    // chunk cursor (t, kc) advanced one chunk at a time; the operator id and
    // the multipole row of this lane's source cell change only with t
    struct Cursor {
        int t, kc;
        size_t base;     // first vec4 entry of the chunk
        const T *src;    // this lane's 4 coefficients of the source multipole
    };
    auto set_t = [&](Cursor &c, int t) {
        c.t = t;
        c.kc = 0;
        const int oid = ilp[min(t, t1 - 1)];  // past the end: stay on a valid chunk
        const uint32_t sx = (tx + (uint32_t)offs[3 * oid]) & nmask;
        const uint32_t sy = (ty + (uint32_t)offs[3 * oid + 1]) & nmask;
        const uint32_t sz = (tz + (uint32_t)offs[3 * oid + 2]) & nmask;
        c.src = M + (size_t)morton3(sx, sy, sz) * Kp + 4 * (lane >> 4);
        c.base = (size_t)oid * op_stride + (size_t)rb0 * 64;
    };
    auto advance = [&](Cursor &c) {
        if (++c.kc == NB) set_t(c, c.t + 1);
        else c.base += (size_t)NB * 64;
    };

    V acc[NRB];
    double hi[F64 ? NRB : 1][4];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) acc[rb] = V{0, 0, 0, 0};
    if constexpr (F64)
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) hi[rb][r] = 0.0;

    Cursor pc;  // prefetch cursor; the compute side only needs kc
    set_t(pc, t0);
    int kc = 0;

    // prologue: stage 0 into LDS buffer 0
    V bcur;
    {
#pragma unroll
        for (int v = 0; v < PER_T - 1; ++v) lds[0][tid + 256 * v] = opsv[pc.base + tid + 256 * v];
        const V x = opsv[pc.base + e_last];
        if (last_in) lds[0][e_last] = x;
        bcur = *reinterpret_cast<const V *>(pc.src + 16 * pc.kc);
        advance(pc);
    }
    // Drain every prologue load: the compiler's wait bookkeeping would
    // otherwise carry the pending bcur load into the loop and put a full
    // memory wait in front of each stage's first MFMA.
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    for (int st = 0; st < nstage; ++st) {
        const int cur = st & 1;
        // prefetch the next chunk (on the last stage: a harmless re-read of a
        // valid chunk) into registers
        V pre[PER_T];
#pragma unroll
        for (int v = 0; v < PER_T - 1; ++v) pre[v] = opsv[pc.base + tid + 256 * v];
        pre[PER_T - 1] = opsv[pc.base + e_last];
        const V bnext = *reinterpret_cast<const V *>(pc.src + 16 * pc.kc);
        advance(pc);
        // this stage on the matrix cores
        V a[NRB];
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb) a[rb] = lds[cur][rb * 64 + lane];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int rb = 0; rb < NRB; ++rb) acc[rb] = Mfma<T>::mma(a[rb][j], bcur[j], acc[rb]);
        if (++kc == NB) {
            kc = 0;
            if constexpr (F64) {
#pragma unroll
                for (int rb = 0; rb < NRB; ++rb) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) hi[rb][r] += (double)acc[rb][r];
                    acc[rb] = V{0, 0, 0, 0};
                }
            }
        }
        // publish the prefetched chunk for the next stage
#pragma unroll
        for (int v = 0; v < PER_T - 1; ++v) lds[cur ^ 1][tid + 256 * v] = pre[v];
        if (last_in) lds[cur ^ 1][e_last] = pre[PER_T - 1];
        bcur = bnext;
        __syncthreads();
    }

    if (!valid) return;
    T *out = L + (size_t)slice * ((size_t)8 << (3 * nh_bits)) * Kp;
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * (rb0 + rb) + Mfma<T>::row(lane, r);
            out[(size_t)tcell * Kp + row] = F64 ? (T)(hi[rb][r] + (double)acc[rb][r]) : acc[rb][r];
        }
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
    switch (level) {
        case 1: return 64;
        case 2: return 64;
        case 3: return 64;
        case 4: return 32;
        default: return 1;
    }
}

// Levels from this one on use the LDS-shared kernel (measured on the 1M-atom
// box: level 3 in FP64 with 64 slices 0.4 ms faster than the offset-split
// kernel); the two coarsest levels (aliased lists of 8 and 64 entries) use the
// offset-split kernel.  m2l_variant 1 forces the offset-split kernel everywhere
// (tuning and cross-checks).
constexpr int kLdsLevel = 3;
static int g_m2l_variant = 0;
void set_m2l_variant(int v) { g_m2l_variant = v; }
template <typename T> static bool use_lds_kernel(int level) {
    if (level < kLdsLevel) return false;
    return g_m2l_variant != 1;
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
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

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

constexpr int kBf16Stage = 3;  // K chunks per LDS stage

template <bool SPLIT>
__global__ __launch_bounds__(256) void k_m2l_bf16(const bf16x8 *__restrict__ ops, const int32_t *__restrict__ il,
                                                  const int32_t *__restrict__ offs, const float *__restrict__ M,
                                                  float *__restrict__ L, int nh_bits, int NB, int NKC, int Kp,
                                                  int nrg, int nslices_arg) {
    const int nslices = SPLIT ? nslices_arg : 1;
    constexpr int NRW = kRowBlocksPerWave;
    constexpr int CHUNK = NRW * 64;  // 16-byte entries per chunk slot
    constexpr int U = kBf16Stage;
    constexpr int PER_T = (U * CHUNK + 255) / 256;
    __shared__ bf16x8 lds[2][U * CHUNK];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const int parity = blockIdx.x & 7;
    int rest = blockIdx.x >> 3;
    const int rg = rest % nrg;
    rest /= nrg;
    const int slice = rest % nslices;
    const int tile = rest / nslices;
    const int rb0 = rg * NRW;
    const int nrb = min(NRW, NB - rb0);
    const uint32_t ntarget = 1u << (3 * nh_bits);
    const uint32_t nmask = (2u << nh_bits) - 1u;

    const uint32_t P = (uint32_t)tile * 64 + (uint32_t)wid * 16 + (lane & 15);
    const bool valid = P < ntarget;
    uint32_t tx, ty, tz;
    demorton3(valid ? P : 0u, tx, ty, tz);
    tx = 2 * tx + ((parity >> 2) & 1);
    ty = 2 * ty + ((parity >> 1) & 1);
    tz = 2 * tz + (parity & 1);
    const uint32_t tcell = 8 * P + (uint32_t)parity;

    const int t0 = slice * kILSize / nslices, t1 = (slice + 1) * kILSize / nslices;
    const int nchunk = (t1 - t0) * NKC;
    const int nstage = (nchunk + U - 1) / U;
    const size_t op_stride = (size_t)NKC * NB * 64;  // 16-byte entries per offset
    const int32_t *ilp = il + parity * kILSize;
    const int kq = 8 * (lane >> 4);  // this lane's k offset inside a chunk

    struct Cursor {
        int t, kc, oid;
        const float *src;
    };
    auto set_t = [&](Cursor &c, int t) {
        c.t = t;
        c.kc = 0;
        if (t >= t1) return;
        c.oid = ilp[t];
        const uint32_t sx = (tx + (uint32_t)offs[3 * c.oid]) & nmask;
        const uint32_t sy = (ty + (uint32_t)offs[3 * c.oid + 1]) & nmask;
        const uint32_t sz = (tz + (uint32_t)offs[3 * c.oid + 2]) & nmask;
        c.src = M + (size_t)morton3(sx, sy, sz) * Kp + kq;
    };
    auto advance = [&](Cursor &c) {
        if (++c.kc == NKC) set_t(c, c.t + 1);
    };
    auto load_b = [&](const Cursor &c) -> bf16x8 {
        bf16x8 b;
        if (32 * c.kc + kq < Kp) {
            const f32x4 x = *reinterpret_cast<const f32x4 *>(c.src + 32 * c.kc);
            const f32x4 y = *reinterpret_cast<const f32x4 *>(c.src + 32 * c.kc + 4);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                b[i] = (__bf16)x[i];
                b[4 + i] = (__bf16)y[i];
            }
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) b[i] = (__bf16)0.0f;
        }
        return b;
    };

    f32x4 acc[NRW];
#pragma unroll
    for (int rb = 0; rb < NRW; ++rb) acc[rb] = f32x4{0, 0, 0, 0};

    Cursor cc, pc;  // compute cursor, prefetch cursor
    set_t(cc, t0);
    set_t(pc, t0);
    bf16x8 pre[PER_T];
    bf16x8 bcur[U], bnext[U];
    size_t base[U];  // first operator entry of each chunk of the prefetched stage
    bool have[U];

    // entry idx = tid + 256 v of a stage belongs to chunk slot idx / CHUNK
    auto fetch_stage = [&](bf16x8 *dst_regs, bf16x8 *dst_lds, bf16x8 *bdst) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            have[u] = pc.t < t1;
            if (have[u]) {
                base[u] = (size_t)pc.oid * op_stride + ((size_t)pc.kc * NB + rb0) * 64;
                bdst[u] = load_b(pc);
                advance(pc);
            }
        }
#pragma unroll
        for (int v = 0; v < PER_T; ++v) {
            const int idx = tid + 256 * v;
            const int u = idx / CHUNK, e = idx % CHUNK;
            if (u < U && e < nrb * 64 && have[u]) {
                const bf16x8 x = ops[base[u] + e];
                if (dst_lds) dst_lds[idx] = x;
                else dst_regs[v] = x;
            }
        }
    };

    fetch_stage(nullptr, lds[0], bcur);
    __syncthreads();

    for (int st = 0; st < nstage; ++st) {
        const int cur = st & 1;
        const bool more = st + 1 < nstage;
        bool hv[U];
        if (more) {
            fetch_stage(pre, nullptr, bnext);
#pragma unroll
            for (int u = 0; u < U; ++u) hv[u] = have[u];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (cc.t < t1) {
                bf16x8 a[NRW];
#pragma unroll
                for (int rb = 0; rb < NRW; ++rb)
                    if (rb < nrb) a[rb] = lds[cur][u * CHUNK + rb * 64 + lane];
#pragma unroll
                for (int rb = 0; rb < NRW; ++rb)
                    if (rb < nrb) acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rb], bcur[u], acc[rb], 0, 0, 0);
                advance(cc);
            }
        }
        if (more) {
#pragma unroll
            for (int v = 0; v < PER_T; ++v) {
                const int idx = tid + 256 * v;
                const int u = idx / CHUNK, e = idx % CHUNK;
                if (u < U && e < nrb * 64 && hv[u]) lds[cur ^ 1][idx] = pre[v];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) bcur[u] = bnext[u];
        }
        __syncthreads();
    }

    if (!valid) return;
    float *out = L + (size_t)slice * ((size_t)8 << (3 * nh_bits)) * Kp;
#pragma unroll
    for (int rb = 0; rb < NRW; ++rb)
        if (rb < nrb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * (rb0 + rb) + Mfma<float>::row(lane, r);
                out[(size_t)tcell * Kp + row] = acc[rb][r];
            }
}

hipError_t launch_m2l_bf16(int level, const void *ops, const int32_t *il, const int32_t *offs, const float *M,
                           float *L, float *partial, int p, int Kp, hipStream_t s) {
    const int NB = Kp / 16;
    const int NKC = bf16_chunks(p);
    const int nh_bits = level - 1;
    const int64_t ntarget = (int64_t)1 << (3 * nh_bits);
    const int nslices = partial ? m2l_slices(level) : 1;
    const int nrg = (NB + kRowBlocksPerWave - 1) / kRowBlocksPerWave;
    const int64_t ntile = (ntarget + 63) / 64;
    const int64_t grid = 8 * ntile * nslices * nrg;
    const bf16x8 *o = reinterpret_cast<const bf16x8 *>(ops);
    if (nslices > 1)
        hipLaunchKernelGGL((k_m2l_bf16<true>), dim3((unsigned)grid), dim3(256), 0, s, o, il, offs, M, partial,
                           nh_bits, NB, NKC, Kp, nrg, nslices);
    else
        hipLaunchKernelGGL((k_m2l_bf16<false>), dim3((unsigned)grid), dim3(256), 0, s, o, il, offs, M, L, nh_bits,
                           NB, NKC, Kp, nrg, 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nslices == 1) return e;
    const int64_t elems = ((int64_t)8 << (3 * nh_bits)) * Kp;
    int64_t g = (elems + 255) / 256;
    if (g > 65535) g = 65535;
    hipLaunchKernelGGL(k_m2l_reduce<float>, dim3((unsigned)g), dim3(256), 0, s, partial, L, nslices, elems);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_m2l(int level, const T *ops, const int32_t *il, const int32_t *offs, const T *M, T *L,
                      T *partial, int p, int Kp, hipStream_t s, int nil) {
    constexpr int CB = Mfma<T>::CB;
    const int NB = Kp / 16;
    int R = 1;
    if (NB > kRowBlocksPerWave) R = 2;
    if (NB > 2 * kRowBlocksPerWave) R = 4;
    if (NB > 4 * kRowBlocksPerWave) return hipErrorInvalidValue;
    const int nh_bits = level - 1;
    const int64_t ntarget = (int64_t)1 << (3 * nh_bits);
    const int nslices = partial ? std::min(m2l_slices(level), nil) : 1;
    if (use_lds_kernel<T>(level)) {
        if (nil != kILSize) return hipErrorInvalidValue;  // the LDS kernel walks the full list
        const int64_t ntile = (ntarget + 63) / 64;
        const int64_t grid = 8 * ntile * nslices;
        T *out = nslices > 1 ? partial : L;
        // one launch per group of up to kRowBlocksPerWave row blocks
        for (int rb0 = 0; rb0 < NB; rb0 += kRowBlocksPerWave) {
            const int nrb = std::min(kRowBlocksPerWave, NB - rb0);
            hipError_t e = hipSuccess;
            switch (nrb) {
#define FMM_M2L_LDS_CASE(N)                                                                                     \
    case N:                                                                                                     \
        if (nslices > 1)                                                                                        \
            hipLaunchKernelGGL((k_m2l_lds<T, true, N>), dim3((unsigned)grid), dim3(256), 0, s, ops, il, offs, M, \
                               out, nh_bits, NB, Kp, rb0, nslices);                                             \
        else                                                                                                    \
            hipLaunchKernelGGL((k_m2l_lds<T, false, N>), dim3((unsigned)grid), dim3(256), 0, s, ops, il, offs, \
                               M, out, nh_bits, NB, Kp, rb0, 1);                                                \
        break;
                FMM_M2L_LDS_CASE(1) FMM_M2L_LDS_CASE(2) FMM_M2L_LDS_CASE(3) FMM_M2L_LDS_CASE(4)
                FMM_M2L_LDS_CASE(5) FMM_M2L_LDS_CASE(6) FMM_M2L_LDS_CASE(7) FMM_M2L_LDS_CASE(8)
                FMM_M2L_LDS_CASE(9) FMM_M2L_LDS_CASE(10) FMM_M2L_LDS_CASE(11)
#undef FMM_M2L_LDS_CASE
                default: return hipErrorInvalidValue;
            }
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    } else {
        const int64_t ntile = (ntarget + 16 * CB - 1) / (16 * CB);
        const int64_t grid = 8 * ntile * nslices;
        hipLaunchKernelGGL(k_m2l<T>, dim3((unsigned)grid), dim3(256), 0, s, ops, il, offs, M,
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
template hipError_t launch_m2l<float>(int, const float *, const int32_t *, const int32_t *, const float *,
                                      float *, float *, int, int, hipStream_t, int);
template hipError_t launch_m2l<double>(int, const double *, const int32_t *, const int32_t *, const double *,
                                       double *, double *, int, int, hipStream_t, int);

}  // namespace fmm
