// Host side of stage a6 (M2L, eq. Lcoeffdef): the symmetry folding of the
// interaction lists, the row order and operand swizzles of the matrix-core
// kernels in k_m2l.hip, and the split-K slicing of shallow levels.  Plain C++
// run once per plan (no device code), so it builds and runs on the host alone.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "fmm_internal.h"

namespace fmm {

// ---------------------------------------------------------------------------
// Symmetries of the M2L operators.  Reflecting the translation in any set of
// axes changes an operator by signs only: for s in {+-1}^3
//   O_{s t} = D_s O_t D_s,   D_s = diag(sigma_s(k)),
// where for a coefficient of degree n, order m and real or imaginary part
//   x -> -x multiplies it by (-1)^m, and by -1 more for an imaginary part,
//   y -> -y by -1 for an imaginary part,   z -> -z by (-1)^(n+m).
// (the irregular harmonics I_n^m(s t) are +-I_n^m(t) or their conjugates).
// For a group H of reflections and a target whose list holds the images s t,
//   sum_{s in H} O_{s t} M_s = sum_{s} D_s O_t D_s M_s,
// and the rows of a character class chi of H (rows k with sigma_s(k) = chi(s)
// for all s in H) receive  O_t (sum_s chi(s) D_s M_s):  one operator product
// per orbit, class by class.  Two groups are used:
//   scheme 1, H = {identity, -1}: classes even / odd degree; per parity class
//     the 875 offsets form 302 pairs (t, -t) and 271 single offsets: 573
//     entries, sources (t, -t);
//   scheme 2, H = {identity, (-,-,+), (-,+,-), (+,-,-)} (two-axis flips):
//     four classes; 305 orbits of 1 to 4 offsets, sources in the order of H.
// Operators are stored with their rows grouped by class, each class padded to
// whole 16-row blocks (so a matrix-core row block holds one class), columns in
// storage order.  Scheme 2 needs four padded classes; it is taken where its
// matrix-core work (entries x row blocks) is smaller, i.e. for p >= 5.
// ---------------------------------------------------------------------------
struct Coef {
    int n, m;
    bool im;
};
static Coef coef(int k) {
    int n = 0;
    while ((n + 1) * (n + 1) <= k) ++n;
    const int r = k - n * n;
    return Coef{n, (r + 1) / 2, r > 0 && (r % 2 == 0)};
}
static int row_class(int scheme, int k) {
    const Coef c = coef(k);
    if (scheme == 1) return c.n & 1;
    return 2 * (c.m & 1) + ((c.n & 1) ^ (c.im ? 1 : 0));
}
static int class_rows(int p, int scheme, int cls) {
    int r = 0;
    for (int k = 0; k < num_coeffs(p); ++k) r += row_class(scheme, k) == cls;
    return r;
}
static int scheme_blocks(int p, int scheme) {
    int b = 0;
    for (int c = 0; c < (scheme == 1 ? 2 : 4); ++c) b += (class_rows(p, scheme, c) + 15) / 16;
    return b;
}
// launches of a full-list level: one for all classes (FP32, small orders), or
// one per half of the classes (the two classes sharing their partial sums),
// split into groups of at most 11 row blocks
static int scheme_launches(int p, int scheme, bool fp64) {
    if (scheme == 2) {
        const int b0 = (class_rows(p, 2, 0) + 15) / 16;
        bool equal = true;
        for (int c = 1; c < 4; ++c) equal = equal && (class_rows(p, 2, c) + 15) / 16 == b0;
        if (equal && one_launch(b0, fp64)) return 1;
    }
    int n = 0;
    for (int h = 0; h < (scheme == 1 ? 1 : 2); ++h) {
        const int c0 = (class_rows(p, scheme, 2 * h) + 15) / 16, c1 = (class_rows(p, scheme, 2 * h + 1) + 15) / 16;
        if (c0 + c1 == 0) continue;
        n += c0 + c1 <= 11 ? 1 : (c0 + 10) / 11 + (c1 + 10) / 11;
    }
    return n;
}
// The scheme with the smaller cost entries x (row blocks + multipole
// fragments loaded per chunk over all launches): each launch gathers every
// source of an entry (2 for pairs, 4 for orbits) for each column chunk.  On
// the 3M-atom box this picks the pairs at p = 8 (41.8 vs 42.6 ms mixed, 71 vs
// 79 ms FP64) and the orbits from p = 10 (84 vs 105 ms at p = 12).
int m2l_scheme(int p) {
    const int64_t c1 = (int64_t)kM2LPairEntries * (scheme_blocks(p, 1) + 2 * scheme_launches(p, 1, false));
    const int64_t c2 = (int64_t)kM2LOrbitEntries * (scheme_blocks(p, 2) + 4 * scheme_launches(p, 2, false));
    return c2 < c1 ? 2 : 1;
}
int m2l_launches(int p, bool fp64) { return scheme_launches(p, m2l_scheme(p), fp64); }
int m2l_row_blocks(int p) { return scheme_blocks(p, m2l_scheme(p)); }
int m2l_class_blocks(int p, int *blocks) {
    const int sch = m2l_scheme(p), nc = sch == 1 ? 2 : 4;
    for (int c = 0; c < nc; ++c) blocks[c] = (class_rows(p, sch, c) + 15) / 16;
    return nc;
}
int m2l_list_entries(int p) { return m2l_scheme(p) == 1 ? kM2LPairEntries : kM2LOrbitEntries; }
int m2l_list_width(int p) { return m2l_scheme(p) == 1 ? 2 : 4; }

// The padding rows K .. Kp-1 of the storage order take the first unused
// slots (their operator rows are zero), so the kernel writes every stored row.
void m2l_row_map(int p, int32_t *map) {
    const int sch = m2l_scheme(p);
    int blocks[4], start[4];
    const int nc = m2l_class_blocks(p, blocks);
    const int nr = 16 * m2l_row_blocks(p);
    for (int i = 0; i < nr; ++i) map[i] = -1;
    for (int c = 0, at = 0; c < nc; ++c) {
        start[c] = at;
        at += 16 * blocks[c];
    }
    for (int k = 0; k < num_coeffs(p); ++k) map[start[row_class(sch, k)]++] = k;
    int pad = num_coeffs(p);
    for (int i = 0; i < nr && pad < padded_coeffs(p); ++i)
        if (map[i] < 0) map[i] = pad++;
}

// List entries per parity class (m2l_list_width ints each, -1 for an absent
// source): the orbits of the scheme's group within the class's list, each
// orbit at the position of its first offset in list order, each offset in
// exactly one entry.  False if the counts differ from the constants.
bool build_m2l_list(int p, const int32_t *vec, const int32_t *il, int32_t *out) {
    const int sch = m2l_scheme(p), W = m2l_list_width(p), NE = m2l_list_entries(p);
    static const int H1[2][3] = {{1, 1, 1}, {-1, -1, -1}};
    static const int H2[4][3] = {{1, 1, 1}, {-1, -1, 1}, {-1, 1, -1}, {1, -1, -1}};
    for (int par = 0; par < 8; ++par) {
        const int32_t *l = il + par * kILSize;
        int32_t *o = out + (size_t)par * W * NE;
        bool used[kNumOffsets] = {};
        int ne = 0;
        for (int i = 0; i < kILSize; ++i) {
            const int a = l[i];
            if (used[a]) continue;
            if (ne == NE) return false;
            for (int w = 0; w < W; ++w) {
                const int *sg = sch == 1 ? H1[w] : H2[w];
                int found = -1;
                for (int jj = 0; jj < kILSize && found < 0; ++jj) {
                    const int c = l[jj];
                    if (!used[c] && vec[3 * c] == sg[0] * vec[3 * a] && vec[3 * c + 1] == sg[1] * vec[3 * a + 1] &&
                        vec[3 * c + 2] == sg[2] * vec[3 * a + 2])
                        found = c;
                }
                if (found >= 0) used[found] = true;
                o[W * ne + w] = found;
            }
            ++ne;
        }
        if (ne != NE) return false;
    }
    return true;
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

// Slices per level: enough workgroups (>= ~512) to fill 256 CUs at two
// resident workgroups each; levels >= 5 have enough targets on their own.
// Level 4 (FP32 all-classes kernel, two workgroups per CU): 8 slices = 512
// workgroups, one resident round; with the partials in FP64 the slicing no
// longer changes the result (1M-atom box: 10.05 ms per step against 10.13 /
// 10.23 with 16 / 32 slices, identical errors).
int m2l_slices(int level) {
    switch (level) {
        case 1: return 64;
        case 2: return 64;
        case 3: return 64;
        case 4: return 8;
        default: return 1;
    }
}

size_t m2l_flip_bytes(int level, int p, size_t elem) {
    return (size_t)m2l_flip_copies(p) * ((size_t)1 << (3 * level)) * (size_t)padded_coeffs(p) * elem;
}

size_t m2l_partial_bytes(int level, int p, int nil, size_t elem) {
    const int nslices = std::min(m2l_slices(level), nil);
    if (nslices <= 1) return 0;
    // FP32 operands on the full list keep their split-K partials in FP64
    const size_t pe = (elem == 4 && nil == kILSize) ? 8 : elem;
    return (size_t)nslices * ((size_t)1 << (3 * level)) * (size_t)padded_coeffs(p) * pe;
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

size_t m2l_bf16_ops_elems(int p) {
    return (size_t)kNumOffsets * m2l_k32_chunks(p) * (padded_coeffs(p) / 16) * 64 * 8;
}

void swizzle_m2l_ops_bf16(int p, const double *ops, uint16_t *out) {
    const int K = num_coeffs(p), NB = padded_coeffs(p) / 16, NKC = m2l_k32_chunks(p);
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

// ---------------------------------------------------------------------------
// Split FP16 operators (k_m2l_f16rows, PolF16x3F): per storage row r and
// column k the powers of two 2^{a_r} and 2^{b_k}, b_k = round(3/4 n(k)) (the multipoles of degree
// n fall off about as 0.87^n, the operators' columns as 3^-n: this keeps both
// near the middle of FP16's range), a_r chosen so that the row's largest
// scaled entry over all offsets lies in [2^9, 2^10).  cscale[k] = 2^{-b_k}
// multiplies the multipoles, rscale[r] = 2^{-a_r} the results (padding: 1).
// Layout [1206][ceil(K/32)][Kp/16][64 lanes][hi 8 | lo 8] in the lane order of
// v_mfma_f32_16x16x32_f16 (lane l: row l % 16, columns 8 (l / 16) + i).
// ---------------------------------------------------------------------------
static uint16_t f16_bits(double v) {
    // round to nearest even into IEEE binary16 (normal, subnormal, zero)
    if (v == 0.0) return 0;
    const uint16_t sign = v < 0 ? 0x8000 : 0;
    double a = std::fabs(v);
    int e;
    std::frexp(a, &e);  // a = f 2^e, f in [0.5, 1)
    int ex = e - 1;     // a = 1.x 2^ex
    if (ex > 15) return sign | 0x7bff;  // not reached with the scales above
    if (ex < -14) ex = -14;             // subnormal: fixed quantum 2^-24
    const double q = std::ldexp(1.0, ex - 10);
    double m = std::nearbyint(a / q);   // significand in units of q (ties to even)
    if (m >= 2048.0) { m /= 2.0; ++ex; }
    if (ex > 15) return sign | 0x7bff;
    if (m < 1024.0) return sign | (uint16_t)m;  // subnormal (ex == -14)
    return sign | (uint16_t)(((ex + 15) << 10) | ((int)m - 1024));
}
static double f16_value(uint16_t b) {
    const int ex = (b >> 10) & 31, mt = b & 1023;
    const double v = ex == 0 ? std::ldexp((double)mt, -24) : std::ldexp(1024.0 + mt, ex - 25);
    return (b & 0x8000) ? -v : v;
}

// row blocks of the split operators: class-ordered for the folded list
static int split16_row_blocks(int p) { return m2l_split16_folded(p) ? m2l_row_blocks(p) : padded_coeffs(p) / 16; }

size_t m2l_split16_ops_elems(int p) {
    return (size_t)kNumOffsets * m2l_k32_chunks(p) * split16_row_blocks(p) * 64 * 16;
}

void swizzle_m2l_ops_split16(int p, const double *ops, uint16_t *out, float *rscale, float *cscale) {
    const int K = num_coeffs(p), Kp = padded_coeffs(p), NB = split16_row_blocks(p), NKC = m2l_k32_chunks(p);
    // operator row of each position (class order when folded; -1: padding)
    std::vector<int32_t> map((size_t)16 * NB);
    if (m2l_split16_folded(p)) {
        m2l_row_map(p, map.data());
    } else {
        for (int i = 0; i < 16 * NB; ++i) map[i] = i;
    }
    std::vector<int> b(Kp, 0), a(Kp, 0);
    for (int k = 0; k < K; ++k) {
        int n = 0;
        while ((n + 1) * (n + 1) <= k) ++n;
        b[k] = (int)std::lround(0.75 * n);
    }
    for (int r = 0; r < K; ++r) {
        double mx = 0.0;
        for (int oid = 0; oid < kNumOffsets; ++oid)
            for (int k = 0; k < K; ++k)
                mx = std::max(mx, std::fabs(ops[((size_t)oid * K + r) * K + k]) * std::ldexp(1.0, b[k]));
        if (mx > 0.0) {
            int e;
            std::frexp(mx, &e);  // mx in [2^(e-1), 2^e)
            a[r] = 10 - e;
        }
    }
    for (int k = 0; k < Kp; ++k) {
        cscale[k] = (float)std::ldexp(1.0, -b[k]);
        rscale[k] = (float)std::ldexp(1.0, -a[k]);
    }
    for (int oid = 0; oid < kNumOffsets; ++oid) {
        const double *A = ops + (size_t)oid * K * K;
        for (int kc = 0; kc < NKC; ++kc)
            for (int rb = 0; rb < NB; ++rb)
                for (int lane = 0; lane < 64; ++lane)
                    for (int i = 0; i < 8; ++i) {
                        const int row = map[16 * rb + (lane & 15)];
                        const int col = 32 * kc + 8 * (lane >> 4) + i;
                        double v = 0.0;
                        if (row >= 0 && row < K && col < K)
                            v = std::ldexp(A[(size_t)row * K + col], a[row] + b[col]);
                        const uint16_t hi = f16_bits(v);
                        const uint16_t lo = f16_bits(v - f16_value(hi));
                        const size_t at = ((((size_t)oid * NKC + kc) * NB + rb) * 64 + lane) * 16;
                        out[at + i] = hi;
                        out[at + 8 + i] = lo;
                    }
    }
}


// Row groups of the class-ordered operators of order p (scheme 1 or 2), or of
// plain storage-ordered operators with NB row blocks (scheme 0).  A group
// holds at most kRowBlocksPerWave blocks and one or two classes of the same
// half (the two classes that share the partial sums w0 +- w1 and w2 +- w3).
int m2l_row_groups(int scheme, int p, int NB, bool fp64, RowGroup *g, int maxrb) {
    int ng = 0;
    auto chunks = [&](int from, int n, bool first, int sym) {
        for (int r = 0; r < n; r += maxrb) {
            const int k = std::min(maxrb, n - r);
            g[ng++] = RowGroup{from + r, k, first ? k : 0, sym};
        }
    };
    if (scheme == 0) {
        chunks(0, NB, false, 0);
        return ng;
    }
    int b[4];
    const int nc = m2l_class_blocks(p, b);
    if (nc == 4 && b[0] == b[1] && b[0] == b[2] && b[0] == b[3] && one_launch(b[0], fp64)) {
        g[ng++] = RowGroup{0, 4 * b[0], b[0], 4};
        return ng;
    }
    int at = 0;
    for (int h = 0; h < nc / 2; ++h) {
        const int c0 = b[2 * h], c1 = b[2 * h + 1], sym = scheme == 1 ? 1 : 2 + h;
        if (c0 + c1 == 0) continue;
        if (c0 + c1 <= maxrb) {
            g[ng++] = RowGroup{at, c0 + c1, c0, sym};
        } else {
            chunks(at, c0, true, sym);
            chunks(at + c0, c1, false, sym);
        }
        at += c0 + c1;
    }
    return ng;
}


// The row group of the folded split kernel for order p: the four row classes
// of the two-axis flips in one launch when each takes three row blocks
// (p = 11, 12), else 0 and the plain list is used.  The split operands cost
// about 4.5 vector instructions per multipole value converted, and the orbit
// list converts four class combinations per entry (1220 per column chunk and
// parity class against 875 on the plain list), so folding only pays where it
// saves the most matrix work: the finest level of the 3M-atom box takes
// 18.9 ms on the plain list against 21.5 ms folded at p = 8, and 72.9 against
// 46.9 ms at p = 12.
int m2l_split16_fold_groups(int p, RowGroup *grp) {
    int b[4];
    if (m2l_scheme(p) != 2 || m2l_class_blocks(p, b) != 4) return 0;
    if (b[0] != 3 || b[1] != 3 || b[2] != 3 || b[3] != 3) return 0;
    grp[0] = RowGroup{0, 12, 3, 4};
    return 1;
}

int m2l_split16_plain_groups(int NB, RowGroup *grp) {
    // full groups first: a group of n blocks runs 4 ceil(n / 4) of them (its
    // four wavefronts take equal shares), so with 12 = 3 x 4 only the last
    // group is padded and the total, 4 ceil(NB / 4), is the least possible
    int ng = 0;
    for (int r = 0; r < NB; r += kSplit16RowBlocks)
        grp[ng++] = RowGroup{r, std::min(kSplit16RowBlocks, NB - r), 0, 0};
    return ng;
}

bool m2l_split16_folded(int p) {
    RowGroup grp[kMaxRowGroups];
    return m2l_split16_fold_groups(p, grp) > 0;
}

int m2l_split16_launches(int p) {
    RowGroup grp[kMaxRowGroups];
    const int ng = m2l_split16_fold_groups(p, grp);
    return ng > 0 ? ng : m2l_split16_plain_groups(padded_coeffs(p) / 16, grp);
}


}  // namespace fmm
