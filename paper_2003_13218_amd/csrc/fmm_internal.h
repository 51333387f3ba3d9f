// Internal declarations shared by the host orchestration and the HIP kernels
// of libfmm.  Nothing here is part of the public ABI (see include/fmm.h).
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

namespace fmm {

constexpr int kWS = 2;            // near field / well-separatedness: +-2 cells
constexpr int kNumOffsets = 1206; // distinct M2L offsets: [-5,5]^3 minus [-2,2]^3
constexpr int kILSize = 875;      // interaction list size per parity class
constexpr int kM2LPairEntries = 573;   // list entries per class, scheme 1: 302 (t, -t) pairs + 271 singles
constexpr int kM2LOrbitEntries = 305;  // list entries per class, scheme 2: orbits of the two-axis flips
constexpr int kMaxP = 20;
constexpr int kMaxP2PGroups = 16;  // largest source-group count of the P2P kernel
// source-group counts of the P2P kernel (0: chosen from the leaf occupancy)
constexpr bool valid_p2p_groups(int g) { return g == 0 || g == 1 || g == 2 || g == 4 || g == 8 || g == kMaxP2PGroups; }
constexpr int kMaxLevels = 10;

// ---------------------------------------------------------------------------
// Coefficient storage ("real storage"), K = (p+1)^2 reals per expansion:
//   index n*n           : m = 0 part
//   index n*n + 2m - 1  : real part of order m > 0
//   index n*n + 2m      : imaginary part of order m > 0
// Multipoles hold  M^_n^m = sum_j q_j conj(R^_n^m(r_j - c))  (no factor 2).
// Locals hold      L^_n^0 and 2 Re / 2 Im of L^_n^m (m > 0), so that the
// potential is the plain dot product  phi(c + x) = sum_k Rr_k(x) Lr_k  with
// Rr = (R^_n^0, Re R^_n^m, Im R^_n^m).
// R^_n^m = sqrt((n+m)!(n-m)!) R_n^m and I^_n^m = I_n^m / sqrt((n+m)!(n-m)!)
// where R_n^m = r^n P_n^m e^{im phi}/(n+m)!, I_n^m = (n-m)! P_n^m e^{im phi}/r^{n+1}.
// Expansions at level l are stored scaled by the cell edge h_l:
//   M~_n = M^_n / h^n,   L~_n = L^_n h^{n+1},
// which makes every M2M, M2L and L2L operator independent of the level and
// of the box size.
// ---------------------------------------------------------------------------

constexpr inline int num_coeffs(int p) { return (p + 1) * (p + 1); }
constexpr inline int padded_coeffs(int p) { return ((num_coeffs(p) + 15) / 16) * 16; }

// Host FP64 precompute (harmonics_host.cpp) ---------------------------------
using cplx = std::complex<double>;

// Complex solid harmonics at (x,y,z) for 0 <= n <= J, all -n <= m <= n,
// stored at n*n + n + m.
void regular_complex(double x, double y, double z, int J, cplx *out);
void irregular_complex(double x, double y, double z, int J, cplx *out);
double norm_factor(int n, int m);  // sqrt((n+|m|)!(n-|m|)!)

struct Offsets {
    std::vector<int> vec;  // kNumOffsets x 3
    std::vector<int> il;   // 8 x kILSize offset ids (parity code = 4 px + 2 py + pz)
};
Offsets build_offsets();

// Real operators, row-major [out][in], K x K.
void build_m2l_operator(int p, const double t[3], double *A);
void build_lattice_operator(int p, const cplx *T, double *A);
void build_m2m_operator(int p, int octant, double *A);  // child octant -> parent
void build_l2l_operator(int p, int octant, double *A);  // parent -> child octant

// Lattice tensor for a unit box: T_j^k = sum_{|nu|_inf > 2} I_j^k(nu), j <= J,
// evaluated as in eq. 12 with split parameter kappa_b (= kappa * b) for j = 0
// and j <= kEwaldMaxJ; direct absolutely convergent sums above.
void lattice_tensor(int J, double kappa_b, cplx *T);

// Recurrence coefficient tables for the normalised regular harmonics
// (index n(n+1)/2 + m): a = (2n-1)/sqrt((n+m)(n-m)),
// b = sqrt((n+m-1)(n-m-1)/((n+m)(n-m))); diagonal c_m = sqrt((2m-1)/(2m)),
// sub-diagonal d_m = sqrt(2m+1).
struct RecTables {
    double a[(kMaxP + 1) * (kMaxP + 2) / 2];
    double b[(kMaxP + 1) * (kMaxP + 2) / 2];
    double c[kMaxP + 1];
    double d[kMaxP + 1];
};
void build_rec_tables(RecTables *t);

// Kernel launchers (defined in the .hip files) ------------------------------
// All return the first HIP error they meet.

// k_expand.hip
hipError_t upload_rec_tables(const RecTables &t);

// k_sort.hip
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t s);
hipError_t launch_bin(int64_t n, const double *pos, const double *q, double box, int levels,
                      uint32_t *key, uint32_t *count, int *flag, hipStream_t s);
hipError_t launch_scan(const uint32_t *in, int32_t *out_exclusive, int64_t n,
                       int32_t *scratch, int64_t scratch_len, hipStream_t s);
int64_t scan_scratch_len(int64_t n);
hipError_t launch_scatter(int64_t n, const uint32_t *key, const int32_t *start, uint32_t *cursor,
                          int32_t *perm, hipStream_t s);
hipError_t launch_cell_sort(int64_t nleaf, const int32_t *start, int32_t *perm, hipStream_t s);
hipError_t launch_pad_counts(int64_t nleaf, const uint32_t *count, int G, uint32_t *pcount, hipStream_t s);
hipError_t launch_pad_gather(int64_t nleaf, const int32_t *start, const int32_t *pstart, bool fp64,
                             const void *xq, double far, void *xqp, hipStream_t s);
hipError_t launch_gather(int64_t n, const int32_t *perm, const double *pos, const double *q,
                         double box, int levels, bool fp64, void *xq, double *xs, hipStream_t s);
hipError_t launch_mask_charges(int64_t n, const int32_t *perm, const uint8_t *mask, bool fp64,
                               const void *xq, void *xq_u, hipStream_t s);
hipError_t launch_invert_mask(int64_t n, const uint8_t *mask, uint8_t *out, hipStream_t s);

// k_expand.hip (T = float for mixed, double for fp64)
template <typename T>
hipError_t launch_p2m(int64_t nleaf, const void *xq, const int32_t *start, T *M, int p, int Kp,
                      double inv_h, hipStream_t s);
hipError_t launch_lattice(const double *M0, double *L0, const double *AT, int p, int Kp,
                          hipStream_t s);
// natoms: atoms of the tree (sets the leaves per workgroup)
template <typename T>
hipError_t launch_l2p(int64_t nleaf, const void *xq, const int32_t *start, const T *L, int p,
                      int Kp, double h, double *phi, T *field, hipStream_t s, int64_t natoms);

// ---------------------------------------------------------------------------
// The solute-solvent pass of several boxes, one launch per stage for all of
// them (a batch plan; a single-box plan is a batch of one box).  UvBox holds
// one box's arrays in device memory; a stage launch takes the table of boxes
// and, per box, the first block of that box in the launch (nbox + 1 int64,
// non-decreasing): block b works for the box w with start[w] <= b < start[w+1].
// ---------------------------------------------------------------------------
struct UvBox {
    int64_t n;          // atoms of the box
    int levels, p, K, Kp;
    int invert;         // solute = atoms with mask == 0 (u and v exchanged)
    int soft_c;         // soft-core exponent c, 0: no soft-core sums
    double box, h;      // box edge, leaf edge
    double asc, kd;     // soft-core alpha lambda sigma^c and alpha sigma^c / c
    const double *xs;   // sorted: wrapped position from the box centre, q (FP64)
    const void *xq;     // sorted: leaf-local position, q (the evaluation's type)
    const uint32_t *key;    // leaf key by original index
    const int32_t *perm;    // sorted -> original index
    const int32_t *start;   // leaf ranges (8^levels + 1)
    const uint8_t *mask;    // caller's order, nonzero = solute
    uint8_t *ms;            // solute flag in sorted order (written by the mask stage)
    uint32_t *flag;         // cell flags: level 0 at [0], level l >= 1 at [1 + sum_{k<l} 8^k]
    double *M, *L;          // FP64 level arrays of levels 1..levels (Kp per cell)
    double *M0, *L0;        // level 0
    const double *lat;      // level-0 lattice operator, transposed, FP64
    const double *phi_uv;   // sorted far-field potential of the evaluation
    double *phi_u;          // sorted far-field potential of the solute charges
    double *nfuv, *nfsc, *nfdl;  // near-field u-v sums per solute atom
    double *partials;       // reduction scratch
    double *sc;             // scalar block of the box (see fmm_api.cpp)
};

__device__ inline int box_of(const int64_t *__restrict__ start, int nbox, int64_t b) {
    int lo = 0, hi = nbox;  // start[lo] <= b < start[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Stages of the solute-solvent pass (each returns the first HIP error):
//   mask   zero every box's cell flags, then sorted solute flags ms and the
//          flags of the leaves holding solute atoms and of all their ancestors
//   p2m    FP64 P2M of the solute atoms of flagged leaves (sparse pass)
//   m2m    step k = 1 .. levels: parents at level levels - k from flagged children
//          (level 0: every box's M0, whatever the flags)
//   lat    level-0 lattice operator L0 = A M0
//   m2l    level l: flagged targets from flagged sources of their list; the
//          FP64 operators with their plain lists (nil entries per parity class):
//          the row-ordered full-list operators with rowpos (storage row ->
//          operator row) and nbr = m2l_row_blocks, or the aliased operators of
//          levels 1, 2 in storage order with rowpos NULL
//   l2l    level l: flagged cells from their parents (level 1: from L0)
//   l2p    far-field potential of the solute charges at the solute atoms
//          (phi_u, 0 at the others)
//   p2p_uv near-field u-v pair sums per solute atom (and soft-core sums)
//   sums   A = sum_u q phi_uv, B = sum_u q phi_u, C = sum_v q phi_u,
//          D = sum nf_uv, soft-core sums (sc[40..45]); moments of u (sc[24..28])
//          and v (sc[32..36]); sc[20] = M0[0]
// Block tables: `blocks(w)` blocks per box, as built by the host.
hipError_t launch_uv_mask(const UvBox *b, int nbox, const int64_t *st_fill, int64_t nb_fill,
                          const int64_t *st_atoms, int64_t nb_atoms, hipStream_t s);
hipError_t launch_uv_p2m(const UvBox *b, int nbox, const int64_t *st_leaf, int64_t nb, hipStream_t s);
hipError_t launch_uv_l2p(const UvBox *b, int nbox, const int64_t *st_atoms, int64_t nb, hipStream_t s);
hipError_t launch_uv_lattice(const UvBox *b, int nbox, const int64_t *st_one, int64_t nb, hipStream_t s);
// k_sparse.hip: ops = the 16 swizzled FP64 octant operators (M2M then L2L)
hipError_t launch_uv_m2m(const UvBox *b, int nbox, int step, const int64_t *st, int64_t nb, const void *ops,
                         hipStream_t s);
hipError_t launch_uv_m2l(const UvBox *b, int nbox, int level, const int64_t *st, int64_t nb, const int32_t *il,
                         const int32_t *offs, const double *ops, const int32_t *rowpos, int nbr, int nil,
                         hipStream_t s);
hipError_t launch_uv_l2l(const UvBox *b, int nbox, int level, const int64_t *st, int64_t nb, const void *ops,
                         hipStream_t s);
// k_p2p.hip (T: type of xq)
template <typename T>
hipError_t launch_uv_p2p(const UvBox *b, int nbox, const int64_t *st_leaf, int64_t nb, hipStream_t s);
// k_reduce.hip: st_red per box moments_blocks(n) blocks, st_one one block
// (partials: 32 moments_blocks(n) doubles per box)
hipError_t launch_uv_sums(const UvBox *b, int nbox, const int64_t *st_red, int64_t nb_red, const int64_t *st_one,
                          int64_t nb_one, hipStream_t s);

// m2l_layout.cpp (host) and k_m2l.hip (kernels)
// Row blocks of 16 operator rows: at most kRowBlocksPerWave per launch of the
// LDS kernel (176 rows: K <= 169, p <= 12, in one row group), at most
// kMaxRowGroups launches per level.  FP32 orbit lists whose four row classes
// fit kAllClassBlocks blocks run in one launch, the four source fragments
// gathered once for all classes (measured on the 1M-atom box, p = 12: 8.22 vs
// 8.42 ms for the level); FP64 keeps two launches (one launch of 12 FP64 row
// blocks: 16.1 vs 14.5 ms).  The split-FP16 M2L takes at most
// kSplit16RowBlocks blocks per launch on the plain list (k_m2l_f16rows: three
// blocks per wavefront, with their FP64 flush accumulators for 64 targets, at
// two wavefronts per SIMD), and all kAllClassBlocks blocks in one launch on
// the orbit list (one wavefront per SIMD).
constexpr int kRowBlocksPerWave = 11;
constexpr int kMaxRowGroups = 16;
constexpr int kAllClassBlocks = 12;
constexpr int kSplit16RowBlocks = 12;
inline bool one_launch(int blocks_per_class, bool fp64) { return !fp64 && 4 * blocks_per_class <= kAllClassBlocks; }
// chunks of 32 coefficients (the k depth of the 16x16x32 BF16 / FP16 MFMA)
inline int m2l_k32_chunks(int p) { return (num_coeffs(p) + 31) / 32; }

// One launch of the LDS-shared M2L kernel: operator rows [rb0, rb0 + nrb) in
// blocks, the first ne blocks on the first source combination, kernel
// variant sym (0 plain list, 1 pairs (t, -t), 2 / 3 orbit halves, 4 all orbit
// classes; see k_m2l_lds).
struct RowGroup {
    int rb0, nrb, ne, sym;
};
// Row groups of the class-ordered operators of order p (scheme 1 or 2), or of
// plain storage-ordered operators with NB row blocks (scheme 0), at most maxrb
// blocks each; returns the count (<= kMaxRowGroups)
int m2l_row_groups(int scheme, int p, int NB, bool fp64, RowGroup *g, int maxrb = kRowBlocksPerWave);
// split-FP16 M2L: the row group of its folded list (the four classes of three
// blocks each in one launch, p = 11, 12; 0 for other orders, which take the
// plain list), whether it folds, and its launches per level
int m2l_split16_fold_groups(int p, RowGroup *grp);
bool m2l_split16_folded(int p);
// row groups of the plain split-FP16 kernel for NB row blocks: as few as fit
// kSplit16RowBlocks each, all full but the last
int m2l_split16_plain_groups(int NB, RowGroup *grp);

// Levels with few target cells split the interaction list into slices
// (split-K) whose partial sums go to `partial` and are added in a fixed order.
// offs: 3 ints per operator id (the source cell is the target cell + offset,
// wrapped on the level's grid).
//   nil == 875: the full interaction list, as the symmetry-folded entries
//     `list` (8 x m2l_list_entries x m2l_list_width operator ids, -1 for an
//     absent source; see build_m2l_list) with the class-ordered operators of
//     swizzle_m2l_ops and `rowmap` (m2l_row_map) to put the result rows back
//     in storage order; Mflip: scratch for the level's sign-flipped
//     multipoles (m2l_flip_copies(p) x cells x Kp elements); zeros: Kp zero
//     elements (the source of an absent image);
//   nil < 875 (the aliased levels 1 and 2): `list` holds 8 x nil operator ids
//     of operators in the plain swizzle_ops layout; rowmap, Mflip, zeros unused.
// flip_cap / part_cap: bytes available in Mflip / partial; a launch that
// would need more returns hipErrorInvalidValue before touching the GPU.
int m2l_slices(int level);
// bytes of the sign-flipped copies of one full-list level of elem-byte
// coefficients, and of its split-K partials (0 when it is not split)
size_t m2l_flip_bytes(int level, int p, size_t elem);
size_t m2l_partial_bytes(int level, int p, int nil, size_t elem);
template <typename T>
hipError_t launch_m2l(int level, const T *ops, const int32_t *list, const int32_t *offs, const int32_t *rowmap,
                      const T *M, T *Mflip, size_t flip_cap, const T *zeros, T *L, T *partial, size_t part_cap, int p,
                      int Kp, hipStream_t s, int nil = kILSize);
// Symmetry scheme of the full-list operators for order p (1: (t, -t) pairs,
// 2: orbits of the two-axis flips), their row blocks (rows grouped by class,
// each class padded to 16), the blocks per class (returns the class count),
// list entries per parity class and ints per entry, flipped copies needed
int m2l_scheme(int p);
int m2l_row_blocks(int p);
int m2l_class_blocks(int p, int *blocks /*4*/);
int m2l_list_entries(int p);
int m2l_list_width(int p);
int m2l_launches(int p, bool fp64);  // launches of the LDS kernel for one full-list level
inline int m2l_flip_copies(int p) { return m2l_scheme(p) == 1 ? 1 : 3; }
// map[16 * m2l_row_blocks] = storage row of each operator row (every row of
// 0 .. Kp-1 once, the padding rows K .. Kp-1 on zero operator rows) or -1
void m2l_row_map(int p, int32_t *map);
bool build_m2l_list(int p, const int32_t *vec /*1206 x 3*/, const int32_t *il /*8 x 875*/, int32_t *out);
template <typename T>
size_t m2l_ops_elems(int p);  // element count of the swizzled, row-ordered operator array
template <typename T>
void swizzle_m2l_ops(int p, const double *ops_rowmajor /*1206 x K x K*/, T *out);
// M2L operators as bfloat16 (round to nearest even) in the lane order of
// v_mfma_f32_16x16x32_bf16: [1206][NKC][NB][64 lanes][8], NKC = ceil(K/32)
size_t m2l_bf16_ops_elems(int p);
void swizzle_m2l_ops_bf16(int p, const double *ops_rowmajor, uint16_t *out);
hipError_t launch_m2l_bf16(int level, const void *ops, const int32_t *il, const int32_t *offs, const float *M,
                           float *L, float *partial, size_t part_cap, int p, int Kp, hipStream_t s);
// M2L operators split into two FP16 parts, with power-of-two row and column
// scales (rscale, cscale: Kp floats each), in the lane order of
// v_mfma_f32_16x16x32_f16: [1206][ceil(K/32)][row blocks][64 lanes][hi 8,
// lo 8], rows in the class order of m2l_row_map (m2l_row_blocks blocks) when
// m2l_split16_folded(p), else in storage order (Kp / 16 blocks)
size_t m2l_split16_ops_elems(int p);
void swizzle_m2l_ops_split16(int p, const double *ops_rowmajor, uint16_t *out, float *rscale, float *cscale);
int m2l_split16_launches(int p);
// list / offs / rowmap: the folded list, offsets and row map of the FP32
// kernel when m2l_split16_folded(p), else the plain list and offsets (rowmap
// unused); ops in the matching layout (swizzle_m2l_ops_split16); Mc: scratch
// for the column-scaled multipoles of the level (plain list: as FP16 hi / lo
// pairs, the same size) and, folded, their sign-flipped copies (mc_cap
// bytes); zeros: Kp zero floats (absent images);
// partial: FP64 split-K partials (part_cap bytes) or NULL
hipError_t launch_m2l_split16(int level, const void *ops, const int32_t *list, const int32_t *offs,
                              const int32_t *rowmap, const float *M, float *Mc, size_t mc_cap, const float *cscale,
                              const float *rscale, const float *zeros, float *L, double *partial, size_t part_cap,
                              int p, int Kp, hipStream_t s);
// any nops row-major K x K operators into the matrix-core lane order
template <typename T>
void swizzle_ops(int p, int nops, const double *ops_rowmajor, T *out);

// k_tree.hip: M2M / L2L on the matrix cores; ops = 8 swizzled octant
// operators in the compute precision (FP64 if either side is FP64)
template <typename Tin, typename Tout>
hipError_t launch_m2m_mfma(int64_t nparent, const Tin *Mchild, Tout *Mparent, const void *ops, int p,
                           int Kp, hipStream_t s);
template <typename Tin, typename Tout>
hipError_t launch_l2l_mfma(int64_t nparent, const Tin *Lparent, Tout *Lchild, const void *ops, int p,
                           int Kp, hipStream_t s);

// k_p2p.hip
template <typename T>
hipError_t launch_p2p(int64_t nleaf, int levels, const void *xqp, const int32_t *pstart, const int32_t *start,
                      double h, double *phi, T *field, int groups, int nsplit, int max_wg, int64_t nsrc_max,
                      hipStream_t s);

// k_reduce.hip
struct Moments {  // device-side FP64 results of the moment reduction
    double Q, mux, muy, muz, S2;
};
hipError_t launch_moments(int64_t n, const double *xs, const int32_t *perm, const uint8_t *mask,
                          int want, double *partials, int nblocks, double *out5, hipStream_t s);
int moments_blocks(int64_t n);
// mu_w: weight of the dipole parts of the background terms, 1 under the
// conducting boundary, 0 under vacuum (the dipole surface term cancels them)
template <typename T>
hipError_t launch_finalize(int64_t n, const int32_t *perm, const double *xs, double box, double kappa,
                           double t00b, double mu_w, const double *moments, const double *m0, const double *phi_nf,
                           const T *field_nf, const double *phi_ff, const T *field_ff, double *forces,
                           double *phi, double *partials, int nblocks, double *energy_out, hipStream_t s);
template <typename T>
hipError_t launch_parts_out(int64_t n, const int32_t *perm, const double *phi_s, const T *field_s,
                            const double *m0, double cq, double *phi, double *field, hipStream_t s);

// tuning_cache.cpp: the autotune cache file of batch plans (host code)
std::string tuning_cache_key(const std::string &arch, int p, int prec, int fp64_levels, size_t nbox,
                             const double *box, const int64_t *natoms);
bool tuning_cache_lookup(const char *path, const std::string &key, size_t nbox, std::vector<int> &levels,
                         std::vector<int> &groups);
bool tuning_cache_append(const char *path, const std::string &key, const std::vector<int> &levels,
                         const std::vector<int> &groups);

}  // namespace fmm
