// libfmm C ABI: plan construction, validation, workspace and the ordering of
// the GPU stages.  Every arithmetic step of the evaluation runs in the HIP
// kernels declared in fmm_internal.h; this file only prepares operators (FP64,
// once per plan) and launches work on the plan's stream.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "fmm.h"
#include "fmm_internal.h"

using namespace fmm;

namespace {

thread_local std::string g_plan_error;

struct DeviceBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    bool borrowed = false;  // a view of memory the buffer does not own (never freed or grown)
    void release() {
        if (ptr && !borrowed) (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
        borrowed = false;
    }
    bool ensure(size_t b) {
        if (b <= bytes && ptr) return true;
        if (borrowed) return false;
        release();
        if (b == 0) b = 16;
        if (hipMalloc(&ptr, b) != hipSuccess) { ptr = nullptr; bytes = 0; return false; }
        bytes = b;
        return true;
    }
    template <typename T> T *as() const { return reinterpret_cast<T *>(ptr); }
};

// Device copies of the order-p operators that do not depend on the box.
struct OpSet {
    int p = 0;
    Offsets offs;
    DeviceBuf ops32, ops64, opsbf, il, offv;  // M2L (FP32 / FP64 / bfloat16), interaction lists
    DeviceBuf ops16, scale16;                 // M2L split into two FP16 parts; its row and column scales
    // symmetry-folded list entries of the FP32/FP64 M2L (m2l_scheme), the row
    // order of its operators (row -> storage row) and its inverse (storage
    // row -> row), and Kp zeros (the source of an absent image)
    DeviceBuf pairs, rowmap, rowpos, zeros;
    DeviceBuf tree32, tree64;                 // swizzled M2M (8) then L2L (8) octant operators
    // levels 1 and 2 (grids of 2 and 4 cells per axis): FP64 operators summed
    // over the offsets that reach the same source cell (alias_ops), their
    // lists (8 x n^3 ids) and offsets (the residues of t modulo n)
    DeviceBuf alias_ops[2], alias_il[2], alias_off[2];
    ~OpSet() {
        DeviceBuf *b[] = {&ops32, &ops64, &opsbf, &ops16, &scale16, &il, &offv, &pairs, &rowmap, &rowpos, &zeros,
                          &tree32, &tree64,
                          &alias_ops[0], &alias_ops[1],
                          &alias_il[0], &alias_il[1], &alias_off[0], &alias_off[1]};
        for (DeviceBuf *x : b) x->release();
    }
};

struct Status {
    fmm_status code;
    std::string msg;
};

}  // namespace

struct fmm_plan {
    double box = 0.0;
    int levels = 0, p = 0, K = 0, Kp = 0;
    int prec = FMM_FP64;
    double kappa = 0.0;
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;                      // near field, concurrent with the far field
    hipStream_t side_up = nullptr;                   // upper M2L levels, concurrent with the lower ones
    hipEvent_t ev_up_fork = nullptr, ev_up_join = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;  // main -> side after the repack, side -> main
    int device = 0;
    std::string err;

    // host operators (FP64)
    std::vector<double> latT;  // transposed [col][row]
    // T_0^0 of the unit box: the net-charge (monopole-monopole) lattice
    // constant, applied exactly in FP64 as phi += t00 Q / b instead of through
    // the level-0 operator, so it never passes through FP32 arrays
    double t00 = 0.0;
    int top_fp64 = 3;  // mixed mode: tree levels 1..3 in FP64 (see top_fp64_levels)
    double q_tree = 0.0;  // level-0 monopole of the last fmm_energy_forces tree
    double last_energy = 0.0;  // energy of the last fmm_energy_forces call
    std::vector<cplx> T;                  // lattice tensor, unit box

    // scale-invariant translation operators of order p, shared by every plan
    // of a batch (they do not depend on the box)
    std::shared_ptr<OpSet> op;
    DeviceBuf lat;  // level-0 lattice operator (depends on kappa b)
    // per-call workspace
    DeviceBuf key, count, cursor, start, perm, scan, xq, xq_u, xs, Mlev, Llev, M0, L0, m2l_part;
    DeviceBuf pstart, xqp;  // near-field copy of xq, leaves padded to the P2P group count
    DeviceBuf mflip;        // sign-flipped multipoles of the level in M2L (symmetry-folded list)
    DeviceBuf m2l_part_up, mflip_up;  // the same two scratch buffers for the upper levels on side_up
    DeviceBuf phi_nf, field_nf, phi_ff, field_ff, phi_u, field_u, nfuv, partials, scalars, flag;
    DeviceBuf sflag;    // sparse solute pass: one flag per cell, level 0 first, then levels 1..L
    DeviceBuf mask_sw;  // exchanged solute mask (FMM_UV_SWAP)
    DeviceBuf mask_s;   // solute mask in sorted order
    DeviceBuf nfsc, nfdl;  // soft-core near-field u-v sums per solute atom
    // solute-solvent stage tables (UvBox entries + block tables) and the host
    // copy of what was last uploaded
    DeviceBuf uvtab;
    std::vector<unsigned char> uvtab_host;
    // batch plans: the boxes' solute-solvent scalar blocks, contiguous, and
    // their pinned host mirror
    DeviceBuf uvsc;
    double *h_uvsc = nullptr;
    // soft-core near-field u-v pairs of the lambda-coupled energy (alpha 0: off)
    double sc_alpha = 0.0, sc_sigma = 1.0;
    int sc_c = 6;
    double uv_d0 = 0.0, uv_dsc = 0.0, uv_dl = 0.0;  // near-field sums of the last solute-solvent pass
    int boundary = FMM_BOUNDARY_CONDUCTING;
    int uv_scheme = FMM_UV_SYMMETRIC;
    double *h_scalars = nullptr;  // pinned host mirror of `scalars`
    int64_t cap_n = -1;
    bool tree_ready = false;

    // stage timing (fmm_profile)
    bool profiling = false;
    hipEvent_t ev_begin[FMM_NUM_STAGES] = {}, ev_end[FMM_NUM_STAGES] = {};
    bool ev_used[FMM_NUM_STAGES] = {};
    double stage_ms[FMM_NUM_STAGES] = {};
    int64_t profiled_calls = 0;

    // state cached for fmm_solute_solvent_energy (sorted copies live in xq, xs)
    bool have_state = false;
    int64_t n_state = 0;
    int p2p_g = 0;  // P2P source groups; 0 = chosen from the leaf occupancy
    bool in_batch = false;  // sub-plan of a batch plan

    // batch plans (fmm_plan_batch): one sub-plan per box, run as parallel
    // branches of one captured HIP graph per call signature
    bool is_batch = false;
    std::vector<fmm_plan_t> sub;
    std::vector<int64_t> sub_natoms;  // atom counts the levels were chosen for
    std::vector<hipStream_t> sub_stream;
    std::vector<hipEvent_t> sub_done;
    hipEvent_t fork = nullptr, input_ready = nullptr;
    hipStream_t own_stream = nullptr;
    struct Graph {
        hipGraphExec_t exec = nullptr;
        std::vector<int64_t> key;
    } g_ef, g_uv;
    std::vector<int64_t> batch_off;  // offsets of the last batch evaluation
    bool batch_state = false;
};

static const int kScalars = 64;

static fmm_status fail(fmm_plan_t pl, fmm_status code, const std::string &m) {
    if (pl) pl->err = m;
    else g_plan_error = m;
    return code;
}

static fmm_status hip_fail(fmm_plan_t pl, hipError_t e, const char *where) {
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(pl, e == hipErrorOutOfMemory ? FMM_ERR_NOMEM : FMM_ERR_DEVICE, m);
}

#define HIPCHK(pl, expr, where)                         \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return hip_fail(pl, e_, where); \
    } while (0)

static int64_t level_cells(int l) { return (int64_t)1 << (3 * l); }
// offset (in cells) of level l >= 1 inside the concatenated level arrays
static int64_t level_offset(int l) {
    int64_t o = 0;
    for (int k = 1; k < l; ++k) o += level_cells(k);
    return o;
}

static bool rec_uploaded[64] = {false};

// ---------------------------------------------------------------------------
// Scratch of fmm_energy_forces_noalloc: one fixed array in device memory per
// GPU (the module's own copy on each device), shared by every plan and call
// on that device.  Host code never uses the array's name as an address: its
// device address is taken once per device, with that device current, when
// the first plan is made there, and only that address is passed on.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = (size_t)FMM_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64] = {};
static hipError_t g_scratch_err[64] = {};

// with `device` current
static void scratch_setup(int device) {
    if (device < 0 || device >= 64) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e == hipSuccess && ptr) g_scratch_ptr[device] = ptr;
    else g_scratch_err[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
}

static void batch_drop_graphs(fmm_plan_t pl) {
    for (auto *g : {&pl->g_ef, &pl->g_uv}) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        g->exec = nullptr;
        g->key.clear();
    }
}

// Stage events: begin/end recorded on the plan stream when profiling.
static void stage_begin(fmm_plan_t pl, int st, hipStream_t on = nullptr) {
    if (!pl->profiling || pl->ev_used[st]) return;
    (void)hipEventRecord(pl->ev_begin[st], on ? on : pl->stream);
}
static void stage_end(fmm_plan_t pl, int st, hipStream_t on = nullptr) {
    if (!pl->profiling || pl->ev_used[st]) return;
    (void)hipEventRecord(pl->ev_end[st], on ? on : pl->stream);
    pl->ev_used[st] = true;
}
static void stage_reset(fmm_plan_t pl) {
    for (int i = 0; i < FMM_NUM_STAGES; ++i) pl->ev_used[i] = false;
}
static void stage_collect(fmm_plan_t pl) {
    if (!pl->profiling) return;
    for (int i = 0; i < FMM_NUM_STAGES; ++i)
        if (pl->ev_used[i]) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, pl->ev_begin[i], pl->ev_end[i]) == hipSuccess) pl->stage_ms[i] += ms;
        }
    pl->profiled_calls++;
    stage_reset(pl);
}

// ---------------------------------------------------------------------------
// Plan construction
// ---------------------------------------------------------------------------
static void build_m2l_all(int p, const Offsets &o, std::vector<double> &out) {
    const int K = num_coeffs(p);
    out.assign((size_t)kNumOffsets * K * K, 0.0);
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (unsigned w = 0; w < nt; ++w)
        th.emplace_back([&, w] {
            for (int oid = (int)w; oid < kNumOffsets; oid += (int)nt) {
                const double t[3] = {(double)o.vec[3 * oid], (double)o.vec[3 * oid + 1],
                                     (double)o.vec[3 * oid + 2]};
                build_m2l_operator(p, t, out.data() + (size_t)oid * K * K);
            }
        });
    for (auto &t : th) t.join();
}

static void transpose_into(const double *A, int K, double *AT) {
    for (int r = 0; r < K; ++r)
        for (int c = 0; c < K; ++c) AT[(size_t)c * K + r] = A[(size_t)r * K + c];
}

// Offsets, interaction lists and the M2M / L2L operators of order p; the
// M2L operators are added on first use (ensure_m2l_ops).
static fmm_status make_opset(int p, std::shared_ptr<OpSet> &out, std::string &msg) {
    auto op = std::make_shared<OpSet>();
    op->p = p;
    op->offs = build_offsets();
    const int K = num_coeffs(p), Kp = padded_coeffs(p);
    // octant operators, row-major, M2M then L2L, swizzled for the matrix cores
    std::vector<double> rm((size_t)16 * K * K);
    for (int o = 0; o < 8; ++o) {
        build_m2m_operator(p, o, rm.data() + (size_t)o * K * K);
        build_l2l_operator(p, o, rm.data() + (size_t)(8 + o) * K * K);
    }
    const size_t ne = (size_t)16 * Kp * Kp;
    std::vector<float> s32(ne);
    std::vector<double> s64(ne);
    swizzle_ops<float>(p, 16, rm.data(), s32.data());
    swizzle_ops<double>(p, 16, rm.data(), s64.data());
    std::vector<int32_t> pairs((size_t)8 * m2l_list_entries(p) * m2l_list_width(p));
    if (!build_m2l_list(p, op->offs.vec.data(), op->offs.il.data(), pairs.data())) {
        msg = "fmm_plan: interaction list does not fold into the expected entries";
        return FMM_ERR_INVALID;
    }
    const std::vector<double> zeros((size_t)Kp, 0.0);
    const int nrow = 16 * m2l_row_blocks(p);
    std::vector<int32_t> rowmap(nrow), rowpos(Kp, -1);
    m2l_row_map(p, rowmap.data());
    for (int i = 0; i < nrow; ++i)
        if (rowmap[i] >= 0) rowpos[rowmap[i]] = i;
    if (!op->tree32.ensure(ne * sizeof(float)) || !op->tree64.ensure(ne * sizeof(double)) ||
        !op->il.ensure(sizeof(int32_t) * 8 * kILSize) || !op->offv.ensure(sizeof(int32_t) * 3 * kNumOffsets) ||
        !op->pairs.ensure(sizeof(int32_t) * pairs.size()) || !op->rowmap.ensure(sizeof(int32_t) * nrow) ||
        !op->rowpos.ensure(sizeof(int32_t) * Kp) || !op->zeros.ensure(sizeof(double) * Kp)) {
        msg = "fmm_plan: device allocation";
        return FMM_ERR_NOMEM;
    }
    if (hipMemcpy(op->tree32.ptr, s32.data(), ne * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(op->tree64.ptr, s64.data(), ne * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(op->il.ptr, op->offs.il.data(), sizeof(int32_t) * 8 * kILSize, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(op->offv.ptr, op->offs.vec.data(), sizeof(int32_t) * 3 * kNumOffsets, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(op->pairs.ptr, pairs.data(), sizeof(int32_t) * pairs.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(op->rowmap.ptr, rowmap.data(), sizeof(int32_t) * nrow, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(op->rowpos.ptr, rowpos.data(), sizeof(int32_t) * Kp, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(op->zeros.ptr, zeros.data(), sizeof(double) * Kp, hipMemcpyHostToDevice) != hipSuccess) {
        msg = "fmm_plan: upload failed";
        return FMM_ERR_DEVICE;
    }
    out = op;
    return FMM_OK;
}

static fmm_status upload_lattice(fmm_plan_t pl) {
    const int K = pl->K;
    pl->T.assign((size_t)(2 * pl->p + 1) * (2 * pl->p + 1), cplx(0.0));
    lattice_tensor(2 * pl->p, pl->kappa * pl->box, pl->T.data());
    std::vector<double> A((size_t)K * K);
    build_lattice_operator(pl->p, pl->T.data(), A.data());
    pl->t00 = A[0];
    A[0] = 0.0;
    pl->latT.assign((size_t)K * K, 0.0);
    transpose_into(A.data(), K, pl->latT.data());
    if (!pl->lat.ensure(sizeof(double) * K * K)) return fail(pl, FMM_ERR_NOMEM, "lattice operator allocation");
    HIPCHK(pl, hipMemcpy(pl->lat.ptr, pl->latT.data(), sizeof(double) * K * K, hipMemcpyHostToDevice),
           "lattice upload");
    return FMM_OK;
}

// Levels 1..top_fp64_levels(pl) of the tree run in FP64 in every mode.  At
// shallow levels the cells are large and their M2L sums add big, nearly
// cancelling monopole terms; in FP32 that cancellation leaves an error of a
// few 1e-6 in every atom's potential (measured on the 1M-atom box), so the
// top of the tree -- a few hundred cells -- stays in FP64, as does level 0.
static int top_fp64_levels(fmm_plan_t pl) {
    if (pl->prec == FMM_FP64) return pl->levels;
    return std::min(pl->levels - 1, pl->top_fp64);
}

// M2L levels 1..upper_m2l_levels(pl) run on the plan's second side stream,
// concurrently with the two finest levels on the plan stream (they read
// different multipoles and write different locals; each stream has its own
// split-K and sign-flip scratch).  They are the FP64 top of the tree in mixed
// mode: small launches that leave most of the chip idle when run alone.
static int upper_m2l_levels(fmm_plan_t pl) {
    return std::max(0, std::min(top_fp64_levels(pl), pl->levels - 2));
}

// The M2L operator sets the plan's current mode needs; want64: the FP64
// operators whatever the precision (sparse solute pass).
struct OpNeeds {
    bool alias, f64, f32, bf, f16;
};
static OpNeeds m2l_needs(fmm_plan_t pl, bool want64) {
    OpNeeds n;
    n.alias = top_fp64_levels(pl) > 0 || want64;
    n.f64 = n.alias || want64;
    n.f32 = pl->prec == FMM_MIXED;
    n.bf = pl->prec == FMM_MIXED_BF16_M2L;
    n.f16 = pl->prec == FMM_MIXED_SPLIT16_M2L;
    return n;
}
static bool m2l_ops_ready(fmm_plan_t pl, bool want64) {
    const OpNeeds n = m2l_needs(pl, want64);
    return (!n.f64 || pl->op->ops64.ptr) && (!n.alias || pl->op->alias_ops[0].ptr) && (!n.f32 || pl->op->ops32.ptr) &&
           (!n.bf || pl->op->opsbf.ptr) && (!n.f16 || pl->op->ops16.ptr);
}

static fmm_status ensure_m2l_ops(fmm_plan_t pl, bool want64 = false) {
    if (m2l_ops_ready(pl, want64)) return FMM_OK;
    const OpNeeds nd = m2l_needs(pl, want64);
    const bool needalias = nd.alias, need64 = nd.f64, need32 = nd.f32, needbf = nd.bf, need16 = nd.f16;
    std::vector<double> rm;
    build_m2l_all(pl->p, pl->op->offs, rm);
    const size_t ne = m2l_ops_elems<float>(pl->p);
    if (need16 && !pl->op->ops16.ptr) {
        const size_t nh = m2l_split16_ops_elems(pl->p);
        std::vector<uint16_t> sw(nh);
        std::vector<float> sc((size_t)2 * pl->Kp);
        swizzle_m2l_ops_split16(pl->p, rm.data(), sw.data(), sc.data(), sc.data() + pl->Kp);
        if (!pl->op->ops16.ensure(nh * sizeof(uint16_t)) || !pl->op->scale16.ensure(sc.size() * sizeof(float)))
            return fail(pl, FMM_ERR_NOMEM, "M2L operator allocation");
        HIPCHK(pl, hipMemcpy(pl->op->ops16.ptr, sw.data(), nh * sizeof(uint16_t), hipMemcpyHostToDevice), "M2L upload");
        HIPCHK(pl, hipMemcpy(pl->op->scale16.ptr, sc.data(), sc.size() * sizeof(float), hipMemcpyHostToDevice),
               "M2L upload");
    }
    if (needbf && !pl->op->opsbf.ptr) {
        const size_t nb = m2l_bf16_ops_elems(pl->p);
        std::vector<uint16_t> sw(nb);
        swizzle_m2l_ops_bf16(pl->p, rm.data(), sw.data());
        if (!pl->op->opsbf.ensure(nb * sizeof(uint16_t))) return fail(pl, FMM_ERR_NOMEM, "M2L operator allocation");
        HIPCHK(pl, hipMemcpy(pl->op->opsbf.ptr, sw.data(), nb * sizeof(uint16_t), hipMemcpyHostToDevice), "M2L upload");
    }
    if (needalias && !pl->op->alias_ops[0].ptr) {
        // On a grid of n <= 4 cells per axis the 875 offsets t of a parity
        // class reach only n^3 distinct source cells (t modulo n), so
        //   sum_t O_t M(c + t) = sum_d (sum_{t = d mod n} O_t) M(c + d):
        // the same sum, reassociated, with n^3 instead of 875 products.
        const int K = pl->K;
        for (int lv = 1; lv <= 2; ++lv) {
            const int n = 1 << lv, n3 = n * n * n;
            std::vector<double> comb((size_t)8 * n3 * K * K, 0.0);
            std::vector<int32_t> il(8 * n3), off(3 * 8 * n3);
            for (int par = 0; par < 8; ++par) {
                for (int k = 0; k < n3; ++k) {
                    il[par * n3 + k] = par * n3 + k;
                    off[3 * (par * n3 + k) + 0] = k / (n * n);
                    off[3 * (par * n3 + k) + 1] = (k / n) % n;
                    off[3 * (par * n3 + k) + 2] = k % n;
                }
                for (int t = 0; t < kILSize; ++t) {
                    const int oid = pl->op->offs.il[par * kILSize + t];
                    int d[3];
                    for (int a = 0; a < 3; ++a) d[a] = ((pl->op->offs.vec[3 * oid + a] % n) + n) % n;
                    const int k = (d[0] * n + d[1]) * n + d[2];
                    double *dst = comb.data() + (size_t)(par * n3 + k) * K * K;
                    const double *src = rm.data() + (size_t)oid * K * K;
                    for (size_t e = 0; e < (size_t)K * K; ++e) dst[e] += src[e];
                }
            }
            const size_t ne = (size_t)8 * n3 * pl->Kp * pl->Kp;
            std::vector<double> sw(ne);
            swizzle_ops<double>(pl->p, 8 * n3, comb.data(), sw.data());
            OpSet &o = *pl->op;
            if (!o.alias_ops[lv - 1].ensure(ne * sizeof(double)) || !o.alias_il[lv - 1].ensure(il.size() * 4) ||
                !o.alias_off[lv - 1].ensure(off.size() * 4))
                return fail(pl, FMM_ERR_NOMEM, "M2L operator allocation");
            HIPCHK(pl, hipMemcpy(o.alias_ops[lv - 1].ptr, sw.data(), ne * sizeof(double), hipMemcpyHostToDevice),
                   "M2L upload");
            HIPCHK(pl, hipMemcpy(o.alias_il[lv - 1].ptr, il.data(), il.size() * 4, hipMemcpyHostToDevice), "M2L upload");
            HIPCHK(pl, hipMemcpy(o.alias_off[lv - 1].ptr, off.data(), off.size() * 4, hipMemcpyHostToDevice),
                   "M2L upload");
        }
    }
    if (need64 && !pl->op->ops64.ptr) {
        std::vector<double> sw(ne);
        swizzle_m2l_ops<double>(pl->p, rm.data(), sw.data());
        if (!pl->op->ops64.ensure(ne * sizeof(double))) return fail(pl, FMM_ERR_NOMEM, "M2L operator allocation");
        HIPCHK(pl, hipMemcpy(pl->op->ops64.ptr, sw.data(), ne * sizeof(double), hipMemcpyHostToDevice), "M2L upload");
    }
    if (need32 && !pl->op->ops32.ptr) {
        std::vector<float> sw(ne);
        swizzle_m2l_ops<float>(pl->p, rm.data(), sw.data());
        if (!pl->op->ops32.ensure(ne * sizeof(float))) return fail(pl, FMM_ERR_NOMEM, "M2L operator allocation");
        HIPCHK(pl, hipMemcpy(pl->op->ops32.ptr, sw.data(), ne * sizeof(float), hipMemcpyHostToDevice), "M2L upload");
    }
    return FMM_OK;
}

static fmm_status ensure_side_streams(fmm_plan_t pl);

// member: a box of a batch plan (or an autotuning candidate for one), which
// never forks and so gets no side streams
static fmm_status plan_create(double box, int levels, int p, const std::shared_ptr<OpSet> &shared, bool member,
                              fmm_plan_t *out) {
    *out = nullptr;
    if (!(box > 0.0) || !std::isfinite(box)) return fail(nullptr, FMM_ERR_INVALID, "fmm_plan: box must be finite and > 0");
    if (levels < 1 || levels > kMaxLevels) return fail(nullptr, FMM_ERR_INVALID, "fmm_plan: levels must be in [1, 10]");
    if (p < 0 || p > kMaxP) return fail(nullptr, FMM_ERR_INVALID, "fmm_plan: p must be in [0, 20]");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(nullptr, FMM_ERR_DEVICE, "fmm_plan: no HIP device available");
    fmm_plan_t pl = new (std::nothrow) struct fmm_plan;
    if (!pl) return fail(nullptr, FMM_ERR_NOMEM, "fmm_plan: host allocation");
    pl->box = box;
    pl->levels = levels;
    pl->p = p;
    pl->K = num_coeffs(p);
    pl->Kp = padded_coeffs(p);
    pl->kappa = 3.0 / box;
    if (hipGetDevice(&pl->device) != hipSuccess) {
        delete pl;
        return fail(nullptr, FMM_ERR_DEVICE, "fmm_plan: hipGetDevice failed");
    }
    fmm_status st = FMM_OK;
    auto bail = [&](fmm_status s) {
        g_plan_error = pl->err;
        fmm_destroy(pl);
        return s;
    };
    scratch_setup(pl->device);
    if (pl->device < 64 && !rec_uploaded[pl->device]) {
        RecTables t;
        build_rec_tables(&t);
        hipError_t e = upload_rec_tables(t);
        if (e != hipSuccess) { hip_fail(pl, e, "recurrence tables"); return bail(FMM_ERR_DEVICE); }
        rec_uploaded[pl->device] = true;
    }
    if (shared) {
        pl->op = shared;
    } else {
        std::string msg;
        fmm_status os = make_opset(p, pl->op, msg);
        if (os != FMM_OK) {
            fail(pl, os, msg);
            return bail(os);
        }
    }
    if ((st = upload_lattice(pl)) != FMM_OK) return bail(st);
    if (hipEventCreateWithFlags(&pl->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&pl->ev_join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&pl->ev_up_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&pl->ev_up_join, hipEventDisableTiming) != hipSuccess) {
        fail(pl, FMM_ERR_DEVICE, "fmm_plan: stream or event creation failed");
        return bail(FMM_ERR_DEVICE);
    }
    if (hipHostMalloc((void **)&pl->h_scalars, sizeof(double) * kScalars, hipHostMallocDefault) != hipSuccess) {
        pl->h_scalars = nullptr;
        fail(pl, FMM_ERR_NOMEM, "fmm_plan: pinned host allocation");
        return bail(FMM_ERR_NOMEM);
    }
    pl->in_batch = member;
    // A single-box plan forks the near field and the upper tree onto two
    // streams of its own: they are made here, with the plan, so that no
    // evaluation (captured into a graph or not) ever creates a stream.
    if (!member && (st = ensure_side_streams(pl)) != FMM_OK) return bail(st);
    *out = pl;
    return FMM_OK;
}

extern "C" fmm_status fmm_plan(double box, int levels, int p, fmm_plan_t *out) {
    if (!out) return fail(nullptr, FMM_ERR_INVALID, "fmm_plan: out is NULL");
    fmm_status st = plan_create(box, levels, p, nullptr, false, out);
    if (st != FMM_OK) return st;
    // the operators of the default precision are uploaded with the plan
    // (fmm_plan_config and fmm_plan_tuning add what a new mode needs), so an
    // evaluation allocates only its per-call workspace
    if ((st = ensure_m2l_ops(*out, false)) != FMM_OK) {
        g_plan_error = (*out)->err;
        fmm_destroy(*out);
        *out = nullptr;
    }
    return st;
}

extern "C" fmm_status fmm_plan_config(fmm_plan_t pl, int precision, double kappa, void *hip_stream) {
    if (!pl) return fail(nullptr, FMM_ERR_INVALID, "fmm_plan_config: plan is NULL");
    if (precision != FMM_FP64 && precision != FMM_MIXED && precision != FMM_MIXED_BF16_M2L &&
        precision != FMM_MIXED_SPLIT16_M2L)
        return fail(pl, FMM_ERR_INVALID, "fmm_plan_config: unknown precision");
    if (!std::isfinite(kappa)) return fail(pl, FMM_ERR_INVALID, "fmm_plan_config: kappa must be finite");
    if (pl->is_batch) {
        if (kappa != 0.0) return fail(pl, FMM_ERR_INVALID, "fmm_plan_config: a batch plan takes kappa = 0 (3/b per box)");
        pl->prec = precision;
        pl->stream = hip_stream ? (hipStream_t)hip_stream : pl->own_stream;
        pl->batch_state = false;
        for (fmm_plan_t b : pl->sub) {
            b->prec = precision;
            b->have_state = false;
        }
        batch_drop_graphs(pl);
        return FMM_OK;
    }
    pl->prec = precision;
    pl->stream = (hipStream_t)hip_stream;
    pl->have_state = false;
    if (kappa > 0.0 && kappa != pl->kappa) {
        pl->kappa = kappa;
        fmm_status st = upload_lattice(pl);
        if (st != FMM_OK) return st;
    }
    HIPCHK(pl, hipSetDevice(pl->device), "hipSetDevice");
    return ensure_m2l_ops(pl, false);
}

extern "C" fmm_status fmm_plan_tuning(fmm_plan_t pl, int fp64_levels, int p2p_groups) {
    if (!pl) return fail(nullptr, FMM_ERR_INVALID, "fmm_plan_tuning: plan is NULL");
    if (fp64_levels < -1 || fp64_levels > kMaxLevels)
        return fail(pl, FMM_ERR_INVALID, "fmm_plan_tuning: fp64_levels must be in [-1, 10]");
    if (p2p_groups != -1 && !valid_p2p_groups(p2p_groups))
        return fail(pl, FMM_ERR_INVALID, "fmm_plan_tuning: p2p_groups must be -1, 0, 1, 2, 4, 8 or 16");
    auto set = [&](fmm_plan_t b) {
        if (fp64_levels >= 0) b->top_fp64 = fp64_levels;
        if (p2p_groups >= 0) b->p2p_g = p2p_groups;
        b->have_state = false;
    };
    set(pl);
    for (fmm_plan_t b : pl->sub) set(b);
    if (pl->is_batch) {
        pl->batch_state = false;
        batch_drop_graphs(pl);
        return FMM_OK;
    }
    HIPCHK(pl, hipSetDevice(pl->device), "hipSetDevice");
    return ensure_m2l_ops(pl, false);
}

extern "C" fmm_status fmm_plan_info(fmm_plan_t pl, int64_t *info, int n) {
    if (!pl) return fail(nullptr, FMM_ERR_INVALID, "fmm_plan_info: plan is NULL");
    if (n < 0 || (n > 0 && !info)) return fail(pl, FMM_ERR_INVALID, "fmm_plan_info: bad info array");
    // the finest level's M2L in the plan's mode: the folded list of the FP32 /
    // FP64 kernels, the plain list of the BF16 kernel, and for the split
    // operands whichever of the two that order takes
    const bool plain = pl->prec == FMM_MIXED_BF16_M2L ||
                       (pl->prec == FMM_MIXED_SPLIT16_M2L && !m2l_split16_folded(pl->p));
    int64_t launches = m2l_launches(pl->p, pl->prec == FMM_FP64);
    if (pl->prec == FMM_MIXED_SPLIT16_M2L) launches = m2l_split16_launches(pl->p);
    if (pl->prec == FMM_MIXED_BF16_M2L) launches = 1;
    // rows run per entry: the plain split-FP16 kernel gives each of its four
    // wavefronts an equal number of row blocks per group (m2l_split16_plain_groups)
    int64_t rows = plain ? pl->Kp : 16 * (int64_t)m2l_row_blocks(pl->p);
    if (pl->prec == FMM_MIXED_SPLIT16_M2L && plain) {
        RowGroup grp[kMaxRowGroups];
        const int ng = m2l_split16_plain_groups(pl->Kp / 16, grp);
        rows = 0;
        for (int i = 0; i < ng; ++i) rows += 64 * (int64_t)((grp[i].nrb + 3) / 4);
    }
    const int64_t v[FMM_INFO_COUNT] = {pl->is_batch ? 0 : pl->levels, pl->p, pl->K, pl->Kp, pl->prec,
                                       plain ? 0 : m2l_scheme(pl->p), plain ? kILSize : m2l_list_entries(pl->p),
                                       launches, pl->is_batch ? pl->top_fp64 : top_fp64_levels(pl), pl->p2p_g,
                                       rows};
    for (int i = 0; i < n && i < FMM_INFO_COUNT; ++i) info[i] = v[i];
    return FMM_OK;
}

extern "C" fmm_status fmm_plan_options(fmm_plan_t pl, int boundary, int uv_scheme) {
    if (!pl) return fail(nullptr, FMM_ERR_INVALID, "fmm_plan_options: plan is NULL");
    if (boundary != FMM_BOUNDARY_CONDUCTING && boundary != FMM_BOUNDARY_VACUUM)
        return fail(pl, FMM_ERR_INVALID, "fmm_plan_options: unknown boundary");
    if (uv_scheme < 0 || uv_scheme > (FMM_UV_SPARSE | FMM_UV_SWAP))
        return fail(pl, FMM_ERR_INVALID, "fmm_plan_options: unknown uv_scheme");
    const bool changed = boundary != pl->boundary;
    pl->boundary = boundary;
    pl->uv_scheme = uv_scheme;
    if (pl->is_batch) {
        if (changed) pl->batch_state = false;
        for (fmm_plan_t b : pl->sub) {
            b->boundary = boundary;
            b->uv_scheme = uv_scheme;
            if (changed) b->have_state = false;
        }
    } else if (changed) {
        pl->have_state = false;
    }
    return FMM_OK;
}

// ---------------------------------------------------------------------------
// Evaluation
// ---------------------------------------------------------------------------
// The per-call workspace, as (buffer, bytes, used by fmm_energy_forces):
// the tree part depends on the plan only, the atom part on n.
struct WsItem {
    DeviceBuf *buf;
    size_t bytes;
    bool eval;  // needed by an energy / forces evaluation (else only by the solute-solvent pass)
};
static void tree_layout(fmm_plan_t pl, std::vector<WsItem> &v) {
    const int64_t nleaf = level_cells(pl->levels);
    const int64_t cells = level_offset(pl->levels + 1);
    const size_t tb = sizeof(double) * (size_t)cells * pl->Kp;
    // M2L scratch of the plan stream (any level) and of the upper-level side
    // stream.  Sized for the largest need of every precision and tuning the
    // plan can be switched to without a new plan: the side stream takes at
    // most levels 1 .. levels - 2 (upper_m2l_levels).
    size_t part = 8, part_up = 8;
    for (int l = 1; l <= pl->levels; ++l) {
        const size_t b = m2l_partial_bytes(l, pl->p, kILSize, sizeof(double));
        part = std::max(part, b);
        if (l <= pl->levels - 2) part_up = std::max(part_up, b);
    }
    const int lup_max = std::max(0, pl->levels - 2);
    v.push_back({&pl->Mlev, tb, true});
    v.push_back({&pl->Llev, tb, true});
    v.push_back({&pl->M0, sizeof(double) * pl->Kp, true});
    v.push_back({&pl->L0, sizeof(double) * pl->Kp, true});
    v.push_back({&pl->mflip, m2l_flip_bytes(pl->levels, pl->p, sizeof(double)), true});
    v.push_back({&pl->m2l_part, part, true});
    v.push_back({&pl->mflip_up, lup_max > 0 ? m2l_flip_bytes(lup_max, pl->p, sizeof(double)) : 8, true});
    v.push_back({&pl->m2l_part_up, part_up, true});
    v.push_back({&pl->count, sizeof(uint32_t) * nleaf, true});
    v.push_back({&pl->cursor, sizeof(uint32_t) * nleaf, true});
    v.push_back({&pl->start, sizeof(int32_t) * (nleaf + 1), true});
    v.push_back({&pl->pstart, sizeof(int32_t) * (nleaf + 1), true});
    v.push_back({&pl->scan, sizeof(int32_t) * scan_scratch_len(nleaf), true});
    v.push_back({&pl->scalars, sizeof(double) * kScalars, true});
    v.push_back({&pl->flag, sizeof(int) * 4, true});
    v.push_back({&pl->partials, sizeof(double) * 2 * 16 * 1024, true});
    v.push_back({&pl->sflag, sizeof(uint32_t) * (size_t)(1 + cells), false});
}
static void atom_layout(fmm_plan_t pl, int64_t n, std::vector<WsItem> &v) {
    const int64_t nleaf = level_cells(pl->levels);
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    v.push_back({&pl->key, sizeof(uint32_t) * nn, true});
    v.push_back({&pl->perm, sizeof(int32_t) * nn, true});
    v.push_back({&pl->xq, sizeof(double) * 4 * nn, true});
    v.push_back({&pl->xs, sizeof(double) * 4 * nn, true});
    v.push_back({&pl->xqp, sizeof(double) * 4 * (nn + (size_t)kMaxP2PGroups * nleaf), true});
    v.push_back({&pl->phi_nf, sizeof(double) * nn, true});
    v.push_back({&pl->field_nf, sizeof(double) * 3 * nn, true});
    v.push_back({&pl->phi_ff, sizeof(double) * nn, true});
    v.push_back({&pl->field_ff, sizeof(double) * 3 * nn, true});
    v.push_back({&pl->xq_u, sizeof(double) * 4 * nn, false});
    v.push_back({&pl->phi_u, sizeof(double) * nn, false});
    v.push_back({&pl->field_u, sizeof(double) * 3 * nn, false});
    v.push_back({&pl->nfuv, sizeof(double) * nn, false});
    v.push_back({&pl->mask_sw, nn, false});
    v.push_back({&pl->mask_s, nn, false});
    v.push_back({&pl->nfsc, sizeof(double) * nn, false});
    v.push_back({&pl->nfdl, sizeof(double) * nn, false});
}

static fmm_status ensure_workspace(fmm_plan_t pl, int64_t n) {
    std::vector<WsItem> v;
    if (!pl->tree_ready) {
        tree_layout(pl, v);
        for (const WsItem &w : v)
            if (!w.buf->ensure(w.bytes)) return fail(pl, FMM_ERR_NOMEM, "tree workspace allocation");
        pl->tree_ready = true;
    }
    if (n > pl->cap_n) {
        v.clear();
        atom_layout(pl, n, v);
        for (const WsItem &w : v)
            if (!w.buf->ensure(w.bytes)) return fail(pl, FMM_ERR_NOMEM, "per-atom workspace allocation");
        pl->cap_n = n;
    }
    return FMM_OK;
}

// a1 + a2: wrap, bin, Morton key, stable sort, leaf ranges.
static fmm_status sort_atoms(fmm_plan_t pl, int64_t n, const double *pos, const double *q) {
    hipStream_t s = pl->stream;
    const int64_t nleaf = level_cells(pl->levels);
    stage_begin(pl, FMM_STAGE_TOTAL);
    stage_begin(pl, FMM_STAGE_SORT);
    HIPCHK(pl, launch_fill_u32(pl->count.as<uint32_t>(), 0u, nleaf, s), "fill");
    HIPCHK(pl, launch_fill_u32(pl->cursor.as<uint32_t>(), 0u, nleaf, s), "fill");
    HIPCHK(pl, launch_fill_u32(pl->flag.as<uint32_t>(), 0u, 4, s), "fill");
    HIPCHK(pl, launch_bin(n, pos, q, pl->box, pl->levels, pl->key.as<uint32_t>(), pl->count.as<uint32_t>(),
                          pl->flag.as<int>(), s), "bin");
    HIPCHK(pl, launch_scan(pl->count.as<uint32_t>(), pl->start.as<int32_t>(), nleaf, pl->scan.as<int32_t>(),
                           scan_scratch_len(nleaf), s), "scan");
    HIPCHK(pl, launch_scatter(n, pl->key.as<uint32_t>(), pl->start.as<int32_t>(), pl->cursor.as<uint32_t>(),
                              pl->perm.as<int32_t>(), s), "scatter");
    HIPCHK(pl, launch_cell_sort(nleaf, pl->start.as<int32_t>(), pl->perm.as<int32_t>(), s), "cell sort");
    stage_end(pl, FMM_STAGE_SORT);
    return FMM_OK;
}

// a3 - a8 on the repacked atoms xq: far-field potential and field per sorted
// atom.  Leaf level in the mode's type T; levels 1..top in FP64; level 0 FP64.
// The two side streams of a single-box plan, created with the plan (an
// evaluation never creates a stream, so none is made while a graph is being
// captured).  Sub-plans of a batch never fork and create none: every stream
// takes one of the device's few hardware queues in turn, and unused streams
// created beside the batch's per-box streams pushed several boxes onto one
// queue (32-window batch: energies and forces 10.6 -> 13.8 ms).
static fmm_status ensure_side_streams(fmm_plan_t pl) {
    if (!pl->side && hipStreamCreateWithFlags(&pl->side, hipStreamNonBlocking) != hipSuccess) {
        pl->side = nullptr;
        return fail(pl, FMM_ERR_DEVICE, "side stream creation failed");
    }
    if (!pl->side_up && hipStreamCreateWithFlags(&pl->side_up, hipStreamNonBlocking) != hipSuccess) {
        pl->side_up = nullptr;
        return fail(pl, FMM_ERR_DEVICE, "side stream creation failed");
    }
    return FMM_OK;
}

template <typename T>
static fmm_status far_field(fmm_plan_t pl, int64_t n, const void *xq, double *phi, T *field) {
    hipStream_t s = pl->stream;
    const int L = pl->levels, p = pl->p, Kp = pl->Kp;
    const int top = top_fp64_levels(pl);
    const double h_leaf = pl->box / (double)(1 << L);
    // level arrays hold 8-byte slots, so a level may be read as T or double
    auto at = [&](const DeviceBuf &b, int l) { return (char *)b.ptr + (size_t)level_offset(l) * Kp * sizeof(double); };
    auto MT = [&](int l) { return reinterpret_cast<T *>(at(pl->Mlev, l)); };
    auto LT = [&](int l) { return reinterpret_cast<T *>(at(pl->Llev, l)); };
    auto MD = [&](int l) { return reinterpret_cast<double *>(at(pl->Mlev, l)); };
    auto LD = [&](int l) { return reinterpret_cast<double *>(at(pl->Llev, l)); };
    // octant operators: M2M block first, L2L block second, in FP32 and FP64
    const size_t blk = (size_t)8 * Kp * Kp;
    const void *m2m32 = pl->op->tree32.as<float>(), *l2l32 = pl->op->tree32.as<float>() + blk;
    const void *m2m64 = pl->op->tree64.as<double>(), *l2l64 = pl->op->tree64.as<double>() + blk;
    auto m2m_ops = [&](bool fp64) { return fp64 ? m2m64 : m2m32; };
    auto l2l_ops = [&](bool fp64) { return fp64 ? l2l64 : l2l32; };
    constexpr bool TD = sizeof(T) == 8;
    stage_begin(pl, FMM_STAGE_P2M);
    HIPCHK(pl, launch_p2m<T>(level_cells(L), xq, pl->start.as<int32_t>(), MT(L), p, Kp, 1.0 / h_leaf, s), "P2M");
    stage_end(pl, FMM_STAGE_P2M);
    // Levels 1..lup (the upper tree: M2M, the level-0 lattice operator, M2L)
    // run on the second side stream once the M2M has produced level lup + 1,
    // beside the M2L of the two finest levels on the plan stream (not inside a
    // batch, whose boxes already run as parallel graph branches).  The upper
    // tree's small launches wait behind the near field for CU slots; off the
    // plan stream they no longer hold back the finest levels.
    const int lup = pl->in_batch ? 0 : upper_m2l_levels(pl);
    if (lup > 0 && !pl->side_up) return fail(pl, FMM_ERR_STATE, "plan has no side stream for the upper tree");
    hipStream_t su = lup > 0 ? pl->side_up : s;
    auto m2m = [&](int l, hipStream_t ms) {
        const int64_t nc = level_cells(l);
        if (l > top) return launch_m2m_mfma<T, T>(nc, MT(l + 1), MT(l), m2m_ops(TD), p, Kp, ms);
        if (l + 1 > top) return launch_m2m_mfma<T, double>(nc, MT(l + 1), MD(l), m2m_ops(true), p, Kp, ms);
        return launch_m2m_mfma<double, double>(nc, MD(l + 1), MD(l), m2m_ops(true), p, Kp, ms);
    };
    stage_begin(pl, FMM_STAGE_M2M);
    for (int l = L - 1; l > lup; --l) HIPCHK(pl, m2m(l, s), "M2M");
    if (lup > 0) {
        HIPCHK(pl, hipEventRecord(pl->ev_up_fork, s), "event record");
        HIPCHK(pl, hipStreamWaitEvent(su, pl->ev_up_fork, 0), "stream wait");
    }
    for (int l = lup; l >= 1; --l) HIPCHK(pl, m2m(l, su), "M2M");
    HIPCHK(pl, (top >= 1 ? launch_m2m_mfma<double, double>(1, MD(1), pl->M0.as<double>(), m2m_ops(true), p, Kp, su)
                         : launch_m2m_mfma<T, double>(1, MT(1), pl->M0.as<double>(), m2m_ops(true), p, Kp, su)),
           "M2M");
    stage_end(pl, FMM_STAGE_M2M, su);
    stage_begin(pl, FMM_STAGE_LATTICE, su);
    HIPCHK(pl, launch_lattice(pl->M0.as<double>(), pl->L0.as<double>(), pl->lat.as<double>(), p, Kp, su), "lattice");
    stage_end(pl, FMM_STAGE_LATTICE, su);
    stage_begin(pl, FMM_STAGE_M2L);
    for (int l = 1; l <= L; ++l) {
        if (l == L) stage_begin(pl, FMM_STAGE_M2L_LEAF);
        const bool up = l <= lup;
        hipStream_t ls = up ? su : s;
        DeviceBuf &part = up ? pl->m2l_part_up : pl->m2l_part;
        DeviceBuf &flip = up ? pl->mflip_up : pl->mflip;
        hipError_t e;
        const OpSet &o = *pl->op;
        if (l <= top && l <= 2)
            e = launch_m2l<double>(l, o.alias_ops[l - 1].as<double>(), o.alias_il[l - 1].as<int32_t>(),
                                   o.alias_off[l - 1].as<int32_t>(), nullptr, MD(l), nullptr, 0, nullptr, LD(l),
                                   part.as<double>(), part.bytes, p, Kp, ls, 1 << (3 * l));
        else if (l <= top)
            e = launch_m2l<double>(l, o.ops64.as<double>(), o.pairs.as<int32_t>(), o.offv.as<int32_t>(),
                                   o.rowmap.as<int32_t>(), MD(l), flip.as<double>(), flip.bytes, o.zeros.as<double>(),
                                   LD(l), part.as<double>(), part.bytes, p, Kp, ls);
        else if (!TD && pl->prec == FMM_MIXED_SPLIT16_M2L)
            e = launch_m2l_split16(l, pl->op->ops16.ptr,
                                   m2l_split16_folded(p) ? o.pairs.as<int32_t>() : o.il.as<int32_t>(),
                                   o.offv.as<int32_t>(), o.rowmap.as<int32_t>(),
                                   reinterpret_cast<const float *>(MT(l)), flip.as<float>(), flip.bytes,
                                   o.scale16.as<float>() + Kp, o.scale16.as<float>(), o.zeros.as<float>(),
                                   reinterpret_cast<float *>(LT(l)), part.as<double>(), part.bytes, p, Kp, ls);
        else if (!TD && pl->prec == FMM_MIXED_BF16_M2L)
            e = launch_m2l_bf16(l, pl->op->opsbf.ptr, pl->op->il.as<int32_t>(), pl->op->offv.as<int32_t>(),
                                reinterpret_cast<const float *>(MT(l)), reinterpret_cast<float *>(LT(l)),
                                part.as<float>(), part.bytes, p, Kp, ls);
        else
            e = launch_m2l<T>(l, sizeof(T) == 8 ? (const T *)o.ops64.ptr : (const T *)o.ops32.ptr,
                              o.pairs.as<int32_t>(), o.offv.as<int32_t>(), o.rowmap.as<int32_t>(), MT(l),
                              flip.as<T>(), flip.bytes, o.zeros.as<T>(), LT(l), part.as<T>(), part.bytes, p, Kp, ls);
        if (e == hipErrorInvalidValue)
            return fail(pl, FMM_ERR_DEVICE, "M2L level " + std::to_string(l) +
                                                ": launch shape or scratch capacity rejected by the launcher");
        HIPCHK(pl, e, "M2L");
        if (l == L) stage_end(pl, FMM_STAGE_M2L_LEAF);
    }
    // L2L into level l (from level l - 1; level 1 from the lattice's L0)
    auto l2l = [&](int l, hipStream_t ls) -> hipError_t {
        if (l == 1)
            return top >= 1 ? launch_l2l_mfma<double, double>(1, pl->L0.as<double>(), LD(1), l2l_ops(true), p, Kp, ls)
                            : launch_l2l_mfma<double, T>(1, pl->L0.as<double>(), LT(1), l2l_ops(true), p, Kp, ls);
        const int64_t np = level_cells(l - 1);  // parents
        if (l <= top) return launch_l2l_mfma<double, double>(np, LD(l - 1), LD(l), l2l_ops(true), p, Kp, ls);
        if (l - 1 <= top) return launch_l2l_mfma<double, T>(np, LD(l - 1), LT(l), l2l_ops(true), p, Kp, ls);
        return launch_l2l_mfma<T, T>(np, LT(l - 1), LT(l), l2l_ops(TD), p, Kp, ls);
    };
    // The upper tree's own L2L steps (into levels 1 .. lup, whose M2L ran on
    // the second side stream) follow its M2L there, before the join, so after
    // the leaf M2L the plan stream only pushes down into levels lup + 1 .. L
    // (the L2L stage timing covers those).
    for (int l = 1; l <= lup; ++l) HIPCHK(pl, l2l(l, su), "L2L");
    if (lup > 0) {
        HIPCHK(pl, hipEventRecord(pl->ev_up_join, pl->side_up), "event record");
        HIPCHK(pl, hipStreamWaitEvent(s, pl->ev_up_join, 0), "stream wait");
    }
    stage_end(pl, FMM_STAGE_M2L);
    stage_begin(pl, FMM_STAGE_L2L);
    for (int l = lup + 1; l <= L; ++l) HIPCHK(pl, l2l(l, s), "L2L");
    stage_end(pl, FMM_STAGE_L2L);
    stage_begin(pl, FMM_STAGE_L2P);
    HIPCHK(pl, launch_l2p<T>(level_cells(L), xq, pl->start.as<int32_t>(), LT(L), p, Kp, h_leaf, phi, field, s, n),
           "L2P");
    stage_end(pl, FMM_STAGE_L2P);
    return FMM_OK;
}

static int p2p_groups(int64_t n, int levels) {
    // 4 groups of 16 target slots fit the 10-40 atom leaves of water boxes at
    // 4-7 A leaf edges best (measured: 30 atoms/leaf G 4 < 2 < 8; 11 atoms/leaf
    // G 4 < 8); sparse leaves take more groups, crowded ones fewer
    const double occ = (double)n / (double)level_cells(levels);
    if (occ > 48.0) return 2;
    if (occ > 5.0) return 4;
    if (occ > 2.5) return 8;
    return 16;
}

template <typename T>
static fmm_status run_fields(fmm_plan_t pl, int64_t n, const double *pos, const double *q) {
    hipStream_t s = pl->stream;
    fmm_status st;
    if ((st = sort_atoms(pl, n, pos, q)) != FMM_OK) return st;
    stage_begin(pl, FMM_STAGE_GATHER);
    HIPCHK(pl, launch_gather(n, pl->perm.as<int32_t>(), pos, q, pl->box, pl->levels, pl->prec == FMM_FP64,
                             pl->xq.ptr, pl->xs.as<double>(), s), "gather");
    stage_end(pl, FMM_STAGE_GATHER);
    // The near field depends only on the sorted atoms: it runs on the plan's
    // side stream concurrently with the upward pass and the upper M2L levels,
    // which leave most of the chip idle (measured on the 1M-atom box: forking
    // here saves 0.85 ms per step, forking after M2M none); the main stream
    // joins it before the corrections.  The side stream first builds the near-field
    // copy with leaves padded to a multiple of the P2P group count (the sort's
    // cursor array is free again and holds the padded counts).  Plans of a
    // batch keep the near field on their own stream: a batch is already one
    // parallel graph branch per box, and the nested fork inside a captured
    // graph is not used (one such run ended in a host-side crash).
    const bool fork = !pl->in_batch;
    if (fork && !pl->side) return fail(pl, FMM_ERR_STATE, "plan has no side stream for the near field");
    hipStream_t ns = fork ? pl->side : s;
    auto near_field = [&]() -> fmm_status {
        if (fork) {
            HIPCHK(pl, hipEventRecord(pl->ev_fork, s), "event record");
            HIPCHK(pl, hipStreamWaitEvent(ns, pl->ev_fork, 0), "stream wait");
        }
        const int64_t nleaf = level_cells(pl->levels);
        const int groups = pl->p2p_g ? pl->p2p_g : p2p_groups(n, pl->levels);
        const double h_leaf = pl->box / (double)(1 << pl->levels);
        stage_begin(pl, FMM_STAGE_P2P, ns);
        HIPCHK(pl, launch_pad_counts(nleaf, pl->count.as<uint32_t>(), groups, pl->cursor.as<uint32_t>(), ns), "pad");
        HIPCHK(pl, launch_scan(pl->cursor.as<uint32_t>(), pl->pstart.as<int32_t>(), nleaf, pl->scan.as<int32_t>(),
                               scan_scratch_len(nleaf), ns), "scan");
        HIPCHK(pl, launch_pad_gather(nleaf, pl->start.as<int32_t>(), pl->pstart.as<int32_t>(), pl->prec == FMM_FP64,
                                     pl->xq.ptr, 16.0 * pl->box, pl->xqp.ptr, ns), "pad gather");
        // target chunks of TS = 64 / groups atoms; enough wavefronts per leaf
        // to cover the mean occupancy once, and at least 64k wavefronts
        const double occ = (double)n / (double)nleaf;
        int nsplit = (int)std::ceil(occ / (64.0 / groups));
        while (nsplit < 8 && nleaf * nsplit < 65536) nsplit *= 2;
        nsplit = std::max(1, std::min(nsplit, 8));
        while (nsplit > 1 && nleaf * nsplit >= ((int64_t)1 << 31)) nsplit /= 2;  // wavefront ids stay int
        HIPCHK(pl, launch_p2p<T>(nleaf, pl->levels, pl->xqp.ptr, pl->pstart.as<int32_t>(), pl->start.as<int32_t>(),
                                 h_leaf, pl->phi_nf.as<double>(), pl->field_nf.as<T>(), groups, nsplit, 0,
                                 n + (int64_t)groups * nleaf, ns),
               "P2P");
        stage_end(pl, FMM_STAGE_P2P, ns);
        if (fork) HIPCHK(pl, hipEventRecord(pl->ev_join, ns), "event record");
        return FMM_OK;
    };
    if ((st = near_field()) != FMM_OK) return st;
    if ((st = far_field<T>(pl, n, pl->xq.ptr, pl->phi_ff.as<double>(), pl->field_ff.as<T>())) != FMM_OK) return st;
    if (fork) HIPCHK(pl, hipStreamWaitEvent(s, pl->ev_join, 0), "stream wait");
    return FMM_OK;
}

static fmm_status check_eval_args(fmm_plan_t pl, int64_t n, const double *pos, const double *q) {
    if (!pl) return fail(nullptr, FMM_ERR_INVALID, "plan is NULL");
    if (pl->is_batch) return fail(pl, FMM_ERR_INVALID, "batch plan: use the *_batch calls");
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(pl, FMM_ERR_INVALID, "n must be in [0, 2^31)");
    if (n > 0 && (!pos || !q)) return fail(pl, FMM_ERR_INVALID, "pos and q must be non-NULL when n > 0");
    return FMM_OK;
}

// Device scalars (and the input-check flag) to the pinned host mirror, on the
// plan stream; check_readback runs once that stream has been synchronised.
static fmm_status enqueue_readback(fmm_plan_t pl, int nscalars) {
    hipStream_t s = pl->stream;
    HIPCHK(pl, hipMemcpyAsync(pl->h_scalars, pl->scalars.ptr, sizeof(double) * nscalars, hipMemcpyDeviceToHost, s),
           "readback");
    HIPCHK(pl, hipMemcpyAsync(&pl->h_scalars[kScalars - 1], pl->flag.ptr, sizeof(int), hipMemcpyDeviceToHost, s),
           "readback");
    return FMM_OK;
}
static fmm_status check_readback(fmm_plan_t pl) {
    int flag = 0;
    std::memcpy(&flag, &pl->h_scalars[kScalars - 1], sizeof(int));
    if (flag) return fail(pl, FMM_ERR_INVALID, "non-finite position or charge");
    return FMM_OK;
}
static fmm_status finish_readback(fmm_plan_t pl, int nscalars) {
    fmm_status st = enqueue_readback(pl, nscalars);
    if (st != FMM_OK) return st;
    HIPCHK(pl, hipStreamSynchronize(pl->stream), "synchronize");
    return check_readback(pl);
}

// All device work of one evaluation plus the readback copies, enqueued on the
// plan stream without synchronising (also used under stream capture).
template <typename T>
static fmm_status enqueue_energy_forces(fmm_plan_t pl, int64_t n, const double *pos, const double *q,
                                        double *forces, double *phi) {
    hipStream_t s = pl->stream;
    fmm_status st;
    if ((st = run_fields<T>(pl, n, pos, q)) != FMM_OK) return st;
    const int nb = moments_blocks(n);
    double *sc = pl->scalars.as<double>();
    stage_begin(pl, FMM_STAGE_FINAL);
    HIPCHK(pl, launch_moments(n, pl->xs.as<double>(), pl->perm.as<int32_t>(), nullptr, 0, pl->partials.as<double>(),
                              nb, sc, s), "moments");
    HIPCHK(pl, hipMemcpyAsync(sc + 10, pl->M0.ptr, sizeof(double), hipMemcpyDeviceToDevice, s), "copy");
    HIPCHK(pl, launch_finalize<T>(n, pl->perm.as<int32_t>(), pl->xs.as<double>(), pl->box, pl->kappa,
                                  pl->t00 / pl->box, pl->boundary == FMM_BOUNDARY_VACUUM ? 0.0 : 1.0, sc,
                                  pl->M0.as<double>(), pl->phi_nf.as<double>(),
                                  pl->field_nf.as<T>(), pl->phi_ff.as<double>(), pl->field_ff.as<T>(), forces, phi,
                                  pl->partials.as<double>(), nb, sc + 8, s), "finalize");
    stage_end(pl, FMM_STAGE_FINAL);
    stage_end(pl, FMM_STAGE_TOTAL);
    return enqueue_readback(pl, 11);
}

// after the plan stream has been synchronised
static fmm_status finish_energy(fmm_plan_t pl, double *energy) {
    fmm_status st = check_readback(pl);
    if (st != FMM_OK) return st;
    stage_collect(pl);
    *energy = pl->h_scalars[8];
    pl->last_energy = *energy;
    pl->q_tree = pl->h_scalars[10];
    return FMM_OK;
}

template <typename T>
static fmm_status energy_forces_t(fmm_plan_t pl, int64_t n, const double *pos, const double *q, double *energy,
                                  double *forces, double *phi) {
    fmm_status st = enqueue_energy_forces<T>(pl, n, pos, q, forces, phi);
    if (st != FMM_OK) return st;
    HIPCHK(pl, hipStreamSynchronize(pl->stream), "synchronize");
    return finish_energy(pl, energy);
}

extern "C" fmm_status fmm_energy_forces(fmm_plan_t pl, int64_t n, const double *pos, const double *q,
                                        double *energy, double *forces, double *phi) {
    fmm_status st = check_eval_args(pl, n, pos, q);
    if (st != FMM_OK) return st;
    if (!energy) return fail(pl, FMM_ERR_INVALID, "energy must be non-NULL");
    pl->have_state = false;
    if (n == 0) {
        *energy = 0.0;
        pl->last_energy = 0.0;
        pl->have_state = true;
        pl->n_state = 0;
        return FMM_OK;
    }
    HIPCHK(pl, hipSetDevice(pl->device), "hipSetDevice");
    if ((st = ensure_workspace(pl, n)) != FMM_OK) return st;
    if ((st = ensure_m2l_ops(pl)) != FMM_OK) return st;
    stage_reset(pl);
    st = pl->prec == FMM_FP64 ? energy_forces_t<double>(pl, n, pos, q, energy, forces, phi)
                              : energy_forces_t<float>(pl, n, pos, q, energy, forces, phi);
    if (st == FMM_OK) {
        pl->have_state = true;
        pl->n_state = n;
    }
    return st;
}

// Evaluation on the library's fixed device scratch instead of the plan's own
// workspace: the plan's workspace buffers are pointed at consecutive
// 256-byte-aligned pieces of the scratch for the duration of the call and
// put back on every return path.
struct ScratchViews {
    std::vector<std::pair<DeviceBuf *, DeviceBuf>> saved;
    ~ScratchViews() {
        for (auto &s : saved) *s.first = s.second;
    }
};

extern "C" fmm_status fmm_energy_forces_noalloc(fmm_plan_t pl, int64_t n, const double *pos, const double *q,
                                                double *energy, double *forces, double *phi) {
    fmm_status st = check_eval_args(pl, n, pos, q);
    if (st != FMM_OK) return st;
    if (!energy) return fail(pl, FMM_ERR_INVALID, "energy must be non-NULL");
    pl->have_state = false;
    if (n == 0) {
        *energy = 0.0;
        pl->last_energy = 0.0;
        return FMM_OK;
    }
    HIPCHK(pl, hipSetDevice(pl->device), "hipSetDevice");
    if (pl->device < 0 || pl->device >= 64 || !g_scratch_ptr[pl->device])
        return hip_fail(pl, pl->device >= 0 && pl->device < 64 ? g_scratch_err[pl->device] : hipErrorInvalidDevice,
                        "fmm_energy_forces_noalloc: device address of the scratch array");
    if (!m2l_ops_ready(pl, false))
        return fail(pl, FMM_ERR_STATE, "fmm_energy_forces_noalloc: the operators of the current mode are not on the "
                                       "device (fmm_plan, fmm_plan_config and fmm_plan_tuning upload them)");
    std::vector<WsItem> items;
    tree_layout(pl, items);
    atom_layout(pl, n, items);
    size_t need = 0;
    for (const WsItem &w : items)
        if (w.eval) need = (need + 255) / 256 * 256 + w.bytes;
    if (need > kNoAllocScratchBytes)
        return fail(pl, FMM_ERR_INVALID,
                    "fmm_energy_forces_noalloc: " + std::to_string(n) + " atoms on this plan need " +
                        std::to_string(need) + " bytes of scratch, more than the " +
                        std::to_string(kNoAllocScratchBytes) + " available");
    char *base = static_cast<char *>(g_scratch_ptr[pl->device]);
    ScratchViews views;
    size_t at = 0;
    for (const WsItem &w : items) {
        if (!w.eval) continue;
        at = (at + 255) / 256 * 256;
        views.saved.emplace_back(w.buf, *w.buf);
        w.buf->ptr = base + at;
        w.buf->bytes = w.bytes;
        w.buf->borrowed = true;
        at += w.bytes;
    }
    stage_reset(pl);
    st = pl->prec == FMM_FP64 ? energy_forces_t<double>(pl, n, pos, q, energy, forces, phi)
                              : energy_forces_t<float>(pl, n, pos, q, energy, forces, phi);
    // the sorted atoms live in the shared scratch, which the next call on this
    // device overwrites: no state is kept for fmm_solute_solvent_energy
    pl->have_state = false;
    return st;
}

template <typename T>
static fmm_status parts_t(fmm_plan_t pl, int64_t n, const double *pos, const double *q, double *phi_nf,
                          double *field_nf, double *phi_ff, double *field_ff) {
    hipStream_t s = pl->stream;
    fmm_status st;
    if ((st = run_fields<T>(pl, n, pos, q)) != FMM_OK) return st;
    double *sc = pl->scalars.as<double>();
    HIPCHK(pl, launch_moments(n, pl->xs.as<double>(), pl->perm.as<int32_t>(), nullptr, 0, pl->partials.as<double>(),
                              moments_blocks(n), sc, s), "moments");
    HIPCHK(pl, launch_parts_out<T>(n, pl->perm.as<int32_t>(), pl->phi_nf.as<double>(), pl->field_nf.as<T>(),
                                   pl->M0.as<double>(), 0.0, phi_nf, field_nf, s), "parts");
    // the far field includes the net-charge lattice constant t00 Q_tree / b
    HIPCHK(pl, launch_parts_out<T>(n, pl->perm.as<int32_t>(), pl->phi_ff.as<double>(), pl->field_ff.as<T>(),
                                   pl->M0.as<double>(), pl->t00 / pl->box, phi_ff, field_ff, s), "parts");
    HIPCHK(pl, hipMemcpyAsync(sc + 10, pl->M0.ptr, sizeof(double), hipMemcpyDeviceToDevice, s), "copy");
    if ((st = finish_readback(pl, 11)) != FMM_OK) return st;
    pl->q_tree = pl->h_scalars[10];
    return FMM_OK;
}

extern "C" fmm_status fmm_potential_parts(fmm_plan_t pl, int64_t n, const double *pos, const double *q,
                                          double *phi_nf, double *field_nf, double *phi_ff, double *field_ff) {
    fmm_status st = check_eval_args(pl, n, pos, q);
    if (st != FMM_OK) return st;
    pl->have_state = false;
    if (n == 0) return FMM_OK;
    HIPCHK(pl, hipSetDevice(pl->device), "hipSetDevice");
    if ((st = ensure_workspace(pl, n)) != FMM_OK) return st;
    if ((st = ensure_m2l_ops(pl)) != FMM_OK) return st;
    st = pl->prec == FMM_FP64 ? parts_t<double>(pl, n, pos, q, phi_nf, field_nf, phi_ff, field_ff)
                              : parts_t<float>(pl, n, pos, q, phi_nf, field_nf, phi_ff, field_ff);
    if (st == FMM_OK) {
        pl->have_state = true;
        pl->n_state = n;
    }
    return st;
}

// ---------------------------------------------------------------------------
// The solute-solvent pass (eq. FMMcalc) of one box or of every box of a batch,
// each stage one launch for all boxes (block tables built here).
//   FMM_UV_SPARSE: the far field of the masked charges alone, at the masked
//     atoms alone (phi_u, 0 at the others): the tree of those charges is
//     non-zero only in the cells above the leaves that hold them, and their
//     potential is wanted only in the same leaves, so every stage runs over
//     the flagged cells (all in FP64, in the level arrays of the evaluation,
//     which are free again): the dense algorithm restricted to the cells
//     whose terms are not identically zero.
//   FMM_UV_SYMMETRIC: a dense far-field pass over the masked charges per box
//     (far_field), before the shared stages.
// Shared stages: solute flags in sorted order, near-field u-v pairs, sums.
// ---------------------------------------------------------------------------
enum { kStFill, kStAtom, kStLeaf, kStLat, kStRed, kStOne, kStFixed };  // then M2M steps, then levels

struct UvTables {
    std::vector<UvBox> box;
    int maxL = 0;
    std::vector<int64_t> tab;    // tables of nbox + 1 block starts
    std::vector<int64_t> total;  // blocks of each table
    int ntab() const { return kStFixed + 2 * maxL; }
    int m2m(int step) const { return kStFixed + step - 1; }
    int lvl(int l) const { return kStFixed + maxL + l - 1; }
};

static int64_t uv_blocks(int k, const UvTables &t, const UvBox &b) {
    if (b.n == 0) return 0;
    const int L = b.levels;
    if (k == kStFill) return (1 + level_offset(L + 1) + 255) / 256;
    if (k == kStAtom) return (b.n + 255) / 256;
    if (k == kStLeaf) return level_cells(L);
    if (k == kStLat) return (b.Kp + 63) / 64;
    if (k == kStRed) return moments_blocks(b.n);
    if (k == kStOne) return 1;
    if (k < kStFixed + t.maxL) {
        const int step = k - kStFixed + 1;
        return L >= step ? level_cells(L - step) : 0;
    }
    const int l = k - kStFixed - t.maxL + 1;
    return L >= l ? level_cells(l) : 0;
}

static void uv_build_tables(UvTables &t) {
    const size_t nb = t.box.size();
    t.maxL = 0;
    for (const UvBox &b : t.box)
        if (b.n > 0) t.maxL = std::max(t.maxL, b.levels);
    t.tab.assign((size_t)t.ntab() * (nb + 1), 0);
    t.total.assign(t.ntab(), 0);
    for (int k = 0; k < t.ntab(); ++k) {
        int64_t run = 0;
        for (size_t w = 0; w < nb; ++w) {
            t.tab[(size_t)k * (nb + 1) + w] = run;
            run += uv_blocks(k, t, t.box[w]);
        }
        t.tab[(size_t)k * (nb + 1) + nb] = run;
        t.total[k] = run;
    }
}

// The UvBox entry of plan b (a single-box plan or a box of a batch) for its
// last evaluation; mask: the box's rows of the caller's mask; lam >= 0 with a
// soft-core set: the soft-core sums at lam; sc: the box's scalar block
static UvBox uv_box(fmm_plan_t b, const uint8_t *mask, double lam, double *sc) {
    UvBox u{};
    u.n = b->n_state;
    u.levels = b->levels;
    u.p = b->p;
    u.K = b->K;
    u.Kp = b->Kp;
    u.invert = (b->uv_scheme & FMM_UV_SWAP) ? 1 : 0;
    const bool soft = lam >= 0.0 && b->sc_alpha > 0.0;
    u.soft_c = soft ? b->sc_c : 0;
    u.box = b->box;
    u.h = b->box / (double)(1 << b->levels);
    if (soft) {
        const double sigc = std::pow(b->sc_sigma, (double)b->sc_c);
        u.asc = b->sc_alpha * lam * sigc;
        u.kd = b->sc_alpha * sigc / b->sc_c;
    }
    u.xs = b->xs.as<double>();
    u.xq = b->xq.ptr;
    u.key = b->key.as<uint32_t>();
    u.perm = b->perm.as<int32_t>();
    u.start = b->start.as<int32_t>();
    u.mask = mask;
    u.ms = b->mask_s.as<uint8_t>();
    u.flag = b->sflag.as<uint32_t>();
    u.M = b->Mlev.as<double>();
    u.L = b->Llev.as<double>();
    u.M0 = b->M0.as<double>();
    u.L0 = b->L0.as<double>();
    u.lat = b->lat.as<double>();
    u.phi_uv = b->phi_ff.as<double>();
    u.phi_u = b->phi_u.as<double>();
    u.nfuv = b->nfuv.as<double>();
    u.nfsc = b->nfsc.as<double>();
    u.nfdl = b->nfdl.as<double>();
    u.partials = b->partials.as<double>();
    u.sc = sc;
    return u;
}

// Uploads the tables into owner->uvtab (synchronously, before anything that
// reads them is enqueued or captured; skipped when unchanged).
static fmm_status uv_upload(fmm_plan_t owner, const UvTables &t) {
    const size_t bb = sizeof(UvBox) * t.box.size(), tb = sizeof(int64_t) * t.tab.size();
    std::vector<unsigned char> host(bb + tb);
    std::memcpy(host.data(), t.box.data(), bb);
    std::memcpy(host.data() + bb, t.tab.data(), tb);
    if (host == owner->uvtab_host && owner->uvtab.ptr) return FMM_OK;
    if (!owner->uvtab.ensure(host.size())) return fail(owner, FMM_ERR_NOMEM, "solute-solvent table allocation");
    HIPCHK(owner, hipMemcpy(owner->uvtab.ptr, host.data(), host.size(), hipMemcpyHostToDevice), "table upload");
    owner->uvtab_host.swap(host);
    return FMM_OK;
}

// The shared stages (and, for FMM_UV_SPARSE, the sparse solute tree) of the
// boxes of t, on stream s; ops: the plan's operator set (shared by all boxes)
template <typename T>
static fmm_status enqueue_uv_stages(fmm_plan_t owner, const UvTables &t, bool sparse, const OpSet &ops,
                                    hipStream_t s) {
    const int nb = (int)t.box.size();
    if (t.maxL == 0) return FMM_OK;
    const UvBox *dB = owner->uvtab.as<UvBox>();
    const int64_t *tab0 = reinterpret_cast<const int64_t *>(owner->uvtab.as<unsigned char>() + sizeof(UvBox) * nb);
    auto T_ = [&](int k) { return tab0 + (size_t)k * (nb + 1); };
    const int p = t.box[0].p;
    HIPCHK(owner, launch_uv_mask(dB, nb, T_(kStFill), t.total[kStFill], T_(kStAtom), t.total[kStAtom], s), "mask");
    if (sparse) {
        HIPCHK(owner, launch_uv_p2m(dB, nb, T_(kStLeaf), t.total[kStLeaf], s), "P2M");
        for (int k = 1; k <= t.maxL; ++k)
            HIPCHK(owner, launch_uv_m2m(dB, nb, k, T_(t.m2m(k)), t.total[t.m2m(k)], ops.tree64.ptr, s), "M2M");
        HIPCHK(owner, launch_uv_lattice(dB, nb, T_(kStLat), t.total[kStLat], s), "lattice");
        // levels 1 and 2 with the operators summed over aliased offsets (as
        // the dense pass), where the 875 offsets reach only 8 or 64 source cells
        for (int l = 1; l <= t.maxL; ++l) {
            const bool alias = l <= 2;
            HIPCHK(owner,
                   launch_uv_m2l(dB, nb, l, T_(t.lvl(l)), t.total[t.lvl(l)],
                                 alias ? ops.alias_il[l - 1].as<int32_t>() : ops.il.as<int32_t>(),
                                 alias ? ops.alias_off[l - 1].as<int32_t>() : ops.offv.as<int32_t>(),
                                 alias ? ops.alias_ops[l - 1].as<double>() : ops.ops64.as<double>(),
                                 alias ? nullptr : ops.rowpos.as<int32_t>(), m2l_row_blocks(p),
                                 alias ? 1 << (3 * l) : kILSize, s),
                   "M2L");
        }
        for (int l = 1; l <= t.maxL; ++l)
            HIPCHK(owner, launch_uv_l2l(dB, nb, l, T_(t.lvl(l)), t.total[t.lvl(l)], ops.tree64.ptr, s), "L2L");
        HIPCHK(owner, launch_uv_l2p(dB, nb, T_(kStAtom), t.total[kStAtom], s), "L2P");
    }
    HIPCHK(owner, launch_uv_p2p<T>(dB, nb, T_(kStLeaf), t.total[kStLeaf], s), "P2P uv");
    HIPCHK(owner, launch_uv_sums(dB, nb, T_(kStRed), t.total[kStRed], T_(kStOne), t.total[kStOne], s), "uv sums");
    return FMM_OK;
}

// The dense second pass of FMM_UV_SYMMETRIC for one box, on its stream: the
// far field of the masked charges (the solvent's with FMM_UV_SWAP)
template <typename T>
static fmm_status enqueue_uv_dense(fmm_plan_t pl, const uint8_t *mask) {
    hipStream_t s = pl->stream;
    const int64_t n = pl->n_state;
    if (pl->uv_scheme & FMM_UV_SWAP) {
        HIPCHK(pl, launch_invert_mask(n, mask, pl->mask_sw.as<uint8_t>(), s), "mask");
        mask = pl->mask_sw.as<uint8_t>();
    }
    HIPCHK(pl, launch_mask_charges(n, pl->perm.as<int32_t>(), mask, pl->prec == FMM_FP64, pl->xq.ptr, pl->xq_u.ptr, s),
           "mask charges");
    return far_field<T>(pl, n, pl->xq_u.ptr, pl->phi_u.as<double>(), pl->field_u.as<T>());
}

// lam >= 0 with a soft-core set: also the soft-core near-field sums at lam
template <typename T>
static fmm_status enqueue_solute_solvent(fmm_plan_t pl, const uint8_t *mask, double lam = -1.0) {
    fmm_status st;
    const bool sparse = (pl->uv_scheme & FMM_UV_SPARSE) != 0;
    UvTables t;
    t.box.push_back(uv_box(pl, mask, lam, pl->scalars.as<double>()));
    uv_build_tables(t);
    if ((st = uv_upload(pl, t)) != FMM_OK) return st;
    if (!sparse && (st = enqueue_uv_dense<T>(pl, mask)) != FMM_OK) return st;
    if ((st = enqueue_uv_stages<T>(pl, t, sparse, *pl->op, pl->stream)) != FMM_OK) return st;
    return enqueue_readback(pl, 46);
}

// W_uv from the pass-2 scalars, after the plan stream has been synchronised
static fmm_status finish_solute_solvent(fmm_plan_t pl, double *e_uv) {
    fmm_status st = check_readback(pl);
    if (st != FMM_OK) return st;
    const double *h = pl->h_scalars;
    const double A = h[40], B = h[41], C = h[42], D = h[43];
    pl->uv_d0 = D;
    pl->uv_dsc = h[44];
    pl->uv_dl = h[45];
    const double Qu = h[24], mux = h[25], muy = h[26], muz = h[27], Su = h[28];
    const double Qv = h[32], mvx = h[33], mvy = h[34], mvz = h[35], Sv = h[36];
    const double V = pl->box * pl->box * pl->box;
    // FF cross term.  The net-charge lattice constant enters phi_uv as
    // t00 Q_tree / b and phi_u as t00 Q_u,tree / b (tree monopoles of the two
    // passes); its share of (A - B + C) / 2 is added here in FP64.
    const double qt = pl->q_tree, qut = h[20];
    // one-sided form: sum_u q (phi_uv - phi_u), C unused (phi_u is 0 at v)
    const double w_ff = (pl->uv_scheme & FMM_UV_SPARSE)
                            ? (A - B) + pl->t00 / pl->box * Qu * (qt - qut)
                            : 0.5 * (A - B + C) + 0.5 * pl->t00 / pl->box * (Qu * qt - Qu * qut + Qv * qut);
    // the vacuum boundary's dipole surface term adds (4 pi / 3V) mu_u.mu_v,
    // which cancels the dipole cross part of the background terms
    const double mu_w = pl->boundary == FMM_BOUNDARY_VACUUM ? 0.0 : 1.0;
    const double w_bc = -M_PI * Qu * Qv / (V * pl->kappa * pl->kappa) +
                        (2.0 * M_PI / (3.0 * V)) *
                            (Qu * Sv + Qv * Su - 2.0 * mu_w * (mux * mvx + muy * mvy + muz * mvz));
    *e_uv = w_ff + D + w_bc;
    return FMM_OK;
}

template <typename T>
static fmm_status solute_solvent_t(fmm_plan_t pl, const uint8_t *mask, double lam, double *e_uv) {
    fmm_status st = enqueue_solute_solvent<T>(pl, mask, lam);
    if (st != FMM_OK) return st;
    HIPCHK(pl, hipStreamSynchronize(pl->stream), "synchronize");
    return finish_solute_solvent(pl, e_uv);
}

// e_uv; with lam >= 0 and a soft-core set, also the soft-core near-field sums
// (pl->uv_d0, uv_dsc, uv_dl) at lam
static fmm_status solute_solvent_single(fmm_plan_t pl, const uint8_t *mask, double lam, double *e_uv) {
    if (!pl) return fail(nullptr, FMM_ERR_INVALID, "plan is NULL");
    if (pl->is_batch) return fail(pl, FMM_ERR_INVALID, "batch plan: use fmm_solute_solvent_energy_batch");
    if (!e_uv) return fail(pl, FMM_ERR_INVALID, "e_uv must be non-NULL");
    if (!pl->have_state) return fail(pl, FMM_ERR_STATE, "fmm_solute_solvent_energy needs a preceding fmm_energy_forces");
    pl->uv_d0 = pl->uv_dsc = pl->uv_dl = 0.0;
    if (pl->n_state == 0) { *e_uv = 0.0; return FMM_OK; }
    if (!mask) return fail(pl, FMM_ERR_INVALID, "mask must be non-NULL");
    HIPCHK(pl, hipSetDevice(pl->device), "hipSetDevice");
    fmm_status st = ensure_m2l_ops(pl, (pl->uv_scheme & FMM_UV_SPARSE) != 0);
    if (st != FMM_OK) return st;
    return pl->prec == FMM_FP64 ? solute_solvent_t<double>(pl, mask, lam, e_uv)
                                : solute_solvent_t<float>(pl, mask, lam, e_uv);
}

extern "C" fmm_status fmm_solute_solvent_energy(fmm_plan_t pl, const uint8_t *mask, double *e_uv) {
    return solute_solvent_single(pl, mask, -1.0, e_uv);
}

// eq. Vswucheme: the solute-solvent coupling scaled by (1 - lambda), V = E -
// lambda W.  With the soft-core near field the u-v NF pairs' share (1 -
// lambda) D0 of that is replaced by (1 - lambda) Dsc(lambda).
static void lambda_values(const struct fmm_plan *b, double e, double w, double lam, double *v, double *dv) {
    double vv = e - lam * w, dd = -w;
    if (b->sc_alpha > 0.0) {
        vv += (1.0 - lam) * (b->uv_dsc - b->uv_d0);
        dd += b->uv_d0 - b->uv_dsc + (1.0 - lam) * b->uv_dl;
    }
    if (v) *v = vv;
    if (dv) *dv = dd;
}

static fmm_status check_lambda(fmm_plan_t pl, double lambda) {
    if (!std::isfinite(lambda)) return fail(pl, FMM_ERR_INVALID, "lambda must be finite");
    if (pl->sc_alpha > 0.0 && (lambda < 0.0 || lambda > 1.0))
        return fail(pl, FMM_ERR_INVALID, "lambda must be in [0, 1] with a soft-core near field");
    return FMM_OK;
}

extern "C" fmm_status fmm_lambda_energy(fmm_plan_t pl, const uint8_t *mask, double lambda, double *v_lambda,
                                        double *dv_dlambda) {
    if (!pl) return fail(nullptr, FMM_ERR_INVALID, "plan is NULL");
    fmm_status st = check_lambda(pl, lambda);
    if (st != FMM_OK) return st;
    double w = 0.0;
    if ((st = solute_solvent_single(pl, mask, lambda, &w)) != FMM_OK) return st;
    lambda_values(pl, pl->last_energy, w, lambda, v_lambda, dv_dlambda);
    return FMM_OK;
}

extern "C" fmm_status fmm_plan_softcore(fmm_plan_t pl, double alpha, double sigma, int c) {
    if (!pl) return fail(nullptr, FMM_ERR_INVALID, "fmm_plan_softcore: plan is NULL");
    if (!std::isfinite(alpha) || alpha < 0.0) return fail(pl, FMM_ERR_INVALID, "fmm_plan_softcore: alpha must be >= 0");
    if (!std::isfinite(sigma) || sigma <= 0.0) return fail(pl, FMM_ERR_INVALID, "fmm_plan_softcore: sigma must be > 0");
    if (c < 1 || c > 12) return fail(pl, FMM_ERR_INVALID, "fmm_plan_softcore: c must be in [1, 12]");
    auto set = [&](fmm_plan_t b) {
        b->sc_alpha = alpha;
        b->sc_sigma = sigma;
        b->sc_c = c;
    };
    set(pl);
    for (fmm_plan_t b : pl->sub) set(b);
    return FMM_OK;
}

extern "C" fmm_status fmm_bin(fmm_plan_t pl, int64_t n, const double *pos, uint32_t *keys, int32_t *perm,
                              int32_t *cell_start) {
    if (!pl) return fail(nullptr, FMM_ERR_INVALID, "plan is NULL");
    if (pl->is_batch) return fail(pl, FMM_ERR_INVALID, "batch plan: fmm_bin takes a single-box plan");
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(pl, FMM_ERR_INVALID, "n must be in [0, 2^31)");
    if (n > 0 && !pos) return fail(pl, FMM_ERR_INVALID, "pos must be non-NULL when n > 0");
    HIPCHK(pl, hipSetDevice(pl->device), "hipSetDevice");
    fmm_status st;
    if ((st = ensure_workspace(pl, n)) != FMM_OK) return st;
    pl->have_state = false;
    hipStream_t s = pl->stream;
    if ((st = sort_atoms(pl, n, pos, nullptr)) != FMM_OK) return st;
    const int64_t nleaf = level_cells(pl->levels);
    if (keys && n > 0) HIPCHK(pl, hipMemcpyAsync(keys, pl->key.ptr, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s), "copy");
    if (perm && n > 0) HIPCHK(pl, hipMemcpyAsync(perm, pl->perm.ptr, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s), "copy");
    if (cell_start)
        HIPCHK(pl, hipMemcpyAsync(cell_start, pl->start.ptr, sizeof(int32_t) * (nleaf + 1), hipMemcpyDeviceToDevice, s),
               "copy");
    return finish_readback(pl, 1);
}

extern "C" fmm_status fmm_lattice_tensor(fmm_plan_t pl, double *out, int64_t cap) {
    if (!pl) return fail(nullptr, FMM_ERR_INVALID, "plan is NULL");
    if (pl->is_batch) return fail(pl, FMM_ERR_INVALID, "batch plan: fmm_lattice_tensor takes a single-box plan");
    const int64_t need = 2 * (int64_t)(2 * pl->p + 1) * (2 * pl->p + 1);
    if (!out || cap < need) return fail(pl, FMM_ERR_INVALID, "output too small");
    // stored for a unit box: T_j(nu b) = b^{-(j+1)} T_j(nu)
    for (int j = 0; j <= 2 * pl->p; ++j) {
        const double sc = std::pow(pl->box, -(double)(j + 1));
        for (int k = -j; k <= j; ++k) {
            const cplx v = pl->T[(size_t)j * j + j + k] * sc;
            out[2 * ((int64_t)j * j + j + k)] = v.real();
            out[2 * ((int64_t)j * j + j + k) + 1] = v.imag();
        }
    }
    return FMM_OK;
}

static void free_events(fmm_plan_t pl) {
    for (int i = 0; i < FMM_NUM_STAGES; ++i) {
        if (pl->ev_begin[i]) (void)hipEventDestroy(pl->ev_begin[i]);
        if (pl->ev_end[i]) (void)hipEventDestroy(pl->ev_end[i]);
        pl->ev_begin[i] = pl->ev_end[i] = nullptr;
    }
    pl->profiling = false;
}

extern "C" fmm_status fmm_profile(fmm_plan_t pl, int enable) {
    if (!pl) return fail(nullptr, FMM_ERR_INVALID, "plan is NULL");
    if (pl->is_batch && enable) return fail(pl, FMM_ERR_INVALID, "batch plan: stage profiling takes a single-box plan");
    HIPCHK(pl, hipSetDevice(pl->device), "hipSetDevice");
    free_events(pl);
    for (int i = 0; i < FMM_NUM_STAGES; ++i) pl->stage_ms[i] = 0.0;
    pl->profiled_calls = 0;
    stage_reset(pl);
    if (!enable) return FMM_OK;
    for (int i = 0; i < FMM_NUM_STAGES; ++i) {
        hipError_t e = hipEventCreate(&pl->ev_begin[i]);
        if (e == hipSuccess) e = hipEventCreate(&pl->ev_end[i]);
        if (e != hipSuccess) {
            free_events(pl);
            return hip_fail(pl, e, "hipEventCreate");
        }
    }
    pl->profiling = true;
    return FMM_OK;
}

extern "C" fmm_status fmm_profile_read(fmm_plan_t pl, double *ms, int64_t *calls) {
    if (!pl) return fail(nullptr, FMM_ERR_INVALID, "plan is NULL");
    if (ms)
        for (int i = 0; i < FMM_NUM_STAGES; ++i) ms[i] = pl->stage_ms[i];
    if (calls) *calls = pl->profiled_calls;
    return FMM_OK;
}

extern "C" const char *fmm_last_error(fmm_plan_t pl) {
    if (!pl) return g_plan_error.c_str();
    return pl->err.c_str();
}

extern "C" void fmm_destroy(fmm_plan_t pl) {
    if (!pl) return;
    if (pl->is_batch) {
        batch_drop_graphs(pl);
        for (fmm_plan_t b : pl->sub) fmm_destroy(b);
        for (hipStream_t x : pl->sub_stream)
            if (x) (void)hipStreamDestroy(x);
        for (hipEvent_t e : pl->sub_done)
            if (e) (void)hipEventDestroy(e);
        if (pl->fork) (void)hipEventDestroy(pl->fork);
        if (pl->input_ready) (void)hipEventDestroy(pl->input_ready);
        if (pl->own_stream) (void)hipStreamDestroy(pl->own_stream);
        pl->uvtab.release();
        pl->uvsc.release();
        if (pl->h_uvsc) (void)hipHostFree(pl->h_uvsc);
        delete pl;
        return;
    }
    DeviceBuf *bufs[] = {&pl->lat, &pl->key,
                         &pl->count, &pl->cursor, &pl->start, &pl->pstart, &pl->xqp, &pl->perm, &pl->scan, &pl->xq, &pl->xq_u, &pl->xs, &pl->m2l_part,
                         &pl->Mlev, &pl->Llev, &pl->mflip, &pl->m2l_part_up, &pl->mflip_up, &pl->M0, &pl->L0, &pl->phi_nf, &pl->field_nf, &pl->phi_ff,
                         &pl->field_ff, &pl->phi_u, &pl->field_u, &pl->nfuv, &pl->partials, &pl->scalars, &pl->flag,
                         &pl->sflag, &pl->mask_sw, &pl->mask_s, &pl->nfsc, &pl->nfdl, &pl->uvtab};
    for (DeviceBuf *b : bufs) b->release();
    free_events(pl);
    if (pl->h_scalars) (void)hipHostFree(pl->h_scalars);
    if (pl->ev_fork) (void)hipEventDestroy(pl->ev_fork);
    if (pl->ev_join) (void)hipEventDestroy(pl->ev_join);
    if (pl->ev_up_fork) (void)hipEventDestroy(pl->ev_up_fork);
    if (pl->ev_up_join) (void)hipEventDestroy(pl->ev_up_join);
    if (pl->side) (void)hipStreamDestroy(pl->side);
    if (pl->side_up) (void)hipStreamDestroy(pl->side_up);
    pl->op.reset();
    delete pl;
}

// ---------------------------------------------------------------------------
// Batches of independent boxes (charging windows of different size)
// ---------------------------------------------------------------------------

// Cost model for the tree depth of one box (seconds, MI355X): P2P pairs
// N * 125 N / 8^L, M2L flops 2 Kp^2 * 875 per cell summed over levels 1..L,
// a fixed per-level launch cost, and the per-atom expansion work.  The rates
// were measured with the kernels of this library on the 1M-atom box; the
// autotuner (fmm_autotune_batch) replaces the model's choice by timings.
static double depth_cost(int64_t n, int levels, int p, int prec) {
    const double Kp = padded_coeffs(p);
    const double pair_s = prec == FMM_FP64 ? 1.2e-12 : 6.5e-13;
    const double flop_s = prec == FMM_FP64 ? 2.0e-14 : 1.0e-14;
    double cells = 0.0;
    for (int l = 1; l <= levels; ++l) cells += (double)level_cells(l);
    const double pairs = (double)n * 125.0 * (double)n / (double)level_cells(levels);
    return pair_s * pairs + flop_s * 2.0 * Kp * Kp * 875.0 * cells + 2.5e-5 * levels + 2.0e-11 * n * Kp;
}

static int model_levels(int64_t n, int p, int prec) {
    int best = 1;
    double bc = depth_cost(n, 1, p, prec);
    for (int L = 2; L <= 7; ++L) {
        const double c = depth_cost(n, L, p, prec);
        if (c < bc) { bc = c; best = L; }
    }
    return best;
}

extern "C" fmm_status fmm_plan_batch(int nbox, const double *box, const int64_t *natoms, const int *levels, int p,
                                     fmm_plan_t *out) {
    if (!out) return fail(nullptr, FMM_ERR_INVALID, "fmm_plan_batch: out is NULL");
    *out = nullptr;
    if (nbox < 1 || nbox > 4096) return fail(nullptr, FMM_ERR_INVALID, "fmm_plan_batch: nbox must be in [1, 4096]");
    if (!box) return fail(nullptr, FMM_ERR_INVALID, "fmm_plan_batch: box is NULL");
    if (!levels && !natoms) return fail(nullptr, FMM_ERR_INVALID, "fmm_plan_batch: give levels or natoms");
    if (p < 0 || p > kMaxP) return fail(nullptr, FMM_ERR_INVALID, "fmm_plan_batch: p must be in [0, 20]");
    fmm_plan_t pl = new (std::nothrow) struct fmm_plan;
    if (!pl) return fail(nullptr, FMM_ERR_NOMEM, "fmm_plan_batch: host allocation");
    pl->is_batch = true;
    pl->p = p;
    pl->K = num_coeffs(p);
    pl->Kp = padded_coeffs(p);
    auto bail = [&](fmm_status st, const std::string &m) {
        g_plan_error = m;
        fmm_destroy(pl);
        return st;
    };
    if (hipGetDevice(&pl->device) != hipSuccess) return bail(FMM_ERR_DEVICE, "fmm_plan_batch: hipGetDevice failed");
    if (hipStreamCreateWithFlags(&pl->own_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&pl->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&pl->input_ready, hipEventDisableTiming) != hipSuccess)
        return bail(FMM_ERR_DEVICE, "fmm_plan_batch: stream or event creation failed");
    pl->stream = pl->own_stream;
    if (!pl->uvsc.ensure(sizeof(double) * kScalars * (size_t)nbox) ||
        hipHostMalloc((void **)&pl->h_uvsc, sizeof(double) * kScalars * (size_t)nbox, hipHostMallocDefault) !=
            hipSuccess) {
        pl->h_uvsc = nullptr;
        return bail(FMM_ERR_NOMEM, "fmm_plan_batch: scalar buffers");
    }
    std::shared_ptr<OpSet> ops;
    for (int w = 0; w < nbox; ++w) {
        if (natoms && natoms[w] < 0) return bail(FMM_ERR_INVALID, "fmm_plan_batch: natoms must be >= 0");
        const int L = levels ? levels[w] : model_levels(natoms[w], p, FMM_MIXED);
        fmm_plan_t b = nullptr;
        fmm_status st = plan_create(box[w], L, p, ops, true, &b);
        if (st != FMM_OK) return bail(st, "fmm_plan_batch: box " + std::to_string(w) + ": " + g_plan_error);
        ops = b->op;
        pl->sub.push_back(b);
        pl->sub_natoms.push_back(natoms ? natoms[w] : -1);
        hipStream_t x = nullptr;
        hipEvent_t e = nullptr;
        if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            if (x) (void)hipStreamDestroy(x);
            return bail(FMM_ERR_DEVICE, "fmm_plan_batch: stream or event creation failed");
        }
        pl->sub_stream.push_back(x);
        pl->sub_done.push_back(e);
        b->stream = x;
    }
    pl->op = ops;
    *out = pl;
    return FMM_OK;
}

extern "C" fmm_status fmm_batch_levels(fmm_plan_t pl, int *levels, int *p2p_groups_out) {
    if (!pl) return fail(nullptr, FMM_ERR_INVALID, "plan is NULL");
    if (!pl->is_batch) return fail(pl, FMM_ERR_INVALID, "fmm_batch_levels: not a batch plan");
    for (size_t w = 0; w < pl->sub.size(); ++w) {
        if (levels) levels[w] = pl->sub[w]->levels;
        if (p2p_groups_out) p2p_groups_out[w] = pl->sub[w]->p2p_g;
    }
    return FMM_OK;
}

static fmm_status check_batch_offsets(fmm_plan_t pl, const int64_t *off) {
    if (!off) return fail(pl, FMM_ERR_INVALID, "offsets is NULL");
    if (off[0] < 0) return fail(pl, FMM_ERR_INVALID, "offsets[0] must be >= 0");
    for (size_t w = 0; w < pl->sub.size(); ++w) {
        const int64_t n = off[w + 1] - off[w];
        if (n < 0 || n >= ((int64_t)1 << 31)) return fail(pl, FMM_ERR_INVALID, "offsets must be non-decreasing, boxes < 2^31 atoms");
    }
    return FMM_OK;
}

// Capture `enqueue(w)` for every non-empty box as parallel branches of one
// graph (fork from and join into the batch stream), or reuse the graph that
// was captured for the same key.  Launches it; the caller synchronises.
struct NoTail {
    fmm_status operator()() const { return FMM_OK; }
};

// branches: false to capture no per-box branch (only the tail); tail: work
// enqueued on the batch stream after every branch has joined it
template <typename F, typename G = NoTail>
static fmm_status batch_run(fmm_plan_t pl, fmm_plan::Graph &g, const std::vector<int64_t> &key,
                            const int64_t *off, F enqueue, bool branches = true, G tail = G()) {
    hipStream_t cs = pl->stream;
    if (!g.exec || g.key != key) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g.exec = nullptr;
        g.key.clear();
        HIPCHK(pl, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "graph capture");
        fmm_status st = FMM_OK;
        hipError_t e = hipEventRecord(pl->fork, cs);
        for (size_t w = 0; branches && w < pl->sub.size() && st == FMM_OK && e == hipSuccess; ++w) {
            if (off[w + 1] == off[w]) continue;
            fmm_plan_t b = pl->sub[w];
            b->stream = pl->sub_stream[w];
            e = hipStreamWaitEvent(b->stream, pl->fork, 0);
            if (e != hipSuccess) break;
            st = enqueue(w);
            if (st != FMM_OK) {
                pl->err = "box " + std::to_string(w) + ": " + b->err;
                break;
            }
            e = hipEventRecord(pl->sub_done[w], b->stream);
            if (e == hipSuccess) e = hipStreamWaitEvent(cs, pl->sub_done[w], 0);
        }
        if (st == FMM_OK && e == hipSuccess) st = tail();
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(cs, &graph);
        if (st != FMM_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess || ec != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(pl, e != hipSuccess ? e : ec, "graph capture");
        }
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(pl, e, "graph instantiate");
        g.exec = exec;
        g.key = key;
    }
    if (cs == pl->own_stream) {
        // the plan's own stream does not order itself after the null stream,
        // on which the caller's inputs may still be in flight
        HIPCHK(pl, hipEventRecord(pl->input_ready, nullptr), "event record");
        HIPCHK(pl, hipStreamWaitEvent(cs, pl->input_ready, 0), "stream wait");
    }
    HIPCHK(pl, hipGraphLaunch(g.exec, cs), "graph launch");
    return FMM_OK;
}

extern "C" fmm_status fmm_energy_forces_batch(fmm_plan_t pl, const int64_t *offsets, const double *pos,
                                              const double *q, double *energies, double *forces) {
    if (!pl) return fail(nullptr, FMM_ERR_INVALID, "plan is NULL");
    if (!pl->is_batch) return fail(pl, FMM_ERR_INVALID, "fmm_energy_forces_batch: not a batch plan");
    fmm_status st = check_batch_offsets(pl, offsets);
    if (st != FMM_OK) return st;
    if (!energies) return fail(pl, FMM_ERR_INVALID, "energies is NULL");
    const size_t nb = pl->sub.size();
    if (offsets[nb] > offsets[0] && (!pos || !q)) return fail(pl, FMM_ERR_INVALID, "pos and q must be non-NULL");
    HIPCHK(pl, hipSetDevice(pl->device), "hipSetDevice");
    pl->batch_state = false;
    for (size_t w = 0; w < nb; ++w) {
        fmm_plan_t b = pl->sub[w];
        b->have_state = false;
        const int64_t n = offsets[w + 1] - offsets[w];
        if (n == 0) continue;
        if ((st = ensure_workspace(b, n)) != FMM_OK || (st = ensure_m2l_ops(b)) != FMM_OK) {
            pl->err = "box " + std::to_string(w) + ": " + b->err;
            return st;
        }
    }
    std::vector<int64_t> key(offsets, offsets + nb + 1);
    key.push_back((int64_t)(uintptr_t)pos);
    key.push_back((int64_t)(uintptr_t)q);
    key.push_back((int64_t)(uintptr_t)forces);
    key.push_back(pl->prec);
    key.push_back(pl->boundary);
    st = batch_run(pl, pl->g_ef, key, offsets, [&](size_t w) -> fmm_status {
        fmm_plan_t b = pl->sub[w];
        const int64_t o = offsets[w], n = offsets[w + 1] - o;
        double *f = forces ? forces + 3 * o : nullptr;
        return b->prec == FMM_FP64 ? enqueue_energy_forces<double>(b, n, pos + 3 * o, q + o, f, nullptr)
                                   : enqueue_energy_forces<float>(b, n, pos + 3 * o, q + o, f, nullptr);
    });
    if (st != FMM_OK) return st;
    HIPCHK(pl, hipStreamSynchronize(pl->stream), "synchronize");
    for (size_t w = 0; w < nb; ++w) {
        fmm_plan_t b = pl->sub[w];
        const int64_t n = offsets[w + 1] - offsets[w];
        energies[w] = 0.0;
        if (n > 0 && (st = finish_energy(b, &energies[w])) != FMM_OK) {
            pl->err = "box " + std::to_string(w) + ": " + b->err;
            return st;
        }
        b->have_state = true;
        b->n_state = n;
    }
    pl->batch_off.assign(offsets, offsets + nb + 1);
    pl->batch_state = true;
    return FMM_OK;
}

// lams (host, nbox) or NULL: with a soft-core set, the per-box lambda of the
// soft-core near-field sums
static fmm_status solute_solvent_batch(fmm_plan_t pl, const uint8_t *mask, const double *lams, double *e_uv) {
    if (!pl) return fail(nullptr, FMM_ERR_INVALID, "plan is NULL");
    if (!pl->is_batch) return fail(pl, FMM_ERR_INVALID, "fmm_solute_solvent_energy_batch: not a batch plan");
    if (!e_uv) return fail(pl, FMM_ERR_INVALID, "e_uv is NULL");
    if (!pl->batch_state)
        return fail(pl, FMM_ERR_STATE, "fmm_solute_solvent_energy_batch needs a preceding fmm_energy_forces_batch");
    const size_t nb = pl->sub.size();
    const int64_t *off = pl->batch_off.data();
    if (off[nb] > off[0] && !mask) return fail(pl, FMM_ERR_INVALID, "mask is NULL");
    HIPCHK(pl, hipSetDevice(pl->device), "hipSetDevice");
    for (size_t w = 0; w < nb; ++w) {
        if (off[w + 1] == off[w]) continue;
        const fmm_status so = ensure_m2l_ops(pl->sub[w], (pl->uv_scheme & FMM_UV_SPARSE) != 0);
        if (so != FMM_OK) {
            pl->err = "box " + std::to_string(w) + ": " + pl->sub[w]->err;
            return so;
        }
    }
    std::vector<int64_t> key(pl->batch_off);
    key.push_back((int64_t)(uintptr_t)mask);
    key.push_back(pl->prec);
    key.push_back(pl->uv_scheme);
    const bool soft = lams && pl->sc_alpha > 0.0;
    if (soft) {
        // the soft-core parameters and lambdas are kernel arguments of the graph
        const double prm[2] = {pl->sc_alpha, pl->sc_sigma};
        for (double x : prm) {
            int64_t bits;
            std::memcpy(&bits, &x, sizeof bits);
            key.push_back(bits);
        }
        key.push_back(pl->sc_c);
        for (size_t w = 0; w < nb; ++w) {
            int64_t bits;
            std::memcpy(&bits, &lams[w], sizeof bits);
            key.push_back(bits);
        }
    }
    key.push_back(soft ? 1 : 0);
    for (fmm_plan_t b : pl->sub) b->uv_d0 = b->uv_dsc = b->uv_dl = 0.0;
    // every box's stages in one launch per stage; the symmetric scheme first
    // runs each box's dense second pass as a parallel branch
    const bool sparse = (pl->uv_scheme & FMM_UV_SPARSE) != 0;
    UvTables t;
    for (size_t w = 0; w < nb; ++w) {
        fmm_plan_t b = pl->sub[w];
        UvBox u = uv_box(b, mask ? mask + off[w] : nullptr, soft ? lams[w] : -1.0, pl->uvsc.as<double>() + w * kScalars);
        if (off[w + 1] == off[w]) u.n = 0;
        t.box.push_back(u);
    }
    uv_build_tables(t);
    void *const tab_before = pl->uvtab.ptr;
    fmm_status st = uv_upload(pl, t);
    if (st != FMM_OK) return st;
    if (pl->uvtab.ptr != tab_before && pl->g_uv.exec) {  // a captured graph reads the old table
        (void)hipGraphExecDestroy(pl->g_uv.exec);
        pl->g_uv.exec = nullptr;
        pl->g_uv.key.clear();
    }
    const bool fp64 = pl->prec == FMM_FP64;
    st = batch_run(
        pl, pl->g_uv, key, off,
        [&](size_t w) -> fmm_status {
            fmm_plan_t b = pl->sub[w];
            return fp64 ? enqueue_uv_dense<double>(b, mask + off[w]) : enqueue_uv_dense<float>(b, mask + off[w]);
        },
        !sparse,
        [&]() -> fmm_status {
            const fmm_status s2 = fp64 ? enqueue_uv_stages<double>(pl, t, sparse, *pl->op, pl->stream)
                                       : enqueue_uv_stages<float>(pl, t, sparse, *pl->op, pl->stream);
            if (s2 != FMM_OK) return s2;
            HIPCHK(pl, hipMemcpyAsync(pl->h_uvsc, pl->uvsc.ptr, sizeof(double) * kScalars * nb, hipMemcpyDeviceToHost,
                                      pl->stream),
                   "readback");
            return FMM_OK;
        });
    if (st != FMM_OK) return st;
    HIPCHK(pl, hipStreamSynchronize(pl->stream), "synchronize");
    for (size_t w = 0; w < nb; ++w) {
        e_uv[w] = 0.0;
        if (off[w + 1] == off[w]) continue;
        fmm_plan_t b = pl->sub[w];
        std::memcpy(b->h_scalars, pl->h_uvsc + w * kScalars, sizeof(double) * 46);
        std::memset(&b->h_scalars[kScalars - 1], 0, sizeof(double));  // no input-check flag in this pass
        if ((st = finish_solute_solvent(b, &e_uv[w])) != FMM_OK) {
            pl->err = "box " + std::to_string(w) + ": " + pl->sub[w]->err;
            return st;
        }
    }
    return FMM_OK;
}

extern "C" fmm_status fmm_solute_solvent_energy_batch(fmm_plan_t pl, const uint8_t *mask, double *e_uv) {
    return solute_solvent_batch(pl, mask, nullptr, e_uv);
}

extern "C" fmm_status fmm_lambda_energy_batch(fmm_plan_t pl, const uint8_t *mask, const double *lambdas,
                                              double *v_lambda, double *dv_dlambda) {
    if (!pl) return fail(nullptr, FMM_ERR_INVALID, "plan is NULL");
    if (!pl->is_batch) return fail(pl, FMM_ERR_INVALID, "fmm_lambda_energy_batch: not a batch plan");
    if (!lambdas) return fail(pl, FMM_ERR_INVALID, "lambdas is NULL");
    const size_t nb = pl->sub.size();
    fmm_status st;
    for (size_t w = 0; w < nb; ++w)
        if ((st = check_lambda(pl, lambdas[w])) != FMM_OK) return st;
    std::vector<double> e_uv(nb);
    if ((st = solute_solvent_batch(pl, mask, lambdas, e_uv.data())) != FMM_OK) return st;
    for (size_t w = 0; w < nb; ++w) {
        const double e = (pl->batch_off[w + 1] > pl->batch_off[w]) ? pl->sub[w]->last_energy : 0.0;
        lambda_values(pl->sub[w], e, e_uv[w], lambdas[w], v_lambda ? &v_lambda[w] : nullptr,
                      dv_dlambda ? &dv_dlambda[w] : nullptr);
    }
    return FMM_OK;
}

// Box w of a batch at depth L with g P2P source groups (0: from the leaf
// occupancy).  A new depth means a new sub-plan, sharing the box-independent
// operators and taking over the box's settings.
static fmm_status batch_set_box(fmm_plan_t pl, size_t w, int L, int g) {
    fmm_plan_t cur = pl->sub[w];
    if (L != cur->levels) {
        fmm_plan_t b = nullptr;
        fmm_status st = plan_create(cur->box, L, pl->p, pl->op, true, &b);
        if (st != FMM_OK) return fail(pl, st, "box " + std::to_string(w) + ": " + g_plan_error);
        b->top_fp64 = cur->top_fp64;
        b->boundary = cur->boundary;
        b->uv_scheme = cur->uv_scheme;
        b->sc_alpha = cur->sc_alpha;
        b->sc_sigma = cur->sc_sigma;
        b->sc_c = cur->sc_c;
        b->prec = pl->prec;
        b->stream = pl->sub_stream[w];
        fmm_destroy(cur);
        pl->sub[w] = b;
        cur = b;
    }
    cur->p2p_g = g;
    cur->have_state = false;
    return FMM_OK;
}

// Autotuner: for every non-empty box, time whole evaluations (energy and
// forces, hipEvent-timed on the box's stream after one warm-up) for the tree
// depths L-1, L, L+1 around the current one and the P2P source-group counts
// 2, 4, 8, and keep the fastest configuration.  Scratch plans share the
// box-independent operators.
extern "C" fmm_status fmm_autotune_batch(fmm_plan_t pl, const int64_t *offsets, const double *pos, const double *q,
                                         double *forces_scratch) {
    if (!pl) return fail(nullptr, FMM_ERR_INVALID, "plan is NULL");
    if (!pl->is_batch) return fail(pl, FMM_ERR_INVALID, "fmm_autotune_batch: not a batch plan");
    fmm_status st = check_batch_offsets(pl, offsets);
    if (st != FMM_OK) return st;
    HIPCHK(pl, hipSetDevice(pl->device), "hipSetDevice");
    HIPCHK(pl, hipDeviceSynchronize(), "synchronize");  // inputs written on any stream
    batch_drop_graphs(pl);
    pl->batch_state = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(pl, hipEventCreate(&e0), "hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(pl, FMM_ERR_DEVICE, "hipEventCreate");
    }
    auto time_eval = [&](fmm_plan_t b, int64_t o, int64_t n, float &ms) -> fmm_status {
        fmm_status s2;
        if ((s2 = ensure_workspace(b, n)) != FMM_OK || (s2 = ensure_m2l_ops(b)) != FMM_OK) return s2;
        double e = 0.0;
        double *f = forces_scratch ? forces_scratch + 3 * o : nullptr;
        ms = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            if (hipEventRecord(e0, b->stream) != hipSuccess) return FMM_ERR_DEVICE;
            s2 = b->prec == FMM_FP64 ? energy_forces_t<double>(b, n, pos + 3 * o, q + o, &e, f, nullptr)
                                     : energy_forces_t<float>(b, n, pos + 3 * o, q + o, &e, f, nullptr);
            if (s2 != FMM_OK) return s2;
            if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return FMM_ERR_DEVICE;
            float t = 0.f;
            (void)hipEventElapsedTime(&t, e0, e1);
            if (rep > 0) ms = std::min(ms, t);  // rep 0 is the warm-up
        }
        return FMM_OK;
    };
    for (size_t w = 0; w < pl->sub.size() && st == FMM_OK; ++w) {
        const int64_t o = offsets[w], n = offsets[w + 1] - o;
        if (n == 0) continue;
        fmm_plan_t cur = pl->sub[w];
        float best_ms = 1e30f;
        int best_L = cur->levels, best_g = 0;
        for (int L = std::max(1, cur->levels - 1); L <= std::min(kMaxLevels, cur->levels + 1) && st == FMM_OK; ++L) {
            fmm_plan_t b = nullptr;
            if (L == cur->levels) b = cur;
            else if ((st = plan_create(cur->box, L, pl->p, pl->op, true, &b)) != FMM_OK) {
                pl->err = "autotune box " + std::to_string(w) + ": " + g_plan_error;
                break;
            }
            b->top_fp64 = cur->top_fp64;
            b->boundary = cur->boundary;
            b->prec = pl->prec;
            b->stream = pl->sub_stream[w];
            for (int g : {2, 4, 8}) {
                b->p2p_g = g;
                float ms = 0.f;
                if ((st = time_eval(b, o, n, ms)) != FMM_OK) {
                    pl->err = "autotune box " + std::to_string(w) + ": " + b->err;
                    break;
                }
                if (ms < best_ms) { best_ms = ms; best_L = L; best_g = g; }
            }
            if (b != cur) fmm_destroy(b);
        }
        if (st != FMM_OK) break;
        st = batch_set_box(pl, w, best_L, best_g);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

extern "C" fmm_status fmm_batch_set_tuning(fmm_plan_t pl, const int *levels, const int *p2p_groups) {
    if (!pl) return fail(nullptr, FMM_ERR_INVALID, "plan is NULL");
    if (!pl->is_batch) return fail(pl, FMM_ERR_INVALID, "fmm_batch_set_tuning: not a batch plan");
    for (size_t w = 0; w < pl->sub.size(); ++w) {
        if (levels && (levels[w] < 1 || levels[w] > kMaxLevels))
            return fail(pl, FMM_ERR_INVALID, "fmm_batch_set_tuning: levels must be in [1, 10]");
        if (p2p_groups && !valid_p2p_groups(p2p_groups[w]))
            return fail(pl, FMM_ERR_INVALID, "fmm_batch_set_tuning: p2p_groups must be 0, 1, 2, 4, 8 or 16");
    }
    HIPCHK(pl, hipSetDevice(pl->device), "hipSetDevice");
    HIPCHK(pl, hipDeviceSynchronize(), "synchronize");  // no queued work still uses a sub-plan
    batch_drop_graphs(pl);
    pl->batch_state = false;
    for (size_t w = 0; w < pl->sub.size(); ++w) {
        const fmm_status st = batch_set_box(pl, w, levels ? levels[w] : pl->sub[w]->levels,
                                            p2p_groups ? p2p_groups[w] : pl->sub[w]->p2p_g);
        if (st != FMM_OK) return st;
    }
    return FMM_OK;
}

extern "C" fmm_status fmm_autotune_batch_cached(fmm_plan_t pl, const int64_t *offsets, const double *pos,
                                                const double *q, double *forces_scratch, const char *cache_path,
                                                int *hit) {
    if (hit) *hit = 0;
    if (!pl) return fail(nullptr, FMM_ERR_INVALID, "plan is NULL");
    if (!pl->is_batch) return fail(pl, FMM_ERR_INVALID, "fmm_autotune_batch_cached: not a batch plan");
    if (!cache_path || !*cache_path) return fail(pl, FMM_ERR_INVALID, "fmm_autotune_batch_cached: no cache path");
    fmm_status st = check_batch_offsets(pl, offsets);
    if (st != FMM_OK) return st;
    const size_t nb = pl->sub.size();
    hipDeviceProp_t prop;
    HIPCHK(pl, hipGetDeviceProperties(&prop, pl->device), "hipGetDeviceProperties");
    std::vector<double> edge(nb);
    std::vector<int64_t> natoms(nb);
    for (size_t w = 0; w < nb; ++w) {
        edge[w] = pl->sub[w]->box;
        natoms[w] = offsets[w + 1] - offsets[w];
    }
    const std::string key = tuning_cache_key(prop.gcnArchName, pl->p, (int)pl->prec, pl->sub[0]->top_fp64, nb,
                                             edge.data(), natoms.data());
    std::vector<int> lv, gr;
    if (tuning_cache_lookup(cache_path, key, nb, lv, gr)) {
        if ((st = fmm_batch_set_tuning(pl, lv.data(), gr.data())) != FMM_OK) return st;
        if (hit) *hit = 1;
        return FMM_OK;
    }
    if ((st = fmm_autotune_batch(pl, offsets, pos, q, forces_scratch)) != FMM_OK) return st;
    lv.assign(nb, 0);
    gr.assign(nb, 0);
    for (size_t w = 0; w < nb; ++w) {
        lv[w] = pl->sub[w]->levels;
        gr[w] = pl->sub[w]->p2p_g;
    }
    if (!tuning_cache_append(cache_path, key, lv, gr))
        return fail(pl, FMM_ERR_INVALID, "fmm_autotune_batch_cached: cannot write the cache file");
    return FMM_OK;
}

extern "C" const char *fmm_version(void) { return "libfmm 0.1 (gfx950)"; }
