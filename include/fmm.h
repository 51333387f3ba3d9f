/*
 * fmm.h -- C ABI of libfmm: periodic fast multipole evaluation of the
 * electrostatic energy, per-atom potential and forces of N point charges in a
 * cubic cell whose net charge is neutralised by a uniform background charge,
 * on one AMD Instinct MI355X (gfx950).
 *
 * Method (Urano, Shinoda, Yoshii, Okazaki, arXiv:2003.13218):
 *   E = NF + FF - pi Q^2 / (2 V kappa^2) + (2 pi / 3V) Q sum_i q_i r_i^2
 *       - (2 pi / 3V) mu.mu                                   (eq. Velecfull)
 * NF is the direct sum over each leaf's +-2 neighbour leaves (eq. EqNF), FF
 * the octree expansion P2M -> M2M -> M2L -> L2L -> L2P (Appendix B, eqs. P2M,
 * Lcoeffdef, EqFF) whose level-0 translation is the Ewald-split image-lattice
 * sum of eq. 12 (with the self term of Appendix C), kappa is the same in the
 * lattice sum and in the charged-system term (eq. 6), and the last two terms
 * are the quadrupole surface term (eq. surfchargedend) and the dipole term
 * that turns the tree's vacuum boundary into a conducting one (Appendix D).
 *
 * Conventions
 *   Units   Gaussian: E = sum q_i q_j / r with no 1/(4 pi eps0).  With charges
 *           in e and lengths in Angstrom, energies are in e^2/A.
 *   Forces  F_i = -dE/dr_i.   Potential phi_i = dE/dq_i, so E = 1/2 sum q_i phi_i.
 *   Box     cubic, edge b, origin at 0; positions may lie anywhere (they are
 *           wrapped into [0, b) internally and never modified).
 *   Memory  every array argument named "device" is device memory of the GPU
 *           current when the plan was created; the caller owns it.  Scalars
 *           marked "host" are host memory.  Device arrays are FP64,
 *           array-of-structs where 3-vectors are involved ([n][3]).
 *   Streams a call's GPU work is ordered on the plan's stream (default: the
 *           null stream): it starts after the work queued there before the
 *           call, and everything it does (including the near field and the
 *           upper tree, which a single-box plan runs on two streams of its
 *           own, created with the plan and joined back) is done before the
 *           call returns with its result on the host.  No evaluation creates
 *           a stream.
 *   Config  the library reads no environment variables: every choice that
 *           changes numerics or schedules is an argument of fmm_plan,
 *           fmm_plan_config, fmm_plan_options, fmm_plan_tuning or
 *           fmm_plan_softcore, and fmm_plan_info reports it.
 *   Threads a plan is not thread-safe; distinct plans are independent.
 *   Errors  every call returns a negative fmm_status on failure and leaves a
 *           message in fmm_last_error(plan); nothing is thrown across the ABI.
 */
#ifndef FMM_H
#define FMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmm_plan *fmm_plan_t;

typedef enum {
    FMM_OK = 0,
    FMM_ERR_INVALID = -1, /* bad argument, or non-finite position / charge  */
    FMM_ERR_NOMEM = -2,   /* device or host allocation failed                */
    FMM_ERR_DEVICE = -3,  /* HIP runtime error or no usable GPU              */
    FMM_ERR_STATE = -4    /* call order violated (see fmm_solute_solvent_energy) */
} fmm_status;

typedef enum {
    /* everything in FP64 */
    FMM_FP64 = 0,
    /* P2P, P2M, L2P and the expansions of levels >= 4 (their M2M, M2L and
     * L2L) in FP32 with cell-local coordinates; the P2P potential and the
     * leaf multipoles summed in FP64; levels 0-3, the lattice operator, the
     * charged-system, quadrupole and dipole terms and the energy reduction
     * in FP64 */
    FMM_MIXED = 1,
    /* as FMM_MIXED, but the FP32 levels' M2L takes BF16 operands (operators
     * and multipoles rounded to bfloat16, 8 significant bits) with FP32
     * accumulation on the matrix cores: a precision/speed trade-off whose
     * far-field error is of the order of the BF16 unit roundoff 2^-8.  It
     * does NOT meet the 1e-5 accuracy of the other modes: on water boxes
     * the RMS relative potential error is about 1.4e-2 and the force error
     * about 4e-4 at every order p */
    FMM_MIXED_BF16_M2L = 2,
    /* as FMM_MIXED, but the FP32 levels' M2L writes every operator and
     * multipole entry as the sum of two FP16 numbers (hi + lo, with exact
     * power-of-two row and column scales keeping them in FP16's range) and
     * forms hi*hi + hi*lo + lo*hi on the FP16 matrix cores with FP32
     * accumulation, partial sums flushed to FP64 after every list entry: about
     * 2^-22 relative per product against 2^-24 for FP32 operands.  Orders
     * 11 and 12 run the folded orbit list (all four row classes in one
     * launch), the others the plain 875-offset list */
    FMM_MIXED_SPLIT16_M2L = 3
} fmm_precision;

/*
 * fmm_plan -- build a plan for a cubic box of edge `box` (> 0, finite),
 * an octree of `levels` divisions (1..10; 8^levels leaves; Appendix B,
 * division of cells) and expansion order `p` (0..20, the paper's n_max; the
 * truncation n <= p, lambda <= p of eq. Lcoeffdef).  Near field is the
 * +-2-leaf block (the "second nearest neighbours" of eq. EqNF), the
 * interaction list at every level is the children of the parent's +-2
 * neighbours minus the own +-2 block (875 cells, 1206 distinct offsets).
 * Defaults: FMM_FP64, kappa = 3/box, null stream.
 * Precomputes in FP64 on the host the scale-invariant M2M / M2L / L2L
 * operators and the lattice tensor of eq. 12, and uploads them.
 * On success *out owns them until fmm_destroy.  On failure *out is NULL.
 */
fmm_status fmm_plan(double box, int levels, int p, fmm_plan_t *out);

/*
 * fmm_plan_config -- precision mode, Ewald split parameter and stream.
 * kappa > 0 sets the splitting parameter used by BOTH the j = 0 lattice sum
 * (eq. 12a-c) and the charged-system term (eq. 6), as the paper requires;
 * kappa <= 0 keeps the current value.  hip_stream is a hipStream_t (NULL =
 * null stream).  Rebuilds the lattice operator when kappa changes.  Clears
 * the cached state used by fmm_solute_solvent_energy.
 */
fmm_status fmm_plan_config(fmm_plan_t plan, int precision, double kappa, void *hip_stream);

/*
 * fmm_plan_tuning -- schedule and precision split of the plan's tree.
 *   fp64_levels  in the mixed modes, tree levels 1 .. fp64_levels run in
 *                FP64 (M2M, M2L, L2L; clamped to levels - 1); default 3.  At
 *                shallow levels the cells are large and their M2L terms
 *                cancel strongly, so FP32 there costs accuracy: on the
 *                1,000,000-atom water box (levels 5, p 12) the default
 *                gives an RMS potential error of 1.8e-6 against the FP64
 *                Ewald sum, 4 gives 7e-7 at about 0.8 ms more per
 *                evaluation.  Ignored in FMM_FP64 (everything is FP64).
 *                -1 keeps the current value.
 *   p2p_groups   source groups of the near-field kernel (1, 2, 4, 8, 16; the
 *                atoms of a leaf are split in that many target chunks of
 *                64 / groups slots), or 0 to choose from the mean leaf
 *                occupancy (default); -1 keeps the current value.  Changes
 *                the schedule only: results are identical up to the order of
 *                FP64 partial sums.
 * On a batch plan it applies to every box (fmm_autotune_batch then replaces
 * the group counts).  Clears the cached state used by
 * fmm_solute_solvent_energy.  FMM_ERR_INVALID for other values.
 */
fmm_status fmm_plan_tuning(fmm_plan_t plan, int fp64_levels, int p2p_groups);

/* Boundary condition at infinity (Appendix A, eq. surfdipole). */
typedef enum {
    FMM_BOUNDARY_CONDUCTING = 0, /* tin-foil boundary of the Ewald sum (default) */
    FMM_BOUNDARY_VACUUM = 1      /* adds the dipole surface term               */
} fmm_boundary;

/* Far-field scheme of fmm_solute_solvent_energy (bit flags). */
typedef enum {
    FMM_UV_SYMMETRIC = 0, /* eq. FMMcalc: a dense second pass over the solute charges       */
    FMM_UV_SPARSE = 1,    /* one-sided W_FF = sum_u q (phi_uv - phi_u), phi_u at u only     */
    FMM_UV_SWAP = 2       /* exchange the roles of u and v in the second pass               */
} fmm_uv_scheme;

/*
 * fmm_plan_options -- boundary condition and solute-solvent scheme.
 *   boundary   FMM_BOUNDARY_CONDUCTING or FMM_BOUNDARY_VACUUM.  Vacuum adds
 *              the dipole surface term (2 pi / 3V) mu.mu of eq. surfdipole to
 *              E, with mu = sum q r over the atoms wrapped into the box and
 *              measured from its centre (the level-0 expansion centre); the
 *              forces gain -(4 pi / 3V) q_i mu, the potential (4 pi / 3V)
 *              mu.r_i, and e_uv the cross part (4 pi / 3V) mu_u.mu_v.
 *              Changing it clears the cached state (as fmm_plan_config).
 *   uv_scheme  FMM_UV_SYMMETRIC or FMM_UV_SPARSE, optionally | FMM_UV_SWAP.
 *              SYMMETRIC is eq. FMMcalc with a full far-field pass over the
 *              masked charges.  SPARSE uses the one-sided form the same
 *              derivation gives, W_FF = sum_u q (phi_uv - phi_u): phi_u is
 *              needed at the solute atoms only, and the tree of the solute
 *              charges is non-zero only above the leaves that hold them, so
 *              that pass runs (in FP64) over those cells alone -- the cheap
 *              choice for a few ions in a large box.  phi_uv carries the
 *              precision of the preceding fmm_energy_forces call: in the
 *              mixed modes the one-sided sum over a LARGE masked set adds
 *              that call's FP32 error at every masked atom, so SPARSE is
 *              meant for a masked set of few atoms.  SWAP evaluates the
 *              second pass over the solvent charges instead (the exchanged
 *              form the paper notes after eq. FMMcalc); e_uv is symmetric in
 *              u and v, so every scheme returns the same value up to the
 *              truncation and rounding of the far field.
 * On a batch plan the options apply to every box.  FMM_ERR_INVALID for
 * values outside the enums.
 */
fmm_status fmm_plan_options(fmm_plan_t plan, int boundary, int uv_scheme);

/*
 * fmm_energy_forces -- E of eq. Velecfull, forces and per-atom potential.
 *   n       number of atoms (0 <= n < 2^31); n == 0 gives E = 0
 *   pos     device, n x 3 FP64 (AoS), any range
 *   q       device, n FP64
 *   energy  host out, 1 FP64 (required)
 *   forces  device out, n x 3 FP64, or NULL
 *   phi     device out, n FP64, or NULL
 * Non-finite positions or charges give FMM_ERR_INVALID (detected on the GPU).
 * Keeps its own sorted copy of the atoms and the far-field potential for a
 * following fmm_solute_solvent_energy (pos and q may change or be freed
 * after this call returns).
 */
fmm_status fmm_energy_forces(fmm_plan_t plan, int64_t n, const double *pos, const double *q,
                             double *energy, double *forces, double *phi);

/*
 * fmm_energy_forces_noalloc -- fmm_energy_forces for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, same kernels and the same
 * results bit for bit; it calls no hipMalloc, hipFree or allocating library
 * routine.  Its per-call workspace (sorted atoms, expansions, M2L scratch,
 * near-field copy, reductions) is carved from one fixed array of
 * FMM_NOALLOC_SCRATCH_BYTES bytes of device memory that the library holds on
 * each GPU it runs on until the process ends, shared by every plan and call
 * on that GPU and keeping the last call's contents (every piece is written
 * before it is read).  Calls that overlap on one GPU (two threads, or two
 * plans on different streams) race on it: the caller serialises them.
 * The plan's operators must be on the device already (fmm_plan,
 * fmm_plan_config and fmm_plan_tuning upload them; FMM_ERR_STATE otherwise).
 * A workspace larger than the array gives FMM_ERR_INVALID before any GPU
 * work, with the bytes needed in fmm_last_error: about 170 bytes per atom
 * plus, per tree, 16 (8^(levels+1) / 7) Kp bytes for the expansions and the
 * M2L scratch of the deepest level (3 x 8^levels x 8 Kp bytes) and of the
 * split-K levels; e.g. 30,000 atoms at levels 4, p 10 fit, 1,000,000 atoms at
 * levels 5, p 12 do not.  No state is kept for fmm_solute_solvent_energy (it
 * returns FMM_ERR_STATE after this call).  Batch plans are rejected.
 */
#define FMM_NOALLOC_SCRATCH_BYTES (128ull << 20)
fmm_status fmm_energy_forces_noalloc(fmm_plan_t plan, int64_t n, const double *pos, const double *q,
                                     double *energy, double *forces, double *phi);

/*
 * fmm_solute_solvent_energy -- the solute-solvent interaction energy
 *   e_uv = E(u + Bu  U  v + Bv) - E(u + Bu) - E(v + Bv)
 * for the partition mask[i] = 1 (solute u) / 0 (solvent v), each part with
 * its own neutralising background, of the atoms of the preceding
 * fmm_energy_forces call on this plan.  Far field by the two-pass scheme
 * of eq. FMMcalc (the full-system potential of the preceding call plus one
 * pass with solute sources only):
 *   W_FF = 1/2 [ sum_u q phi_uv - (sum_u q phi_u - sum_v q phi_u) ],
 * plus the near-field u-v pairs and the background cross terms
 *   -pi Q_u Q_v / (V kappa^2) + (2 pi / 3V)(Q_u S_v + Q_v S_u - 2 mu_u.mu_v),
 * S = sum q r^2.  This is minus the derivative of V_lambda (eq. Vswucheme)
 * with respect to lambda.
 *   mask  device, n uint8 (nonzero = solute)
 *   e_uv  host out
 * FMM_ERR_STATE if no fmm_energy_forces has run since the plan was made or
 * reconfigured.
 */
fmm_status fmm_solute_solvent_energy(fmm_plan_t plan, const uint8_t *mask, double *e_uv);

/*
 * fmm_lambda_energy -- the lambda-coupled energy of eq. Vswucheme, in which
 * the solute-solvent coupling (u-v, u-Bv, v-Bu, Bu-Bv) is scaled by
 * (1 - lambda) and everything else is kept:
 *   V_lambda = E(u+Bu) + E(v+Bv) + (1 - lambda) e_uv = E - lambda e_uv,
 *   dV_lambda/dlambda = -e_uv,
 * with E the energy of the preceding fmm_energy_forces call on this plan and
 * e_uv as returned by fmm_solute_solvent_energy for the same mask (which this
 * call computes).  lambda = 0: the solute fully in solution; lambda = 1: the
 * solute decoupled from the solvent (each part still neutralised by its own
 * background).  This is eq. FMMVTI with the signs of its background terms
 * taken from eq. Velecfull and eq. 6.  v_lambda, dv_dlambda: host out (either
 * may be NULL).  Same errors as fmm_solute_solvent_energy.
 */
fmm_status fmm_lambda_energy(fmm_plan_t plan, const uint8_t *mask, double lambda, double *v_lambda,
                             double *dv_dlambda);

/*
 * fmm_plan_softcore -- soft-core near-field solute-solvent Coulomb pairs in
 * fmm_lambda_energy and fmm_lambda_energy_batch.  The paper gives the
 * soft-core form for the solute-solvent LJ term of its charging path
 * (section "Calculation detail") and notes that it applies to the
 * electrostatic near-field term as well; here every u-v pair of the near field
 * (eq. EqNF: the +-2-leaf neighbourhood of the plan's tree) takes
 *   q_u q_v / s,  s = (alpha lambda sigma^c + r^c)^(1/c),
 * in place of q_u q_v / r inside the (1 - lambda)-scaled coupling, so that
 *   V_lambda    = E - lambda e_uv + (1 - lambda)(Dsc - D0),
 *   dV/dlambda  = -e_uv + D0 - Dsc + (1 - lambda) dDsc/dlambda,
 * with D0 and Dsc the hard and soft sums over those pairs (the far field and
 * the background terms keep their plain form).  alpha = 0 (the default)
 * turns it off; sigma > 0 is a length, c an integer in [1, 12]; with it on,
 * lambda must lie in [0, 1].  The near-field pair set depends on the tree
 * depth, so results are comparable between plans of equal depth only.  On a
 * batch plan it applies to every box.  fmm_solute_solvent_energy is not
 * affected.
 */
fmm_status fmm_plan_softcore(fmm_plan_t plan, double alpha, double sigma, int c);

/*
 * fmm_potential_parts -- near- and far-field parts separately (no charged,
 * quadrupole or dipole terms), per atom in the caller's order, for checking
 * the stages on their own.  phi_nf / phi_ff: device n FP64 (or NULL);
 * field_nf / field_ff: device n x 3 FP64 (or NULL), field = -grad phi.
 * Same input contract as fmm_energy_forces; also refreshes the cached state.
 */
fmm_status fmm_potential_parts(fmm_plan_t plan, int64_t n, const double *pos, const double *q,
                               double *phi_nf, double *field_nf, double *phi_ff, double *field_ff);

/*
 * fmm_bin -- stages wrap + bin + Morton key + stable sort (by key, then by
 * original index) only.  keys: device n uint32 (leaf Morton key of each atom
 * in the caller's order; bit k of the x leaf index at bit 3k+2, of y at 3k+1,
 * of z at 3k); perm: device n int32 (perm[s] = original index of sorted atom
 * s); cell_start: device 8^levels + 1 int32 (atoms of leaf with key c are
 * sorted positions cell_start[c] .. cell_start[c+1]-1).  Any output may be NULL.
 */
fmm_status fmm_bin(fmm_plan_t plan, int64_t n, const double *pos,
                   uint32_t *keys, int32_t *perm, int32_t *cell_start);

/*
 * fmm_lattice_tensor -- copy of the plan's lattice tensor (host out):
 * T_j^k = sum over images nu with max|nu_a| > 2 of I_j^k(nu b), for
 * 0 <= j <= 2p, -j <= k <= j, as complex pairs (re, im) at index
 * 2 (j*j + j + k), with I_j^k(r) = (j-k)! P_j^k(cos theta) e^{i k phi} / r^{j+1}
 * (P with the Condon-Shortley phase).  The sum is taken as in eq. 12 (real,
 * reciprocal k != 0 and self term, kappa of the plan) minus the explicit
 * images with max|nu_a| <= 2.  cap = number of doubles available in out
 * (>= 2 (2p+1)^2).
 */
fmm_status fmm_lattice_tensor(fmm_plan_t plan, double *out, int64_t cap);

/*
 * Batches of independent boxes -- e.g. the charging windows lambda_w of a
 * free-energy calculation (the lambda-scaled solute-solvent interaction of
 * eq. Vswucheme), each window its own periodic box with its own atom count
 * and edge.  All boxes share the order p, the precision and the
 * box-independent operators; each has its own tree depth.
 *
 * fmm_plan_batch -- nbox boxes of edges box[w] (host, nbox doubles).
 *   levels: host nbox ints (1..10), or NULL to choose each depth from a cost
 *           model of this library's P2P and M2L rates and natoms[w];
 *   natoms: host nbox expected atom counts (used only when levels is NULL).
 *   Default precision FMM_FP64; kappa is 3/box[w] per box (fmm_plan_config on
 *   a batch plan takes kappa = 0).  The plan owns one HIP stream per box and
 *   one of its own (used when the configured stream is NULL).
 *
 * fmm_energy_forces_batch -- energies of all boxes.  Box w holds the atoms
 *   offsets[w] .. offsets[w+1]-1 (host, nbox + 1 non-decreasing int64) of
 *   pos (device, x 3 FP64) and q (device FP64); energies: host out, nbox;
 *   forces: device out (same rows as pos) or NULL.  The boxes run as
 *   parallel branches of one HIP graph launch on the plan stream; the graph
 *   is captured on the first call and replayed while offsets, the three
 *   pointers and the precision stay the same (inputs may change in place).
 *   Empty boxes give 0.  Caches the per-box state for
 *   fmm_solute_solvent_energy_batch and fmm_lambda_energy_batch.
 *
 * fmm_solute_solvent_energy_batch -- e_uv[w] (host out, nbox) of every box
 *   (see fmm_solute_solvent_energy) for mask (device, same rows as pos),
 *   one graph launch.  FMM_ERR_STATE without a preceding
 *   fmm_energy_forces_batch on this plan.
 *
 * fmm_autotune_batch -- times, on the given inputs, whole evaluations of
 *   every box at depths L-1, L, L+1 around its current one and with 2, 4 and
 *   8 P2P source groups, and keeps the fastest; forces_scratch: device, same
 *   rows as pos x 3, or NULL.  fmm_batch_levels reports the chosen depths and
 *   P2P group counts (0 = from the leaf occupancy), host nbox ints each, either
 *   may be NULL.
 *
 * fmm_batch_set_tuning -- sets every box's depth (levels[w] in [1, 10]) and
 *   P2P source-group count (p2p_groups[w]: 0, 1, 2, 4, 8 or 16), host nbox ints
 *   each; NULL keeps that setting.  Every value is checked before any box
 *   changes (FMM_ERR_INVALID).  Waits for the device; the next batch call
 *   captures its graph anew.
 *
 * fmm_autotune_batch_cached -- fmm_autotune_batch with a cache file
 *   (cache_path: a text file, created if absent, one line per tuned batch).
 *   The key of a line is the device architecture, p, the precision mode, the
 *   FP64 top levels and every box's edge and atom count (from offsets).  On
 *   a key found in the file the stored depths and group counts are applied
 *   as by fmm_batch_set_tuning, nothing is timed and *hit = 1; otherwise the
 *   batch is tuned, the result appended as one line and *hit = 0 (hit may be
 *   NULL).  Lines that do not parse are skipped; the last valid line of a
 *   key wins.  If the file cannot be written the tuning stays applied and
 *   the call returns FMM_ERR_INVALID.  Concurrent writers may interleave
 *   lines but each line is one write.
 *
 * Single-box calls (fmm_energy_forces, fmm_bin, ...) reject a batch plan and
 * the *_batch calls reject a single-box plan (FMM_ERR_INVALID).
 */
fmm_status fmm_plan_batch(int nbox, const double *box, const int64_t *natoms, const int *levels, int p,
                          fmm_plan_t *out);
fmm_status fmm_energy_forces_batch(fmm_plan_t plan, const int64_t *offsets, const double *pos, const double *q,
                                   double *energies, double *forces);
fmm_status fmm_solute_solvent_energy_batch(fmm_plan_t plan, const uint8_t *mask, double *e_uv);
/* Batched fmm_lambda_energy: lambdas (host, nbox) in, v_lambda and dv_dlambda
 * (host, nbox; either may be NULL) out, one graph launch. */
fmm_status fmm_lambda_energy_batch(fmm_plan_t plan, const uint8_t *mask, const double *lambdas, double *v_lambda,
                                   double *dv_dlambda);
fmm_status fmm_autotune_batch(fmm_plan_t plan, const int64_t *offsets, const double *pos, const double *q,
                              double *forces_scratch);
fmm_status fmm_batch_levels(fmm_plan_t plan, int *levels, int *p2p_groups);
fmm_status fmm_batch_set_tuning(fmm_plan_t plan, const int *levels, const int *p2p_groups);
fmm_status fmm_autotune_batch_cached(fmm_plan_t plan, const int64_t *offsets, const double *pos, const double *q,
                                     double *forces_scratch, const char *cache_path, int *hit);

/*
 * Stage timing.  fmm_profile(plan, 1) creates HIP events on the plan's stream
 * and from then on every fmm_energy_forces call records one event pair around
 * each stage group below and adds the elapsed milliseconds to per-stage
 * accumulators (read after the call's own synchronisation, so no extra host
 * round trip); fmm_profile(plan, 0) stops and frees them.  Enabling resets the
 * accumulators.  fmm_profile_read copies FMM_NUM_STAGES doubles (ms, summed
 * over calls) and the number of profiled calls.
 */
enum {
    FMM_STAGE_SORT = 0,      /* wrap, bin, Morton keys, counting sort        */
    FMM_STAGE_GATHER = 1,    /* repack into sorted leaf-local coordinates    */
    FMM_STAGE_P2M = 2,
    FMM_STAGE_M2M = 3,
    FMM_STAGE_LATTICE = 4,   /* level-0 image-lattice operator (eq. 12)      */
    FMM_STAGE_M2L = 5,       /* all levels                                   */
    FMM_STAGE_M2L_LEAF = 6,  /* finest level only (also counted in M2L)      */
    FMM_STAGE_L2L = 7,
    FMM_STAGE_L2P = 8,
    FMM_STAGE_P2P = 9,
    FMM_STAGE_FINAL = 10,    /* moments, corrections, energy reduction       */
    FMM_STAGE_TOTAL = 11,    /* first to last event of the call              */
    FMM_NUM_STAGES = 12
};
fmm_status fmm_profile(fmm_plan_t plan, int enable);
fmm_status fmm_profile_read(fmm_plan_t plan, double *ms, int64_t *calls);

/*
 * fmm_plan_info -- layout facts of a plan, for tools and benchmarks.
 * Writes min(n, FMM_INFO_COUNT) int64 values to info (host):
 *   [0] levels (0 for a batch plan: see fmm_batch_levels)   [1] p
 *   [2] K = (p+1)^2   [3] Kp (K padded to 16)   [4] precision mode
 *   [5]-[7] and [10] describe the finest level's M2L in the plan's current
 *   precision mode (FP32 in the mixed modes, FP64 in FMM_FP64):
 *   [5] symmetry folding of its interaction list: 0 = none (the 875 offsets:
 *       the BF16 M2L, and the split-FP16 one except at p = 11, 12),
 *       1 = (t, -t) pairs, 2 = orbits of the two-axis flips (the operators of
 *       reflected offsets differ by signs only, so each pair or orbit is one
 *       operator product per row class)
 *   [6] list entries per cell under that folding (875, 573 or 305)
 *   [7] launches of the M2L kernel per full-list level
 *   [8] tree levels run in FP64 (1 .. [8]; all of them in FMM_FP64; for a
 *       batch plan the fmm_plan_tuning setting)
 *   [9] near-field source groups set by fmm_plan_tuning (0 = automatic)
 *   [10] operator rows the matrix cores run per list entry (folded: each row
 *       class padded to whole 16-row blocks; plain: Kp, and for the plain
 *       split-FP16 kernel 64 ceil(n / 4) per row group of n blocks; >= K)
 */
#define FMM_INFO_COUNT 11
fmm_status fmm_plan_info(fmm_plan_t plan, int64_t *info, int n);

/* Message of the last failed call on this plan (never NULL; "" if none).
 * fmm_last_error(NULL) reports failures of fmm_plan itself. */
const char *fmm_last_error(fmm_plan_t plan);

/* Frees the plan and its device memory.  NULL is ignored. */
void fmm_destroy(fmm_plan_t plan);

/* Library version string. */
const char *fmm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FMM_H */
