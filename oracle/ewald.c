/*
 * oracle/ewald.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct FP64 CPU reference for the periodic
 * Coulomb energy, potential and forces of N point charges in a cubic cell
 * neutralised by a uniform background charge, under the conducting
 * ("tin-foil") boundary at infinity.  Only tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library; the product path never
 * does.  It shares no code, header or table with the GPU library.
 *
 * What it computes (Appendix A of the paper, Ewald split of eq. Velec, the
 * terms of Table A-1):
 *   E      = E_real + E_rec + E_self + E_charged
 *   E_real = 1/2 sum_nu' sum_ij q_i q_j erfc(kappa d)/d,  d = |r_i - r_j + nu b|
 *            (the prime drops i == j at nu == 0; the paper's r_i - r_i is read
 *            as r_i - r_j)                                   -- eq. Ereal
 *   E_rec  = (2 pi / V) sum_{k != 0} exp(-k^2/4kappa^2)/k^2 |S(k)|^2,
 *            S(k) = sum_j q_j exp(i k.r_j), k = 2 pi n / b    -- eq. VPPrec
 *   E_self = -(kappa/sqrt(pi)) sum_i q_i^2                    -- eq. Eself
 *   E_charged = -pi Q^2 / (2 V kappa^2), Q = sum_i q_i        -- eq. 6
 * The k = 0 term is dropped: with the conducting boundary the surface term
 * of eq. surftotal is zero.  Units are Gaussian (no 1/(4 pi eps0)).
 *
 * phi_i = dE/dq_i (so E = 1/2 sum_i q_i phi_i) and F_i = -dE/dr_i follow by
 * differentiating the four terms above.
 *
 * The solute-solvent energy W = E(u+v) - E(u) - E(v), each set with its own
 * background, is the cross part of the same four terms:
 *   W = sum_{i in u, j in v} sum_nu q_i q_j erfc(kappa d)/d
 *     + (4 pi / V) sum_{k != 0} A_k Re(S_u(k) conj(S_v(k)))
 *     - pi Q_u Q_v / (V kappa^2).
 *
 * Sums that produce energies use Neumaier compensated summation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Neumaier compensated accumulator. */
typedef struct { double s, c; } nsum_t;
static inline void nadd(nsum_t *a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static inline double nval(const nsum_t *a) { return a->s + a->c; }

static inline double wrap_coord(double x, double b) {
    double y = x - b * floor(x / b);
    if (y >= b) y = 0.0;
    if (y < 0.0) y = 0.0;
    return y;
}

/* ----------------------------------------------------------------------- */
/* Real-space part over a cell list with explicit periodic images.          */
/* For every target atom i (listed in idx) and every source atom j, every   */
/* image j + nu b with |r_i - r_j - nu b| < rcut is visited exactly once:    */
/* the cell offsets (dx,dy,dz) in [-m, m]^3 around i's cell each name one    */
/* image of one wrapped cell, so nothing is deduplicated.                    */
/* ----------------------------------------------------------------------- */
typedef struct {
    int nc;            /* cells per dimension */
    double cs;         /* cell size */
    int64_t *start;    /* nc^3 + 1 */
    int64_t *list;     /* atom indices grouped by cell */
} clist_t;

static int build_clist(clist_t *cl, int64_t n, const double *w, double box, double rcut) {
    int nc = (int)floor(box / rcut);
    if (nc < 1) nc = 1;
    if (nc > 256) nc = 256;
    cl->nc = nc;
    cl->cs = box / nc;
    int64_t ncell = (int64_t)nc * nc * nc;
    cl->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    cl->list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *cell = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *fill = (int64_t *)calloc((size_t)ncell, sizeof(int64_t));
    if (!cl->start || !cl->list || !cell || !fill) { free(cell); free(fill); return -1; }
    for (int64_t i = 0; i < n; ++i) {
        int c[3];
        for (int a = 0; a < 3; ++a) {
            c[a] = (int)floor(w[3 * i + a] / cl->cs);
            if (c[a] >= nc) c[a] = nc - 1;
            if (c[a] < 0) c[a] = 0;
        }
        cell[i] = ((int64_t)c[0] * nc + c[1]) * nc + c[2];
        cl->start[cell[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) cl->start[c + 1] += cl->start[c];
    for (int64_t i = 0; i < n; ++i) cl->list[cl->start[cell[i]] + fill[cell[i]]++] = i;
    free(cell);
    free(fill);
    return 0;
}

static void free_clist(clist_t *cl) { free(cl->start); free(cl->list); }

/* Real-space potential and field at atom i from all sources (optionally only
 * those with srcmask[j] == want).  Returns phi (sum q_j erfc/d) and grad
 * accumulates  sum q_j [erfc(kd)/d + 2k/sqrt(pi) exp(-k^2 d^2)] dvec/d^2,
 * which is -(d phi / d r_i). */
static void real_one(int64_t i, const double *w, const double *q, double box, double kappa,
                     double rcut, const clist_t *cl, const uint8_t *srcmask, int want,
                     double *phi_out, double efield[3]) {
    const int nc = cl->nc;
    const double cs = cl->cs;
    const int m = (int)ceil(rcut / cs);
    const double rc2 = rcut * rcut;
    const double two_k_sqrtpi = 2.0 * kappa / sqrt(M_PI);
    int ci[3];
    for (int a = 0; a < 3; ++a) {
        ci[a] = (int)floor(w[3 * i + a] / cs);
        if (ci[a] >= nc) ci[a] = nc - 1;
        if (ci[a] < 0) ci[a] = 0;
    }
    nsum_t ph = {0, 0}, ex = {0, 0}, ey = {0, 0}, ez = {0, 0};
    for (int dx = -m; dx <= m; ++dx)
        for (int dy = -m; dy <= m; ++dy)
            for (int dz = -m; dz <= m; ++dz) {
                int u[3] = {ci[0] + dx, ci[1] + dy, ci[2] + dz};
                int s[3];
                double shift[3];
                for (int a = 0; a < 3; ++a) {
                    int img = (int)floor((double)u[a] / nc);
                    s[a] = u[a] - img * nc;
                    shift[a] = img * box;
                }
                int64_t sc = ((int64_t)s[0] * nc + s[1]) * nc + s[2];
                /* the zero image of cell ci is only reached at offset (0,0,0) */
                int self_image = (shift[0] == 0.0 && shift[1] == 0.0 && shift[2] == 0.0);
                for (int64_t p = cl->start[sc]; p < cl->start[sc + 1]; ++p) {
                    int64_t j = cl->list[p];
                    if (srcmask && (int)srcmask[j] != want) continue;
                    if (j == i && self_image) continue;
                    double d0 = w[3 * i + 0] - (w[3 * j + 0] + shift[0]);
                    double d1 = w[3 * i + 1] - (w[3 * j + 1] + shift[1]);
                    double d2 = w[3 * i + 2] - (w[3 * j + 2] + shift[2]);
                    double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                    if (r2 >= rc2) continue;
                    double r = sqrt(r2);
                    double e = erfc(kappa * r) / r;
                    nadd(&ph, q[j] * e);
                    double g = q[j] * (e + two_k_sqrtpi * exp(-kappa * kappa * r2)) / r2;
                    nadd(&ex, g * d0);
                    nadd(&ey, g * d1);
                    nadd(&ez, g * d2);
                }
            }
    *phi_out = nval(&ph);
    efield[0] = nval(&ex);
    efield[1] = nval(&ey);
    efield[2] = nval(&ez);
}

/* ----------------------------------------------------------------------- */
/* Reciprocal-space structure factors over the half space of n vectors.     */
/* ----------------------------------------------------------------------- */
typedef struct {
    int64_t nk;
    int *n;         /* nk x 3 integer vectors */
    double *ak;     /* exp(-k^2/4kappa^2)/k^2 */
} kset_t;

static int build_kset(kset_t *ks, double box, double kappa, double kmax, int *nmax_out) {
    int nmax = (int)floor(kmax * box / (2.0 * M_PI));
    if (nmax < 0) nmax = 0;
    *nmax_out = nmax;
    int64_t cap = (int64_t)(2 * nmax + 1) * (2 * nmax + 1) * (2 * nmax + 1);
    ks->n = (int *)malloc(sizeof(int) * 3 * (size_t)(cap > 0 ? cap : 1));
    ks->ak = (double *)malloc(sizeof(double) * (size_t)(cap > 0 ? cap : 1));
    if (!ks->n || !ks->ak) return -1;
    int64_t nk = 0;
    const double kk = 2.0 * M_PI / box;
    for (int a = 0; a <= nmax; ++a)
        for (int b = -nmax; b <= nmax; ++b)
            for (int c = -nmax; c <= nmax; ++c) {
                /* half space: a > 0, or a == 0 and b > 0, or a == b == 0 and c > 0 */
                int half = (a > 0) || (a == 0 && b > 0) || (a == 0 && b == 0 && c > 0);
                if (!half) continue;
                double k2 = kk * kk * (double)(a * a + b * b + c * c);
                if (k2 > kmax * kmax) continue;
                ks->n[3 * nk + 0] = a;
                ks->n[3 * nk + 1] = b;
                ks->n[3 * nk + 2] = c;
                ks->ak[nk] = exp(-k2 / (4.0 * kappa * kappa)) / k2;
                ++nk;
            }
    ks->nk = nk;
    return 0;
}

/* Per-axis phase table: tab[(i*3 + axis)*(2nmax+1) + (m+nmax)] = exp(i 2pi m x_a / b),
 * evaluated by direct cos/sin (no recurrence). */
static double *phase_table(int64_t n, const double *w, double box, int nmax) {
    int64_t width = 2 * nmax + 1;
    double *t = (double *)malloc(sizeof(double) * 2 * (size_t)(n * 3 * width > 0 ? n * 3 * width : 1));
    if (!t) return NULL;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a)
            for (int m = -nmax; m <= nmax; ++m) {
                double ang = 2.0 * M_PI * (double)m * w[3 * i + a] / box;
                int64_t o = ((i * 3 + a) * width + (m + nmax)) * 2;
                t[o] = cos(ang);
                t[o + 1] = sin(ang);
            }
    return t;
}

static inline void phase_of(const double *tab, int64_t i, const int *nv, int nmax, double *re, double *im) {
    int64_t width = 2 * nmax + 1;
    double r = 1.0, s = 0.0;
    for (int a = 0; a < 3; ++a) {
        int64_t o = ((i * 3 + a) * width + (nv[a] + nmax)) * 2;
        double cr = tab[o], ci = tab[o + 1];
        double nr = r * cr - s * ci;
        double ni = r * ci + s * cr;
        r = nr;
        s = ni;
    }
    *re = r;
    *im = s;
}

/* Structure factor S(k) = sum_j q_j exp(i k.r_j) for every k in the set,
 * restricted to atoms with mask[j] == want when mask is given. */
static void structure_factors(int64_t n, const double *q, const uint8_t *mask, int want,
                              const double *tab, int nmax, const kset_t *ks,
                              double *sre, double *sim) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < ks->nk; ++k) {
        nsum_t a = {0, 0}, b = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (mask && (int)mask[j] != want) continue;
            double re, im;
            phase_of(tab, j, &ks->n[3 * k], nmax, &re, &im);
            nadd(&a, q[j] * re);
            nadd(&b, q[j] * im);
        }
        sre[k] = nval(&a);
        sim[k] = nval(&b);
    }
}

/* ----------------------------------------------------------------------- */
/* Public entry points (plain C ABI, host pointers).                        */
/* ----------------------------------------------------------------------- */

/*
 * oracle_ewald: energy terms, per-atom potential and force.
 *   n, pos[n*3], q[n]   : atoms (any coordinates; wrapped into [0,b) here)
 *   box                 : cubic cell edge b
 *   kappa, rcut, kmax   : Ewald split parameter, real-space cutoff, |k| cutoff
 *   n_eval, eval_idx    : atoms at which phi/force are returned; eval_idx
 *                         NULL means all atoms (n_eval must equal n)
 *   terms[5]            : E_real, E_rec, E_self, E_charged, E_total; filled
 *                         only when all atoms are evaluated (else NaN)
 *   phi[n_eval], force[n_eval*3] : outputs (may be NULL)
 * Returns 0 on success, -1 on bad arguments, -2 on allocation failure.
 */
int oracle_ewald(int64_t n, const double *pos, const double *q, double box,
                 double kappa, double rcut, double kmax,
                 int64_t n_eval, const int64_t *eval_idx,
                 double *terms, double *phi, double *force) {
    if (n < 0 || !(box > 0) || !(kappa > 0) || !(rcut > 0) || !(kmax >= 0)) return -1;
    if (!eval_idx && n_eval != n) return -1;
    const double V = box * box * box;
    double *w = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!w) return -2;
    for (int64_t i = 0; i < 3 * n; ++i) w[i] = wrap_coord(pos[i], box);

    clist_t cl;
    if (build_clist(&cl, n, w, box, rcut)) { free(w); return -2; }
    kset_t ks;
    int nmax = 0;
    if (build_kset(&ks, box, kappa, kmax, &nmax)) { free(w); free_clist(&cl); return -2; }
    double *tab = phase_table(n, w, box, nmax);
    double *sre = (double *)malloc(sizeof(double) * (size_t)(ks.nk > 0 ? ks.nk : 1));
    double *sim = (double *)malloc(sizeof(double) * (size_t)(ks.nk > 0 ? ks.nk : 1));
    if (!tab || !sre || !sim) { free(w); free_clist(&cl); free(tab); free(sre); free(sim); return -2; }
    structure_factors(n, q, NULL, 0, tab, nmax, &ks, sre, sim);

    nsum_t qtot = {0, 0}, q2 = {0, 0};
    for (int64_t i = 0; i < n; ++i) { nadd(&qtot, q[i]); nadd(&q2, q[i] * q[i]); }
    const double Q = nval(&qtot);
    const double kk = 2.0 * M_PI / box;
    const double self_c = 2.0 * kappa / sqrt(M_PI);
    const double bg_phi = -M_PI * Q / (V * kappa * kappa);

    double *phr = (double *)malloc(sizeof(double) * (size_t)(n_eval > 0 ? n_eval : 1));
    double *php = (double *)malloc(sizeof(double) * (size_t)(n_eval > 0 ? n_eval : 1));
    if (!phr || !php) { free(w); free_clist(&cl); free(tab); free(sre); free(sim); free(phr); free(php); return -2; }

#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t e = 0; e < n_eval; ++e) {
        int64_t i = eval_idx ? eval_idx[e] : e;
        double pr, ef[3];
        real_one(i, w, q, box, kappa, rcut, &cl, NULL, 0, &pr, ef);
        /* reciprocal: phi_rec = (4pi/V) sum_{all k} A_k Re(S e^{-ik r_i})
         *           = 2 (4pi/V) sum_{half} ... ; force as in the header. */
        nsum_t rp = {0, 0}, fx = {0, 0}, fy = {0, 0}, fz = {0, 0};
        for (int64_t k = 0; k < ks.nk; ++k) {
            double cr, ci;
            phase_of(tab, i, &ks.n[3 * k], nmax, &cr, &ci);
            /* S * conj(e^{ik r_i}) */
            double re = sre[k] * cr + sim[k] * ci;
            double im = sim[k] * cr - sre[k] * ci;
            nadd(&rp, ks.ak[k] * re);
            double g = ks.ak[k] * im;
            nadd(&fx, g * kk * ks.n[3 * k + 0]);
            nadd(&fy, g * kk * ks.n[3 * k + 1]);
            nadd(&fz, g * kk * ks.n[3 * k + 2]);
        }
        double rec_phi = 2.0 * (4.0 * M_PI / V) * nval(&rp);
        phr[e] = pr;
        php[e] = rec_phi;
        if (phi) phi[e] = pr + rec_phi - self_c * q[i] + bg_phi;
        if (force) {
            const double cf = -2.0 * (4.0 * M_PI / V) * q[i];
            force[3 * e + 0] = q[i] * ef[0] + cf * nval(&fx);
            force[3 * e + 1] = q[i] * ef[1] + cf * nval(&fy);
            force[3 * e + 2] = q[i] * ef[2] + cf * nval(&fz);
        }
    }

    if (terms) {
        if (!eval_idx) {
            nsum_t er = {0, 0}, ek = {0, 0};
            for (int64_t i = 0; i < n; ++i) nadd(&er, 0.5 * q[i] * phr[i]);
            for (int64_t k = 0; k < ks.nk; ++k)
                nadd(&ek, 2.0 * (2.0 * M_PI / V) * ks.ak[k] * (sre[k] * sre[k] + sim[k] * sim[k]));
            terms[0] = nval(&er);
            terms[1] = nval(&ek);
            terms[2] = -(kappa / sqrt(M_PI)) * nval(&q2);
            terms[3] = -M_PI * Q * Q / (2.0 * V * kappa * kappa);
            nsum_t t = {0, 0};
            for (int a = 0; a < 4; ++a) nadd(&t, terms[a]);
            terms[4] = nval(&t);
        } else {
            for (int a = 0; a < 5; ++a) terms[a] = NAN;
        }
    }
    free(w); free_clist(&cl); free(tab); free(sre); free(sim); free(phr); free(php);
    free(ks.n); free(ks.ak);
    return 0;
}

/*
 * oracle_ewald_uv: the solute-solvent interaction energy of the header,
 * mask[i] = 1 for solute (u), 0 for solvent (v).
 *   terms[4] : W_real, W_rec, W_charged, W_total.
 */
int oracle_ewald_uv(int64_t n, const double *pos, const double *q, const uint8_t *mask,
                    double box, double kappa, double rcut, double kmax, double *terms) {
    if (n < 0 || !(box > 0) || !(kappa > 0) || !(rcut > 0) || !(kmax >= 0) || !mask || !terms) return -1;
    const double V = box * box * box;
    double *w = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!w) return -2;
    for (int64_t i = 0; i < 3 * n; ++i) w[i] = wrap_coord(pos[i], box);
    clist_t cl;
    if (build_clist(&cl, n, w, box, rcut)) { free(w); return -2; }
    kset_t ks;
    int nmax = 0;
    if (build_kset(&ks, box, kappa, kmax, &nmax)) { free(w); free_clist(&cl); return -2; }
    double *tab = phase_table(n, w, box, nmax);
    double *s = (double *)malloc(sizeof(double) * 4 * (size_t)(ks.nk > 0 ? ks.nk : 1));
    if (!tab || !s) { free(w); free_clist(&cl); free(tab); free(s); return -2; }
    double *su_re = s, *su_im = s + ks.nk, *sv_re = s + 2 * ks.nk, *sv_im = s + 3 * ks.nk;
    structure_factors(n, q, mask, 1, tab, nmax, &ks, su_re, su_im);
    structure_factors(n, q, mask, 0, tab, nmax, &ks, sv_re, sv_im);

    nsum_t qu = {0, 0}, qv = {0, 0};
    int64_t nu = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (mask[i]) { nadd(&qu, q[i]); ++nu; } else nadd(&qv, q[i]);
    }
    /* real space: loop over solute atoms, sources restricted to solvent. */
    int64_t *ui = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nu > 0 ? nu : 1));
    double *part = (double *)malloc(sizeof(double) * (size_t)(nu > 0 ? nu : 1));
    if (!ui || !part) { free(w); free_clist(&cl); free(tab); free(s); free(ui); free(part); return -2; }
    for (int64_t i = 0, c = 0; i < n; ++i) if (mask[i]) ui[c++] = i;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t e = 0; e < nu; ++e) {
        double pr, ef[3];
        real_one(ui[e], w, q, box, kappa, rcut, &cl, mask, 0, &pr, ef);
        part[e] = q[ui[e]] * pr;
    }
    nsum_t wr = {0, 0}, wk = {0, 0};
    for (int64_t e = 0; e < nu; ++e) nadd(&wr, part[e]);
    for (int64_t k = 0; k < ks.nk; ++k)
        nadd(&wk, 2.0 * (4.0 * M_PI / V) * ks.ak[k] * (su_re[k] * sv_re[k] + su_im[k] * sv_im[k]));
    terms[0] = nval(&wr);
    terms[1] = nval(&wk);
    terms[2] = -M_PI * nval(&qu) * nval(&qv) / (V * kappa * kappa);
    nsum_t t = {0, 0};
    for (int a = 0; a < 3; ++a) nadd(&t, terms[a]);
    terms[3] = nval(&t);
    free(w); free_clist(&cl); free(tab); free(s); free(ui); free(part);
    free(ks.n); free(ks.ak);
    return 0;
}

/*
 * oracle_nearfield: the near-field sum of eq. EqNF as a plain definition.
 * Atoms are binned into 2^levels leaves per axis after wrapping into [0,b)
 * (leaf index floor(x * 2^levels / b), clamped).  For every atom i in leaf c
 * and every offset t in [-ws, ws]^3, the source leaf is c + t taken modulo
 * 2^levels, and its atoms are shifted by the image vector that the modulo
 * removed; i == j is skipped only for the zero image.  Returns
 *   phi[i]   = sum q_j / d
 *   field[i] = sum q_j dvec / d^3  (dvec = r_i - r_j_image), i.e. -grad phi.
 * Results are in the caller's atom order.
 */
int oracle_nearfield(int64_t n, const double *pos, const double *q, double box, int levels, int ws,
                     double *phi, double *field) {
    if (n < 0 || !(box > 0) || levels < 0 || levels > 10 || ws < 0) return -1;
    const int nc = 1 << levels;
    int64_t ncell = (int64_t)nc * nc * nc;
    double *w = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    int *cc = (int *)malloc(sizeof(int) * 3 * (size_t)(n > 0 ? n : 1));
    int64_t *start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t *fill = (int64_t *)calloc((size_t)ncell, sizeof(int64_t));
    int64_t *list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!w || !cc || !start || !fill || !list) { free(w); free(cc); free(start); free(fill); free(list); return -2; }
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {
            w[3 * i + a] = wrap_coord(pos[3 * i + a], box);
            int c = (int)floor(w[3 * i + a] * ((double)nc / box));
            if (c > nc - 1) c = nc - 1;
            if (c < 0) c = 0;
            cc[3 * i + a] = c;
        }
        int64_t id = ((int64_t)cc[3 * i] * nc + cc[3 * i + 1]) * nc + cc[3 * i + 2];
        start[id + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
    for (int64_t i = 0; i < n; ++i) {
        int64_t id = ((int64_t)cc[3 * i] * nc + cc[3 * i + 1]) * nc + cc[3 * i + 2];
        list[start[id] + fill[id]++] = i;
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        nsum_t ph = {0, 0}, ex = {0, 0}, ey = {0, 0}, ez = {0, 0};
        for (int tx = -ws; tx <= ws; ++tx)
            for (int ty = -ws; ty <= ws; ++ty)
                for (int tz = -ws; tz <= ws; ++tz) {
                    int u[3] = {cc[3 * i] + tx, cc[3 * i + 1] + ty, cc[3 * i + 2] + tz};
                    int s[3];
                    double shift[3];
                    int zero_img = 1;
                    for (int a = 0; a < 3; ++a) {
                        int img = (int)floor((double)u[a] / nc);
                        s[a] = u[a] - img * nc;
                        shift[a] = img * box;
                        if (img != 0) zero_img = 0;
                    }
                    int64_t sc = ((int64_t)s[0] * nc + s[1]) * nc + s[2];
                    for (int64_t p = start[sc]; p < start[sc + 1]; ++p) {
                        int64_t j = list[p];
                        if (j == i && zero_img) continue;
                        double d0 = w[3 * i] - (w[3 * j] + shift[0]);
                        double d1 = w[3 * i + 1] - (w[3 * j + 1] + shift[1]);
                        double d2 = w[3 * i + 2] - (w[3 * j + 2] + shift[2]);
                        double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                        double r = sqrt(r2);
                        nadd(&ph, q[j] / r);
                        double g = q[j] / (r2 * r);
                        nadd(&ex, g * d0);
                        nadd(&ey, g * d1);
                        nadd(&ez, g * d2);
                    }
                }
        if (phi) phi[i] = nval(&ph);
        if (field) {
            field[3 * i] = nval(&ex);
            field[3 * i + 1] = nval(&ey);
            field[3 * i + 2] = nval(&ez);
        }
    }
    free(w); free(cc); free(start); free(fill); free(list);
    return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
