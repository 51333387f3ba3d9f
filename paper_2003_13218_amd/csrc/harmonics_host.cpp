// Host-side FP64 precompute for libfmm: solid harmonics, the scale-invariant
// translation operators in real storage, the interaction-list offsets and the
// periodic lattice tensor of eq. 12.
//
// Conventions (complex, Condon-Shortley phase):
//   R_n^m(r) = r^n P_n^m(cos t) e^{i m phi} / (n+m)!
//   I_n^m(r) = (n-m)! P_n^m(cos t) e^{i m phi} / r^{n+1}
// so that R_n^{-m} = (-1)^m conj(R_n^m) (same for I) and
//   1/|r - s| = sum_{n,m} conj(R_n^m(s)) I_n^m(r)                (|s| < |r|)
//   R_n^m(a + b) = sum_{k,l} R_k^l(a) R_{n-k}^{m-l}(b)
//   I_n^m(a + s) = sum_{k,l} (-1)^k conj(R_k^l(s)) I_{n+k}^{m+l}(a) (|s| < |a|).
// With M_n^m = sum_j q_j conj(R_n^m(r_j - c)) and L_n^m = sum_j q_j I_n^m(r_j - c')
// the far-field potential near c' is phi(c' + x) = sum conj(R_n^m(x)) L_n^m, and
//   M2M  M_n^m(P)  = sum_{k,l} conj(R_{n-k}^{m-l}(c - P)) M_k^l(c)
//   M2L  L_n^m(c') = sum_{k,l} (-1)^k I_{n+k}^{m+l}(c - c') M_k^l(c)   (eq. Lcoeffdef)
//   L2L  L_k^l(c'') = sum_{n,m} conj(R_{n-k}^{m-l}(c'' - c')) L_n^m(c')
// These are the paper's P2M / M2M / M2L / L2L / L2P steps (Appendix B)
// written in one consistent normalisation; the paper leaves the
// normalisation of R and I open.
#include <cmath>
#include <cstring>
#include <algorithm>
#include <functional>

#include "fmm_internal.h"

namespace fmm {

static inline int cidx(int n, int m) { return n * n + n + m; }

void regular_complex(double x, double y, double z, int J, cplx *R) {
    const double r2 = x * x + y * y + z * z;
    cplx mm(1.0, 0.0);
    for (int m = 0; m <= J; ++m) {
        if (m > 0) mm *= cplx(-x, -y) / double(2 * m);
        R[cidx(m, m)] = mm;
        if (m + 1 <= J) R[cidx(m + 1, m)] = z * mm;
        for (int n = m + 2; n <= J; ++n)
            R[cidx(n, m)] = (double(2 * n - 1) * z * R[cidx(n - 1, m)] - r2 * R[cidx(n - 2, m)]) /
                            double((n + m) * (n - m));
    }
    for (int n = 0; n <= J; ++n)
        for (int m = 1; m <= n; ++m) R[cidx(n, -m)] = ((m & 1) ? -1.0 : 1.0) * std::conj(R[cidx(n, m)]);
}

void irregular_complex(double x, double y, double z, int J, cplx *I) {
    const double r2 = x * x + y * y + z * z;
    cplx mm(1.0 / std::sqrt(r2), 0.0);
    for (int m = 0; m <= J; ++m) {
        if (m > 0) mm *= -double(2 * m - 1) * cplx(x, y) / r2;
        I[cidx(m, m)] = mm;
        if (m + 1 <= J) I[cidx(m + 1, m)] = double(2 * m + 1) * z / r2 * mm;
        for (int n = m + 2; n <= J; ++n)
            I[cidx(n, m)] = (double(2 * n - 1) * z * I[cidx(n - 1, m)] -
                             double((n - 1 - m) * (n - 1 + m)) * I[cidx(n - 2, m)]) / r2;
    }
    for (int n = 0; n <= J; ++n)
        for (int m = 1; m <= n; ++m) I[cidx(n, -m)] = ((m & 1) ? -1.0 : 1.0) * std::conj(I[cidx(n, m)]);
}

// sqrt((n+|m|)!(n-|m|)!) for n <= 2 kMaxP, tabulated once.
double norm_factor(int n, int m) {
    static const std::vector<double> tab = [] {
        const int J = 2 * kMaxP + 1;
        std::vector<double> t((size_t)(J + 1) * (J + 1));
        for (int a = 0; a <= J; ++a)
            for (int b = 0; b <= a; ++b)
                t[(size_t)a * (J + 1) + b] = std::sqrt(std::tgamma(double(a + b + 1)) * std::tgamma(double(a - b + 1)));
        return t;
    }();
    if (m < 0) m = -m;
    return tab[(size_t)n * (2 * kMaxP + 2) + m];
}

// Build a real-storage operator from a complex coefficient function
// c(no, mo, ni, mi) defined for all signed orders (out = sum c * in, in the
// normalised complex basis).  in_f2 / out_f2: whether that side stores
// 2 Re / 2 Im for m > 0 (local expansions) or Re / Im (multipoles).
static void build_real(int p_out, int p_in, bool in_f2, bool out_f2,
                       const std::function<cplx(int, int, int, int)> &c, double *A) {
    const int Ko = num_coeffs(p_out), Ki = num_coeffs(p_in);
    std::memset(A, 0, sizeof(double) * (size_t)Ko * Ki);
    const double fo = out_f2 ? 2.0 : 1.0;
    const double si = in_f2 ? 0.5 : 1.0;
    for (int n = 0; n <= p_out; ++n)
        for (int m = 0; m <= n; ++m)
            for (int k = 0; k <= p_in; ++k)
                for (int l = 0; l <= k; ++l) {
                    cplx a = c(n, m, k, l);
                    // (column index, contribution to the complex output per unit input)
                    int col[2];
                    cplx w[2];
                    int ncol;
                    if (l == 0) {
                        col[0] = k * k;
                        w[0] = a;
                        ncol = 1;
                    } else {
                        cplx b = ((l & 1) ? -1.0 : 1.0) * c(n, m, k, -l);
                        // input X = x + i y at order l, X_{-l} = (-1)^l conj(X)
                        col[0] = k * k + 2 * l - 1;  // x
                        w[0] = si * (a + b);
                        col[1] = k * k + 2 * l;      // y
                        w[1] = si * cplx(0.0, 1.0) * (a - b);
                        ncol = 2;
                    }
                    for (int u = 0; u < ncol; ++u) {
                        if (m == 0) {
                            A[(size_t)(n * n) * Ki + col[u]] += w[u].real();
                        } else {
                            A[(size_t)(n * n + 2 * m - 1) * Ki + col[u]] += fo * w[u].real();
                            A[(size_t)(n * n + 2 * m) * Ki + col[u]] += fo * w[u].imag();
                        }
                    }
                }
}

void build_m2l_operator(int p, const double t[3], double *A) {
    std::vector<cplx> I((size_t)(2 * p + 1) * (2 * p + 1));
    irregular_complex(t[0], t[1], t[2], 2 * p, I.data());
    build_real(p, p, false, true, [&](int n, int m, int k, int l) -> cplx {
        if (std::abs(m + l) > n + k) return cplx(0.0);
        return ((k & 1) ? -1.0 : 1.0) * I[cidx(n + k, m + l)] / (norm_factor(n, m) * norm_factor(k, l));
    }, A);
}

void build_lattice_operator(int p, const cplx *T, double *A) {
    build_real(p, p, false, true, [&](int n, int m, int k, int l) -> cplx {
        if (std::abs(m + l) > n + k) return cplx(0.0);
        return ((k & 1) ? -1.0 : 1.0) * T[cidx(n + k, m + l)] / (norm_factor(n, m) * norm_factor(k, l));
    }, A);
}

// Child octant o = 4 ox + 2 oy + oz of a parent of edge 2 (scaled units: child
// edge 1).  Child centre - parent centre = (o - 1/2) per axis.  Scaled
// multipoles: M~_P,n = 2^{-n} sum_k A(delta)_{nk} M~_c,k.
void build_m2m_operator(int p, int o, double *A) {
    const double d[3] = {((o >> 2) & 1) - 0.5, ((o >> 1) & 1) - 0.5, (o & 1) - 0.5};
    std::vector<cplx> R((size_t)(p + 1) * (p + 1));
    regular_complex(d[0], d[1], d[2], p, R.data());
    build_real(p, p, false, false, [&](int n, int m, int k, int l) -> cplx {
        if (k > n || std::abs(m - l) > n - k) return cplx(0.0);
        return std::conj(R[cidx(n - k, m - l)]) * norm_factor(n, m) / norm_factor(k, l) *
               std::pow(0.5, n);
    }, A);
}

// Parent (edge 2) -> child octant o (edge 1): L~_c,k = sum_n A(delta)_{kn} L~_P,n / 2^{n+1},
// with L_k^l(c'') = sum_{n,m} conj(R_{n-k}^{m-l}(c'' - c')) L_n^m(c').
void build_l2l_operator(int p, int o, double *A) {
    const double d[3] = {((o >> 2) & 1) - 0.5, ((o >> 1) & 1) - 0.5, (o & 1) - 0.5};
    std::vector<cplx> R((size_t)(p + 1) * (p + 1));
    regular_complex(d[0], d[1], d[2], p, R.data());
    build_real(p, p, true, true, [&](int k, int l, int n, int m) -> cplx {
        if (n < k || std::abs(m - l) > n - k) return cplx(0.0);
        return std::conj(R[cidx(n - k, m - l)]) * norm_factor(n, m) / norm_factor(k, l) *
               std::pow(0.5, n + 1);
    }, A);
}

Offsets build_offsets() {
    Offsets o;
    // all offsets with 2 < max|t| <= 5, in a fixed order
    std::vector<int> id(11 * 11 * 11, -1);
    for (int x = -5; x <= 5; ++x)
        for (int y = -5; y <= 5; ++y)
            for (int z = -5; z <= 5; ++z) {
                int mx = std::max(std::abs(x), std::max(std::abs(y), std::abs(z)));
                if (mx <= kWS) continue;
                id[(x + 5) * 121 + (y + 5) * 11 + (z + 5)] = (int)(o.vec.size() / 3);
                o.vec.push_back(x);
                o.vec.push_back(y);
                o.vec.push_back(z);
            }
    // per parity class: children of the parent's +-2 neighbours minus the own +-2 block
    o.il.assign(8 * kILSize, 0);
    for (int par = 0; par < 8; ++par) {
        const int px = (par >> 2) & 1, py = (par >> 1) & 1, pz = par & 1;
        int cnt = 0;
        for (int x = -5; x <= 5; ++x)
            for (int y = -5; y <= 5; ++y)
                for (int z = -5; z <= 5; ++z) {
                    // t = 2 delta + sigma - parity with delta in [-2,2], sigma in {0,1}
                    auto ok = [](int t, int pp) { int u = t + pp; return u >= -4 && u <= 5; };
                    if (!ok(x, px) || !ok(y, py) || !ok(z, pz)) continue;
                    int mx = std::max(std::abs(x), std::max(std::abs(y), std::abs(z)));
                    if (mx <= kWS) continue;
                    o.il[par * kILSize + cnt++] = id[(x + 5) * 121 + (y + 5) * 11 + (z + 5)];
                }
        (void)cnt;
    }
    return o;
}

// ---------------------------------------------------------------------------
// Lattice tensor of eq. 12 (unit box, b = 1).
// Real space  (eq. 12a): sum_{nu != 0} I_j^k(nu) Q(j + 1/2, kappa^2 |nu|^2),
//             Q(a, x) = Gamma(a, x) / Gamma(a) (regularised upper incomplete gamma,
//             upward recurrence Q(a+1, x) = Q(a, x) + x^a e^{-x} / Gamma(a+1) from
//             Q(1/2, x) = erfc(sqrt x); every term is positive, so it is stable).
// Reciprocal  (eq. 12b): pi^{3/2} i^j / (2^{j-2} Gamma(j + 1/2) V)
//             * sum_{k != 0} I_j^k(k) |k|^{2j-1} exp(-|k|^2 / 4 kappa^2), k = 2 pi n.
//             The k = 0 term is left out: with a background charge it is carried
//             by the charged-system and quadrupole terms (eqs. surfcharged1-3).
// Self        (eq. 12c): -2 kappa / sqrt(pi) for j = k = 0.
// From the Ewald value the explicit images 0 < max|nu| <= 2 are subtracted:
// those reach every target through the tree's own M2L at levels >= 1 and the
// near field, so the level-0 operator carries only max|nu| > 2.
// For j > kEwaldMaxJ the sum over max|nu| > 2 converges absolutely and fast
// (terms fall as |nu|^{-(j+1)}); it is then summed directly, which avoids the
// cancellation of subtracting the large near images.
// ---------------------------------------------------------------------------
static constexpr int kEwaldMaxJ = 12;

void lattice_tensor(int J, double kappa0, cplx *T) {
    const int KJ = (J + 1) * (J + 1);
    for (int i = 0; i < KJ; ++i) T[i] = cplx(0.0);
    const int JE = std::min(J, kEwaldMaxJ);

    // j = 0 uses the plan's kappa (it must match the charged-system term);
    // j >= 1 are kappa-independent, use a fixed well-balanced split.
    for (int pass = 0; pass < 2; ++pass) {
        const int jlo = pass == 0 ? 0 : 1;
        const int jhi = pass == 0 ? 0 : JE;
        if (jhi < jlo) continue;
        const double kap = pass == 0 ? kappa0 : 2.5;
        // real-space radius: Q(jhi + 1/2, kappa^2 r^2) below ~1e-18
        const double xcut = 45.0 + 2.5 * jhi;
        const double rmax = std::sqrt(xcut) / kap;
        const int nr = std::max((int)std::ceil(rmax) + 1, kWS);
        std::vector<cplx> I((size_t)(jhi + 1) * (jhi + 1));
        std::vector<double> Qv(jhi + 1);
        for (int a = -nr; a <= nr; ++a)
            for (int b = -nr; b <= nr; ++b)
                for (int c = -nr; c <= nr; ++c) {
                    if (a == 0 && b == 0 && c == 0) continue;
                    const double r2 = double(a * a + b * b + c * c);
                    const bool near = std::max(std::abs(a), std::max(std::abs(b), std::abs(c))) <= kWS;
                    const double x = kap * kap * r2;
                    if (x > xcut && !near) continue;
                    irregular_complex(a, b, c, jhi, I.data());
                    double q = std::erfc(std::sqrt(x));
                    for (int j = 0; j <= jhi; ++j) {
                        if (j > 0) q += std::exp((j - 0.5) * std::log(x) - x - std::lgamma(j + 0.5));
                        Qv[j] = q;
                    }
                    for (int j = jlo; j <= jhi; ++j) {
                        const double w = Qv[j] - (near ? 1.0 : 0.0);
                        for (int k = -j; k <= j; ++k) T[cidx(j, k)] += I[cidx(j, k)] * w;
                    }
                }
        // reciprocal space, k = 2 pi n; summand ~ |k|^{j-2} exp(-k^2/4kappa^2)
        const double kcut = 2.0 * kap * std::sqrt(xcut);
        const int nk = (int)std::ceil(kcut / (2.0 * M_PI)) + 1;
        for (int a = -nk; a <= nk; ++a)
            for (int b = -nk; b <= nk; ++b)
                for (int c = -nk; c <= nk; ++c) {
                    if (a == 0 && b == 0 && c == 0) continue;
                    const double kx = 2.0 * M_PI * a, ky = 2.0 * M_PI * b, kz = 2.0 * M_PI * c;
                    const double k2 = kx * kx + ky * ky + kz * kz;
                    const double kk = std::sqrt(k2);
                    if (kk > kcut) continue;
                    irregular_complex(kx, ky, kz, jhi, I.data());
                    const double g = std::exp(-k2 / (4.0 * kap * kap));
                    for (int j = jlo; j <= jhi; ++j) {
                        // i^j
                        cplx ij = (j % 4 == 0) ? cplx(1, 0) : (j % 4 == 1) ? cplx(0, 1)
                                : (j % 4 == 2) ? cplx(-1, 0) : cplx(0, -1);
                        const double pref = std::pow(M_PI, 1.5) / (std::pow(2.0, j - 2) * std::tgamma(j + 0.5));
                        const cplx f = ij * pref * std::pow(kk, 2 * j - 1) * g;
                        for (int k = -j; k <= j; ++k) T[cidx(j, k)] += I[cidx(j, k)] * f;
                    }
                }
        if (pass == 0) T[cidx(0, 0)] += -2.0 * kap / std::sqrt(M_PI);
    }

    // direct sums for kEwaldMaxJ < j <= J over 2 < max|nu| <= R
    if (J > JE) {
        const int R = 30;
        std::vector<cplx> I((size_t)(J + 1) * (J + 1));
        for (int a = -R; a <= R; ++a)
            for (int b = -R; b <= R; ++b)
                for (int c = -R; c <= R; ++c) {
                    if (std::max(std::abs(a), std::max(std::abs(b), std::abs(c))) <= kWS) continue;
                    irregular_complex(a, b, c, J, I.data());
                    for (int j = JE + 1; j <= J; ++j)
                        for (int k = -j; k <= j; ++k) T[cidx(j, k)] += I[cidx(j, k)];
                }
    }
}

void build_rec_tables(RecTables *t) {
    std::memset(t, 0, sizeof(*t));
    for (int n = 0; n <= kMaxP; ++n)
        for (int m = 0; m <= n; ++m) {
            const int i = n * (n + 1) / 2 + m;
            if (n >= m + 2) {
                t->a[i] = double(2 * n - 1) / std::sqrt(double((n + m) * (n - m)));
                t->b[i] = std::sqrt(double((n + m - 1) * (n - m - 1)) / double((n + m) * (n - m)));
            }
        }
    for (int m = 0; m <= kMaxP; ++m) {
        t->c[m] = m > 0 ? std::sqrt(double(2 * m - 1) / double(2 * m)) : 0.0;
        t->d[m] = std::sqrt(double(2 * m + 1));
    }
}

}  // namespace fmm
