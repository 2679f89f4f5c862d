// krt_tables.cpp -- FP64 host construction of the per-line lookup tables that
// the transport kernel stages into LDS.
//
//  (i)  Voigt profile H(a, x) (Sec. 2.1) as cubic polynomials per interval:
//       512 intervals of width 1/64 on 0 <= |x| < 8, and 128 intervals in
//       w = 8/|x| on |x| >= 8 for G(w) = H x^2 (so H = G w^2 / 64), which tends
//       to a/sqrt(pi) in the far wing.  H and dH/dx come from direct adaptive
//       Gauss-Legendre quadrature of H = (1/pi) int exp(-(x + a tan t)^2) dt,
//       the Voigt integral after the substitution y = x + a tan t.
//  (ii) The atom-velocity sampler of Sec. 2.1.1 (the USampler): the density
//       p(u | x) ~ exp(-u^2)/(a^2 + (x-u)^2) is split, for x >= 0, into four
//       pieces (see krt_internal.h): the resonant core S (|u - x| < DELTA), the
//       Lorentz wing just below it L1, the thermal bump L2 (u <= x - SMID) and
//       the wing above R.  Each piece has a single feature and is smooth in a
//       variable of its own; its quantile function is tabulated on 64 rows of x
//       (48 uniform rows on [0, 8), 16 logarithmic rows on [8, 300]) and the
//       piece probabilities on a fine 1/128 grid of x.  Tabulating quantiles
//       rather than the cumulative distribution moves the narrow resonant peak
//       continuously between rows, and keeping separated features in separate
//       pieces stops interpolation between rows from mixing them.  Symmetry
//       p(u | -x) = p(-u | x) covers x < 0.
//
// Everything here is computed once per line in FP64 and rounded to binary32.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <functional>
#include <algorithm>

#include "krt_internal.h"

namespace krt {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrtPi = 1.77245385090551602730;

// ---- Gauss-Legendre nodes by Newton iteration on P_n (n = 20) -------------
struct GL {
    static constexpr int N = 20;
    double x[N], w[N];
    GL() {
        for (int i = 0; i < N; ++i) {
            double z = std::cos(kPi * (i + 0.75) / (N + 0.5));
            for (int it = 0; it < 100; ++it) {
                double p1 = 1.0, p2 = 0.0;
                for (int j = 1; j <= N; ++j) {
                    double p3 = p2;
                    p2 = p1;
                    p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
                }
                double pp = N * (z * p1 - p2) / (z * z - 1.0);
                double dz = p1 / pp;
                z -= dz;
                if (std::fabs(dz) < 1e-16) {
                    x[i] = z;
                    w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
                    break;
                }
                x[i] = z;
                w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
            }
        }
    }
};

const GL &gl() {
    static GL g;
    return g;
}

using Fn = std::function<double(double)>;

double gl_fixed(const Fn &f, double a, double b) {
    const GL &g = gl();
    double c = 0.5 * (a + b), h = 0.5 * (b - a), s = 0.0;
    for (int i = 0; i < GL::N; ++i) s += g.w[i] * f(c + h * g.x[i]);
    return s * h;
}

double adapt_rec(const Fn &f, double a, double b, double whole, double abstol, int depth) {
    double m = 0.5 * (a + b);
    double l = gl_fixed(f, a, m), r = gl_fixed(f, m, b);
    if (depth <= 0 || std::fabs(l + r - whole) <= abstol) return l + r;
    return adapt_rec(f, a, m, l, 0.5 * abstol, depth - 1) + adapt_rec(f, m, b, r, 0.5 * abstol, depth - 1);
}

// adaptive bisection; the absolute tolerance is relative to the integral of |f|
double integrate(const Fn &f, double a, double b, double rtol) {
    if (b <= a) return 0.0;
    Fn af = [&](double t) { return std::fabs(f(t)); };
    double scale = 0.0;
    for (int k = 0; k < 8; ++k) scale += gl_fixed(af, a + (b - a) * k / 8, a + (b - a) * (k + 1) / 8);
    if (scale == 0.0) return 0.0;
    return adapt_rec(f, a, b, gl_fixed(f, a, b), rtol * scale, 18);
}

// H(a, x) and dH/dx by quadrature of the Voigt integral
//   H(a, x) = (a/pi) int g(y) / ((x - y)^2 + a^2) dy,   g = exp(-y^2),
// and of its x-derivative (g -> -2 y exp(-y^2), after shifting y -> x + s).
// Near the Lorentz peak (|y - x| < 1) the substitution y = x + a tan t makes
// the integrand smooth; elsewhere the integrand is smooth in y and negligible
// beyond |y| = 10.
double voigt_part(double a, double x, const Fn &g) {
    const double c = 1.0, ymax = 10.0;
    double tot = 0.0;
    double Th = std::atan(c / a);
    Fn fp = [&](double t) { return g(x + a * std::tan(t)) / a; };
    if (x - c < ymax && x + c > -ymax) tot += integrate(fp, -Th, Th, 1e-15);
    Fn fo = [&](double y) { double d = x - y; return g(y) / (d * d + a * a); };
    double l1 = -ymax, r1 = std::min(ymax, x - c), l2 = std::max(-ymax, x + c), r2 = ymax;
    if (r1 > l1) {
        if (l1 < 0.0 && r1 > 0.0) tot += integrate(fo, l1, 0.0, 1e-15) + integrate(fo, 0.0, r1, 1e-15);
        else tot += integrate(fo, l1, r1, 1e-15);
    }
    if (r2 > l2) {
        if (l2 < 0.0 && r2 > 0.0) tot += integrate(fo, l2, 0.0, 1e-15) + integrate(fo, 0.0, r2, 1e-15);
        else tot += integrate(fo, l2, r2, 1e-15);
    }
    return tot * a / kPi;
}

void voigt_quad(double a, double x, double *H, double *dH) {
    *H = voigt_part(a, x, [](double y) { return std::exp(-y * y); });
    *dH = voigt_part(a, x, [](double y) { return -2.0 * y * std::exp(-y * y); });
}

// cubic on [0,1] through (y0, m0) and (y1, m1) (values and derivatives times the step)
void hermite_coefs(double y0, double m0, double y1, double m1, float *c) {
    c[0] = (float)y0;
    c[1] = (float)m0;
    c[2] = (float)(3.0 * (y1 - y0) - 2.0 * m0 - m1);
    c[3] = (float)(2.0 * (y0 - y1) + m0 + m1);
}

// ---- sampler pieces -------------------------------------------------------
// density of each piece in its own variable (u-measure times the Jacobian), with
// exp(-x^2) factored out of S and R so that large x does not underflow.
double smid_of(double xa) { return std::max(0.5 * xa, 2.0 * kDelta); }

struct Piece {
    int kind;  // 0 = S (t), 1 = L1 (l), 2 = L2 (u), 3 = R (l)
    double xa, a, thd, smid;
    double vlo, vhi;
    double dens(double v) const {
        if (kind == 0) {
            double tt = a * std::tan(v * thd);
            return std::exp(-2.0 * xa * tt - tt * tt);
        }
        if (kind == 2) {
            double s = xa - v;
            return std::exp(-v * v) / (a * a + s * s);
        }
        double s = kDelta * std::exp(v);
        if (kind == 1) {
            double y = xa - s;
            return std::exp(-y * y) * s / (a * a + s * s);
        }
        return std::exp(-2.0 * xa * s - s * s) * s / (a * a + s * s);
    }
    double vmin() const { return vlo; }
    double vmax_() const { return vhi; }
};

Piece make_piece(int kind, double xa, double a) {
    Piece p;
    p.kind = kind; p.xa = xa; p.a = a; p.thd = std::atan(kDelta / a);
    p.smid = smid_of(xa);
    if (kind == 0) { p.vlo = -1.0; p.vhi = 1.0; }
    else if (kind == 1) { p.vlo = 0.0; p.vhi = std::log(p.smid / kDelta); }
    else if (kind == 2) { p.vlo = std::min(-7.0, xa - p.smid - 1.0); p.vhi = xa - p.smid; }
    else { p.vlo = 0.0; p.vhi = std::log(7.0 / kDelta); }
    return p;
}

// Fine cumulative distribution of a piece on nf intervals; returns the total.
double fine_cdf(const Piece &p, int nf, std::vector<double> &v, std::vector<double> &F,
                std::vector<double> &f) {
    v.resize(nf + 1); F.resize(nf + 1); f.resize(nf + 1);
    double lo = p.vmin(), hi = p.vmax_();
    for (int i = 0; i <= nf; ++i) { v[i] = lo + (hi - lo) * i / nf; f[i] = p.dens(v[i]); }
    F[0] = 0.0;
    Fn fn = [&](double t) { return p.dens(t); };
    for (int i = 0; i < nf; ++i) F[i + 1] = F[i] + gl_fixed(fn, v[i], v[i + 1]);
    return F[nf];
}

// quantile of the fine CDF at probability q (0..1) by a cubic Hermite model of
// F on the bracketing interval (F' = density), solved by bisection.
double fine_quantile(const std::vector<double> &v, const std::vector<double> &F,
                     const std::vector<double> &f, double q) {
    double target = q * F.back();
    int n = (int)v.size() - 1;
    if (target <= 0.0) return v[0];
    if (target >= F[n]) return v[n];
    int i = (int)(std::upper_bound(F.begin(), F.end(), target) - F.begin()) - 1;
    i = std::max(0, std::min(n - 1, i));
    double h = v[i + 1] - v[i];
    double y0 = F[i], y1 = F[i + 1], m0 = f[i] * h, m1 = f[i + 1] * h;
    double c2 = 3.0 * (y1 - y0) - 2.0 * m0 - m1, c3 = 2.0 * (y0 - y1) + m0 + m1;
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 60; ++it) {
        double t = 0.5 * (lo + hi);
        double val = y0 + t * (m0 + t * (c2 + t * c3));
        if (val < target) lo = t; else hi = t;
    }
    return v[i] + h * 0.5 * (lo + hi);
}

double log_mass(const Piece &p) {
    std::vector<double> v, F, f;
    double tot = fine_cdf(p, 256, v, F, f);
    double lm = std::log(std::max(tot, 1e-300));
    if (p.kind == 0) lm += std::log(p.thd / p.a) - p.xa * p.xa;  // dtheta = thd dt, u-measure 1/a
    if (p.kind == 3) lm += -p.xa * p.xa;
    return lm;
}

}  // namespace

double row_x(int j) {
    if (j < kRowsLin) return j * (kXLin / kRowsLin);
    return kXLin * std::pow(kXMax / kXLin, (double)(j - kRowsLin) / (kRows - kRowsLin - 1));
}

void build_voigt_block(double a, float *tab) {
    // (i) Voigt core: nodes x_i = i / 64, i = 0..512
    {
        std::vector<double> H(kVoigtCoreN + 1), D(kVoigtCoreN + 1);
        for (int i = 0; i <= kVoigtCoreN; ++i) voigt_quad(a, i * kVoigtCoreH, &H[i], &D[i]);
        for (int i = 0; i < kVoigtCoreN; ++i)
            hermite_coefs(H[i], D[i] * kVoigtCoreH, H[i + 1], D[i + 1] * kVoigtCoreH,
                          &tab[kOffVoigtCore + 4 * i]);
    }
    // (i) Voigt wing: G(w) = H(8/w) (8/w)^2, w_j = j / 128
    {
        std::vector<double> G(kVoigtWingN + 1), Gd(kVoigtWingN + 1);
        G[0] = a / kSqrtPi;
        Gd[0] = 0.0;
        for (int j = 1; j <= kVoigtWingN; ++j) {
            double w = (double)j / kVoigtWingN;
            double x = kXLin / w, h, d;
            voigt_quad(a, x, &h, &d);
            G[j] = h * x * x;
            Gd[j] = (d * x * x + 2.0 * x * h) * (-x * x / kXLin);
        }
        for (int j = 0; j < kVoigtWingN; ++j)
            hermite_coefs(G[j], Gd[j] / kVoigtWingN, G[j + 1], Gd[j + 1] / kVoigtWingN,
                          &tab[kOffVoigtWing + 4 * j]);
    }
}

void build_sampler_block(double a, float *tab) {
    // (ii) cumulative piece probabilities on x_i = i / 64, i = 0..512
    for (int i = 0; i <= kMassN; ++i) {
        double xa = i * (kXLin / kMassN);
        double lm[4], m = -1e300;
        for (int k = 0; k < 4; ++k) { lm[k] = log_mass(make_piece(k, xa, a)); m = std::max(m, lm[k]); }
        double e[4], tot = 0.0;
        for (int k = 0; k < 4; ++k) { e[k] = std::exp(lm[k] - m); tot += e[k]; }
        tab[kOffMass + 4 * i + 0] = (float)(e[0] / tot);
        tab[kOffMass + 4 * i + 1] = (float)((e[0] + e[1]) / tot);
        tab[kOffMass + 4 * i + 2] = (float)((e[0] + e[1] + e[2]) / tot);
        tab[kOffMass + 4 * i + 3] = 1.0f;
    }
    // (ii) quantile rows.  The wing pieces use nodes dense at both ends,
    // q = 4 xi^3 (xi < 1/2), q = 1 - 4 (1 - xi)^3 (xi >= 1/2), and their first and
    // last nodes are the 1e-9 and 1 - 1e-9 quantiles: no interval spans a stretch
    // of the variable that carries no probability, and the outermost intervals
    // hold so little probability that interpolating across the Gaussian tails
    // does not inflate the second moment of the kick.
    std::vector<double> v, F, f;
    const int nqs[4] = {kQS, kQL1, kQL2, kQR};
    const int offs[4] = {kOffSpike, kOffL1, kOffL2, kOffRight};
    for (int j = 0; j < kRows; ++j) {
        double xa = row_x(j);
        for (int kind = 0; kind < 4; ++kind) {
            Piece p = make_piece(kind, xa, a);
            fine_cdf(p, 4096, v, F, f);
            int nq = nqs[kind], off = offs[kind];
            for (int k = 0; k < nq; ++k) {
                double xi = (double)k / (nq - 1);
                double q;
                if (kind == 0) q = xi;
                else if (k == 0) q = 1e-9;
                else if (k == nq - 1) q = 1.0 - 1e-9;
                else q = (xi < 0.5) ? 4.0 * xi * xi * xi : 1.0 - 4.0 * (1.0 - xi) * (1.0 - xi) * (1.0 - xi);
                tab[off + j * nq + k] = (float)fine_quantile(v, F, f, q);
            }
        }
    }
}

void build_line_tables(double a, std::vector<float> &tab) {
    tab.assign(kTabFloats, 0.0f);
    build_voigt_block(a, tab.data());
    build_sampler_block(a, tab.data());
}

// ---- host reference evaluation of the staged tables (same arithmetic as the
// kernel's lookups, in FP64), used by the library's own self-check.
double table_voigt(const std::vector<float> &tab, double x) {
    double xa = std::fabs(x);
    if (xa < kXLin) {
        double t = xa / kVoigtCoreH;
        int i = std::min((int)t, kVoigtCoreN - 1);
        double fr = t - i;
        const float *c = &tab[kOffVoigtCore + 4 * i];
        return c[0] + fr * (c[1] + fr * (c[2] + fr * c[3]));
    }
    double w = kXLin / xa, t = w * kVoigtWingN;
    int j = std::min((int)t, kVoigtWingN - 1);
    double fr = t - j;
    const float *c = &tab[kOffVoigtWing + 4 * j];
    double G = c[0] + fr * (c[1] + fr * (c[2] + fr * c[3]));
    return G * w * w / (kXLin * kXLin);
}

double voigt_reference(double a, double x) {
    double h, d;
    voigt_quad(a, std::fabs(x), &h, &d);
    return h;
}

}  // namespace krt
