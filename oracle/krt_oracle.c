/*
 * krt_oracle.c -- plain FP64 CPU oracle for the Monte Carlo line-transfer pass.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP library: it is an independent statement of what the
 * pass computes, written for a reader who checks it against the paper by eye.
 *
 * Paper: "Kratos-linerad: GPU-accelerated Monte Carlo radiative transfer of
 * lines with efficient imaging" (L. Wang).  Citations name the section or
 * equation label of that paper.
 *
 * What is computed, in the paper's order:
 *   - Doppler units: x is the frequency offset in Doppler widths, velocities
 *     in units of b (Sec. 2.1, eq. xdef).  Gas-frame x_c = x_lab - n.v_bulk.
 *   - Line opacity per unit length k0 * H(a, x_c), with k0 = n_l sigma_0
 *     (eq. sigma0) and H the Voigt function.
 *   - Free flights through cell-wise constant fields, full optical depth, no
 *     core-skipping (Sec. 2.3.2).
 *   - Resonant scattering with partial frequency redistribution: the atom's
 *     parallel velocity u_par drawn from p(u|x) ~ exp(-u^2)/(a^2+(x-u)^2)
 *     (Sec. 2.1.1), the perpendicular component Gaussian of variance 1/2, and
 *     x_out = x_in + u_par (g-1) + u_perp sin(gamma) (eq. riia-scatter).
 *     Outgoing direction isotropic (Sec. 2.1.2) or dipole (3/8)(1+g^2).
 *   - Collisional destruction with probability eps per scattering (eq. eps).
 *   - Optional grey absorption (dust) per cell added to the flight opacity;
 *     an interaction is an absorption with probability kabs / (k0 H + kabs)
 *     (Sec. 3.2, the dusty slab).
 *   - Tallies: escaped spectrum, scattering counts, the camera-directed
 *     velocity-resolved scattering emissivity per (cell, channel)
 *     (Sec. 2.2.1, eq. scat-line; collision estimator, see below) and the
 *     profile-weighted mean intensity per cell that feeds the level
 *     populations (Sec. 2.1.3).
 *   - Statistical equilibrium of a multi-level system per cell (Sec. 2.1.3,
 *     eq. boltzmann for two levels), solved by Gaussian elimination.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - Random numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11),
 *     key = (seed_lo, seed_hi), counter = (event, packet_lo, packet_hi,
 *     purpose).  Event 0 is the emission; event n >= 1 is the n-th flight and
 *     the scattering that ends it.  Purposes 0 and 1 of an event are shared
 *     with the GPU path word for word; this oracle draws u_par by exact
 *     rejection from purposes 2, 3, ... (one block per trial).
 *   - Uniform variate: u = (w >> 9) * 2^-23 + 2^-24, an odd multiple of 2^-24
 *     in (0, 1), exactly representable in binary32.
 *   - Emissivity estimator: at each non-destroyed scattering in cell c the
 *     same atom (u_par, u_perp vector) is re-emitted virtually toward the
 *     camera; the tally (cell c, channel of the lab-frame camera frequency)
 *     receives the phase-function value at g_cam = n_in . n_cam.  Its
 *     expectation is the camera-directed emissivity of eq. scat-line.
 *   - Mean intensity: track-length estimator sum(dl * H(a, x_c)) / sqrt(pi).
 *
 * Parity pins live in tests/ (closed forms, invariants, brute force).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>
#include <complex.h>

#define ORC_PI 3.14159265358979323846
#define ORC_SQRTPI 1.77245385090551602730

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al. 2011, SC'11, Sec. 5 and the Random123 spec)  */
/* ------------------------------------------------------------------------ */
static const uint32_t PHILOX_M0 = 0xD2511F53u, PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u, PHILOX_W1 = 0xBB67AE85u;

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Batch form for the tests: ctr[n][4], key[n][2] -> out[n][4]. */
void orc_philox_batch(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i) orc_philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

static double u01(uint32_t w) { return (double)(w >> 9) * 0x1p-23 + 0x1p-24; }

double orc_u01(uint32_t w) { return u01(w); }

typedef struct { uint32_t key[2]; uint64_t packet; } rng_t;

static void draw_block(const rng_t *r, uint32_t event, uint32_t purpose, uint32_t out[4])
{
    uint32_t ctr[4] = { event, (uint32_t)r->packet, (uint32_t)(r->packet >> 32), purpose };
    orc_philox4x32_10(ctr, r->key, out);
}

/* ------------------------------------------------------------------------ */
/* Voigt function H(a,x) = Re w(x + i a), Sec. 2.1 (line profile).          */
/* w is the Faddeeva function.  |z| < 7: Weideman (1994, SIAM J. Numer.     */
/* Anal. 31, 1497) rational expansion with N = 36 terms, coefficients from   */
/* the discrete Fourier transform that paper prescribes.  |z| >= 7: the      */
/* Laplace continued fraction  w = (i/sqrt(pi)) / (z - (1/2)/(z - 1/(z -      */
/* (3/2)/(z - ...)))).                                                        */
/* ------------------------------------------------------------------------ */
#define WEID_N 36
static double weid_coef[WEID_N + 1];
static double weid_L;
static pthread_once_t weid_once = PTHREAD_ONCE_INIT;

static void weid_init(void)
{
    const int N = WEID_N, M = 2 * N, M2 = 2 * M;
    weid_L = sqrt((double)N / sqrt(2.0));
    /* f_k at k = -M+1 .. M-1 with t_k = L tan(k pi / M2), plus f = 0 in front:
       a vector of length M2, fftshift-ed, then a real DFT / M2. */
    double f[4 * WEID_N];
    f[0] = 0.0;
    for (int j = 1; j < M2; ++j) {
        int k = j - M; /* k runs -M+1 .. M-1 */
        double t = weid_L * tan(k * ORC_PI / M2);
        f[j] = exp(-t * t) * (weid_L * weid_L + t * t);
    }
    /* fftshift of a length-M2 vector: g[i] = f[(i + M2/2) % M2] */
    double g[4 * WEID_N];
    for (int i = 0; i < M2; ++i) g[i] = f[(i + M2 / 2) % M2];
    /* real part of the DFT, indices 1..N (descending order is applied at use) */
    for (int n = 0; n <= N; ++n) {
        double s = 0.0;
        for (int i = 0; i < M2; ++i) s += g[i] * cos(2.0 * ORC_PI * (double)n * i / M2);
        weid_coef[n] = s / M2;
    }
}

static double complex faddeeva(double complex z)
{
    double az = cabs(z);
    if (az >= 7.0) {
        /* continued fraction, evaluated bottom-up */
        double complex r = 0.0;
        for (int k = 40; k >= 1; --k) r = (k * 0.5) / (z - r);
        return (I / ORC_SQRTPI) / (z - r);
    }
    pthread_once(&weid_once, weid_init);
    double L = weid_L;
    double complex iz = I * z;
    double complex Z = (L + iz) / (L - iz);
    /* p(Z) = sum_{n=1}^{N} a_n Z^{N-n}   (Horner, highest power first) */
    double complex p = 0.0;
    for (int n = 1; n <= WEID_N; ++n) p = p * Z + weid_coef[WEID_N + 1 - n];
    /* coefficient order: the polynomial uses a reversed list a(N..1) */
    double complex lmiz = L - iz;
    return 2.0 * p / (lmiz * lmiz) + (1.0 / ORC_SQRTPI) / lmiz;
}

double orc_voigt_H(double a, double x)
{
    /* w(z) for Im z >= 0; H is even in x */
    double complex w = faddeeva(fabs(x) + I * a);
    return creal(w);
}

void orc_voigt_batch(int64_t n, double a, const double *x, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_voigt_H(a, x[i]);
}

/* ------------------------------------------------------------------------ */
/* Atom parallel velocity, Sec. 2.1.1: p(u | x) ~ exp(-u^2)/(a^2 + (x-u)^2). */
/* Exact rejection sampling in the manner of Zheng & Miralda-Escude (2002,   */
/* ApJ 578, 33, appendix): propose from the Lorentzian centred at |x| with   */
/* weight 1 below a split point u0 >= 0 and exp(-u0^2) above it; accept with  */
/* exp(-u^2) resp. exp(-u^2)/exp(-u0^2).  Both ratios are <= 1 for any        */
/* u0 >= 0, so the draw is exact whatever u0 is; u0 only sets the acceptance  */
/* rate and is picked from a fixed candidate list to minimise the envelope    */
/* mass.  Symmetry p(u|x) = p(-u|-x) handles x < 0.                           */
/* ------------------------------------------------------------------------ */
static double envelope_mass(double xa, double a, double u0, double *plow)
{
    double th0 = atan((u0 - xa) / a);
    double pl = (th0 + 0.5 * ORC_PI) / ORC_PI; /* Lorentz probability below u0 */
    *plow = pl;
    return pl + exp(-u0 * u0) * (1.0 - pl);
}

static const double U0_OFFSETS[] = { 1e-3, 3e-3, 1e-2, 3e-2, 0.1, 0.2, 0.3, 0.5, 0.7,
                                      1.0, 1.3, 1.6, 2.0, 2.5, 3.0, 4.0, 6.0, 9.0 };

/* returns u_par; *trials receives the number of proposals used */
static double sample_upar(double x, double a, const rng_t *r, uint32_t event, int *trials)
{
    double s = (x < 0.0) ? -1.0 : 1.0;
    double xa = fabs(x);
    double u0 = 0.0, pl0;
    double best = envelope_mass(xa, a, 0.0, &pl0);
    for (size_t i = 0; i < sizeof(U0_OFFSETS) / sizeof(U0_OFFSETS[0]); ++i) {
        double c = xa - U0_OFFSETS[i];
        if (c <= 0.0) continue;
        double pl;
        double m = envelope_mass(xa, a, c, &pl);
        if (m < best) { best = m; u0 = c; pl0 = pl; }
    }
    double th0 = atan((u0 - xa) / a);
    double e0 = exp(-u0 * u0);
    double p_low = pl0 / (pl0 + e0 * (1.0 - pl0));
    for (int t = 0; t < 1000000; ++t) {
        uint32_t w[4];
        draw_block(r, event, 2u + (uint32_t)t, w);
        double r1 = u01(w[0]), r2 = u01(w[1]), r3 = u01(w[2]);
        double th;
        if (r1 < p_low) th = -0.5 * ORC_PI + r2 * (th0 + 0.5 * ORC_PI);
        else            th = th0 + r2 * (0.5 * ORC_PI - th0);
        double u = xa + a * tan(th);
        double acc = (u <= u0) ? exp(-u * u) : exp(-(u * u - u0 * u0));
        if (r3 <= acc) { *trials = t + 1; return s * u; }
    }
    *trials = -1;
    return 0.0;
}

/* test hook: draw u_par for event indices [ev0, ev0+n) of one packet */
void orc_sample_upar_batch(int64_t n, double x, double a, uint64_t seed, uint64_t packet,
                           uint32_t ev0, double *out, int64_t *total_trials)
{
    rng_t r = { { (uint32_t)seed, (uint32_t)(seed >> 32) }, packet };
    int64_t tt = 0;
    for (int64_t i = 0; i < n; ++i) {
        int t;
        out[i] = sample_upar(x, a, &r, ev0 + (uint32_t)i, &t);
        tt += t;
    }
    if (total_trials) *total_trials = tt;
}

/* ------------------------------------------------------------------------ */
/* Directions.                                                                */
/* ------------------------------------------------------------------------ */
/* Orthonormal basis (e1, e2) perpendicular to unit n: the branch-free       */
/* construction of Duff, Burgess, Christensen et al. (2017, JCGT 6(1)).       */
static void ortho_basis(const double n[3], double e1[3], double e2[3])
{
    double sign = (n[2] >= 0.0) ? 1.0 : -1.0;
    double A = -1.0 / (sign + n[2]);
    double B = n[0] * n[1] * A;
    e1[0] = 1.0 + sign * n[0] * n[0] * A; e1[1] = sign * B; e1[2] = -sign * n[0];
    e2[0] = B; e2[1] = sign + n[1] * n[1] * A; e2[2] = -n[1];
}

/* Dipole phase (3/8)(1+g^2): invert F(g) = (g^3 + 3g + 4)/8 = u.           */
/* With g = 2 sinh(t): g^3 + 3g = 2 sinh(3t), so g = 2 sinh(asinh(4u-2)/3).  */
static double dipole_g(double u) { return 2.0 * sinh(asinh(4.0 * u - 2.0) / 3.0); }

/* ------------------------------------------------------------------------ */
/* Bins: the edges are binary32 values of lo + k (hi-lo)/nb (computed in     */
/* FP64, then rounded); bin = 1 + largest k with edge[k] <= x, 0 below the    */
/* first edge, nb+1 at or above the last edge.  x is compared as binary32.   */
/* ------------------------------------------------------------------------ */
static int bin_index(float xf, int nb, double lo, double hi)
{
    if (!(xf == xf)) return -1; /* NaN */
    int lo_k = 0, hi_k = nb;    /* edges 0..nb */
    float e0 = (float)lo, en = (float)(lo + (hi - lo) * nb / nb);
    if (xf < e0) return 0;
    if (xf >= en) return nb + 1;
    /* binary search for largest k in [0, nb) with edge[k] <= xf */
    while (hi_k - lo_k > 1) {
        int mid = (lo_k + hi_k) / 2;
        float em = (float)(lo + (hi - lo) * (double)mid / (double)nb);
        if (em <= xf) lo_k = mid; else hi_k = mid;
    }
    return lo_k + 1;
}

void orc_bin_batch(int64_t n, const float *x, int nb, double lo, double hi, int32_t *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = bin_index(x[i], nb, lo, hi);
}

/* ------------------------------------------------------------------------ */
/* Problem description (input data are binary32 arrays shared with the GPU   */
/* path as plain data; the oracle widens them to FP64).                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n[3];
    double lo[3], hi[3];
    int32_t bc[3];             /* 0 vacuum, 1 periodic */
    const float *k0;           /* [ncell] */
    const float *vel;          /* [3][ncell], may be NULL (static) */
    const float *eps;          /* [ncell], may be NULL */
    const float *emis;         /* [ncell] volume emission weights, may be NULL */
    const float *bratio;       /* [ncell] Doppler width b_cell / b_ref, may be NULL (all 1) */
    const float *kabs;         /* [ncell] grey absorption coefficient (dust, units of k0), may be NULL */
    double a;                  /* damping at b_ref; a cell's is a b_ref / b_cell */
    int32_t phase;             /* 0 isotropic, 1 dipole */
    int32_t source;            /* 0 point, 1 plane z = src_pos[2], 2 volume, 3 beam */
    double src_pos[3];
    double src_dir[3];         /* beam direction (unit) */
    int32_t src_profile;       /* 0 delta at x0, 1 Voigt, 2 Gaussian (thermal) */
    double src_x0;
    int32_t spec_nbins;
    double spec_lo, spec_hi;
    int32_t emis_nch;          /* 0 disables */
    double ch_lo, ch_hi;
    double n_cam[3];
    int32_t jbar;              /* tally mean intensity */
    uint64_t max_events;
} orc_problem;

enum { C_EMITTED = 0, C_ESCAPED, C_DESTROYED, C_SCATTER, C_CROSS, C_STUCK, C_TRIALS, C_STATUS, C_NCOUNT };

typedef struct {
    const orc_problem *P;
    uint64_t seed, p0, p1;
    /* private tallies */
    int64_t *spec;
    double *emis;
    double *jbar;
    int64_t cnt[C_NCOUNT];
    double *packet_log;        /* [n][8] or NULL, indexed from the run's first packet */
    uint64_t log_base;
    /* volume-source CDF (shared, read-only) */
    const double *cdf; int64_t ncdf;
} worker_t;

static int64_t cell_lin(const orc_problem *P, const int c[3])
{
    return ((int64_t)c[2] * P->n[1] + c[1]) * P->n[0] + c[0];
}

/* one packet */
static void run_packet(worker_t *W, uint64_t pid)
{
    const orc_problem *P = W->P;
    rng_t r = { { (uint32_t)W->seed, (uint32_t)(W->seed >> 32) }, pid };
    const int64_t ncell = (int64_t)P->n[0] * P->n[1] * P->n[2];
    double dx[3];
    for (int d = 0; d < 3; ++d) dx[d] = (P->hi[d] - P->lo[d]) / P->n[d];

    uint32_t w0[4], w1[4], w2[4];
    draw_block(&r, 0, 0, w0);
    draw_block(&r, 0, 1, w1);
    draw_block(&r, 0, 2, w2);

    /* direction: mu = 2u-1, phi = 2 pi u */
    double mu = 2.0 * u01(w0[0]) - 1.0, ph = 2.0 * ORC_PI * u01(w0[1]);
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double n[3] = { st * cos(ph), st * sin(ph), mu };
    if (P->source == 3) for (int d = 0; d < 3; ++d) n[d] = P->src_dir[d];

    /* position and cell */
    double X[3];
    int c[3];
    if (P->source == 2) {
        /* volume: cell by inverse CDF of the emission weights */
        double uc = u01(w0[2]) * W->cdf[W->ncdf - 1];
        int64_t lo = 0, hi = W->ncdf - 1;
        while (lo < hi) { int64_t m = (lo + hi) / 2; if (W->cdf[m] > uc) hi = m; else lo = m + 1; }
        int64_t cl = lo;
        c[0] = (int)(cl % P->n[0]); c[1] = (int)((cl / P->n[0]) % P->n[1]); c[2] = (int)(cl / ((int64_t)P->n[0] * P->n[1]));
        for (int d = 0; d < 3; ++d) X[d] = P->lo[d] + (c[d] + u01(w1[d])) * dx[d];
    } else {
        for (int d = 0; d < 3; ++d) X[d] = P->src_pos[d];
        if (P->source == 1) { /* plane z = src: uniform transverse position */
            X[0] = P->lo[0] + u01(w1[0]) * (P->hi[0] - P->lo[0]);
            X[1] = P->lo[1] + u01(w1[1]) * (P->hi[1] - P->lo[1]);
        }
        for (int d = 0; d < 3; ++d) {
            double f = (X[d] - P->lo[d]) / dx[d];
            int ci = (int)floor(f);
            /* on a face: the cell the packet moves into */
            if ((double)ci == f && n[d] < 0.0) ci -= 1;
            if (ci < 0) ci = 0;
            if (ci >= P->n[d]) ci = P->n[d] - 1;
            c[d] = ci;
        }
    }
    int64_t cl = cell_lin(P, c);
    double vc[3] = { 0, 0, 0 };
    if (P->vel) for (int d = 0; d < 3; ++d) vc[d] = P->vel[(int64_t)d * ncell + cl];
    /* per-cell temperature (Sec. 2.1: frequencies in units of the local Doppler
     * width): s = b_ref / b_cell scales the gas-frame frequency and the damping */
    double sc = P->bratio ? 1.0 / (double)P->bratio[cl] : 1.0;
    double ac = P->a * sc;

    /* gas-frame emission frequency */
    double xg;
    if (P->src_profile == 0) xg = P->src_x0;
    else {
        double rr = sqrt(-log(u01(w2[0]))), th = 2.0 * ORC_PI * u01(w2[1]);
        double gsn = rr * cos(th);           /* N(0, 1/2) */
        if (P->src_profile == 1) xg = gsn + ac * tan(ORC_PI * (u01(w2[2]) - 0.5)); /* Voigt = Gauss (*) Cauchy */
        else xg = gsn;
        xg /= sc;  /* the profile is in the emitting cell's Doppler units */
    }
    double x = xg + n[0] * vc[0] + n[1] * vc[1] + n[2] * vc[2];
    W->cnt[C_EMITTED] += 1;

    double sqrtpi_inv = 1.0 / ORC_SQRTPI;
    int64_t nscat = 0;
    int outcome = 0; /* 1 escaped, 2 destroyed, 3 stuck */
    uint64_t ev;
    for (ev = 1; ev <= P->max_events; ++ev) {
        uint32_t A[4], B[4];
        draw_block(&r, (uint32_t)ev, 0, A);
        draw_block(&r, (uint32_t)ev, 1, B);
        double tau = -log(u01(A[0]));
        /* ---- flight ---- */
        int escaped = 0;
        for (;;) {
            double k0 = P->k0[cl];
            double xc = (x - (n[0] * vc[0] + n[1] * vc[1] + n[2] * vc[2])) * sc;
            double H = (k0 > 0.0) ? orc_voigt_H(ac, xc) : 0.0;
            /* line opacity plus the cell's grey absorption (Sec. 3.2) */
            double kap = k0 * H + (P->kabs ? (double)P->kabs[cl] : 0.0);
            /* distance to the cell boundary */
            double dmin = INFINITY; int ax = -1;
            for (int d = 0; d < 3; ++d) {
                if (n[d] > 0.0) {
                    double t = (P->lo[d] + (c[d] + 1) * dx[d] - X[d]) / n[d];
                    if (t < dmin) { dmin = t; ax = d; }
                } else if (n[d] < 0.0) {
                    double t = (P->lo[d] + c[d] * dx[d] - X[d]) / n[d];
                    if (t < dmin) { dmin = t; ax = d; }
                }
            }
            if (dmin < 0.0) dmin = 0.0;
            if (kap > 0.0 && kap * dmin >= tau) {
                double l = tau / kap;
                for (int d = 0; d < 3; ++d) X[d] += l * n[d];
                if (P->jbar && W->jbar) W->jbar[cl] += l * H * sqrtpi_inv;
                break; /* interaction */
            }
            /* cross the face */
            tau -= kap * dmin;
            if (P->jbar && W->jbar) W->jbar[cl] += dmin * H * sqrtpi_inv;
            for (int d = 0; d < 3; ++d) X[d] += dmin * n[d];
            W->cnt[C_CROSS] += 1;
            int step = (n[ax] > 0.0) ? 1 : -1;
            c[ax] += step;
            X[ax] = P->lo[ax] + ((step > 0) ? c[ax] : c[ax] + 1) * dx[ax];
            if (c[ax] < 0 || c[ax] >= P->n[ax]) {
                if (P->bc[ax] == 1) {
                    c[ax] = (c[ax] < 0) ? P->n[ax] - 1 : 0;
                    X[ax] = (step > 0) ? P->lo[ax] : P->hi[ax];
                } else { escaped = 1; break; }
            }
            cl = cell_lin(P, c);
            if (P->vel) for (int d = 0; d < 3; ++d) vc[d] = P->vel[(int64_t)d * ncell + cl];
            sc = P->bratio ? 1.0 / (double)P->bratio[cl] : 1.0;
            ac = P->a * sc;
        }
        if (escaped) { outcome = 1; break; }
        /* ---- scattering (in the cell's Doppler units) ---- */
        double xc = (x - (n[0] * vc[0] + n[1] * vc[1] + n[2] * vc[2])) * sc;
        if (P->eps || P->kabs) {
            /* the interaction is a grey absorption with probability p_d =
             * kabs / (k0 H + kabs); otherwise a line scattering, destroyed with
             * probability eps (eq. eps): one uniform decides both */
            double e = P->eps ? (double)P->eps[cl] : 0.0;
            double pd = 0.0;
            if (P->kabs && P->kabs[cl] > 0.0f) {
                double ka = (double)P->kabs[cl];
                pd = ka / (P->k0[cl] * orc_voigt_H(ac, xc) + ka);
            }
            if (u01(A[1]) < pd + (1.0 - pd) * e) { outcome = 2; break; }
        }
        int trials;
        double upar = sample_upar(xc, ac, &r, (uint32_t)ev, &trials);
        if (trials < 0) { W->cnt[C_STATUS] |= 4; outcome = 3; break; }
        W->cnt[C_TRIALS] += trials;
        /* perpendicular atom velocity: two N(0, 1/2) components (Box-Muller) */
        double rr = sqrt(-log(u01(B[0]))), th = 2.0 * ORC_PI * u01(B[1]);
        double up1 = rr * cos(th), up2 = rr * sin(th);
        /* outgoing direction about n_in */
        double g = (P->phase == 1) ? dipole_g(u01(B[2])) : 2.0 * u01(B[2]) - 1.0;
        double psi = 2.0 * ORC_PI * u01(B[3]);
        double sg = sqrt(fmax(0.0, 1.0 - g * g));
        double e1[3], e2[3];
        ortho_basis(n, e1, e2);
        double cp = cos(psi), sp = sin(psi);
        double nout[3];
        for (int d = 0; d < 3; ++d) nout[d] = g * n[d] + sg * (cp * e1[d] + sp * e2[d]);
        /* eq. riia-scatter: x_out = x_in + u_par (g-1) + u_perp . n_out */
        double xo = xc + upar * (g - 1.0) + sg * (up1 * cp + up2 * sp);
        /* emissivity toward the camera from the same atom */
        if (P->emis_nch > 0 && W->emis) {
            double gc = n[0] * P->n_cam[0] + n[1] * P->n_cam[1] + n[2] * P->n_cam[2];
            double upc = up1 * (e1[0] * P->n_cam[0] + e1[1] * P->n_cam[1] + e1[2] * P->n_cam[2])
                       + up2 * (e2[0] * P->n_cam[0] + e2[1] * P->n_cam[1] + e2[2] * P->n_cam[2]);
            double xcam = xc + upar * (gc - 1.0) + upc;
            double xcam_lab = xcam / sc + (P->n_cam[0] * vc[0] + P->n_cam[1] * vc[1] + P->n_cam[2] * vc[2]);
            int k = bin_index((float)xcam_lab, P->emis_nch, P->ch_lo, P->ch_hi);
            if (k >= 1 && k <= P->emis_nch) {
                double wph = (P->phase == 1) ? 0.75 * (1.0 + gc * gc) : 1.0;
                W->emis[cl * P->emis_nch + (k - 1)] += wph;
            }
        }
        for (int d = 0; d < 3; ++d) n[d] = nout[d];
        x = xo / sc + (n[0] * vc[0] + n[1] * vc[1] + n[2] * vc[2]);
        nscat += 1;
    }
    if (outcome == 0) { outcome = 3; W->cnt[C_STUCK] += 1; W->cnt[C_STATUS] |= 2; }
    W->cnt[C_SCATTER] += nscat;
    if (outcome == 1) {
        W->cnt[C_ESCAPED] += 1;
        int b = bin_index((float)x, P->spec_nbins, P->spec_lo, P->spec_hi);
        if (b < 0) W->cnt[C_STATUS] |= 1; else W->spec[b] += 1;
    } else if (outcome == 2) {
        W->cnt[C_DESTROYED] += 1;
    }
    if (W->packet_log) {
        double *L = W->packet_log + 8 * (pid - W->log_base);
        L[0] = x; L[1] = (double)nscat; L[2] = (double)outcome;
        L[3] = n[0]; L[4] = n[1]; L[5] = n[2];
        L[6] = (double)cl; L[7] = (double)ev;  /* last cell inside the grid */
    }
}

static void *worker_main(void *arg)
{
    worker_t *W = (worker_t *)arg;
    for (uint64_t p = W->p0; p < W->p1; ++p) run_packet(W, p);
    return NULL;
}

/*
 * Run packets [packet_offset, packet_offset + n_packets) with n_threads threads.
 * Outputs (accumulated, caller zeroes): spec[nb+2] int64 counts, emis[ncell*nch]
 * FP64 weights (may be NULL), jbar[ncell] FP64 sums of dl*H/sqrt(pi) (may be
 * NULL), counters[8], packet_log[n_packets*8] (may be NULL).
 */
int orc_mc_run(const orc_problem *P, uint64_t n_packets, uint64_t packet_offset, uint64_t seed,
               int n_threads, int64_t *spec, double *emis, double *jbar, int64_t *counters,
               double *packet_log)
{
    if (n_threads < 1) n_threads = 1;
    const int64_t ncell = (int64_t)P->n[0] * P->n[1] * P->n[2];
    double *cdf = NULL;
    if (P->source == 2) {
        if (!P->emis) return -1;
        cdf = (double *)malloc(sizeof(double) * ncell);
        double s = 0.0;
        for (int64_t i = 0; i < ncell; ++i) { s += (double)P->emis[i]; cdf[i] = s; }
    }
    pthread_t *th = (pthread_t *)calloc(n_threads, sizeof(pthread_t));
    worker_t *W = (worker_t *)calloc(n_threads, sizeof(worker_t));
    int nb = P->spec_nbins + 2;
    for (int t = 0; t < n_threads; ++t) {
        W[t].P = P; W[t].seed = seed;
        W[t].p0 = packet_offset + n_packets * t / n_threads;
        W[t].p1 = packet_offset + n_packets * (t + 1) / n_threads;
        W[t].spec = (int64_t *)calloc(nb, sizeof(int64_t));
        W[t].emis = (emis && P->emis_nch > 0) ? (double *)calloc(ncell * P->emis_nch, sizeof(double)) : NULL;
        W[t].jbar = (jbar && P->jbar) ? (double *)calloc(ncell, sizeof(double)) : NULL;
        W[t].packet_log = packet_log;
        W[t].log_base = packet_offset;
        W[t].cdf = cdf; W[t].ncdf = ncell;
        pthread_create(&th[t], NULL, worker_main, &W[t]);
    }
    for (int t = 0; t < n_threads; ++t) {
        pthread_join(th[t], NULL);
        for (int b = 0; b < nb; ++b) spec[b] += W[t].spec[b];
        if (W[t].emis) for (int64_t i = 0; i < ncell * P->emis_nch; ++i) emis[i] += W[t].emis[i];
        if (W[t].jbar) for (int64_t i = 0; i < ncell; ++i) jbar[i] += W[t].jbar[i];
        for (int k = 0; k < C_NCOUNT; ++k) {
            if (k == C_STATUS) counters[k] |= W[t].cnt[k];
            else counters[k] += W[t].cnt[k];
        }
        free(W[t].spec); free(W[t].emis); free(W[t].jbar);
    }
    free(th); free(W); free(cdf);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Statistical equilibrium, Sec. 2.1.3.  For each cell: rate matrix of an    */
/* L-level system with radiative decays A[u][l], absorption rate Gamma per    */
/* lower-level molecule for each line (u = l+1 ladder) and stimulated         */
/* emission (g_l/g_u) Gamma per upper-level molecule (Einstein relation),     */
/* collisional rates Cd[u][l] downward per unit collider density, upward by   */
/* detailed balance Cu = (g_u/g_l) Cd exp(-(E_u-E_l)/kT).  The last balance   */
/* equation is replaced by sum n = n_tot; Gaussian elimination with partial  */
/* pivoting.                                                                  */
/* ------------------------------------------------------------------------ */
static int solve_dense(int n, double *M, double *b)
{
    for (int k = 0; k < n; ++k) {
        int p = k; double mx = fabs(M[k * n + k]);
        for (int i = k + 1; i < n; ++i) if (fabs(M[i * n + k]) > mx) { mx = fabs(M[i * n + k]); p = i; }
        if (mx == 0.0) return -1;
        if (p != k) {
            for (int j = 0; j < n; ++j) { double t = M[k * n + j]; M[k * n + j] = M[p * n + j]; M[p * n + j] = t; }
            double t = b[k]; b[k] = b[p]; b[p] = t;
        }
        for (int i = k + 1; i < n; ++i) {
            double f = M[i * n + k] / M[k * n + k];
            for (int j = k; j < n; ++j) M[i * n + j] -= f * M[k * n + j];
            b[i] -= f * b[k];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int j = i + 1; j < n; ++j) s -= M[i * n + j] * b[j];
        b[i] = s / M[i * n + i];
    }
    return 0;
}

/*
 * nl levels; E[nl] energies in units of kT; g[nl]; A[nl*nl] (A[u*nl+l], u>l);
 * Cd[nl*nl] downward collision rate coefficients (u>l); per cell: ncoll[cell],
 * ntot[cell], gamma[(nl-1) * ncell] absorption rate per lower molecule for
 * line l -> l+1 (may be NULL = 0).  Output pops[cell*nl + i].
 */
int orc_levels_solve(int nl, int64_t ncell, const double *E, const double *g, const double *A,
                     const double *Cd, const double *ncoll, const double *ntot,
                     const double *gamma, double *pops)
{
    if (nl < 2 || nl > 16) return -1;
    double R[256], M[256], b[16];
    for (int64_t c = 0; c < ncell; ++c) {
        /* R[i][j] = transition rate per molecule from level i to level j */
        for (int i = 0; i < nl * nl; ++i) R[i] = 0.0;
        for (int u = 1; u < nl; ++u)
            for (int l = 0; l < u; ++l) {
                double cd = Cd[u * nl + l] * ncoll[c];
                double cu = cd * (g[u] / g[l]) * exp(-(E[u] - E[l]));
                R[u * nl + l] += A[u * nl + l] + cd;
                R[l * nl + u] += cu;
            }
        if (gamma)
            for (int l = 0; l + 1 < nl; ++l) {
                int u = l + 1;
                double G = gamma[(int64_t)l * ncell + c];
                R[l * nl + u] += G;
                R[u * nl + l] += (g[l] / g[u]) * G;
            }
        /* balance: for each level i, sum_j n_j R[j][i] - n_i sum_j R[i][j] = 0 */
        for (int i = 0; i < nl; ++i) {
            for (int j = 0; j < nl; ++j) M[i * nl + j] = 0.0;
            double out = 0.0;
            for (int j = 0; j < nl; ++j) if (j != i) { M[i * nl + j] = R[j * nl + i]; out += R[i * nl + j]; }
            M[i * nl + i] = -out;
            b[i] = 0.0;
        }
        for (int j = 0; j < nl; ++j) M[(nl - 1) * nl + j] = 1.0;
        b[nl - 1] = ntot[c];
        if (solve_dense(nl, M, b) != 0) return -2;
        for (int i = 0; i < nl; ++i) pops[c * nl + i] = b[i];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Whole-cell escape (reference for the learned escape; the paper has no     */
/* learned part, this is the plain walk of Sec. 2.1-2.3 confined to one      */
/* cell).  The cell is the homogeneous static cube [-1,1]^3 in units of its  */
/* half-width, of line-centre opacity tau_c per unit length, so tau_c is the */
/* line-centre depth from the centre to a face.  A photon of gas-frame       */
/* frequency x_in arriving along n_in (given, or isotropic from event 0,     */
/* purpose 4, words 0-1) scatters at the point q (event 1, no flight), then  */
/* takes plain flights and resonant scatterings until it leaves the cube.    */
/* Record (ORC_CELL_REC doubles):                                            */
/*   0 log10 tau_c  1 log10 a  2 x_in  3-5 q  6 log10 depth, depth =         */
/*   tau_c (1 - max|q_k|) the line-centre depth to the nearest face          */
/*   7-9 n_in  10 exit face F = 2 axis + (outward normal along +axis)        */
/*   11, 12 ys, yt: offsets of the exit point from q's projection onto the   */
/*   exit face along the two axes following the exit axis cyclically, over  */
/*   q's distance to the face's plane   13 mu = |n_out . normal|             */
/*   14 alpha in [0, pi]: angle between the exit direction's tangential part */
/*   and that offset (0 where either vanishes)   15 x_out   16 ln N_s (N_s   */
/*   scatterings inside, the first one included)   17 ln <x^2> over them     */
/*   18 valid (0 if the scattering cap was reached)   19 0                   */
/* ------------------------------------------------------------------------ */
#define ORC_CELL_REC 20
typedef struct {
    double tau, a, xin, q[3], nin[3];
    int given_dir;
    uint64_t seed, p0, p1, max_scat;
    double *out;
} cell_job_t;

static void cell_escape_one(const cell_job_t *J, uint64_t pid, double *o)
{
    rng_t r = { { (uint32_t)J->seed, (uint32_t)(J->seed >> 32) }, pid };
    double n[3];
    if (J->given_dir) {
        for (int k = 0; k < 3; ++k) n[k] = J->nin[k];
    } else {
        uint32_t d[4];
        draw_block(&r, 0, 4, d);
        double mu0 = 2.0 * u01(d[0]) - 1.0, ph0 = 2.0 * ORC_PI * u01(d[1]);
        double st0 = sqrt(fmax(0.0, 1.0 - mu0 * mu0));
        n[0] = st0 * cos(ph0); n[1] = st0 * sin(ph0); n[2] = mu0;
    }
    double depth = J->tau * (1.0 - fmax(fabs(J->q[0]), fmax(fabs(J->q[1]), fabs(J->q[2]))));
    o[0] = log10(J->tau); o[1] = log10(J->a); o[2] = J->xin;
    for (int k = 0; k < 3; ++k) { o[3 + k] = J->q[k]; o[7 + k] = n[k]; }
    o[6] = log10(fmax(depth, 1e-300));
    double X[3] = { J->q[0], J->q[1], J->q[2] };
    double x = J->xin, sx2 = 0.0;
    uint64_t ns = 0;
    int valid = 0, ax = 0;
    for (uint64_t ev = 1; ev <= J->max_scat + 1; ++ev) {
        uint32_t A[4], B[4];
        draw_block(&r, (uint32_t)ev, 0, A);
        draw_block(&r, (uint32_t)ev, 1, B);
        if (ev > 1) {
            /* free flight: tau = -ln u against k0 H(a, x) (Sec. 2.3.2) */
            double tau = -log(u01(A[0]));
            double kap = J->tau * orc_voigt_H(J->a, x);
            double dm = INFINITY;
            for (int k = 0; k < 3; ++k) {
                double t = (n[k] > 0.0) ? (1.0 - X[k]) / n[k] : ((n[k] < 0.0) ? (-1.0 - X[k]) / n[k] : INFINITY);
                if (t < dm) { dm = t; ax = k; }
            }
            if (dm < 0.0) dm = 0.0;
            if (kap * dm < tau) {
                for (int k = 0; k < 3; ++k) X[k] += dm * n[k];
                valid = 1;
                break;
            }
            double l = tau / kap;
            for (int k = 0; k < 3; ++k) X[k] += l * n[k];
        }
        /* resonant scattering, isotropic phase (eq. riia-scatter) */
        int trials;
        double upar = sample_upar(x, J->a, &r, (uint32_t)ev, &trials);
        double rr = sqrt(-log(u01(B[0]))), th = 2.0 * ORC_PI * u01(B[1]);
        double up1 = rr * cos(th), up2 = rr * sin(th);
        double g = 2.0 * u01(B[2]) - 1.0, psi = 2.0 * ORC_PI * u01(B[3]);
        double sg = sqrt(fmax(0.0, 1.0 - g * g));
        double e1[3], e2[3];
        ortho_basis(n, e1, e2);
        double cp = cos(psi), sp = sin(psi);
        double no[3];
        for (int k = 0; k < 3; ++k) no[k] = g * n[k] + sg * (cp * e1[k] + sp * e2[k]);
        sx2 += x * x;
        x = x + upar * (g - 1.0) + sg * (up1 * cp + up2 * sp);
        for (int k = 0; k < 3; ++k) n[k] = no[k];
        ns += 1;
    }
    if (!valid) {
        for (int k = 10; k < ORC_CELL_REC; ++k) o[k] = 0.0;
        return;
    }
    int a1 = (ax + 1) % 3, a2 = (ax + 2) % 3;
    double side = (n[ax] > 0.0) ? 1.0 : -1.0;
    double dplane = 1.0 - side * J->q[ax];       /* q's distance to the exit face's plane */
    double ds = X[a1] - J->q[a1], dt = X[a2] - J->q[a2];
    o[10] = 2.0 * ax + (side > 0.0 ? 1.0 : 0.0);
    o[11] = ds / dplane;
    o[12] = dt / dplane;
    o[13] = fabs(n[ax]);
    o[14] = atan2(fabs(ds * n[a2] - dt * n[a1]), ds * n[a1] + dt * n[a2]);
    o[15] = x;
    o[16] = log((double)ns);
    o[17] = log(sx2 / (double)ns);
    o[18] = 1.0;
    o[19] = 0.0;
}

static void *cell_escape_main(void *arg)
{
    cell_job_t *J = (cell_job_t *)arg;
    for (uint64_t p = J->p0; p < J->p1; ++p) cell_escape_one(J, p, J->out + ORC_CELL_REC * (p - J->p0));
    return NULL;
}

/* n whole-cell escapes from q (|q_k| < 1) with packet ids [offset, offset+n);
 * n_in NULL = isotropic incoming directions.  out [n][ORC_CELL_REC]. */
int orc_cell_escape_record(int64_t n, double tau_c, double a, double x_in, const double *q, const double *n_in,
                           uint64_t seed, uint64_t offset, int n_threads, double *out)
{
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    for (int k = 0; k < 3; ++k) if (!(fabs(q[k]) < 1.0)) return -1;
    pthread_t th[256];
    cell_job_t J[256];
    for (int t = 0; t < n_threads; ++t) {
        J[t].tau = tau_c; J[t].a = a; J[t].xin = x_in; J[t].seed = seed; J[t].max_scat = 20000000;
        for (int k = 0; k < 3; ++k) { J[t].q[k] = q[k]; J[t].nin[k] = n_in ? n_in[k] : 0.0; }
        J[t].given_dir = n_in != NULL;
        J[t].p0 = offset + (uint64_t)n * t / n_threads;
        J[t].p1 = offset + (uint64_t)n * (t + 1) / n_threads;
        J[t].out = out + ORC_CELL_REC * (J[t].p0 - offset);
        pthread_create(&th[t], NULL, cell_escape_main, &J[t]);
    }
    for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    return 0;
}
