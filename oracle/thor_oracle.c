/*
 * thor_oracle.c -- plain, serial, FP64 CPU oracle of the resonant-line Monte
 * Carlo transport of arXiv 2507.11603 ("THOR"), Sections 2-3.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product library.  It shares no
 * code, headers, tables or constants with the HIP path.
 *
 * Style: each step is written in the order the paper states it, with no
 * blocking, fusion or reordering, so a reader can check it against the
 * paper.  Where the paper is silent (constants, RNG slot map, image plane,
 * u_parallel envelope split) the reading taken is stated in the comment
 * beside the code that takes it.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared thor_oracle.c -lm
 *
 * What pins each part (tests/test_oracle_*.py, all CPU-only):
 *   line constants       literature values at 1e4 K
 *   or_voigt, dawson     scipy's Faddeeva function, 40-digit mpmath, special
 *                        cases, far-wing series, normalisation
 *   Philox               published known-answer vectors; AMD rocRAND's header
 *   u_parallel           exact CDF by quadrature (KS, chi^2), closed-form first
 *                        and second moments, expected trial counts
 *   phase functions      exact inverse CDFs, E[mu^2], Henyey-Greenstein E[mu]
 *   emission             cell frequencies against n^2 / sum n^2, uniform offsets,
 *                        isotropy, thermal gas-frame profile, Gaussian lines
 *   resonant scattering  x_out moments and the direction correlation in closed
 *                        form; core-skip truncation against brute-force
 *                        rejection sampling and the Exp(1) law of rho^2 - x_c^2
 *   transport            flux conservation, pure absorber, optically thin
 *                        limit, single-scattering probability, exact grid peel
 *                        depth, escape fraction by quadrature, peel
 *                        normalisation, frame invariance of a moving grid,
 *                        fitted emergent peaks of the slab and sphere solutions
 *   raytracing           Gunn-Peterson depth, equivalent width, damping wing,
 *                        closed-form projections, transposition invariance
 * Parity unpinned: the spectra and cubes of the expanding-shell and
 * cosmic-web grids, beyond the invariants above (no independent result
 * exists for them).
 */
#include "thor_oracle.h"

#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* Physical and atomic constants (cgs).  The paper fixes none of them; the */
/* CODATA values and the standard Lyman-alpha data are used.               */
/* ---------------------------------------------------------------------- */
static const double C_LIGHT = 2.99792458e10;     /* cm/s */
static const double K_BOLTZ = 1.380649e-16;      /* erg/K */
static const double M_HYDROGEN = 1.6735575e-24;  /* g */
static const double M_ELECTRON = 9.1093837015e-28; /* g */
static const double E_CHARGE = 4.80320471e-10;   /* esu */
static const double LYA_LAMBDA = 1215.67e-8;     /* cm */
static const double LYA_A21 = 6.265e8;           /* s^-1 */
static const double LYA_F12 = 0.4162;
static const double PI = 3.14159265358979323846;

/* The Mg II h and k resonance doublet (Section 2.4: fine-structure        */
/* splitting of one transition; both lines start from the same ground      */
/* level): k = 3s 2S1/2 - 3p 2P3/2 at 2796.352 A, h = 3s 2S1/2 - 3p 2P1/2   */
/* at 2803.531 A; Einstein A and oscillator strengths of Morton (2003).    */
static const double MG2K_LAMBDA = 2796.352e-8, MG2K_A21 = 2.60e8, MG2K_F12 = 0.6155;
static const double MG2H_LAMBDA = 2803.531e-8, MG2H_A21 = 2.57e8, MG2H_F12 = 0.3058;
static const double M_MAGNESIUM = 24.305 * 1.66053906660e-24;   /* g */

/* Section 2.3.1: x = (c/v_th)(nu - nu0)/nu0, v_th = sqrt(2 k T / m).      */
/* Doppler width dnu_D = nu0 v_th / c = v_th / lambda0, damping parameter  */
/* a = A21 / (4 pi dnu_D), line-centre cross-section                        */
/* sigma0 = f12 sqrt(pi) e^2 / (m_e c dnu_D), sigma(x) = sigma0 H(a, x).    */
static void transition_params(double lambda0, double a21, double f12, double mass, double T,
                              double *v_th, double *a, double *sigma0)
{
    double vth = sqrt(2.0 * K_BOLTZ * T / mass);
    double dnu_d = vth / lambda0;
    *v_th = vth;
    *a = a21 / (4.0 * PI * dnu_d);
    *sigma0 = f12 * sqrt(PI) * E_CHARGE * E_CHARGE / (M_ELECTRON * C_LIGHT * dnu_d);
}

void or_line_params(double T, double *v_th, double *a, double *sigma0)
{
    transition_params(LYA_LAMBDA, LYA_A21, LYA_F12, M_HYDROGEN, T, v_th, a, sigma0);
}

void or_species_params(int line, double T, double *v_th, double *a, double *sigma0)
{
    if (line == OR_LINE_MG2 || line == OR_LINE_MG2K)
        transition_params(MG2K_LAMBDA, MG2K_A21, MG2K_F12, M_MAGNESIUM, T, v_th, a, sigma0);
    else
        or_line_params(T, v_th, a, sigma0);
}

/* ---------------------------------------------------------------------- */
/* Voigt-Hjerting function H(a,x) = Re w(x + i a), the profile of eq.      */
/* (uparallel)'s normalisation and of sigma(x) (Section 3.4, Appendix A.3). */
/* ---------------------------------------------------------------------- */

/* Dawson's integral F(x) = exp(-x^2) * int_0^x exp(t^2) dt, by the power   */
/* series of the integral, sum_n x^(2n+1) / (n! (2n+1)), all terms positive, */
/* summed in long double.                                                    */
static long double dawson_ld(long double x)
{
    long double ax = fabsl(x), x2 = ax * ax, term = ax, sum = 0.0L;
    for (int n = 0; n < 2000; ++n) {
        long double add = term / (long double)(2 * n + 1);
        sum += add;
        if (add <= sum * 1e-22L)
            break;
        term *= x2 / (long double)(n + 1);
    }
    long double f = expl(-x2) * sum;
    return x < 0 ? -f : f;
}

double or_dawson(double x) { return (double)dawson_ld(x); }

/* ---------------------------------------------- core-to-wing transition x_cw */
/* Appendix A.2: x_cw(a) is where the Gaussian core exp(-x^2) of H(a,x) meets */
/* its Lorentzian wing a/(sqrt(pi) x^2).  With y = -x^2 the condition reads  */
/* y e^y = -a/sqrt(pi), so x_cw = sqrt(-W_{-1}(-a/sqrt(pi))), W_{-1} the     */
/* lower real branch of Lambert's W (defined for -1/e <= z < 0).             */
double or_lambert_wm1(double z)
{
    const double e = exp(1.0);
    if (!(z >= -1.0 / e && z < 0.0))
        return NAN;
    double w;
    if (z < -0.3) {
        /* near the branch point z = -1/e: w = -1 - p - p^2/3, p = sqrt(2(1 + e z)) */
        const double p = sqrt(fmax(0.0, 2.0 * (1.0 + e * z)));
        w = -1.0 - p - p * p / 3.0;
    } else {
        /* asymptotic start for z -> 0-: w = L1 - L2 + L2/L1 */
        const double L1 = log(-z), L2 = log(-L1);
        w = L1 - L2 + L2 / L1;
    }
    /* Halley's iteration on f(w) = w e^w - z */
    for (int it = 0; it < 64; ++it) {
        const double ew = exp(w);
        const double f = w * ew - z;
        if (w == -1.0)
            break;
        const double step = f / (ew * (w + 1.0) - (w + 2.0) * f / (2.0 * w + 2.0));
        w -= step;
        if (fabs(step) <= 4e-16 * fabs(w))
            break;
    }
    return w;
}

double or_xcw_exact(double a)
{
    return sqrt(-or_lambert_wm1(-a / sqrt(PI)));
}

/* the quartic in ln a of Appendix A.2 (five coefficients printed there) */
double or_xcw_b25(double a)
{
    const double L = log(a);
    const double c[5] = {1.03489162, -6.17680644e-1, -8.73073343e-2, -7.91384757e-3, -2.76037084e-4};
    double s = 0.0, p = 1.0;
    for (int i = 0; i < 5; ++i) {
        s += c[i] * p;
        p *= L;
    }
    return s;
}

/* |x| <= 6.5: Taylor series of the entire function w about the real point */
/* x, w(x + i a) = sum_n (i a)^n w^(n)(x) / n!, with                        */
/*   w(x) = exp(-x^2) + (2i/sqrt(pi)) F(x),                                 */
/*   w'(z) = -2 z w(z) + 2i/sqrt(pi),                                       */
/*   w^(n+1)(z) = -2 z w^(n)(z) - 2 n w^(n-1)(z)   (n >= 1).                */
/* |x| > 6.5: Laplace continued fraction of the non-Gaussian part,          */
/*   w(z) - exp(-z^2) ~ (i/sqrt(pi)) / (z - (1/2)/(z - 1/(z - (3/2)/...))), */
/* truncated at 16 levels (the last Hermite node of that depth lies below   */
/* 6.5, so the truncated fraction has no pole near the real axis there).    */
double or_voigt(double a, double x)
{
    const long double rsqpi = 0.56418958354775628694807945156077258584L; /* 1/sqrt(pi) */
    if (fabs(x) <= 6.5) {
        long double xl = x, al = a;
        long double complex w_prev = expl(-xl * xl) + 2.0L * rsqpi * dawson_ld(xl) * I;
        long double complex w_cur = -2.0L * xl * w_prev + 2.0L * rsqpi * I;
        long double complex ia_pow = 1.0L; /* (i a)^n */
        long double fact = 1.0L;           /* n! */
        long double sum = creall(w_prev);  /* n = 0 */
        for (int n = 1; n <= 24; ++n) {
            ia_pow *= al * I;
            fact *= (long double)n;
            sum += creall(ia_pow * w_cur) / fact;
            long double complex w_next = -2.0L * xl * w_cur - 2.0L * (long double)n * w_prev;
            w_prev = w_cur;
            w_cur = w_next;
        }
        return (double)sum;
    }
    long double complex z = (long double)x + (long double)a * I;
    long double complex t = z;
    for (int k = 16; k >= 1; --k)
        t = z - (0.5L * (long double)k) / t;
    long double complex w_asym = rsqpi * I / t;
    long double gauss = expl((long double)a * a - (long double)x * x) * cosl(2.0L * a * x);
    return (double)(creall(w_asym) + gauss);
}

/* ---------------------------------------------------------------------- */
/* Random numbers (Section 3.4.3).  The paper's generator is replaced by    */
/* the counter-based Philox4x32-10 of Salmon et al. (SC'11): key = (seed,   */
/* request id), counter = (slot, event, photon id low, photon id high).     */
/* ---------------------------------------------------------------------- */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* One keyed draw: two uniforms in [0,1) with 53 random bits each. */
static void draw2(uint32_t seed, uint32_t req, uint32_t slot, uint32_t event, uint64_t id,
                  double *ua, double *ub)
{
    uint32_t ctr[4] = { slot, event, (uint32_t)id, (uint32_t)(id >> 32) };
    uint32_t key[2] = { seed, req };
    uint32_t w[4];
    or_philox4x32_10(ctr, key, w);
    uint64_t hi = ((uint64_t)w[0] << 32) | w[1];
    uint64_t lo = ((uint64_t)w[2] << 32) | w[3];
    *ua = (double)(hi >> 11) * 0x1p-53;
    *ub = (double)(lo >> 11) * 0x1p-53;
}

void or_draw(uint32_t seed, uint32_t request_id, uint32_t slot, uint32_t event, uint64_t id,
             double out[2])
{
    draw2(seed, request_id, slot, event, id, &out[0], &out[1]);
}

/* RNG slot map.  Event 0 is the emission, event e >= 1 the e-th interaction. */
enum { SLOT_E_DIR = 0, SLOT_E_GAUSS = 1, SLOT_E_CELL = 2, SLOT_E_OFFS = 3, SLOT_E_TAU = 4, SLOT_E_LINE = 5 };
enum { SLOT_TYPE = 0, SLOT_UPERP = 1, SLOT_MU = 2, SLOT_TAU = 3, SLOT_UPAR = 4 };

/* ---------------------------------------------------------------------- */
/* u_parallel, eq. (uparallel): f(u) ~ exp(-u^2) / ((x - u)^2 + a^2) for    */
/* |x|, with u -> sign(x) u afterwards.  Rejection sampling (Section 3.4).  */
/*                                                                          */
/* |x| < 2.25: the paper's piecewise comparison function, eq.               */
/* (uparallel_comparisonfunc): g1 = 1/((x-u)^2+a^2) for u <= u0,            */
/* g2 = exp(-u0^2)/((x-u)^2+a^2) for u > u0; exact for any u0 >= 0.         */
/* |x| >= 2.25: same g2 above u0, and below u0 the Gaussian envelope        */
/* exp(-u^2) x^-2 exp(2u/x + c u^2/x^2) >= f, with c = h(u0/x),              */
/* h(t) = (-2 ln(1-t) - 2t)/t^2 (h increases with t, so                      */
/* (1 - u/x)^-2 <= exp(2t + c t^2) for all u <= u0).  Exact as well.        */
/* u0 rules (speed only; any u0 gives exact samples): |x| < 2.25, two steps */
/* of u0 <- x - sqrt(a expm1(u0^2) / (2 pi u0)) from u0 = x; |x| >= 2.25,     */
/* u0 = min(sqrt(ln(sqrt(pi) x^2 / a) + 3), x - 0.3/x).                      */
/* Trial j draws from slot 4 + 2j (choice, acceptance) and, for a Gaussian  */
/* proposal, slot 5 + 2j (radius, angle).                                    */
/* ---------------------------------------------------------------------- */
static const double UPAR_X_SWITCH = 2.25;

static double zheng_u0(double xa, double a)
{
    double u0 = xa;
    for (int it = 0; it < 2; ++it) {
        if (u0 <= 0.0)
            break;
        u0 = xa - sqrt(a * expm1(u0 * u0) / (2.0 * PI * u0));
        if (u0 < 0.0) u0 = 0.0;
        if (u0 > xa) u0 = xa;
    }
    return u0;
}

static double split_u0(double xa, double a)
{
    double u0 = sqrt(log(sqrt(PI) * xa * xa / a) + 3.0);
    double cap = xa - 0.3 / xa;
    return u0 < cap ? u0 : cap;
}

static double h_coef(double t)
{
    return (-2.0 * log1p(-t) - 2.0 * t) / (t * t);
}

double or_upar_expected_trials(double x, double a)
{
    double xa = fabs(x);
    double target = PI * or_voigt(a, xa) / a;   /* integral of f */
    if (xa < UPAR_X_SWITCH) {
        double u0 = zheng_u0(xa, a);
        double th0 = atan((u0 - xa) / a);
        double m = (th0 + PI / 2) + exp(-u0 * u0) * (PI / 2 - th0);
        return (m / a) / target;
    }
    double u0 = split_u0(xa, a);
    double t0 = u0 / xa, c = h_coef(t0);
    double p = 1.0 - c / (xa * xa), mu = 1.0 / (xa * p);
    double za = exp(p * mu * mu) * sqrt(PI / p) / (xa * xa);
    double th0 = atan((u0 - xa) / a);
    double zb = exp(-u0 * u0) * (PI / 2 - th0) / a;
    return (za + zb) / target;
}

static double sample_upar_keyed(double x, double a, uint32_t seed, uint32_t req, uint32_t event,
                                uint64_t id, uint64_t *trials)
{
    double xa = fabs(x);
    double sgn = x < 0 ? -1.0 : 1.0;
    uint64_t n = 0;
    double u;
    if (xa < UPAR_X_SWITCH) {
        double u0 = zheng_u0(xa, a);
        double th0 = atan((u0 - xa) / a);
        double p1 = th0 + PI / 2;
        double e0 = exp(-u0 * u0);
        double m = p1 + e0 * (PI / 2 - th0);
        for (;;) {
            double r1, r2;
            draw2(seed, req, SLOT_UPAR + 2u * (uint32_t)n, event, id, &r1, &r2);
            ++n;
            double r = r1 * m;
            if (r < p1) {
                double th = r - PI / 2;
                u = xa + a * tan(th);
                if (r2 < exp(-u * u))
                    break;
            } else {
                double th = th0 + (r - p1) / e0;
                u = xa + a * tan(th);
                if (r2 < exp(u0 * u0 - u * u))
                    break;
            }
        }
    } else {
        double u0 = split_u0(xa, a);
        double t0 = u0 / xa, c = h_coef(t0);
        double p = 1.0 - c / (xa * xa), mu = 1.0 / (xa * p);
        double za = exp(p * mu * mu) * sqrt(PI / p) / (xa * xa);
        double th0 = atan((u0 - xa) / a);
        double e0 = exp(-u0 * u0);
        double zb = e0 * (PI / 2 - th0) / a;
        for (;;) {
            double r1, r2;
            draw2(seed, req, SLOT_UPAR + 2u * (uint32_t)n, event, id, &r1, &r2);
            double r = r1 * (za + zb);
            if (r < za) {
                double r3, r4;
                draw2(seed, req, SLOT_UPAR + 2u * (uint32_t)n + 1u, event, id, &r3, &r4);
                ++n;
                u = mu + sqrt(-log(1.0 - r3) / p) * cos(2.0 * PI * r4);
                if (u > u0)
                    continue;
                double t = u / xa;
                double env = exp(2.0 * t + c * t * t) / (xa * xa);
                double tgt = 1.0 / ((xa - u) * (xa - u) + a * a);
                if (r2 * env < tgt)
                    break;
            } else {
                ++n;
                double th = th0 + (r - za) * a / e0;
                u = xa + a * tan(th);
                if (r2 < exp(u0 * u0 - u * u))
                    break;
            }
        }
    }
    if (trials)
        *trials = n;
    return sgn * u;
}

double or_sample_upar(double x, double a, uint32_t seed, uint32_t event, uint64_t id,
                      uint64_t *trials)
{
    return sample_upar_keyed(x, a, seed, 0u, event, id, trials);
}

/* ---------------------------------------------------------------------- */
/* Phase functions (Sections 2.3.1, 2.3.2).  Each samples mu = cos(theta)  */
/* by inverting its CDF on [-1, 1].                                          */
/*   isotropic p = 1/2:            mu = 2U - 1                              */
/*   dipole p = 3/8 (1 + mu^2):    mu^3 + 3 mu = 8U - 4 (Cardano)           */
/*   core mix p = 11/24 + 3/24 mu^2: mu^3 + 11 mu = 24U - 12 (Cardano)      */
/*   Henyey-Greenstein:            closed-form inverse                      */
/* ---------------------------------------------------------------------- */
double or_sample_mu(int phase, double U, double g)
{
    if (phase == OR_PHASE_ISO)
        return 2.0 * U - 1.0;
    if (phase == OR_PHASE_DIPOLE || phase == OR_PHASE_CORE_WING) {
        /* depressed cubic mu^3 + p mu = q, one real root */
        double p = (phase == OR_PHASE_DIPOLE) ? 3.0 : 11.0;
        double q = (phase == OR_PHASE_DIPOLE) ? (8.0 * U - 4.0) : (24.0 * U - 12.0);
        double disc = sqrt(q * q / 4.0 + p * p * p / 27.0);
        double s = cbrt(q / 2.0 + disc);
        return s - p / (3.0 * s);
    }
    /* Henyey-Greenstein */
    if (g == 0.0)
        return 2.0 * U - 1.0;
    double frac = (1.0 - g * g) / (1.0 - g + 2.0 * g * U);
    return (1.0 + g * g - frac * frac) / (2.0 * g);
}

static double phase_value(int phase, double mu, double g)
{
    if (phase == OR_PHASE_ISO)
        return 0.5;
    if (phase == OR_PHASE_DIPOLE)
        return 0.375 * (1.0 + mu * mu);
    if (phase == OR_PHASE_CORE_WING)
        return 11.0 / 24.0 + 3.0 / 24.0 * mu * mu;
    return 0.5 * (1.0 - g * g) / pow(1.0 + g * g - 2.0 * g * mu, 1.5);
}

/* Orthonormal basis perpendicular to a unit vector: the branchless          */
/* construction of Duff et al. (2017, JCGT 6(1)).                            */
void or_basis(const double n[3], double e1[3], double e2[3])
{
    double sign = copysign(1.0, n[2]);
    double a = -1.0 / (sign + n[2]);
    double b = n[0] * n[1] * a;
    e1[0] = 1.0 + sign * n[0] * n[0] * a;
    e1[1] = sign * b;
    e1[2] = -sign * n[0];
    e2[0] = b;
    e2[1] = sign + n[1] * n[1] * a;
    e2[2] = -n[1];
}

/* ---------------------------------------------------------------------- */
/* Media (Section 3.3): meshless sphere/shell and slab, uniform Cartesian   */
/* grid.  query(): distance to the next cell face / boundary and the fields */
/* of the current cell (zeroth order, Section 3.4).                          */
/* ---------------------------------------------------------------------- */
typedef struct {
    const or_geometry *g;
    const or_opts *o;
    /* homogeneous meshless medium */
    double n, T, vth, a, sig0, k0, kd, sigd;
    double xcrit;
    /* resonant lines (Section 2.4): nl transitions; line 0 is the reference
     * whose per-cell v_th, a and k0 the medium carries.  Line j sits at lab
     * offset lc[j] (cm/s) from line 0's centre; its dimensionless frequency
     * is x_j = lrho[j] (x - lc[j]/v_th) (lrho = lambda_j/lambda_0, the ratio
     * of the Doppler widths), its damping parameter lam[j] a and its
     * line-centre opacity lk[j] k0; lw[j]: emission probability (oscillator
     * strengths, Section 5.3) */
    int nl;
    double lc[2], lrho[2], lam[2], lk[2], lw[2];
    /* grid */
    double dx[3];
    int dims[3];
    double *cdf;
    double cdf_total;
} model_t;

enum { REG_CAVITY = 0, REG_GAS = 1, REG_OUT = 2 };

typedef struct {
    double p[3];
    int cell[3];
    int region;
} loc_t;

typedef struct {
    double n, vth, a, k0, kd, v[3];
} cellf_t;

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Resonant opacity at gas-frame offset x (units of the reference line's    */
/* v_th): a doublet sums its transitions (Section 2.4).  *k_first: line 0's */
/* share.                                                                    */
static double line_opacity(const model_t *m, double k0, double a, double vth, double x, double *k_first)
{
    double k = k0 * or_voigt(a, x);
    if (k_first)
        *k_first = k;
    for (int j = 1; j < m->nl; ++j)
        k += k0 * m->lk[j] * or_voigt(a * m->lam[j], m->lrho[j] * (x - m->lc[j] / vth));
    return k;
}

/* Lab-frame offset of a photon leaving line j at offset x_j from its centre */
/* (in that line's Doppler units) with gas velocity component vk.            */
static double line_dv(const model_t *m, int j, double xj, double vth, double vk)
{
    if (j == 0)
        return xj * vth + vk;
    return (xj / m->lrho[j]) * vth + m->lc[j] + vk;
}

static void grid_fields(const model_t *m, const int c[3], cellf_t *f)
{
    const or_geometry *g = m->g;
    size_t idx = ((size_t)c[2] * (size_t)g->ny + (size_t)c[1]) * (size_t)g->nx + (size_t)c[0];
    double n = (double)g->f_n[idx];
    f->n = n;
    f->v[0] = (double)g->f_vx[idx];
    f->v[1] = (double)g->f_vy[idx];
    f->v[2] = (double)g->f_vz[idx];
    if (n > 0.0) {
        double sig0;
        or_species_params(g->line, (double)g->f_T[idx], &f->vth, &f->a, &sig0);
        f->k0 = n * sig0;
        f->kd = g->sigma_d * n;
    } else {
        f->vth = 1.0; f->a = 0.0; f->k0 = 0.0; f->kd = 0.0;
    }
}

/* Hubble flow of a grid medium.  The cross-section is taken in the frame of
 * the gas (Section 2.2), whose velocity includes the cosmological expansion:
 * v(p) = v_cell + H (p - p_ref), so along a flight the gas-frame frequency
 * drifts by -H per unit length.  Sub-cell stepping (Section 3.4): a cell
 * crossing of length t is cut into n equal steps, n the smallest integer
 * with H t / n <= hubble_step v_th, each with the profile at its midpoint. */
static int hubble_on(const model_t *m) { return m->g->kind == OR_GRID && m->g->hubble > 0.0; }

static void hubble_velocity(const model_t *m, const double p[3], double vh[3])
{
    for (int i = 0; i < 3; ++i) vh[i] = m->g->hubble * (p[i] - m->g->hubble_ref[i]);
}

static int hubble_steps(const model_t *m, double t, double vth)
{
    double f = m->g->hubble_step > 0.0 ? m->g->hubble_step : 0.1;
    double r = m->g->hubble * t / (f * vth);
    return r > 1.0 ? (int)ceil(r) : 1;
}

static void meshless_velocity(const model_t *m, const double q[3], double v[3])
{
    const or_geometry *g = m->g;
    v[0] = v[1] = v[2] = 0.0;
    if (g->v_profile == OR_VEL_NONE)
        return;
    if (g->kind == OR_SLAB) { /* linear v_z = v_max z / Z */
        v[2] = g->v_max * q[2] / g->r_outer;
        return;
    }
    double r = sqrt(dot3(q, q));
    if (g->v_profile == OR_VEL_CONST_RADIAL) {
        if (r > 0.0)
            for (int i = 0; i < 3; ++i) v[i] = g->v_max * q[i] / r;
    } else {
        for (int i = 0; i < 3; ++i) v[i] = g->v_max * q[i] / g->r_outer;
    }
}

/* Exit distance from a sphere of radius R along k: the far root of
 * |p + t k|^2 = R^2.  A point that rounding put just outside the sphere while
 * it moves inwards still crosses it (far root > 0); a point outside moving
 * away exits at once (0). */
static double sphere_exit(const double p[3], const double k[3], double R)
{
    double b = dot3(p, k);
    double c = dot3(p, p) - R * R;
    double disc = b * b - c;
    if (disc <= 0.0)
        return 0.0;
    double q = sqrt(disc);
    if (b <= 0.0)
        return q - b;
    return c < 0.0 ? -c / (q + b) : 0.0;
}

/* Segment query.  Returns the path length t to the end of the segment and  */
/* fills the fields; *cross tells whether the segment ends on a boundary    */
/* (1) or is a limiter sub-step inside the same region (0).                 */
static double query(const model_t *m, const loc_t *L, const double k[3], cellf_t *f, int *next_region,
                    int *cross_mask)
{
    const or_geometry *g = m->g;
    *cross_mask = 0;
    if (g->kind == OR_GRID) {
        double tmin = INFINITY;
        double tm[3];
        for (int ax = 0; ax < 3; ++ax) {
            if (k[ax] > 0.0)
                tm[ax] = (g->lo[ax] + (double)(L->cell[ax] + 1) * m->dx[ax] - L->p[ax]) / k[ax];
            else if (k[ax] < 0.0)
                tm[ax] = (g->lo[ax] + (double)L->cell[ax] * m->dx[ax] - L->p[ax]) / k[ax];
            else
                tm[ax] = INFINITY;
            if (tm[ax] < tmin) tmin = tm[ax];
        }
        for (int ax = 0; ax < 3; ++ax)
            if (tm[ax] == tmin) *cross_mask |= 1 << ax;
        if (tmin < 0.0) tmin = 0.0;
        grid_fields(m, L->cell, f);
        *next_region = REG_GAS;
        return tmin;
    }
    /* meshless */
    double t;
    int nxt;
    if (g->kind == OR_SLAB) {
        if (k[2] > 0.0) t = (g->r_outer - L->p[2]) / k[2];
        else if (k[2] < 0.0) t = (-g->r_outer - L->p[2]) / k[2];
        else t = INFINITY;
        if (t < 0.0) t = 0.0;
        nxt = REG_OUT;
    } else if (L->region == REG_CAVITY) {
        t = sphere_exit(L->p, k, g->r_inner);
        nxt = REG_GAS;
    } else {
        t = sphere_exit(L->p, k, g->r_outer);
        nxt = REG_OUT;
        if (g->r_inner > 0.0) {
            double b = dot3(L->p, k);
            double ci = dot3(L->p, L->p) - g->r_inner * g->r_inner;
            double disc = b * b - ci;
            if (b < 0.0 && disc > 0.0) {
                double tin = ci / (-b + sqrt(disc));
                if (tin < 0.0) tin = 0.0;
                if (tin < t) {
                    t = tin;
                    nxt = REG_CAVITY;
                }
            }
        }
    }
    if (L->region == REG_CAVITY) {
        f->n = 0.0; f->vth = 1.0; f->a = 0.0; f->k0 = 0.0; f->kd = 0.0;
        f->v[0] = f->v[1] = f->v[2] = 0.0;
        *next_region = nxt;
        *cross_mask = 1;
        return t;
    }
    /* homogeneous gas; velocity fields are sub-stepped with the limiter */
    f->n = m->n; f->vth = m->vth; f->a = m->a; f->k0 = m->k0; f->kd = m->kd;
    *cross_mask = 1;
    if (g->v_profile != OR_VEL_NONE && g->v_max != 0.0) {
        double scale;
        if (g->kind == OR_SLAB || g->v_profile == OR_VEL_LINEAR)
            scale = g->r_outer;
        else {
            double r = sqrt(dot3(L->p, L->p));
            scale = r > 1e-6 * g->r_outer ? r : 1e-6 * g->r_outer;
        }
        double lmax = g->step_f * m->vth * scale / fabs(g->v_max);
        if (t > lmax) {
            t = lmax;
            *cross_mask = 0;
            nxt = L->region;
        }
        double mid[3];
        for (int i = 0; i < 3; ++i) mid[i] = L->p[i] + 0.5 * t * k[i];
        meshless_velocity(m, mid, f->v);
    } else {
        f->v[0] = f->v[1] = f->v[2] = 0.0;
    }
    *next_region = nxt;
    return t;
}

/* Move the location along k by the full segment t and apply the crossing. */
/* Returns 1 when the packet leaves the domain.                             */
static int advance(const model_t *m, loc_t *L, const double k[3], double t, int next_region,
                   int cross_mask)
{
    const or_geometry *g = m->g;
    for (int i = 0; i < 3; ++i)
        L->p[i] += t * k[i];
    if (g->kind == OR_GRID) {
        for (int ax = 0; ax < 3; ++ax) {
            if (!(cross_mask & (1 << ax)))
                continue;
            if (k[ax] > 0.0) {
                L->cell[ax] += 1;
                L->p[ax] = g->lo[ax] + (double)L->cell[ax] * m->dx[ax];
            } else {
                L->cell[ax] -= 1;
                L->p[ax] = g->lo[ax] + (double)(L->cell[ax] + 1) * m->dx[ax];
            }
        }
        for (int ax = 0; ax < 3; ++ax)
            if (L->cell[ax] < 0 || L->cell[ax] >= m->dims[ax])
                return 1;
        return 0;
    }
    if (cross_mask)
        L->region = next_region;
    return L->region == REG_OUT;
}

static void locate(const model_t *m, loc_t *L)
{
    const or_geometry *g = m->g;
    if (g->kind == OR_GRID) {
        for (int ax = 0; ax < 3; ++ax) {
            int c = (int)floor((L->p[ax] - g->lo[ax]) / m->dx[ax]);
            if (c < 0) c = 0;
            if (c >= m->dims[ax]) c = m->dims[ax] - 1;
            L->cell[ax] = c;
        }
        L->region = REG_GAS;
        return;
    }
    if (g->kind == OR_SLAB) {
        L->region = fabs(L->p[2]) < g->r_outer ? REG_GAS : REG_OUT;
        return;
    }
    double r = sqrt(dot3(L->p, L->p));
    if (r < g->r_inner) L->region = REG_CAVITY;
    else if (r < g->r_outer) L->region = REG_GAS;
    else L->region = REG_OUT;
}

/* ---------------------------------------------------------------------- */
/* Peeling off (Section 3.4.1): phase function towards the observer times  */
/* exp(-tau) along a new ray from the event to the boundary.                */
/* ---------------------------------------------------------------------- */
static void obs_dir(int axis, double k[3])
{
    k[0] = k[1] = k[2] = 0.0;
    k[axis % 3] = axis < 3 ? 1.0 : -1.0;
}

static void obs_image(int axis, const double p[3], double *u, double *v)
{
    switch (axis % 3) {
    case 2: *u = p[0]; *v = p[1]; break;   /* +-z: (x, y) */
    case 0: *u = p[1]; *v = p[2]; break;   /* +-x: (y, z) */
    default: *u = p[2]; *v = p[0]; break;  /* +-y: (z, x) */
    }
}

static int bin_of(double v, double lo, double hi, int nb)
{
    double w = (hi - lo) / (double)nb;
    double b = floor((v - lo) / w);
    if (!(b >= 0.0) || b >= (double)nb)
        return -1;
    return (int)b;
}

static void peel(const model_t *m, const loc_t *L0, int o, double weight, double dv_peel,
                 double *cube, or_stats *st)
{
    const or_opts *op = m->o;
    double k[3];
    obs_dir(op->obs_axis[o], k);
    st->peel_contrib++;
    loc_t L = *L0;
    double tau = 0.0;
    int cut = 0;
    for (;;) {
        cellf_t f;
        int nr, cm;
        double t = query(m, &L, k, &f, &nr, &cm);
        st->peel_visits++;
        if (f.k0 > 0.0 || f.kd > 0.0) {
            if (hubble_on(m)) {
                /* gas-frame offset at the segment start, then the sub-steps */
                double vh[3];
                hubble_velocity(m, L.p, vh);
                double u0 = dv_peel - dot3(f.v, k) - dot3(vh, k);
                int n = hubble_steps(m, t, f.vth);
                double ds = t / n;
                for (int j = 0; j < n; ++j) {
                    double x = (u0 - m->g->hubble * ((j + 0.5) * ds)) / f.vth;
                    tau += (line_opacity(m, f.k0, f.a, f.vth, x, NULL) + f.kd) * ds;
                }
            } else {
                double x = (dv_peel - dot3(f.v, k)) / f.vth;
                double kt = line_opacity(m, f.k0, f.a, f.vth, x, NULL) + f.kd;
                if (isinf(t)) { cut = 1; break; }
                tau += kt * t;
            }
        } else if (isinf(t)) {
            break;
        }
        if (tau > op->tau_cut) { cut = 1; break; }
        if (advance(m, &L, k, t, nr, cm))
            break;
    }
    if (cut) {
        st->peel_cut++;
        return;
    }
    double u, v;
    obs_image(op->obs_axis[o], L0->p, &u, &v);
    int ix = bin_of(u, op->img_lo[0], op->img_hi[0], op->cube_nx);
    int iy = bin_of(v, op->img_lo[1], op->img_hi[1], op->cube_ny);
    int ib = bin_of(dv_peel, op->cube_v_lo, op->cube_v_hi, op->cube_nb);
    if (ix < 0 || iy < 0 || ib < 0) {
        st->peel_dropped++;
        return;
    }
    size_t idx = (((size_t)o * op->cube_ny + iy) * op->cube_nx + ix) * op->cube_nb + ib;
    cube[idx] += weight * exp(-tau);
}

/* ---------------------------------------------------------------------- */
/* Transport of one packet (Sections 3.4, 2.2-2.3).                          */
/* ---------------------------------------------------------------------- */
static void rotate(const double kin[3], double mu, double phi, double kout[3], double e1[3], double e2[3])
{
    or_basis(kin, e1, e2);
    double s = sqrt(fmax(0.0, 1.0 - mu * mu));
    double c = cos(phi), sn = sin(phi);
    for (int i = 0; i < 3; ++i)
        kout[i] = mu * kin[i] + s * (c * e1[i] + sn * e2[i]);
}

/* A packet as the generator hands it over (Section 3.4 "Emission"). */
typedef struct {
    loc_t L;
    double k[3];
    cellf_t f0;        /* fields at the emission point */
    double v0[3];      /* gas velocity there (with the Hubble flow of a grid) */
    double dv;         /* lab-frame frequency offset */
    double dv_loc;     /* gas-frame offset (THERMAL spectra; 0 otherwise) */
} emitted_t;

/* Emission (Section 3.4, event 0): isotropic direction, position (the       */
/* source point, or a cell drawn with probability n_HI^2 / sum n_HI^2 and a   */
/* uniform point inside it), frequency (delta, Gaussian, or the gas-frame     */
/* thermal profile of the emitting cell shifted to the lab frame by v.k).     */
static void emit_packet(const model_t *m, const or_source *src, uint64_t id, emitted_t *e)
{
    const or_geometry *g = m->g;
    const uint32_t seed = src->seed, req = src->request_id;
    double ua, ub;
    loc_t L;
    double *k = e->k;

    draw2(seed, req, SLOT_E_DIR, 0, id, &ua, &ub);
    double mu = 2.0 * ua - 1.0, phi = 2.0 * PI * ub;
    double st_ = sqrt(fmax(0.0, 1.0 - mu * mu));
    k[0] = st_ * cos(phi); k[1] = st_ * sin(phi); k[2] = mu;

    if (src->kind == OR_SRC_CELL_N2) {
        double uc, ox, oy, oz;
        draw2(seed, req, SLOT_E_CELL, 0, id, &uc, &ox);
        draw2(seed, req, SLOT_E_OFFS, 0, id, &oy, &oz);
        double target = uc * m->cdf_total;
        size_t ncell = (size_t)g->nx * g->ny * g->nz;
        size_t lo = 0, hi = ncell - 1;           /* first index with cdf > target */
        while (lo < hi) {
            size_t mid = lo + (hi - lo) / 2;
            if (m->cdf[mid] > target) hi = mid; else lo = mid + 1;
        }
        L.cell[0] = (int)(lo % (size_t)g->nx);
        L.cell[1] = (int)((lo / (size_t)g->nx) % (size_t)g->ny);
        L.cell[2] = (int)(lo / ((size_t)g->nx * g->ny));
        double off[3] = { ox, oy, oz };
        for (int ax = 0; ax < 3; ++ax)
            L.p[ax] = g->lo[ax] + ((double)L.cell[ax] + off[ax]) * m->dx[ax];
        L.region = REG_GAS;
    } else {
        for (int i = 0; i < 3; ++i) L.p[i] = src->pos[i];
        locate(m, &L);
    }

    cellf_t f0;
    {
        int nr, cm;
        if (L.region == REG_OUT) {
            f0.n = 0; f0.vth = 1.0; f0.a = 0; f0.k0 = 0; f0.kd = 0; f0.v[0] = f0.v[1] = f0.v[2] = 0;
        } else {
            (void)query(m, &L, k, &f0, &nr, &cm);
        }
    }
    double v0[3] = { f0.v[0], f0.v[1], f0.v[2] };
    if (hubble_on(m) && L.region != REG_OUT) {
        double vh[3];
        hubble_velocity(m, L.p, vh);
        for (int i = 0; i < 3; ++i) v0[i] += vh[i];
    }
    double dv, dv_loc = 0.0;
    double z = 0.0;
    if (src->spectrum != OR_SPEC_DELTA) {
        draw2(seed, req, SLOT_E_GAUSS, 0, id, &ua, &ub);
        if (src->spectrum != OR_SPEC_FLAT)
            z = sqrt(-2.0 * log(1.0 - ua)) * cos(2.0 * PI * ub);
    }
    /* a doublet source emits in line j with probability lw[j] (the ratio of  */
    /* the oscillator strengths), at that line's centre offset                */
    double lcen = 0.0;
    if (src->lines && m->nl > 1) {
        double ul, unused;
        draw2(seed, req, SLOT_E_LINE, 0, id, &ul, &unused);
        if (ul >= m->lw[0])
            lcen = m->lc[1];
    }
    if (src->spectrum == OR_SPEC_THERMAL) {
        /* gas-frame Doppler profile of the emitting cell, then the lab frame */
        dv_loc = src->dv0 + f0.vth * z / sqrt(2.0) + lcen;
        dv = dv_loc + dot3(v0, k);
    } else if (src->spectrum == OR_SPEC_GAUSS) {
        dv = src->dv0 + src->sigma_v * z + lcen;
    } else if (src->spectrum == OR_SPEC_FLAT) {
        /* flat continuum over dv0 +- sigma_v (Section 4's doublet test) */
        dv = src->dv0 + src->sigma_v * (2.0 * ua - 1.0) + lcen;
    } else {
        dv = src->dv0 + lcen;
    }
    e->L = L;
    e->f0 = f0;
    for (int i = 0; i < 3; ++i) e->v0[i] = v0[i];
    e->dv = dv;
    e->dv_loc = dv_loc;
}

/* One resonant scattering (Sections 2.3.1, 3.4, 3.4.2). */
typedef struct {
    double upar;          /* atom velocity along k_in, units of v_th */
    double uperp[2];      /* its components along the basis e1, e2 of k_in */
    double u[3];          /* the atom velocity */
    double x_atom;        /* x - u_par: frequency in the atom's frame */
    int phase;            /* phase function used (core/wing picks per x_atom) */
    double kout[3];
    double x_out;         /* outgoing gas-frame frequency */
    uint64_t trials;      /* u_par proposals */
} scatter_t;

/* Atom velocity u = u_par k + u_perp: u_par from eq. (uparallel), u_perp     */
/* a 2D Gaussian of variance 1/2 per component (eq. uperp) whose radius is    */
/* truncated below x_crit when core skipping applies (|x| < x_crit, Section   */
/* 3.4.2); new direction from the phase function; outgoing frequency          */
/* x_out = x - u_par + u.k_out (eq. doublelorentztransform, recoil ignored).  */
static void resonant_scatter(double x, double a, const double k[3], double xcrit, int phase,
                             uint32_t seed, uint32_t req, uint32_t event, uint64_t id, scatter_t *s)
{
    uint64_t trials = 0;
    double upar = sample_upar_keyed(x, a, seed, req, event, id, &trials);
    double ur, upsi;
    draw2(seed, req, SLOT_UPERP, event, id, &ur, &upsi);
    double rho2 = -log(1.0 - ur);
    if (xcrit > 0.0 && fabs(x) < xcrit)
        rho2 += xcrit * xcrit;
    double rho = sqrt(rho2);
    double up1 = rho * cos(2.0 * PI * upsi), up2 = rho * sin(2.0 * PI * upsi);
    double e1[3], e2[3];
    or_basis(k, e1, e2);
    for (int i = 0; i < 3; ++i)
        s->u[i] = upar * k[i] + up1 * e1[i] + up2 * e2[i];
    double x_atom = x - upar;
    int ph = phase;
    if (ph == OR_PHASE_CORE_WING && fabs(x_atom) >= 0.2)
        ph = OR_PHASE_DIPOLE;
    double um, uf;
    draw2(seed, req, SLOT_MU, event, id, &um, &uf);
    double muo = or_sample_mu(ph, um, 0.0);
    rotate(k, muo, 2.0 * PI * uf, s->kout, e1, e2);
    s->upar = upar;
    s->uperp[0] = up1;
    s->uperp[1] = up2;
    s->x_atom = x_atom;
    s->phase = ph;
    s->x_out = x_atom + dot3(s->u, s->kout);
    s->trials = trials;
}

/* ---------------------------------------------------------------------- */
/* Transport of one packet (Sections 3.4, 2.2-2.3).                          */
/* ---------------------------------------------------------------------- */
static void transport_one(const model_t *m, const or_source *src, uint64_t id, double *spectrum,
                          double *cube, or_stats *st, or_record *rec)
{
    const or_geometry *g = m->g;
    const or_opts *op = m->o;
    const uint32_t seed = src->seed, req = src->request_id;
    double ua, ub;

    /* Emission (Section 3.4): direction, position, frequency, tau_target. */
    emitted_t em;
    emit_packet(m, src, id, &em);
    loc_t L = em.L;
    double k[3] = { em.k[0], em.k[1], em.k[2] };
    cellf_t f0 = em.f0;
    double dv = em.dv, dv_loc = em.dv_loc;
    st->emitted++;
    for (int o = 0; o < op->n_obs; ++o) {
        double ko[3];
        obs_dir(op->obs_axis[o], ko);
        double dvp = (src->spectrum == OR_SPEC_THERMAL) ? dv_loc + dot3(em.v0, ko) : dv;
        if (L.region != REG_OUT)
            peel(m, &L, o, 1.0 / (4.0 * PI), dvp, cube, st);
    }
    draw2(seed, req, SLOT_E_TAU, 0, id, &ua, &ub);
    double tau_target = -log(1.0 - ua);
    double tau_acc = 0.0;
    uint32_t event = 0;
    uint32_t n_res = 0, n_dust = 0;
    int fate = OR_FATE_NONE;
    const double w = 1.0;
    uint64_t max_events = op->max_events ? op->max_events : 100000000ull;

    if (L.region == REG_OUT)
        fate = OR_FATE_ESCAPED;

    while (fate == OR_FATE_NONE) {
        /* Propagation: piecewise-linear integration of tau (Section 3.4). */
        cellf_t f;
        int nr, cm;
        double t = query(m, &L, k, &f, &nr, &cm);
        st->main_visits++;
        double kh = 0.0, kt = 0.0;
        double s = -1.0;          /* interaction site along the segment, if any */
        if (hubble_on(m)) {
            double vh[3];
            hubble_velocity(m, L.p, vh);
            double u0 = dv - dot3(f.v, k) - dot3(vh, k);   /* gas-frame offset at the start */
            if (g->stop_dv > 0.0 && u0 < -g->stop_dv) {
                fate = OR_FATE_REDSHIFTED;
                break;
            }
            if (f.k0 > 0.0 || f.kd > 0.0) {
                int n = hubble_steps(m, t, f.vth);
                double ds = t / n;
                for (int j = 0; j < n; ++j) {
                    double x = (u0 - g->hubble * ((j + 0.5) * ds)) / f.vth;
                    double ktj = line_opacity(m, f.k0, f.a, f.vth, x, NULL) + f.kd;
                    if (tau_acc + ktj * ds >= tau_target) {
                        s = j * ds + (tau_target - tau_acc) / ktj;
                        kt = ktj;
                        break;
                    }
                    tau_acc += ktj * ds;
                }
            }
        } else {
            if (f.k0 > 0.0 || f.kd > 0.0) {
                double x = (dv - dot3(f.v, k)) / f.vth;
                kh = line_opacity(m, f.k0, f.a, f.vth, x, NULL);
                kt = kh + f.kd;
            }
            if (kt > 0.0 && tau_acc + kt * t >= tau_target)
                s = (tau_target - tau_acc) / kt;
        }
        if (s >= 0.0) {
            /* Interaction site: linear step where tau_current = tau_target. */
            for (int i = 0; i < 3; ++i) L.p[i] += s * k[i];
            if (hubble_on(m)) {   /* the gas moves with the Hubble flow at the site */
                double vh[3];
                hubble_velocity(m, L.p, vh);
                for (int i = 0; i < 3; ++i) f.v[i] += vh[i];
            }
            ++event;
            if ((uint64_t)event > max_events) {
                fate = OR_FATE_CAPPED;
                break;
            }
            double utype, ualb;
            draw2(seed, req, SLOT_TYPE, event, id, &utype, &ualb);
            double kout[3], e1[3], e2[3];
            if (utype * kt < f.kd) {
                /* Dust (Section 2.3.2): absorb or Henyey-Greenstein scatter, */
                /* coherent in the gas frame.                                 */
                if (ualb >= g->albedo) {
                    fate = OR_FATE_ABSORBED;
                    st->absorbed++;
                    st->w_absorbed += w;
                    break;
                }
                double um, uf;
                draw2(seed, req, SLOT_MU, event, id, &um, &uf);
                double muo = or_sample_mu(3, um, g->g_hg);
                double dvl = dv - dot3(f.v, k);
                rotate(k, muo, 2.0 * PI * uf, kout, e1, e2);
                for (int o = 0; o < op->n_obs; ++o) {
                    double ko[3];
                    obs_dir(op->obs_axis[o], ko);
                    double c = w * phase_value(3, dot3(k, ko), g->g_hg) / (2.0 * PI);
                    peel(m, &L, o, c, dvl + dot3(f.v, ko), cube, st);
                }
                dv = dvl + dot3(f.v, kout);
                ++n_dust;
                st->n_dust++;
            } else {
                /* Resonant scattering (Sections 2.3.1, 3.4, 3.4.2).  A doublet */
                /* scatters in line j with probability k_j / (k_0 + k_1) at the */
                /* site, from the same uniform rescaled to the resonant share,  */
                /* and re-emits in that line (both decay to the one ground      */
                /* level); the fine-structure line 2P1/2 -> 2S1/2 re-emits       */
                /* isotropically (Section 2.4).                                   */
                double x = (dv - dot3(f.v, k)) / f.vth;
                int j = 0;
                if (m->nl > 1) {
                    double k_first;
                    double kres = line_opacity(m, f.k0, f.a, f.vth, x, &k_first);
                    double u_line = (utype * kt - f.kd) / (kt - f.kd);
                    if (u_line * kres >= k_first)
                        j = 1;
                }
                double xj = j == 0 ? x : m->lrho[j] * (x - m->lc[j] / f.vth);
                double aj = j == 0 ? f.a : f.a * m->lam[j];
                int phj = j == 0 ? op->phase : OR_PHASE_ISO;
                scatter_t sc;
                resonant_scatter(xj, aj, k, m->xcrit, phj, seed, req, event, id, &sc);
                st->upar_trials += sc.trials;
                for (int i = 0; i < 3; ++i) kout[i] = sc.kout[i];
                for (int o = 0; o < op->n_obs; ++o) {
                    double ko[3];
                    obs_dir(op->obs_axis[o], ko);
                    double c = w * phase_value(sc.phase, dot3(k, ko), 0.0) / (2.0 * PI);
                    double xo = sc.x_atom + dot3(sc.u, ko);
                    peel(m, &L, o, c, line_dv(m, j, xo, f.vth, dot3(f.v, ko)), cube, st);
                }
                dv = line_dv(m, j, sc.x_out, f.vth, dot3(f.v, kout));
                ++n_res;
                st->n_res++;
            }
            for (int i = 0; i < 3; ++i) k[i] = kout[i];
            draw2(seed, req, SLOT_TAU, event, id, &ua, &ub);
            tau_target = -log(1.0 - ua);
            tau_acc = 0.0;
            continue;
        }
        if (isinf(t)) { /* a ray that never leaves an empty infinite slab */
            fate = OR_FATE_ESCAPED;
            break;
        }
        if (!hubble_on(m))
            tau_acc += kt * t;
        if (advance(m, &L, k, t, nr, cm))
            fate = OR_FATE_ESCAPED;
    }
    if (fate == OR_FATE_ESCAPED || fate == OR_FATE_REDSHIFTED) {
        st->escaped++;
        st->w_escaped += w;
        if (fate == OR_FATE_REDSHIFTED)
            st->redshifted++;
        else if (g->kind == OR_GRID && g->boundary_handoff)
            st->handed_off++;
        double sv = dv;
        if (op->spec_T_ref > 0.0) {
            double vth, a, s0;
            or_line_params(op->spec_T_ref, &vth, &a, &s0);
            sv = dv / vth;
        }
        int b = bin_of(sv, op->spec_lo, op->spec_hi, op->spec_nb);
        if (b >= 0 && spectrum)
            spectrum[b] += w;
    } else if (fate == OR_FATE_CAPPED) {
        st->capped++;
    }
    if (rec) {
        rec->dv = dv;
        rec->n_res = n_res;
        rec->n_dust = n_dust;
        rec->fate = fate;
        rec->pad = 0;
    }
}

/* Medium constants of a run: meshless line quantities, grid spacing, the    */
/* n_HI^2 emission CDF (inclusive prefix, x-fastest order) and x_crit.        */
static int model_init(model_t *m, const or_geometry *g, const or_source *s, const or_opts *o)
{
    memset(m, 0, sizeof *m);
    m->g = g;
    m->o = o;
    m->nl = 1;
    m->lrho[0] = 1.0; m->lam[0] = 1.0; m->lk[0] = 1.0; m->lw[0] = 1.0;
    if (g->line == OR_LINE_MG2) {
        /* line 0 = k (reference), line 1 = h, redward by c (1 - lambda_k/lambda_h) */
        m->nl = 2;
        m->lc[1] = C_LIGHT * (MG2K_LAMBDA / MG2H_LAMBDA - 1.0);
        m->lrho[1] = MG2H_LAMBDA / MG2K_LAMBDA;
        m->lam[1] = (MG2H_A21 * MG2H_LAMBDA) / (MG2K_A21 * MG2K_LAMBDA);
        m->lk[1] = (MG2H_F12 * MG2H_LAMBDA) / (MG2K_F12 * MG2K_LAMBDA);
        m->lw[0] = MG2K_F12 / (MG2K_F12 + MG2H_F12);
        m->lw[1] = 1.0 - m->lw[0];
    } else if (g->line != OR_LINE_LYA && g->line != OR_LINE_MG2K) {
        return -1;
    }
    if (g->kind == OR_GRID) {
        m->dims[0] = g->nx; m->dims[1] = g->ny; m->dims[2] = g->nz;
        for (int ax = 0; ax < 3; ++ax)
            m->dx[ax] = (g->hi[ax] - g->lo[ax]) / (double)m->dims[ax];
        if (s->kind == OR_SRC_CELL_N2) {
            size_t nc = (size_t)g->nx * g->ny * g->nz;
            m->cdf = (double *)malloc(nc * sizeof(double));
            if (!m->cdf)
                return -2;
            double acc = 0.0;
            for (size_t i = 0; i < nc; ++i) {
                double nn = (double)g->f_n[i];
                acc += nn * nn;
                m->cdf[i] = acc;
            }
            m->cdf_total = acc;
        }
        if (o && o->core_skip == OR_CS_FIXED)
            m->xcrit = o->x_crit;
        else if (o && o->core_skip == OR_CS_ADAPTIVE)
            return -6;
    } else {
        double L = g->r_outer - g->r_inner;
        or_species_params(g->line, g->T, &m->vth, &m->a, &m->sig0);
        m->n = g->tau0 > 0.0 ? g->tau0 / (m->sig0 * L) : g->n_HI;
        m->k0 = m->n * m->sig0;
        m->sigd = g->tau_d > 0.0 ? g->tau_d / (m->n * L) : g->sigma_d;
        m->kd = m->sigd * m->n;
        if (o && o->core_skip == OR_CS_FIXED) {
            m->xcrit = o->x_crit;
        } else if (o && o->core_skip == OR_CS_ADAPTIVE) {
            /* Section 3.4.2: x_crit = 0.2 (a tau0)^(1/3) for a tau0 >= 1 */
            double atau = m->a * m->k0 * L;
            m->xcrit = atau >= 1.0 ? 0.2 * cbrt(atau) : 0.0;
        }
    }
    return 0;
}

struct or_prepared {
    or_geometry g;
    or_source s;
    or_opts o;
    model_t m;
};

or_prepared *or_prepare(const or_geometry *g, const or_source *s, const or_opts *o)
{
    or_prepared *p = (or_prepared *)calloc(1, sizeof *p);
    if (!p)
        return NULL;
    p->g = *g;
    p->s = *s;
    p->o = *o;
    if (model_init(&p->m, &p->g, &p->s, &p->o) != 0) {
        free(p->m.cdf);
        free(p);
        return NULL;
    }
    return p;
}

int or_transport_prepared(const or_prepared *p, uint64_t first_id, uint64_t n, double *spectrum,
                          double *cube, or_stats *st, or_record *records)
{
    if (!p)
        return -1;
    for (uint64_t i = 0; i < n; ++i)
        transport_one(&p->m, &p->s, first_id + i, spectrum, cube, st, records ? &records[i] : NULL);
    return 0;
}

void or_release(or_prepared *p)
{
    if (!p)
        return;
    free(p->m.cdf);
    free(p);
}

int or_transport(const or_geometry *g, const or_source *s, const or_opts *o, uint64_t first_id,
                 uint64_t n, double *spectrum, double *cube, or_stats *st, or_record *records)
{
    model_t m;
    int rc = model_init(&m, g, s, o);
    if (rc != 0) {
        free(m.cdf);
        return rc;
    }
    for (uint64_t i = 0; i < n; ++i)
        transport_one(&m, s, first_id + i, spectrum, cube, st, records ? &records[i] : NULL);
    free(m.cdf);
    return 0;
}

/* Emission only (test access to the generator): rows of 11 doubles per       */
/* packet: position (3), direction (3), lab dv, gas-frame dv_loc, cell (3).   */
int or_emit(const or_geometry *g, const or_source *s, uint64_t first_id, uint64_t n, double *out)
{
    model_t m;
    int rc = model_init(&m, g, s, NULL);
    if (rc != 0) {
        free(m.cdf);
        return rc;
    }
    for (uint64_t i = 0; i < n; ++i) {
        emitted_t e;
        emit_packet(&m, s, first_id + i, &e);
        double *r = out + 11 * i;
        for (int j = 0; j < 3; ++j) {
            r[j] = e.L.p[j];
            r[3 + j] = e.k[j];
            r[8 + j] = (double)e.L.cell[j];
        }
        r[6] = e.dv;
        r[7] = e.dv_loc;
    }
    free(m.cdf);
    return 0;
}

/* n resonant scatterings at fixed (x, a, k_in), photon ids 0..n-1, event    */
/* `event`, key (seed, 0): rows of 10 doubles: u_par, u_perp (2), x_atom,     */
/* x_out, k_out (3), trials, phase used.                                      */
int or_scatter_resonant(double x, double a, const double k[3], double x_crit, int phase,
                        uint32_t seed, uint32_t event, uint64_t n, double *out)
{
    if (!(a > 0.0) || phase < 0 || phase > 2)
        return -1;
    for (uint64_t i = 0; i < n; ++i) {
        scatter_t sc;
        resonant_scatter(x, a, k, x_crit, phase, seed, 0u, event, i, &sc);
        double *r = out + 10 * i;
        r[0] = sc.upar;
        r[1] = sc.uperp[0];
        r[2] = sc.uperp[1];
        r[3] = sc.x_atom;
        r[4] = sc.x_out;
        r[5] = sc.kout[0]; r[6] = sc.kout[1]; r[7] = sc.kout[2];
        r[8] = (double)sc.trials;
        r[9] = (double)sc.phase;
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Raytracing driver (Section 3.5).  Rays run parallel to one grid axis    */
/* through cell centres, from the low face (s = 0) to the high face; the    */
/* fields are constant within a cell (the zeroth-order assumption of        */
/* Section 3.4).  A ray is named by its cell indices (i, j) along the two   */
/* other axes, i along the lower-numbered one: axis z -> (x, y),            */
/* axis y -> (x, z), axis x -> (y, z).                                      */
/* ---------------------------------------------------------------------- */
static size_t ray_cell(int axis, int nx, int ny, int i, int j, int k)
{
    int c[3];
    if (axis == 0) { c[0] = k; c[1] = i; c[2] = j; }
    else if (axis == 1) { c[0] = i; c[1] = k; c[2] = j; }
    else { c[0] = i; c[1] = j; c[2] = k; }
    return ((size_t)c[2] * (size_t)ny + (size_t)c[1]) * (size_t)nx + (size_t)c[0];
}

static void ray_dims(int axis, int nx, int ny, int nz, int *ni, int *nj, int *nk)
{
    int n[3] = {nx, ny, nz};
    *nk = n[axis];
    *ni = axis == 0 ? ny : nx;
    *nj = axis == 2 ? ny : nz;
}

/* Section 3.5.1: the projection Q = int q w ds and its normalisation       */
/* Q_hat = int w ds along every ray of the axis (w = 1 when w is NULL).      */
/* Images are [j][i].  Returns 0, or -1 for invalid arguments.              */
int or_project(const float *q, const float *w, int nx, int ny, int nz, int axis, double ds,
               double *Q, double *W)
{
    if (axis < 0 || axis > 2 || nx <= 0 || ny <= 0 || nz <= 0 || !(ds > 0.0))
        return -1;
    int ni, nj, nk;
    ray_dims(axis, nx, ny, nz, &ni, &nj, &nk);
    for (int j = 0; j < nj; ++j)
        for (int i = 0; i < ni; ++i) {
            double acc_q = 0.0, acc_w = 0.0;
            for (int k = 0; k < nk; ++k) {
                size_t c = ray_cell(axis, nx, ny, i, j, k);
                double wk = w ? (double)w[c] : 1.0;
                acc_q += (double)q[c] * wk * ds;
                acc_w += wk * ds;
            }
            Q[(size_t)j * ni + i] = acc_q;
            if (W)
                W[(size_t)j * ni + i] = acc_w;
        }
    return 0;
}

/* Section 3.5.2, eq. (abs): tau(nu) = int n_HI(s) sigma(nu(s), T(s)) ds     */
/* with nu(s) = nu_i [1 - (v(s) + H s)/c].  The spectrum is sampled at the  */
/* centres u_b of nb bins over [u_lo, u_hi), where u = c (nu_i/nu0 - 1) is  */
/* the photon's velocity offset at s = 0.  To first order in v/c, the gas   */
/* at s sees x = (u - v(s) - H s) / v_th(T(s)), so a cell adds               */
/* n_HI sigma0(T) H(a(T), x) ds to every bin.  Each cell is split into      */
/* n_sub equal steps evaluated at their midpoints (the sub-cell stepping    */
/* that keeps the Hubble shift per step below the line width).  vlos is     */
/* the velocity component along +axis (cm/s); hubble is H(z) in 1/s.        */
/* los holds (i, j) per ray; tau is [n_los][nb].                            */
int or_forest(const float *nHI, const float *T, const float *vlos, int nx, int ny, int nz,
              int axis, double ds, double hubble, int n_sub, const int32_t *los,
              uint32_t n_los, uint32_t nb, double u_lo, double u_hi, double *tau)
{
    if (axis < 0 || axis > 2 || nx <= 0 || ny <= 0 || nz <= 0 || !(ds > 0.0) || n_sub < 1 ||
        nb < 1 || !(u_hi > u_lo))
        return -1;
    int ni, nj, nk;
    ray_dims(axis, nx, ny, nz, &ni, &nj, &nk);
    double du = (u_hi - u_lo) / (double)nb;
    for (uint32_t l = 0; l < n_los; ++l) {
        int i = los[2 * l], j = los[2 * l + 1];
        if (i < 0 || i >= ni || j < 0 || j >= nj)
            return -1;
        double *row = tau + (size_t)l * nb;
        for (uint32_t b = 0; b < nb; ++b)
            row[b] = 0.0;
        for (int k = 0; k < nk; ++k) {
            size_t c = ray_cell(axis, nx, ny, i, j, k);
            double n = (double)nHI[c];
            if (n == 0.0)
                continue;   /* adds exactly zero */
            double vth, a, sigma0;
            or_line_params((double)T[c], &vth, &a, &sigma0);
            double step = ds / (double)n_sub;
            for (int m = 0; m < n_sub; ++m) {
                double s = ((double)k + ((double)m + 0.5) / (double)n_sub) * ds;
                for (uint32_t b = 0; b < nb; ++b) {
                    double u = u_lo + ((double)b + 0.5) * du;
                    double x = (u - (double)vlos[c] - hubble * s) / vth;
                    row[b] += n * sigma0 * or_voigt(a, x) * step;
                }
            }
        }
    }
    return 0;
}
