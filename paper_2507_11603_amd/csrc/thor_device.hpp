// thor_device.hpp -- device code of the MI355X resonant-line Monte Carlo
// transport (arXiv 2507.11603, Sections 2.2-2.3 physics, 3.4 MCRT driver).
//
// Everything here runs on CDNA4 VALU: there is no dense contraction in the
// method, so no MFMA.  The per-packet engine is shared by the plain kernel
// (one thread per packet) and the persistent refilling kernel.
//
// Precision policy R: double for the FP64 path; float for the mixed path,
// where the Voigt evaluation, the direction vector and the frequency
// redistribution run in FP32 while position, cell-boundary distances and
// optical depths stay FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace thor {

// ---------------------------------------------------------------------------
// Physical constants (cgs) and Lyman-alpha atomic data.  The paper prints
// none of them; these are CODATA and the standard Lya values.
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrtPi = 1.77245385090551602730;
constexpr double kClight = 2.99792458e10;
constexpr double kBoltzmann = 1.380649e-16;
constexpr double kMassH = 1.6735575e-24;
constexpr double kMassE = 9.1093837015e-28;
constexpr double kCharge = 4.80320471e-10;
constexpr double kLambda0 = 1215.67e-8;
constexpr double kA21 = 6.265e8;
constexpr double kF12 = 0.4162;
// Section 2.3.1: v_th = sqrt(2kT/m); Doppler width dnu_D = v_th / lambda0,
// a = A21 / (4 pi dnu_D), sigma0 = f12 sqrt(pi) e^2 / (m_e c dnu_D).
// Mg II h and k (a fine-structure doublet from one ground level): k = 3s
// 2S1/2 - 3p 2P3/2 at 2796.352 A, h = 3s 2S1/2 - 3p 2P1/2 at 2803.531 A,
// Einstein A and oscillator strengths of Morton (2003); Mg mass 24.305 u.
constexpr double kMassMg = 24.305 * 1.66053906660e-24;
constexpr double kMgKLambda = 2796.352e-8, kMgKA21 = 2.60e8, kMgKF12 = 0.6155;
constexpr double kMgHLambda = 2803.531e-8, kMgHA21 = 2.57e8, kMgHF12 = 0.3058;
constexpr double kVth2PerT = 2.0 * kBoltzmann / kMassH;
constexpr double kDampTimesVth = kA21 * kLambda0 / (4.0 * kPi);
constexpr double kSigma0TimesVth = kF12 * kSqrtPi * kCharge * kCharge * kLambda0 / (kMassE * kClight);

// ---------------------------------------------------------------------------
// Dawson's integral table (filled at context creation): 52 intervals of
// width 1/8 on [0, 6.5], Taylor coefficients in s = (x - centre) * 16.
// ---------------------------------------------------------------------------
constexpr int kDawsonIntervals = 52;
constexpr int kDawsonDeg64 = 12;
constexpr int kDawsonDeg32 = 6;
extern __constant__ double c_dawson64[kDawsonIntervals * (kDawsonDeg64 + 1)];
extern __constant__ float c_dawson32[kDawsonIntervals * (kDawsonDeg32 + 1)];

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11), the counter-based stream replacing
// the paper's per-work-item generator (Section 3.4.3): key = (seed, request),
// counter = (slot, event, id_lo, id_hi).
// ---------------------------------------------------------------------------
struct Words { uint32_t w0, w1, w2, w3; };

__device__ __forceinline__ Words philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32 -> 64-bit product gives both halves (v_mad_u64_u32)
        const uint64_t p0 = uint64_t(c0) * 0xD2511F53u;
        const uint64_t p1 = uint64_t(c2) * 0xCD9E8D57u;
        const uint32_t n0 = uint32_t(p1 >> 32) ^ c1 ^ k0, n2 = uint32_t(p0 >> 32) ^ c3 ^ k1;
        c0 = n0; c1 = uint32_t(p1); c2 = n2; c3 = uint32_t(p0);
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    return Words{c0, c1, c2, c3};
}

struct Key {
    uint32_t seed, req, id_lo, id_hi;
};

template <class R> struct Uni2 { R a, b; };

// Two uniforms in [0,1): 53 random bits each in FP64 ((w0:w1) >> 11, (w2:w3) >> 11);
// the top 24 bits of the same words in FP32.
template <class R> __device__ __forceinline__ Uni2<R> draw(const Key& k, uint32_t slot, uint32_t event);
template <> __device__ __forceinline__ Uni2<double> draw<double>(const Key& k, uint32_t slot, uint32_t event) {
    const Words w = philox10(slot, event, k.id_lo, k.id_hi, k.seed, k.req);
    const uint64_t hi = (uint64_t(w.w0) << 32) | w.w1;
    const uint64_t lo = (uint64_t(w.w2) << 32) | w.w3;
    return Uni2<double>{double(hi >> 11) * 0x1p-53, double(lo >> 11) * 0x1p-53};
}
template <> __device__ __forceinline__ Uni2<float> draw<float>(const Key& k, uint32_t slot, uint32_t event) {
    const Words w = philox10(slot, event, k.id_lo, k.id_hi, k.seed, k.req);
    return Uni2<float>{float(w.w0 >> 8) * 0x1p-24f, float(w.w2 >> 8) * 0x1p-24f};
}

// Slot map: event 0 = emission, event e >= 1 = e-th interaction.
enum : uint32_t { kSlotEDir = 0, kSlotEGauss = 1, kSlotECell = 2, kSlotEOffs = 3, kSlotETau = 4, kSlotELine = 5 };
enum : uint32_t { kSlotType = 0, kSlotUperp = 1, kSlotMu = 2, kSlotTau = 3, kSlotUpar = 4 };

// Division: IEEE in FP64; reciprocal-based (about 1 ulp) in the FP32 path.
__device__ __forceinline__ double fdiv(double a, double b) { return a / b; }

// FP64 reciprocal from the hardware estimate and two Newton steps (within
// 1 ulp): the mixed path's inverse directions and interaction distances.
__device__ __forceinline__ double rcp64(double b) {
    double r = __builtin_amdgcn_rcp(b);
    r = fma(r, fma(-b, r, 1.0), r);
    return fma(r, fma(-b, r, 1.0), r);
}
// a / b in the FP64 quantities of the mixed path: a * (1/b) with one
// residual correction; IEEE division in the FP64 path.
template <class R> __device__ __forceinline__ double div_tau(double a, double b) {
    if constexpr (sizeof(R) == 8) {
        return a / b;
    } else {
        const double q = a * rcp64(b);
        return fma(rcp64(b), fma(-b, q, a), q);
    }
}
__device__ __forceinline__ float fdiv(float a, float b) { return __fdividef(a, b); }

// ---------------------------------------------------------------------------
// math shims per precision
// ---------------------------------------------------------------------------
template <class R> struct M;
template <> struct M<double> {
    static __device__ __forceinline__ double exp(double v) { return ::exp(v); }
    static __device__ __forceinline__ double expm1(double v) { return ::expm1(v); }
    static __device__ __forceinline__ double log(double v) { return ::log(v); }
    static __device__ __forceinline__ double log1p(double v) { return ::log1p(v); }
    static __device__ __forceinline__ double sqrt(double v) { return ::sqrt(v); }
    static __device__ __forceinline__ double cbrt(double v) { return ::cbrt(v); }
    static __device__ __forceinline__ double atan(double v) { return ::atan(v); }
    static __device__ __forceinline__ double tan(double v) { return ::tan(v); }
    static __device__ __forceinline__ void sincos(double v, double* s, double* c) { ::sincos(v, s, c); }
    static __device__ __forceinline__ double sinpi2(double u, double* c) {  // sin/cos(2 pi u)
        double s; ::sincos(2.0 * kPi * u, &s, c); return s;
    }
};
template <> struct M<float> {
    static __device__ __forceinline__ float exp(float v) { return __expf(v); }
    static __device__ __forceinline__ float expm1(float v) { return ::expm1f(v); }
    static __device__ __forceinline__ float log(float v) { return __logf(v); }
    static __device__ __forceinline__ float log1p(float v) { return ::log1pf(v); }
    static __device__ __forceinline__ float sqrt(float v) { return ::sqrtf(v); }
    static __device__ __forceinline__ float cbrt(float v) { return ::cbrtf(v); }
    static __device__ __forceinline__ float atan(float v) { return ::atanf(v); }
    static __device__ __forceinline__ float tan(float v) { return ::tanf(v); }
    static __device__ __forceinline__ void sincos(float v, float* s, float* c) { ::sincosf(v, s, c); }
    static __device__ __forceinline__ float sinpi2(float u, float* c) {
        float s; ::sincospif(2.0f * u, &s, c); return s;
    }
};

// ---------------------------------------------------------------------------
// Voigt-Hjerting function H(a, x) = Re w(x + i a), the profile of
// sigma(x) = sigma0 H(a, x) evaluated at every march step (Section 3.4,
// Appendix A.3).  |x| <= 6.5: Taylor series of w in i a about the real point
// x, from w(x) = exp(-x^2) + (2i/sqrt(pi)) F(x) and the derivative recurrence
// w^(n+1) = -2x w^(n) - 2n w^(n-1) (w' = -2x w + 2i/sqrt(pi)); the number of
// terms depends on a.  |x| > 6.5: Laplace continued fraction of w - exp(-z^2)
// with the Gaussian term added back.  FP64: <= 1e-13 relative for
// a <= 0.05; FP32: <= 2e-5.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double dawson64(double ax) {
    int i = int(ax * 8.0);
    i = i < kDawsonIntervals - 1 ? i : kDawsonIntervals - 1;
    const double s = (ax - (double(i) + 0.5) * 0.125) * 16.0;
    const double* c = c_dawson64 + i * (kDawsonDeg64 + 1);
    // Estrin evaluation of the degree-12 polynomial
    const double s2 = s * s, s4 = s2 * s2, s8 = s4 * s4;
    const double p01 = fma(c[1], s, c[0]), p23 = fma(c[3], s, c[2]);
    const double p45 = fma(c[5], s, c[4]), p67 = fma(c[7], s, c[6]);
    const double p89 = fma(c[9], s, c[8]), pab = fma(c[11], s, c[10]);
    const double q0 = fma(p23, s2, p01), q1 = fma(p67, s2, p45), q2 = fma(pab, s2, p89);
    const double r0 = fma(q1, s4, q0), r1 = fma(c[12], s4, q2);
    return fma(r1, s8, r0);
}

// `tab`: the FP32 coefficient table (c_dawson32, or a copy of it in LDS)
__device__ __forceinline__ float dawson32(float ax, const float* tab) {
    int i = int(ax * 8.0f);
    i = i < kDawsonIntervals - 1 ? i : kDawsonIntervals - 1;
    const float s = (ax - (float(i) + 0.5f) * 0.125f) * 16.0f;
    const float* c = tab + i * (kDawsonDeg32 + 1);
    const float s2 = s * s, s4 = s2 * s2;
    const float p01 = fmaf(c[1], s, c[0]), p23 = fmaf(c[3], s, c[2]), p45 = fmaf(c[5], s, c[4]);
    return fmaf(fmaf(c[6], s2, p45), s4, fmaf(p23, s2, p01));
}

__device__ __forceinline__ double voigt64(double a, double x) {
    const double ax = fabs(x);
    constexpr double two_rsqpi = 2.0 / kSqrtPi;
    if (ax <= 6.5) {
        const int nterms = a <= 1.2e-3 ? 4 : (a <= 1.2e-2 ? 6 : (a <= 2.5e-2 ? 8 : 12));
        const double e = exp(-ax * ax);
        double wr_p = e, wi_p = two_rsqpi * dawson64(ax);          // w(x)
        double wr = -2.0 * ax * wr_p, wi = fma(-2.0 * ax, wi_p, two_rsqpi);  // w'(x)
        double sum = wr_p;
        double pr = 1.0, pi = 0.0, inv_fact = 1.0;                  // (i a)^n, 1/n!
        for (int n = 1; n <= nterms; ++n) {
            const double npr = -pi * a, npi = pr * a;
            pr = npr; pi = npi;
            inv_fact /= double(n);
            sum = fma(pr * wr - pi * wi, inv_fact, sum);
            const double nr = fma(-2.0 * ax, wr, -2.0 * double(n) * wr_p);
            const double ni = fma(-2.0 * ax, wi, -2.0 * double(n) * wi_p);
            wr_p = wr; wi_p = wi; wr = nr; wi = ni;
        }
        return sum;
    }
    // continued fraction t = z - (1/2)/(z - 1/(z - (3/2)/(...))), 14 levels
    double tr = ax, ti = a;
#pragma unroll
    for (int k = 14; k >= 1; --k) {
        const double inv = 1.0 / (tr * tr + ti * ti);
        const double h = 0.5 * double(k);
        tr = ax - h * tr * inv;
        ti = a + h * ti * inv;
    }
    // Re[(i/sqrt(pi)) / t] = (ti / |t|^2) / sqrt(pi)
    double h = ti / ((tr * tr + ti * ti) * kSqrtPi);
    if (ax < 9.0) h += exp(-ax * ax);
    return h;
}

// Far from the line centre H(a, x) follows the asymptotic series of
// w(z) = (i/pi) int exp(-t^2) / (z - t) dt at z = x + i a:
//   w(z) ~ (i / sqrt(pi)) sum_n (2n - 1)!! / 2^n  z^-(2n+1),
// so H = Re w = -Im(S) / sqrt(pi) with S that sum (the Gaussian part,
// exp(-x^2), is below 1e-18 of H there).  Dropping the terms after n = N
// changes H by about (2N + 3) c_(N+1) / x^(2N+2) relative.  FP64: N = 4 from
// |x| = 40 (3e-14), N = 6 from |x| = 20 (1e-14) and N = 9 from |x| = 12
// (4e-15); nearer the line the FP64 Voigt function.  1 / |z|^2 comes from the
// hardware reciprocal refined by two Newton steps (FP64) or alone (FP32).
// FP32 (the forest kernel): N = 4 beyond |x| = 6.5 (3e-6).
template <class R, int N>
__device__ __forceinline__ R voigt_wing(R a, R x) {
    // c_n = (2n - 1)!! / 2^n
    constexpr R c[10] = {R(1.0), R(0.5), R(0.75), R(1.875), R(6.5625), R(29.53125), R(162.421875),
                         R(1055.7421875), R(7918.06640625), R(67303.564453125)};
    static_assert(N >= 1 && N <= 9, "series length");
    R r;
    if constexpr (sizeof(R) == 8) r = rcp64(x * x + a * a);
    else r = __builtin_amdgcn_rcpf(x * x + a * a);
    const R zr = x * r, zi = -a * r;                        // zeta = 1 / z
    const R qr = zr * zr - zi * zi, qi = R(2) * zr * zi;    // zeta^2
    R pr = c[N], pi = R(0);
#pragma unroll
    for (int k = N - 1; k >= 0; --k) {
        const R nr = pr * qr - pi * qi + c[k];
        pi = pr * qi + pi * qr;
        pr = nr;
    }
    return -(zr * pi + zi * pr) * R(1.0 / kSqrtPi);         // -Im(zeta P) / sqrt(pi)
}

// FP32 H(a, x) in one form for every x, so that the lanes of a wave near the
// line and in the wing run the same instructions except for g below.
// Expanding w(x + i a) = w(x) + i a w'(x) - a^2 w''(x)/2 + ... with
// w(x) = exp(-x^2) + (2i/sqrt(pi)) F(x) (F Dawson's integral) gives
//   H = exp(-x^2) (1 - a^2 (2x^2 - 1)) - (2a/sqrt(pi)) g(x) + O(a^3),
//   g(x) = 1 - 2x F(x).
// |x| <= 6.5: F from the Dawson table; the a^3, a^4 terms are added when
// a > 3e-3.  |x| > 6.5: g from its asymptotic series
//   g = -(r/2)(1 + 3r/2 + 15r^2/4 + 105r^3/8 + 945r^4/16), r = 1/x^2
// (truncation below 3e-6 relative), with the next order in a folded in as
// x^2/(x^2 + a^2) (the first term of the series of w at x + i a is
// a/(sqrt(pi)(x^2 + a^2)); the rest of the a^2 terms are below 1e-6
// relative there).  Relative error below 2e-5 for a <= 0.05.
__device__ __forceinline__ float voigt32(float a, float x, const float* tab = c_dawson32) {
    const float ax = fabsf(x);
    constexpr float two_rsqpi = float(2.0 / kSqrtPi);
    const float x2 = ax * ax;
    const float e = __expf(-x2);
    const bool core = ax <= 6.5f;
    float g, c = 1.0f, wi_p = 0.0f;    // g here: (2/sqrt(pi)) g(x)
    if (core) {
        wi_p = two_rsqpi * dawson32(ax, tab);
        g = fmaf(-2.0f * ax, wi_p, two_rsqpi);
    } else {
        const float r = __builtin_amdgcn_rcpf(x2);
        g = (-0.5f * two_rsqpi) * r * fmaf(r, fmaf(r, fmaf(r, fmaf(r, 59.0625f, 13.125f), 3.75f), 1.5f), 1.0f);
        c = x2 * __builtin_amdgcn_rcpf(fmaf(a, a, x2));
    }
    float sum = fmaf(-a * c, g, e * fmaf(-a * a, fmaf(2.0f, x2, -1.0f), 1.0f));
    if (a > 3e-3f && core) {
        // n = 3: a^3 Im(w''')/6, n = 4: a^4 Re(w'''')/24, from w' = -2x w + 2i/sqrt(pi)
        const float wr = -2.0f * ax * e, wi = g;
        const float nr = fmaf(-2.0f * ax, wr, -2.0f * e), ni = fmaf(-2.0f * ax, wi, -2.0f * wi_p);
        const float r3 = fmaf(-2.0f * ax, nr, -4.0f * wr), i3 = fmaf(-2.0f * ax, ni, -4.0f * wi);
        const float r4 = fmaf(-2.0f * ax, r3, -6.0f * nr);
        const float a2 = a * a;
        sum = fmaf(a2 * a * (1.0f / 6.0f), i3, sum);
        sum = fmaf(a2 * a2 * (1.0f / 24.0f), r4, sum);
    }
    return sum;
}

// A lower bound of H(a, x) that decides sure peel cuts without the profile.
// H is the mean of exp(-(x - l)^2) over a Lorentzian l of half width a, so
// for delta = 1/4, H >= P(|l| <= delta) exp(-(|x| + delta)^2) and
// P(|l| <= delta) = (2/pi) atan(delta/a) >= 1 - 2a/(pi delta).  The factor
// 0.99 keeps the bound below both evaluations of H (FP64 within 1e-13, FP32
// within 2e-5 relative for a <= 0.05); above that a, 0.
__device__ __forceinline__ float voigt_floor(float a, float x) {
    if (!(a <= 0.05f)) return 0.0f;
    const float ax = fabsf(x) + 0.25f;
    return 0.99f * (1.0f - 2.5464790894703255f * a) * __expf(-ax * ax);
}

template <class R> __device__ __forceinline__ R voigt(R a, R x);
template <> __device__ __forceinline__ double voigt<double>(double a, double x) { return voigt64(a, x); }
template <> __device__ __forceinline__ float voigt<float>(float a, float x) { return voigt32(a, x); }

// ---------------------------------------------------------------------------
// Core-to-wing transition x_cw(a) of H(a, x) (Appendix A.2: where exp(-x^2)
// meets a/(sqrt(pi) x^2)), by the quartic in ln a printed there.  FP32 takes
// ln a without the library logarithm: the exponent field gives e ln 2, the
// mantissa m (folded into [sqrt(1/2), sqrt(2))) gives ln m = 2 atanh(s),
// s = (m - 1)/(m + 1), |s| <= 0.172, by four terms of the atanh series
// (truncation below 3e-8).  Positive normal a only.
__device__ __forceinline__ float log_bits(float v) {
    uint32_t b = __float_as_uint(v);
    int e = int((b >> 23) & 0xFFu) - 127;
    float m = __uint_as_float((b & 0x7FFFFFu) | 0x3F800000u);
    if (m > 1.41421356f) { m *= 0.5f; e += 1; }
    const float s = (m - 1.0f) * __builtin_amdgcn_rcpf(m + 1.0f);
    const float s2 = s * s;
    const float lm = 2.0f * s * (1.0f + s2 * (1.0f / 3.0f + s2 * (0.2f + s2 * (1.0f / 7.0f))));
    return float(e) * 0.69314718f + lm;
}
template <class R>
__device__ __forceinline__ R xcw_b25(R a) {
    R L;
    if constexpr (sizeof(R) == 8) L = log(a);
    else L = log_bits(a);
    return R(1.03489162) + L * (R(-6.17680644e-1) + L * (R(-8.73073343e-2) + L * (R(-7.91384757e-3) +
                                                                                  L * R(-2.76037084e-4))));
}

// ---------------------------------------------------------------------------
// u_parallel sampler, eq. (uparallel): f(u) ~ exp(-u^2) / ((x-u)^2 + a^2).
// Exact rejection sampling for any split u0 >= 0.
//   |x| < 2.25: the paper's comparison function (eq. uparallel_comparisonfunc):
//     1/((x-u)^2+a^2) below u0, exp(-u0^2)/((x-u)^2+a^2) above;
//     u0 from two steps of u0 <- x - sqrt(a expm1(u0^2) / (2 pi u0)), u0 = x first.
//   |x| >= 2.25: the same Lorentzian envelope above u0 and, below u0, the
//     Gaussian envelope exp(-u^2) x^-2 exp(2u/x + c u^2/x^2) with
//     c = (-2 ln(1 - t0) - 2 t0)/t0^2, t0 = u0/x;
//     u0 = min(sqrt(ln(sqrt(pi) x^2 / a) + 3), x - 0.3/x).
// Trial j draws slot 4+2j (choice, accept) and, for a Gaussian proposal,
// slot 5+2j (radius, angle).  The FP64 version evaluates the same formulas
// in the same order as the CPU reference so that same-seed runs follow the
// same decisions; the FP32 version uses cancellation-free equivalents.
// ---------------------------------------------------------------------------
constexpr double kUparSwitch = 2.25;
// Hard bound on proposals (never reached for finite x, a > 0: the expected
// count is below 10); keeps a non-finite input from spinning a lane forever.
constexpr uint32_t kUparMaxTrials = 1u << 20;
// The first kPreUpar u_par slots (kSlotUpar ...) may be drawn ahead of the
// event (the draws depend only on the key, the slot and the event number).
constexpr uint32_t kPreUpar = 4;

template <class R>
__device__ __forceinline__ Uni2<R> upar_draw(const Key& key, uint32_t slot, uint32_t event, const Uni2<R>* pre) {
    const uint32_t j = slot - kSlotUpar;
    if (pre && j < kPreUpar) return pre[j];
    return draw<R>(key, slot, event);
}

__device__ __forceinline__ double upar_sample64(double x, double a, const Key& key, uint32_t event,
                                                uint32_t* trials, const Uni2<double>* pre) {
    const double xa = fabs(x);
    const double sgn = x < 0.0 ? -1.0 : 1.0;
    uint32_t n = 0;
    double u = 0.0;
    if (!(xa < 1e300) || !(a > 0.0)) { *trials = 0; return 0.0; }
    if (xa < kUparSwitch) {
        double u0 = xa;
        for (int it = 0; it < 2; ++it) {
            if (u0 <= 0.0) break;
            u0 = xa - sqrt(a * expm1(u0 * u0) / (2.0 * kPi * u0));
            u0 = u0 < 0.0 ? 0.0 : (u0 > xa ? xa : u0);
        }
        const double th0 = atan((u0 - xa) / a);
        const double p1 = th0 + kPi / 2;
        const double e0 = exp(-u0 * u0);
        const double m = p1 + e0 * (kPi / 2 - th0);
        for (;;) {
            if (n >= kUparMaxTrials) break;
            const Uni2<double> r12 = upar_draw<double>(key, kSlotUpar + 2u * n, event, pre);
            ++n;
            const double r = r12.a * m;
            if (r < p1) {
                u = xa + a * tan(r - kPi / 2);
                if (r12.b < exp(-u * u)) break;
            } else {
                u = xa + a * tan(th0 + (r - p1) / e0);
                if (r12.b < exp(u0 * u0 - u * u)) break;
            }
        }
    } else {
        double u0 = sqrt(log(kSqrtPi * xa * xa / a) + 3.0);
        const double cap = xa - 0.3 / xa;
        u0 = u0 < cap ? u0 : cap;
        const double t0 = u0 / xa;
        const double c = (-2.0 * log1p(-t0) - 2.0 * t0) / (t0 * t0);
        const double p = 1.0 - c / (xa * xa), mu = 1.0 / (xa * p);
        const double za = exp(p * mu * mu) * sqrt(kPi / p) / (xa * xa);
        const double th0 = atan((u0 - xa) / a);
        const double e0 = exp(-u0 * u0);
        const double zb = e0 * (kPi / 2 - th0) / a;
        for (;;) {
            if (n >= kUparMaxTrials) break;
            const Uni2<double> r12 = upar_draw<double>(key, kSlotUpar + 2u * n, event, pre);
            const double r = r12.a * (za + zb);
            if (r < za) {
                const Uni2<double> r34 = upar_draw<double>(key, kSlotUpar + 2u * n + 1u, event, pre);
                ++n;
                double cs, sn;
                sincos(2.0 * kPi * r34.b, &sn, &cs);
                u = mu + sqrt(-log(1.0 - r34.a) / p) * cs;
                if (u > u0) continue;
                const double t = u / xa;
                const double env = exp(2.0 * t + c * t * t) / (xa * xa);
                const double tgt = 1.0 / ((xa - u) * (xa - u) + a * a);
                if (r12.b * env < tgt) break;
            } else {
                ++n;
                u = xa + a * tan(th0 + (r - za) * a / e0);
                if (r12.b < exp(u0 * u0 - u * u)) break;
            }
        }
    }
    *trials = n;
    return sgn * u;
}

// FP32 arctangent of z >= 0: atan z = pi/2 - atan(1/z) above 1, and
// atan w = pi/4 + atan((w - 1)/(w + 1)) above tan(pi/8), leaving |t| <=
// tan(pi/8) for the Taylor series t - t^3/3 + ... - t^15/15 + t^17/17
// (truncation below 3e-9 relative).
__device__ __forceinline__ float atan_nonneg(float z) {
    const bool inv = z > 1.0f;
    const float w = inv ? __builtin_amdgcn_rcpf(z) : z;
    const bool mid = w > 0.41421356f;
    const float t = mid ? __fdividef(w - 1.0f, w + 1.0f) : w;
    const float t2 = t * t;
    float p = 1.0f / 17.0f;
    p = fmaf(p, t2, -1.0f / 15.0f);
    p = fmaf(p, t2, 1.0f / 13.0f);
    p = fmaf(p, t2, -1.0f / 11.0f);
    p = fmaf(p, t2, 1.0f / 9.0f);
    p = fmaf(p, t2, -1.0f / 7.0f);
    p = fmaf(p, t2, 1.0f / 5.0f);
    p = fmaf(p, t2, -1.0f / 3.0f);
    p = fmaf(p, t2, 1.0f);
    float r = t * p;
    if (mid) r += float(kPi / 4);
    return inv ? float(kPi / 2) - r : r;
}

// FP32 cotangent on [0, pi): cot(pi - t) = -cot t, cot t = tan(pi/2 - t)
// above pi/4, and sin, cos of t in [0, pi/4] from their Taylor series to
// t^11, t^12 (truncation below 1e-11).  cot 0 = +inf.
__device__ __forceinline__ float cot_0pi(float th) {
    const bool neg = th > float(kPi / 2);
    float t = neg ? float(kPi) - th : th;
    const bool hi = t > float(kPi / 4);
    t = hi ? float(kPi / 2) - t : t;
    const float t2 = t * t;
    float sp = -1.0f / 39916800.0f;
    sp = fmaf(sp, t2, 1.0f / 362880.0f);
    sp = fmaf(sp, t2, -1.0f / 5040.0f);
    sp = fmaf(sp, t2, 1.0f / 120.0f);
    sp = fmaf(sp, t2, -1.0f / 6.0f);
    sp = fmaf(sp, t2, 1.0f);
    const float sn = t * sp;
    float cp = 1.0f / 479001600.0f;
    cp = fmaf(cp, t2, -1.0f / 3628800.0f);
    cp = fmaf(cp, t2, 1.0f / 40320.0f);
    cp = fmaf(cp, t2, -1.0f / 720.0f);
    cp = fmaf(cp, t2, 1.0f / 24.0f);
    cp = fmaf(cp, t2, -0.5f);
    const float cs = fmaf(cp, t2, 1.0f);
    const float c = hi ? __fdividef(sn, cs) : __fdividef(cs, sn);
    return neg ? -c : c;
}

__device__ __forceinline__ float upar_sample32(float x, float a, const Key& key, uint32_t event,
                                               uint32_t* trials, const Uni2<float>* pre) {
    const float xa = fabsf(x);
    const float sgn = x < 0.0f ? -1.0f : 1.0f;
    constexpr float pi = float(kPi), hpi = float(kPi / 2);
    uint32_t n = 0;
    float u = 0.0f;
    if (!(xa < 1e30f) || !(a > 0.0f)) { *trials = 0; return 0.0f; }
    if (xa < float(kUparSwitch)) {
        // any split in [0, xa] keeps the sampler exact: one step of the
        // iteration, on fast (approximate) exp and sqrt, gives the same
        // expected number of proposals as two (within 0.4 % for xa < 2.25)
        float u0 = xa;
        if (u0 > 0.0f) {
            u0 = xa - __builtin_amdgcn_sqrtf(__fdividef(a * (__expf(u0 * u0) - 1.0f), 2.0f * pi * u0));
            u0 = fminf(fmaxf(u0, 0.0f), xa);
        }
        const float d = xa - u0;                    // >= 0
        const float p1 = d > 0.0f ? atan_nonneg(__fdividef(a, d)) : hpi;   // theta0 + pi/2
        const float q2 = d > 0.0f ? pi - p1 : hpi;                        // pi/2 - theta0
        const float e0 = __expf(-u0 * u0);
        const float m = fmaf(e0, q2, p1);
        for (;;) {
            if (n >= kUparMaxTrials) break;
            const Uni2<float> r12 = upar_draw<float>(key, kSlotUpar + 2u * n, event, pre);
            ++n;
            const float r = r12.a * m;
            if (r < p1) {
                u = xa - a * cot_0pi(r);                // tan(r - pi/2) = -cot(r)
                if (r12.b < __expf(-u * u)) break;
            } else {
                u = xa + a * cot_0pi(q2 - __fdividef(r - p1, e0));  // tan(pi/2 - psi) = cot(psi)
                if (r12.b < __expf((u0 - u) * (u0 + u))) break;
            }
        }
    } else {
        float u0 = sqrtf(__logf(__fdividef(float(kSqrtPi) * xa * xa, a)) + 3.0f);
        u0 = fminf(u0, xa - __fdividef(0.3f, xa));
        const float t0 = __fdividef(u0, xa);
        float c;
        if (t0 < 0.125f) {   // h(t) = sum_{k>=2} 2 t^(k-2) / k
            c = 1.0f + t0 * (2.0f / 3.0f + t0 * (0.5f + t0 * (0.4f + t0 * (1.0f / 3.0f + t0 * (2.0f / 7.0f + t0 * 0.25f)))));
            c *= 1.0f + 1e-5f;   // keeps the envelope a strict bound after truncation
        } else {
            c = __fdividef(-2.0f * log1pf(-t0) - 2.0f * t0, t0 * t0) * (1.0f + 1e-5f);
        }
        const float p = 1.0f - __fdividef(c, xa * xa), mu = __builtin_amdgcn_rcpf(xa * p);
        const float za = __fdividef(__expf(p * mu * mu) * sqrtf(__fdividef(pi, p)), xa * xa);
        const float d = xa - u0;
        const float q2 = pi - atan_nonneg(__fdividef(a, d));
        const float e0 = __expf(-u0 * u0);
        const float zb = __fdividef(e0 * q2, a);
        for (;;) {
            if (n >= kUparMaxTrials) break;
            const Uni2<float> r12 = upar_draw<float>(key, kSlotUpar + 2u * n, event, pre);
            const float r = r12.a * (za + zb);
            if (r < za) {
                const Uni2<float> r34 = upar_draw<float>(key, kSlotUpar + 2u * n + 1u, event, pre);
                ++n;
                float sn, cs;
                sincospif(2.0f * r34.b, &sn, &cs);
                u = mu + sqrtf(__fdividef(-__logf(1.0f - r34.a), p)) * cs;
                if (u > u0) continue;
                const float t = __fdividef(u, xa);
                const float env = __fdividef(__expf(fmaf(c * t, t, 2.0f * t)), xa * xa);
                const float tgt = __builtin_amdgcn_rcpf(fmaf(xa - u, xa - u, a * a));
                if (r12.b * env < tgt) break;
            } else {
                ++n;
                u = xa + a * cot_0pi(q2 - __fdividef((r - za) * a, e0));
                if (r12.b < __expf((u0 - u) * (u0 + u))) break;
            }
        }
    }
    *trials = n;
    return sgn * u;
}

template <class R>
__device__ __forceinline__ R upar_sample(R x, R a, const Key& k, uint32_t e, uint32_t* t, const Uni2<R>* pre = nullptr);
template <>
__device__ __forceinline__ double upar_sample<double>(double x, double a, const Key& k, uint32_t e, uint32_t* t,
                                                      const Uni2<double>* pre) {
    return upar_sample64(x, a, k, e, t, pre);
}
template <>
__device__ __forceinline__ float upar_sample<float>(float x, float a, const Key& k, uint32_t e, uint32_t* t,
                                                    const Uni2<float>* pre) {
    return upar_sample32(x, a, k, e, t, pre);
}

// ---------------------------------------------------------------------------
// Phase functions (Sections 2.3.1, 2.3.2): inverse CDFs of mu = cos(theta).
//   isotropic 1/2; dipole 3/8(1+mu^2) (mu^3 + 3mu = 8U - 4); core mix
//   11/24 + 3/24 mu^2 (mu^3 + 11 mu = 24U - 12); Henyey-Greenstein.
// ---------------------------------------------------------------------------
enum : int { kPhaseIso = 0, kPhaseDipole = 1, kPhaseCoreWing = 2, kPhaseHG = 3 };

template <class R> __device__ __forceinline__ R cubic_root_mu(R p, R q) {
    // real root of mu^3 + p mu = q (Cardano, p > 0)
    const R disc = M<R>::sqrt(q * q * R(0.25) + fdiv(p * p * p, R(27)));
    const R s = M<R>::cbrt(q * R(0.5) + disc);
    return s - fdiv(p, R(3) * s);
}

template <class R> __device__ __forceinline__ R sample_mu(int phase, R U, R g) {
    if (phase == kPhaseIso) return R(2) * U - R(1);
    if (phase == kPhaseDipole) return cubic_root_mu<R>(R(3), R(8) * U - R(4));
    if (phase == kPhaseCoreWing) return cubic_root_mu<R>(R(11), R(24) * U - R(12));
    if (g == R(0)) return R(2) * U - R(1);
    const R frac = (R(1) - g * g) / (R(1) - g + R(2) * g * U);
    return (R(1) + g * g - frac * frac) / (R(2) * g);
}

template <class R> __device__ __forceinline__ R phase_value(int phase, R mu, R g) {
    if (phase == kPhaseIso) return R(0.5);
    if (phase == kPhaseDipole) return R(0.375) * (R(1) + mu * mu);
    if (phase == kPhaseCoreWing) return R(11.0 / 24.0) + R(3.0 / 24.0) * mu * mu;
    const R b = R(1) + g * g - R(2) * g * mu;
    return R(0.5) * (R(1) - g * g) / (b * M<R>::sqrt(b));
}

// Orthonormal basis perpendicular to unit n (Duff et al. 2017, JCGT 6(1)).
template <class R> __device__ __forceinline__ void onb(const R n[3], R e1[3], R e2[3]) {
    const R sign = copysign(R(1), n[2]);
    const R a = fdiv(R(-1), sign + n[2]);
    const R b = n[0] * n[1] * a;
    e1[0] = R(1) + sign * n[0] * n[0] * a; e1[1] = sign * b; e1[2] = -sign * n[0];
    e2[0] = b; e2[1] = sign + n[1] * n[1] * a; e2[2] = -n[1];
}

// ---------------------------------------------------------------------------
// Device-side descriptions of the medium, the batch models and the outputs.
// ---------------------------------------------------------------------------
enum : int { kGeomShell = 0, kGeomSlab = 1, kGeomGrid = 2 };
enum : int { kVelNone = 0, kVelConstRadial = 1, kVelLinear = 2 };
enum : int { kSrcPoint = 0, kSrcCellN2 = 1 };
enum : int { kLineLya = 0, kLineMg2 = 1, kLineMg2K = 2 };
enum : int { kSpecDelta = 0, kSpecGauss = 1, kSpecThermal = 2, kSpecFlat = 3 };
enum : int { kFateNone = 0, kFateEscaped = 1, kFateAbsorbed = 2, kFateCapped = 3, kFateRedshifted = 4 };
enum : int { kRegCavity = 0, kRegGas = 1, kRegOut = 2 };

// Grid cell record (32 B, one aligned half cache line): gas velocity and
// density, then the temperature and the FP32 line quantities the mixed path
// uses (thermal speed, Voigt a, line-centre opacity k0 = n_HI sigma0).
struct CellRec {
    float4 lo;   // vx, vy, vz, n_HI
    float4 hi;   // T, v_th, a, k0
};

// Peel-march record of one cell for rays along one axis: velocity component
// on that axis, 1/v_th, k0 and dust opacity (FP32).  One array per axis in
// pencil order (that axis's index fastest), so consecutive cells of a ray
// are consecutive in memory; a = A21 lambda0 / (4 pi v_th) comes from 1/v_th.
struct alignas(16) AxisRec {
    float v, ivth, k0, kd;
};
// The same without the dust opacity (12 B), for grids without dust: a quarter
// fewer bytes per visit for the peel pass, whose time follows the bytes it
// fetches.
struct AxisRec3 {
    float v, ivth, k0;
};
static_assert(sizeof(AxisRec3) == 12, "compact pencil record");
__device__ __forceinline__ float rec_kd(const AxisRec& r) { return r.kd; }
__device__ __forceinline__ float rec_kd(const AxisRec3&) { return 0.0f; }

struct GridDev {
    int nx, ny, nz, handoff;
    double lo[3], dx[3];
    const CellRec* rec;   // [z][y][x]
    const AxisRec* axr[3];   // pencil arrays per axis (built on first use), or null
    const AxisRec3* axc[3];  // the same, compact, on grids without dust (then axr is null)
    const double* cdf;    // inclusive prefix of n_HI^2 (CELL_N2 sources)
    double cdf_total;
    uint64_t ncell;
    double sigma_d;
    double hubble;        // Hubble flow: gas velocity v_cell + hubble (p - href) (0 = none)
    double href[3];
    double hstep;         // largest Hubble shift of a sub-step, in units of v_th
    double stop_dv;       // redshift stop (cm/s; 0 = none)
};

// One batch model: medium constants (meshless), dust, source, output slice.
struct ModelDev {
    int kind, v_profile, src_kind, spectrum;
    double r_in, r_out, n, vth, a, k0, kd, v_max, step_f, xcrit;
    double albedo, g_hg;
    double pos[3];
    double dv0, sigma_v;
    uint32_t seed, req;
    double* spec;               // escape spectrum of this model
    int spec_nb;
    int spec_rep;               // copies of it (workgroup b adds into copy b mod spec_rep), folded after the call
    double spec_lo, spec_w, spec_scale;
    unsigned long long* done;   // packets finished (escaped, absorbed, capped)
    // resonant lines (Section 2.4): nl = 2 for a doublet.  Line 1 sits at lab
    // offset lc1 (cm/s) from line 0's centre; its dimensionless frequency is
    // lrho1 (x - lc1 / v_th), its damping parameter lam1 a, its line-centre
    // opacity lk1 k0; a doublet source (lines = 1) emits in line 0 with
    // probability lw0.
    int nl, lines;
    double lc1, lrho1, lam1, lk1, lw0;
};

struct BatchDev {
    uint64_t q0;          // first queue index of the batch
    uint64_t first_id;    // photon id of its first packet
    uint64_t n;
    int model;
    int pad;
};

// Scalars of one persistent launch, read from device memory so that a
// captured graph can be replayed with new values.
struct StepDesc {
    uint64_t q_end;        // queue indices [0, q_end) exist
    int nbatch;
    uint32_t step_events;  // 0 = run to completion
    uint32_t turn_visits;
    uint32_t wide;         // wide turns at or below this many live lanes (0 = never)
    uint32_t park;         // lanes at their interaction sites that interact together (0 = no parking)
    uint32_t refill;       // a turn ends once refill/64 of the lanes that entered it have left (64: never early)
    uint32_t pad;
};

struct OutDev {
    int phase;
    int n_obs;
    int obs_axis[6];
    int cube_nx, cube_ny, cube_nb;
    double img_lo[2], img_w[2];
    double v_lo, v_w;
    float* cube;
    unsigned long long* cube_fx;   // fixed-point cube (units of 1/fx_scale), used instead of `cube` when set
    double fx_scale;
    double tau_cut;
    uint64_t max_events;
    double* rec_dv;       // optional per-packet records (SoA), indexed by queue index - q_rec0
    uint32_t* rec_nres;
    uint32_t* rec_ndust;
    int32_t* rec_fate;
    uint64_t q_rec0;
};

// Per-lane counters, reduced per wave at the end of a launch.  Event counts
// are 32-bit per lane (a lane handles far fewer than 2^32 events in one
// launch); visit and trial counts are 64-bit.  Packet weights are always 1,
// so escaped / absorbed weights equal the counts.
struct Counters {
    uint32_t emitted, escaped, absorbed, capped, handed_off, n_res, n_dust;
    uint32_t peel_contrib, peel_dropped, peel_cut, redshifted;
    uint64_t main_visits, peel_visits, upar_trials;
    uint32_t max_events;    // longest finished history (interactions)
};
constexpr int kNumU64Counters = 14;

}  // namespace thor
