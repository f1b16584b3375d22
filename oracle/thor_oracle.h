/*
 * thor_oracle.h -- serial FP64 CPU oracle for resonant-line (Lyman-alpha)
 * Monte Carlo transport, written from the paper (arXiv 2507.11603, "THOR").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, tables or constants with the
 * HIP path.
 *
 * Every routine follows the paper's statement of the method in its plainest
 * form; see thor_oracle.c for the per-function citations.
 */
#ifndef THOR_ORACLE_H
#define THOR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* geometry kinds */
enum { OR_SHELL = 0, OR_SLAB = 1, OR_GRID = 2 };
/* velocity profiles of the meshless geometries */
enum { OR_VEL_NONE = 0, OR_VEL_CONST_RADIAL = 1, OR_VEL_LINEAR = 2 };
/* source kinds / spectra */
enum { OR_SRC_POINT = 0, OR_SRC_CELL_N2 = 1 };
enum { OR_SPEC_DELTA = 0, OR_SPEC_GAUSS = 1, OR_SPEC_THERMAL = 2, OR_SPEC_FLAT = 3 };
/* resonant line of the medium: Lyman alpha, the Mg II h and k doublet, or
 * the Mg II k line alone (Mg II: frequencies relative to the k line,
 * densities of Mg II) */
enum { OR_LINE_LYA = 0, OR_LINE_MG2 = 1, OR_LINE_MG2K = 2 };
/* phase functions, core skipping */
enum { OR_PHASE_ISO = 0, OR_PHASE_DIPOLE = 1, OR_PHASE_CORE_WING = 2 };
enum { OR_CS_OFF = 0, OR_CS_FIXED = 1, OR_CS_ADAPTIVE = 2 };
/* packet fates */
/* REDSHIFTED: a grid packet in a Hubble flow whose gas-frame offset fell more
 * than stop_dv below line centre; it escapes (the IGM is taken as transparent
 * beyond that shift). */
enum { OR_FATE_NONE = 0, OR_FATE_ESCAPED = 1, OR_FATE_ABSORBED = 2, OR_FATE_CAPPED = 3, OR_FATE_REDSHIFTED = 4 };

typedef struct {
    int32_t kind;
    double r_inner, r_outer;   /* cm; sphere: r_inner = 0; slab: |z| < r_outer */
    double n_HI;               /* cm^-3, homogeneous meshless media */
    double tau0;               /* > 0: line-centre optical depth of the column r_outer - r_inner */
    double T;                  /* K */
    int32_t v_profile;
    double v_max;              /* cm/s */
    double step_f;             /* sub-step limiter fraction for velocity fields */
    int32_t nx, ny, nz;
    double lo[3], hi[3];       /* cm */
    const float *f_n, *f_T, *f_vx, *f_vy, *f_vz;   /* [z][y][x], x fastest */
    int32_t boundary_handoff;
    double sigma_d;            /* dust cross-section per HI atom, cm^2 */
    double tau_d;              /* > 0 (meshless): dust optical depth of the column */
    double albedo, g_hg;
    /* grid Hubble flow: gas velocity v_cell + hubble (p - hubble_ref) (hubble in
     * s^-1, 0 = none); every cell crossing is split into equal sub-steps whose
     * Hubble shift is at most hubble_step v_th (0 = 0.1), each evaluated at its
     * midpoint; stop_dv > 0: redshift stop (cm/s) */
    double hubble, hubble_ref[3], hubble_step, stop_dv;
    int32_t line;              /* OR_LINE_*: the absorbing species and its transitions */
} or_geometry;

typedef struct {
    int32_t kind;
    double pos[3];
    int32_t spectrum;
    double dv0, sigma_v;       /* cm/s; FLAT: dv0 +- sigma_v */
    uint32_t seed, request_id;
    int32_t lines;             /* doublet media: 1 = emit in either line with probability
                                  in the ratio of the oscillator strengths, 0 = at dv0 */
} or_source;

typedef struct {
    int32_t phase;
    int32_t core_skip;
    double x_crit;
    int32_t n_obs;
    int32_t obs_axis[6];       /* 0:+x 1:+y 2:+z 3:-x 4:-y 5:-z */
    int32_t cube_nx, cube_ny, cube_nb;
    double img_lo[2], img_hi[2];
    double cube_v_lo, cube_v_hi;   /* cm/s */
    int32_t spec_nb;
    double spec_lo, spec_hi;       /* cm/s, or units of v_th(spec_T_ref) when spec_T_ref > 0 */
    double spec_T_ref;
    double tau_cut;
    uint64_t max_events;
} or_opts;

typedef struct {
    uint64_t emitted, escaped, absorbed, capped, handed_off;
    uint64_t n_res, n_dust, main_visits, peel_visits, peel_contrib, peel_dropped, peel_cut, upar_trials;
    double w_escaped, w_absorbed;
    uint64_t redshifted;        /* escaped through the redshift stop (part of escaped) */
} or_stats;

typedef struct {
    double dv;          /* final lab-frame frequency offset, cm/s */
    uint32_t n_res;     /* resonant scatterings */
    uint32_t n_dust;    /* dust scatterings */
    int32_t fate;
    uint32_t pad;
} or_record;

/* line constants at temperature T: thermal speed (cm/s), Voigt a, sigma_0 (cm^2) */
void or_line_params(double T, double *v_th, double *a, double *sigma0);
/* the same for the reference line of a species (OR_LINE_*) */
void or_species_params(int line, double T, double *v_th, double *a, double *sigma0);
/* Voigt-Hjerting function H(a,x) = Re w(x + i a) */
double or_voigt(double a, double x);
/* Dawson's integral (long-double power series), exported for its own pin */
double or_dawson(double x);
/* lower real branch W_{-1}(z) of Lambert's W, -1/e <= z < 0 (NaN outside) */
double or_lambert_wm1(double z);
/* core-to-wing transition x_cw(a): exact (Lambert W) and the quartic in ln a */
double or_xcw_exact(double a);
double or_xcw_b25(double a);
/* Philox4x32-10 block function */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* the two 53-bit uniforms of a keyed draw */
void or_draw(uint32_t seed, uint32_t request_id, uint32_t slot, uint32_t event, uint64_t id,
             double out[2]);
/* u_parallel sampler; returns the sample, writes the trial count */
double or_sample_upar(double x, double a, uint32_t seed, uint32_t event, uint64_t id,
                      uint64_t *trials);
/* envelope mass ratio of the u_parallel sampler: expected trials */
double or_upar_expected_trials(double x, double a);
/* phase-function cosines (phase: 0 iso, 1 dipole, 2 core mix, 3 Henyey-Greenstein) */
double or_sample_mu(int phase, double U, double g);
/* orthonormal basis perpendicular to unit n */
void or_basis(const double n[3], double e1[3], double e2[3]);

/* transport packets [first_id, first_id + n); outputs are accumulated (not cleared) */
int or_transport(const or_geometry *g, const or_source *s, const or_opts *o,
                 uint64_t first_id, uint64_t n,
                 double *spectrum, double *cube, or_stats *st, or_record *records);

/* The same run split over threads: or_prepare copies the three structs and
 * builds the medium constants (the n_HI^2 emission CDF of a grid) once; the
 * field arrays must outlive it.  or_transport_prepared may then run from
 * several threads at once on disjoint id ranges, each with its own outputs. */
typedef struct or_prepared or_prepared;
or_prepared *or_prepare(const or_geometry *g, const or_source *s, const or_opts *o);
int or_transport_prepared(const or_prepared *p, uint64_t first_id, uint64_t n,
                          double *spectrum, double *cube, or_stats *st, or_record *records);
void or_release(or_prepared *p);

/* the generator alone: rows of 11 doubles per packet, position (3),
 * direction (3), lab dv, gas-frame dv (THERMAL; else 0), cell (3) */
int or_emit(const or_geometry *g, const or_source *s, uint64_t first_id, uint64_t n, double *out);

/* n resonant scatterings at fixed (x, a, k_in) with photon ids 0..n-1 at
 * `event`, key (seed, 0); phase 0 iso, 1 dipole, 2 core/wing: rows of 10
 * doubles, u_par, u_perp (2), x_atom, x_out, k_out (3), trials, phase used */
int or_scatter_resonant(double x, double a, const double k[3], double x_crit, int phase,
                        uint32_t seed, uint32_t event, uint64_t n, double *out);

/* raytracing driver (Section 3.5): rays parallel to grid axis `axis` (0 x, 1 y, 2 z)  */
/* projection Q = int q w ds, Q_hat = int w ds (w may be NULL: w = 1); images [j][i]  */
int or_project(const float *q, const float *w, int nx, int ny, int nz, int axis, double ds,
               double *Q, double *W);
/* Lyman-alpha absorption spectra tau[n_los][nb] at bin centres of [u_lo, u_hi) cm/s */
int or_forest(const float *nHI, const float *T, const float *vlos, int nx, int ny, int nz,
              int axis, double ds, double hubble, int n_sub, const int32_t *los,
              uint32_t n_los, uint32_t nb, double u_lo, double u_hi, double *tau);

#ifdef __cplusplus
}
#endif
#endif
