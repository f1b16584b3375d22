/*
 * thor_rays.h -- C ABI of the raytracing driver of libthor.so (arXiv
 * 2507.11603, Section 3.5): integrals along rays that cross a uniform grid
 * parallel to one of its axes.
 *   image projection        -> thor_ray_project  (Section 3.5.1)
 *   Lyman-alpha absorption  -> thor_ray_forest   (Section 3.5.2, eq. abs)
 *
 * Conventions (as in thor.h): cgs units; no call throws; a negative
 * thor_status is a failure, with a thread-local message from
 * thor_ray_last_error().  These calls need no thor_ctx: every pointer named
 * "device" is memory of the current HIP device, owned by the caller, and the
 * work is enqueued on `hip_stream` (a hipStream_t; NULL = the null stream).
 * The calls return once the work is enqueued; results are valid after the
 * stream has reached that point.  Calls on different streams may overlap;
 * outputs must not alias inputs.
 *
 * Grids: fields are float32 arrays [z][y][x] (x fastest) of nx * ny * nz
 * cells.  A ray runs along +axis through cell centres from the low face
 * (s = 0) to the high face, and the fields are constant within a cell.  A
 * ray is named by its cell indices (i, j) along the other two axes, i along
 * the lower-numbered one: axis z -> (i, j) = (x, y), axis y -> (x, z),
 * axis x -> (y, z).  Images are [j][i] float64.
 */
#ifndef THOR_RAYS_H
#define THOR_RAYS_H

#include <stdint.h>

#include "thor.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny, nz;    /* cells along x, y, z (each >= 1) */
    int32_t axis;          /* direction of the rays: 0 = x, 1 = y, 2 = z */
    double ds;             /* cell length along the axis, cm (> 0) */
} thor_ray_grid;

/* Section 3.5.1, image projection: along every ray of the axis,
 *   Q = int q w ds   and   W = int w ds   (w = 1 when w is NULL).
 * The mean of q weighted by w along a ray is Q / W (a mass-weighted
 * temperature map takes q = T and w = the gas mass of a cell).
 * q, w: device float32 fields; Q, W: device float64 images [j][i] (W may be
 * NULL).  Sums are FP64.  When an image has too few rays to fill the GPU,
 * each ray is split into segments whose partial sums are added atomically,
 * so the last bits of Q and W then depend on their order.  Errors:
 * THOR_E_INVAL (bad grid, NULL q or Q), THOR_E_DEVICE (launch failed). */
thor_status thor_ray_project(const thor_ray_grid *g, const float *q, const float *w,
                             double *Q, double *W, void *hip_stream);

typedef struct {
    int32_t i0, ni;        /* rays i0 <= i < i0 + ni ... */
    int32_t j0, nj;        /* ... times j0 <= j < j0 + nj (ni or nj = 0: no rays) */
    double hubble;         /* H(z), 1/s: the Hubble velocity at s is hubble * s */
    int32_t n_sub;         /* equal steps per cell, each evaluated at its midpoint
                              (1 .. 65536); H ds / n_sub well below v_th keeps the
                              Hubble shift per step below the line width */
    uint32_t nb;           /* spectral bins (1 .. 2^22) */
    double u_lo, u_hi;     /* bin range, cm/s (u_hi > u_lo) */
    int32_t precision;     /* THOR_PREC_FP64, or THOR_PREC_MIXED: the Voigt
                              function and its argument in FP32, sums in FP64 */
} thor_forest_opts;

/* Section 3.5.2, eq. (abs): optical depth tau(u) = int n_HI sigma(nu(s), T) ds
 * along each ray, with the gas frequency nu(s) = nu_i [1 - (v(s) + H s)/c].
 * u = c (nu_i / nu0 - 1) is the photon's velocity offset at s = 0, sampled
 * at the nb bin centres of [u_lo, u_hi); to first order in v/c a cell at s
 * with thermal speed v_th(T) adds n_HI sigma0(T) H(a(T), x) ds to bin u with
 * x = (u - v(s) - H s) / v_th.  The flux is exp(-tau).
 * n_HI (cm^-3), T (K, > 0 wherever n_HI > 0), v_los (velocity component
 * along +axis, cm/s): device float32 fields.  tau: device float64
 * [nj][ni][nb].  Errors: THOR_E_INVAL (bad grid, rays outside the grid,
 * n_sub, nb, range or precision; NULL pointers), THOR_E_DEVICE (launch
 * failed). */
thor_status thor_ray_forest(const thor_ray_grid *g, const thor_forest_opts *o,
                            const float *n_HI, const float *T, const float *v_los,
                            double *tau, void *hip_stream);

/* message of the last failed thor_ray_* call on this thread */
const char *thor_ray_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
