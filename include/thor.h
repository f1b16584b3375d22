/*
 * thor.h -- C ABI of the MI355X resonant-line (Lyman-alpha) Monte Carlo
 * transport library (libthor.so).
 *
 * The calls follow the paper's statement of the problem (arXiv 2507.11603,
 * Section 3.2 building blocks and Section 3.4 MCRT driver):
 *   a dataset answers where the next cell face is and what gas fills the cell
 *        -> thor_load_grid      (Section 3.3, dataset "query")
 *   a generator spawns photons with weights, frequencies and directions
 *        -> thor_emit           (Section 3.4, "Emission")
 *   the MCRT driver propagates packets and handles interactions
 *        -> thor_transport      (Section 3.4 "Propagation", "Interaction",
 *                                3.4.1 peeling, 3.4.2 core skipping, 3.4.3 RNG)
 *   output processors reduce finished photons into spectra and cubes
 *        -> thor_read_spectra   (Section 3.2, output processors)
 * plus a continuous-batching extension for stream of shell-model solves
 * (Section 5.1's parameter grid): thor_submit / thor_step / thor_poll.
 *
 * Conventions for every call:
 *   - Units are cgs: lengths in cm, velocities and frequency offsets in cm/s
 *     (a frequency offset dv = c (nu - nu0)/nu0 is stored in the lab frame),
 *     densities in cm^-3, temperatures in K.
 *   - Pointers are plain host or device pointers as stated per argument; a
 *     "device" pointer is memory of the context's HIP device.
 *   - No call throws; failures return a negative thor_status, and
 *     thor_last_error() gives a message (thread-local).  THOR_E_INVAL and
 *     THOR_E_BUDGET leave the context unchanged; THOR_E_DEVICE poisons it
 *     (only thor_destroy is valid afterwards).
 *   - A context must not be used from two host threads at once.
 *   - All device work is ordered on the stream given to thor_create.
 */
#ifndef THOR_H
#define THOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define THOR_ABI_VERSION 1

typedef enum {
    THOR_OK = 0,
    THOR_INCOMPLETE = 1,        /* bounded step ended with work left: call again */
    THOR_E_INVAL = -1,          /* bad argument; context unchanged */
    THOR_E_NOMEM = -2,          /* device allocation failed */
    THOR_E_BUDGET = -3,         /* HBM budget of the context would be exceeded */
    THOR_E_DEVICE = -4,         /* HIP runtime error; context poisoned */
    THOR_E_STATE = -5,          /* call not valid in the current state */
    THOR_E_UNSUPPORTED = -6     /* option combination not implemented */
} thor_status;

typedef struct thor_ctx thor_ctx;

/* ---------------------------------------------------------------- geometry */
typedef enum { THOR_GEOM_SHELL = 0, THOR_GEOM_SLAB = 1, THOR_GEOM_GRID = 2 } thor_geom_kind;
typedef enum { THOR_VEL_NONE = 0, THOR_VEL_CONST_RADIAL = 1, THOR_VEL_LINEAR = 2 } thor_vel_profile;
typedef enum { THOR_MEM_HOST = 0, THOR_MEM_DEVICE = 1 } thor_mem;

/* The medium (Section 3.3).  Meshless kinds (Section 4 validation media):
 *   SHELL: homogeneous gas for r_inner <= r < r_outer around the origin,
 *          vacuum inside (r_inner = 0 gives a sphere);
 *   SLAB:  homogeneous gas for |z| < r_outer, infinite in x and y.
 * Their density is n_HI, or, when tau0 > 0, tau0 / (sigma0(T) (r_outer -
 * r_inner)) (tau0 = line-centre optical depth of the column).  Velocity
 * profiles: CONST_RADIAL v = v_max r_hat; LINEAR v = v_max r / r_outer (slab:
 * v_z = v_max z / r_outer).  Velocity fields are integrated in sub-steps of
 * at most step_f v_th r / |v_max| (CONST_RADIAL) or step_f v_th r_outer /
 * |v_max| (LINEAR), with the fields at each sub-step's midpoint.
 * GRID: uniform Cartesian grid nx * ny * nz over [lo, hi]; five float32
 * fields in C order [z][y][x] (x fastest), each nx*ny*nz values, in host or
 * device memory per `mem`; cells with n_HI = 0 are vacuum.  The fields are
 * copied into the context (the caller may free them on return).
 * Dust (Section 2.3.2): opacity k_d = sigma_d n_HI, or for meshless kinds
 * with tau_d > 0, tau_d / (r_outer - r_inner); interaction is absorption
 * with probability 1 - albedo, else Henyey-Greenstein scattering with
 * asymmetry g_hg, coherent in the gas frame. */
typedef struct {
    int32_t kind;
    double r_inner, r_outer;
    double n_HI;
    double tau0;
    double T;
    int32_t v_profile;
    double v_max;
    double step_f;
    int32_t nx, ny, nz;
    double lo[3], hi[3];
    const float *n_HI_field, *T_field, *vx, *vy, *vz;
    int32_t mem;
    int32_t boundary_handoff;   /* grid exits also counted as hand-offs */
    double sigma_d;
    double tau_d;
    double albedo, g_hg;
    /* GRID Hubble flow (Section 2.2: the cross-section in the frame of the gas,
     * which moves with the expansion; Section 3.4 sub-cell stepping): gas
     * velocity v_cell + hubble (p - hubble_ref), hubble in s^-1 (0 = none).
     * Every cell crossing of a flight or peel ray is cut into n equal steps, n
     * the smallest with hubble t / n <= hubble_step v_th (0 = 0.1), each taking
     * the profile at its midpoint.  stop_dv > 0 (cm/s): a packet whose
     * gas-frame offset falls more than stop_dv below line centre (checked at
     * cell faces) escapes (beyond that shift the IGM is taken as transparent),
     * counted in thor_stats.redshifted and not as a hand-off. */
    double hubble, hubble_ref[3], hubble_step, stop_dv;
    /* Resonant line (THOR_LINE_*).  LYA: Lyman alpha of H I.  MG2: the Mg II
     * h and k doublet (Section 2.4: the two lines' cross-sections add; a
     * resonant scattering picks the line by its share of the opacity at the
     * site and re-emits in it, h isotropically), densities of Mg II, every
     * frequency offset relative to the k line (2796.352 A; h lies 767.6 km/s
     * to the red).  MG2K: the k line alone.  MG2 and MG2K need a meshless
     * medium (THOR_E_UNSUPPORTED on a grid); their packets are not handed to
     * the tail kernel. */
    int32_t line;
} thor_geometry;

typedef enum { THOR_LINE_LYA = 0, THOR_LINE_MG2 = 1, THOR_LINE_MG2K = 2 } thor_line;

/* ---------------------------------------------------------------- sources */
typedef enum { THOR_SRC_POINT = 0, THOR_SRC_CELL_N2 = 1 } thor_source_kind;
typedef enum { THOR_SPEC_DELTA = 0, THOR_SPEC_GAUSS = 1, THOR_SPEC_THERMAL = 2, THOR_SPEC_FLAT = 3 } thor_spectrum_kind;

/* Generator (Section 3.4 "Emission"): isotropic directions; frequency
 * DELTA dv0, GAUSS dv0 + sigma_v N(0,1) (source frame = lab frame), or
 * THERMAL: the gas-frame Doppler profile of the emitting cell,
 * dv0 + v_th N(0,1)/sqrt(2), shifted to the lab frame by v.k; FLAT: a flat
 * continuum, dv0 + sigma_v U(-1, 1).  lines = 1 in a doublet medium: each
 * packet is emitted in line 1 with probability f_1 / (f_0 + f_1) (the
 * oscillator strengths), its frequency shifted to that line's centre.
 * POINT: emitted at pos.  CELL_N2 (grid only): cell drawn with probability
 * proportional to n_HI^2, uniform position inside the cell.
 * Packet ids and (seed, request_id) key the Philox4x32-10 stream. */
typedef struct {
    int32_t kind;
    double pos[3];
    int32_t spectrum;
    double dv0, sigma_v;
    uint32_t seed, request_id;
    int32_t lines;
} thor_source;

/* ---------------------------------------------------------------- transport */
typedef enum { THOR_PREC_FP64 = 0, THOR_PREC_MIXED = 1 } thor_precision;
typedef enum { THOR_PATH_PLAIN = 0, THOR_PATH_PERSISTENT = 1 } thor_path;
typedef enum { THOR_PHASE_ISO = 0, THOR_PHASE_DIPOLE = 1, THOR_PHASE_CORE_WING = 2 } thor_phase;
typedef enum { THOR_CS_OFF = 0, THOR_CS_FIXED = 1, THOR_CS_ADAPTIVE = 2 } thor_core_skip;
typedef enum { THOR_OBS_PX = 0, THOR_OBS_PY = 1, THOR_OBS_PZ = 2,
               THOR_OBS_MX = 3, THOR_OBS_MY = 4, THOR_OBS_MZ = 5 } thor_obs_axis;

/* Options of one transport call.
 *   precision: FP64 everywhere, or MIXED (FP32 Voigt, direction and frequency
 *              redistribution; FP64 position, cell distances, tau).
 *   path:      PLAIN = one thread per packet, one launch per emitted batch,
 *              runs to completion; PERSISTENT = resident waves refill lanes
 *              from a queue over all pending batches.
 *   phase:     resonant phase function (Section 2.3.1); core_skip/x_crit as
 *              in Section 3.4.2 (ADAPTIVE: 0.2 (a tau0)^(1/3) for meshless
 *              media with a tau0 >= 1, from the column of the medium).
 *   observers: n_obs axis-aligned observers at infinity (peeling, Section
 *              3.4.1); image axes: +-z -> (x, y), +-x -> (y, z), +-y -> (z, x).
 *   cube:      [n_obs][cube_ny][cube_nx][cube_nb] float32, pixel of the
 *              projected event position over [img_lo, img_hi), frequency bin
 *              of the peeled dv over [cube_v_lo, cube_v_hi).
 *   spectrum:  escaped weight per bin of dv over [spec_lo, spec_hi), or of
 *              dv / v_th(spec_T_ref) when spec_T_ref > 0 (float64).
 *   tau_cut:   peel rays stop once tau exceeds it (contribution dropped).
 *   max_events: interaction cap per packet (0 = 1e8); capped packets are
 *              counted, not binned.
 *   step_events: PERSISTENT only: 0 = run to completion; else each call
 *              advances every resident packet by at most this many
 *              interactions and returns THOR_INCOMPLETE while work is left.
 *   waves_per_cu, block: PERSISTENT launch shape (0 = automatic);
 *              visits_per_turn: march segments a lane advances its packet
 *              before the wave refills finished lanes (0 = 256). */
typedef struct {
    int32_t precision;
    int32_t path;
    int32_t phase;
    int32_t core_skip;
    double x_crit;
    int32_t n_obs;
    int32_t obs_axis[6];
    int32_t cube_nx, cube_ny, cube_nb;
    double img_lo[2], img_hi[2];
    double cube_v_lo, cube_v_hi;
    int32_t spec_nb;
    double spec_lo, spec_hi, spec_T_ref;
    double tau_cut;
    uint64_t max_events;
    uint64_t step_events;
    int32_t waves_per_cu;
    int32_t block;
    int32_t visits_per_turn;    /* PERSISTENT: march segments per lane turn (0 = 256) */
    int32_t use_graph;          /* thor_step: replay one captured hipGraph per step */
    int32_t inline_peel;        /* PERSISTENT: march peel rays in the scattering lane
                                   instead of the peel-seed pass */
    int32_t records;            /* 1: keep per-packet records of this call */
    uint64_t seed_slots;        /* PERSISTENT, grid, 1-3 observers: slots (48 B each) of
                                   the peel-seed buffer; 0 = the largest power of two
                                   from 2^28 to 2^30 whose seeds and sort arrays (64 B
                                   a slot) fit in half the free device memory (and of the
                                   budget left), else 2^28 (12.9 GB), else max(2^26, 128
                                   per lane of the launch); at least observers x lanes.  A full
                                   buffer ends a transport kernel early (packets wait
                                   in device memory), the peel pass empties it and
                                   transport resumes. */
    int32_t wide_lanes;         /* PERSISTENT, step_events = 0: once the queue is drained, a
                                   wave holding at most this many live packets hands them
                                   to a tail kernel that runs each in a wave of its own,
                                   its idle lanes evaluating the random draws of the
                                   packet's next events ahead (same results; a shorter
                                   serial chain for the packets that end a launch);
                                   0 = 8, negative = never, at most 16 */
    int32_t park_lanes;         /* PERSISTENT: a lane that reaches its interaction site waits
                                   there while its wave mates march on; the waiting lanes
                                   interact together once this many wait, no lane marches,
                                   or the turn ends (same histories; more lanes share the
                                   long interaction code); 0 = the library default,
                                   negative = never, at most 64 */
    int32_t refill_64ths;       /* PERSISTENT: a turn ends early once this many 64ths of the
                                   lanes that entered it have finished, so that the wave
                                   refills them; 0 = 16 (a quarter), 64 = only at the
                                   visits_per_turn bound */
    int32_t accum;              /* cube accumulation: THOR_ACCUM_F32_ATOMIC (float32 atomic
                                   adds; sums depend on their order in the last bits) or
                                   THOR_ACCUM_FIXED64 (each contribution rounded to an
                                   integer number of 2^-fixed_bits units and added as a
                                   uint64: bit-reproducible in any order and launch
                                   shape; a voxel holds at most 2^(64 - fixed_bits)) */
    int32_t fixed_bits;         /* FIXED64: 0 = 40 (units of 9.1e-13, voxel sums up to 1.7e7) */
    int32_t presort;            /* PERSISTENT, unbounded: order in which the queued packets are
                                   taken (keys drawn by a pre-pass, radix-sorted on the device,
                                   inside the call's time); results do not change (each packet's
                                   history depends only on its id).  1 = spatial: the Morton
                                   order of n_HI^2-weighted emission cells (grids), so that the
                                   packets in flight and their peel rays are near each other;
                                   2 = frequency: the emitted offset (Section 7.1's pre-sorting),
                                   so that a wave's packets start alike; 0 = the library default
                                   (1 for grids with CELL_N2 sources, 2 for meshless media whose
                                   sources spread in frequency, else none); -1 = queue order;
                                   other values THOR_E_INVAL */
    int32_t seed_sort;          /* peel-seed path: before each peel pass the buffer's rays are
                                   sorted by (axis, pencil index of their front cell), so that
                                   the rays a wave marches together share cache lines; 0 = the
                                   library default (on), 1 = on, -1 = buffer order.  Only the
                                   order of the cube's additions changes (FIXED64 cubes are
                                   identical) */
    int32_t fuse_bins;          /* peel-seed path, photon fusing (Section 3.4.1), 0 = off.  m > 0:
                                   before each peel pass, rays of one round that start in the
                                   same cell towards the same observer and whose peeled
                                   frequencies fall in the same 1/m of a cube frequency bin
                                   (and the same cube element) are merged into one ray, weight
                                   sum w exp(-tau_first), marched at the first ray's frequency.
                                   Changes results (within the frequency tolerance); which rays
                                   share a round depends on scheduling */
} thor_transport_opts;

typedef enum { THOR_ACCUM_F32_ATOMIC = 0, THOR_ACCUM_FIXED64 = 1 } thor_accum;

/* Counters of one thor_transport call (device counters read back at the end
 * of the call). */
typedef struct {
    uint64_t emitted, escaped, absorbed, capped, handed_off;
    uint64_t n_res, n_dust;         /* resonant / dust scatterings */
    uint64_t main_visits;           /* cell (segment) visits of the main march */
    uint64_t peel_visits;           /* cell visits of peel rays */
    uint64_t peel_contrib, peel_dropped, peel_cut;
    uint64_t upar_trials;           /* u_parallel proposals */
    double w_escaped, w_absorbed;
    double kernel_ms;               /* device time of the call (events around all launches) */
    double transport_ms;            /* of which transport kernels (grid persistent path with
                                       peel seeds: summed per pass; otherwise = kernel_ms) */
    double peel_ms;                 /* of which peel-pass kernels */
    uint64_t passes;                /* transport + peel pass rounds (1 without seeds) */
    double tail_ms;                 /* of transport_ms, the tail kernels (packets handed off
                                       by drained waves, see wide_lanes) */
    uint64_t max_events;            /* longest finished history of the call (interactions;
                                       plain and unbounded persistent calls) */
    uint64_t tail_events;           /* interactions run by the tail kernels (in n_res, n_dust) */
    uint64_t tail_main_visits;      /* main-march cell visits of the tail kernels */
    uint64_t tail_peel_visits;      /* peel cell visits of the tail kernels */
    uint64_t redshifted;            /* escaped through the redshift stop (part of escaped) */
    double presort_ms;              /* of kernel_ms, the presort of the queue */
    double seedsort_ms;             /* of kernel_ms, the sorts of the seed buffer before the peel passes */
    uint64_t peel_fused;            /* peel rays merged away by photon fusing */
} thor_stats;

/* Per-packet record (index = packet id - first id of its batch, batches in
 * emission order). */
typedef struct {
    double dv;          /* final lab-frame frequency offset, cm/s */
    uint32_t n_res;
    uint32_t n_dust;
    int32_t fate;       /* 1 escaped, 2 absorbed, 3 capped, 4 escaped by the redshift stop */
    uint32_t pad;
} thor_record;

typedef enum { THOR_OUT_SPECTRUM = 0, THOR_OUT_CUBE = 1, THOR_OUT_RECORDS = 2,
               THOR_OUT_STATS = 3, THOR_OUT_CUBE_FIXED = 4 } thor_output;

/* ---------------------------------------------------------------- calls */

/* Create a context on HIP device `hip_device`.  `hip_stream` is a
 * hipStream_t of that device (e.g. torch.cuda.current_stream().cuda_stream)
 * or NULL for the device's null stream.  hbm_budget_bytes bounds what the
 * context allocates (0 = no bound); exceeding it gives THOR_E_BUDGET. */
thor_status thor_create(thor_ctx **out, int hip_device, void *hip_stream, uint64_t hbm_budget_bytes);

/* Release the context and all device memory it owns. NULL is ignored. */
void thor_destroy(thor_ctx *ctx);

/* Install the medium (dataset).  Replaces any previous one and discards
 * emitted batches that have not been transported. */
thor_status thor_load_grid(thor_ctx *ctx, const thor_geometry *g);

/* Queue n_packets packets with ids first_photon_id .. + n_packets - 1 from
 * source `src` (generator).  Packets are created lazily inside
 * thor_transport; a CELL_N2 source builds the n_HI^2 emission CDF here once
 * per medium. */
thor_status thor_emit(thor_ctx *ctx, const thor_source *src, uint64_t n_packets,
                      uint64_t first_photon_id);

/* Transport every queued packet (MCRT driver).  Outputs (spectrum, cube)
 * are shaped by `opt` and accumulated across calls until
 * thor_reset_outputs; `out_stats` (may be NULL) receives this call's
 * counters.  Returns THOR_INCOMPLETE for a bounded PERSISTENT step with
 * work left. */
thor_status thor_transport(thor_ctx *ctx, const thor_transport_opts *opt, thor_stats *out_stats);

/* Zero the accumulated spectrum and cube. */
thor_status thor_reset_outputs(thor_ctx *ctx);

/* Copy an output to dst (host memory, or device memory when dst_on_device):
 *   SPECTRUM: float64[spec_nb]; CUBE: float32[n_obs][ny][nx][nb] (index
 *   selects nothing and must be 0; a FIXED64 cube is converted, each voxel
 *   rounded once); CUBE_FIXED: uint64[n_obs][ny][nx][nb], the FIXED64 cube's
 *   integer sums (units of 2^-fixed_bits; THOR_E_STATE for a float cube);
 *   RECORDS: thor_record[packets of the last call]; STATS: thor_stats of the
 *   last call.  dst_bytes must be at least the size of the output
 *   (THOR_E_INVAL otherwise). */
thor_status thor_read_spectra(thor_ctx *ctx, thor_output which, uint32_t index, void *dst,
                              uint64_t dst_bytes, int dst_on_device);

/* Size in bytes of an output as thor_read_spectra would copy it. */
uint64_t thor_output_bytes(thor_ctx *ctx, thor_output which);

/* Message of the last failure in this thread ("" if none). */
const char *thor_last_error(void);

/* ------------------------------------------------ device-function harness */
/* Evaluate H(a, x) (the Voigt-Hjerting function used for sigma(x),
 * Section 3.4 and Appendix A.3) with the transport kernels' own device code
 * on n (a, x) pairs: a, x, out are device float64 arrays; precision FP64 or
 * MIXED (FP32 evaluation, result widened).  For tests of the device code. */
thor_status thor_eval_voigt(thor_ctx *ctx, const double *a, const double *x, double *out,
                            uint64_t n, int32_t precision);

/* Core-to-wing transition x_cw(a) of H(a, x) (Appendix A.2) by the quartic
 * in ln a printed there, with the device code: a, out are device float64
 * arrays of n entries (a > 0, normal); precision FP64 (library logarithm)
 * or MIXED (FP32, logarithm from the exponent bits and an atanh series, the
 * fast form of Appendix A.2).  Within 0.6 % of the exact Lambert-W value for
 * 1.5e-5 <= a <= 1e-2. */
thor_status thor_eval_xcw(thor_ctx *ctx, const double *a, double *out, uint64_t n, int32_t precision);

/* Draw n u_parallel samples (eq. uparallel) at (x, a) with the kernels' own
 * sampler, photon ids 0..n-1, event `event`, key (seed, 0): out_u float64[n]
 * and out_trials uint32[n], device arrays. */
thor_status thor_sample_upar(thor_ctx *ctx, double x, double a, uint32_t seed, uint32_t event,
                             double *out_u, uint32_t *out_trials, uint64_t n, int32_t precision);

/* --------------------------------------------- serving extension (batching) */
/* One shell-model solve (Section 5.1): homogeneous shell r_inner..r_outer
 * (cm) with column N_HI (cm^-2) at temperature T, constant radial expansion
 * v_exp (cm/s), dust optical depth tau_d (albedo, g_hg), central GAUSS source
 * of width sigma_v, n_packets packets keyed (seed, request_id), dipole
 * phase function, adaptive core skipping, spectrum of spec_nb bins over
 * [spec_lo, spec_hi) of dv. */
typedef struct {
    double N_HI, v_exp, T, tau_d, albedo, g_hg;
    double r_inner, r_outer, sigma_v, step_f;
    uint64_t n_packets;
    uint32_t seed, request_id;
    int32_t spec_nb;
    double spec_lo, spec_hi;
} thor_shell_request;

/* Admit a request if its packet slots and output memory fit the context's
 * HBM budget, else THOR_E_BUDGET (nothing changes; submit again later).
 * *req_id receives the handle.  Requests share the device with every other
 * admitted request; each packet's random stream depends only on (seed,
 * request_id, photon id), so a result is the same alone and in any mix. */
thor_status thor_submit(thor_ctx *ctx, const thor_shell_request *r, uint64_t *req_id);

/* Run one bounded persistent step over all admitted requests: every
 * resident packet advances by at most max_events_per_packet interactions
 * (0 = to completion).  Returns THOR_OK when no admitted work is left,
 * THOR_INCOMPLETE otherwise. */
thor_status thor_step(thor_ctx *ctx, uint32_t max_events_per_packet, const thor_transport_opts *opt);

/* Poll a request: *done = 1 once all its packets finished; then spectrum
 * (host float64[spec_nb], may be NULL) and st (may be NULL) are filled and
 * the request's memory is released (the handle becomes invalid). */
thor_status thor_poll(thor_ctx *ctx, uint64_t req_id, double *spectrum, thor_stats *st, int *done);

/* ------------------------------------------------ no-allocation transport */
/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * Transports every packet queued by thor_emit, like thor_transport with
 * path PERSISTENT run to completion (the same kernels, so the same packet
 * histories), but allocates nothing: besides the caller's outputs, every
 * device buffer of the call (step descriptor, batch and model tables,
 * counters, queue cursor, the escape spectrum's 32 partial copies) lives in
 * one static device array of the library, THOR_NOALLOC_SCRATCH_BYTES on each
 * GPU the library runs on, held until the process ends.  Its address is
 * looked up once per device in thor_create.
 *
 * Limits (THOR_E_INVAL beyond them, context unchanged): at most
 * THOR_NOALLOC_MAX_BATCHES queued batches and THOR_NOALLOC_MAX_BINS spectrum
 * bins.  Not supported (THOR_E_UNSUPPORTED): path PLAIN, step_events > 0,
 * records, accum FIXED64.  The last packets of a launch are not handed to a tail kernel,
 * and on a grid with observers every peel ray is marched by the scattering
 * lane (inline_peel), since the tail list and the peel-seed buffer are not
 * of a modest size.  Packet histories, spectrum and counters equal those of
 * thor_transport; cube sums differ only by the order of float atomics.
 *
 * Outputs, device memory of the context's device, added to (not cleared):
 *   d_spectrum  float64[opt->spec_nb], escaped weight per bin as in
 *               thor_transport;
 *   d_cube      float32[n_obs][cube_ny][cube_nx][cube_nb] (NULL when
 *               opt->n_obs = 0).
 * out_stats (host, may be NULL): this call's counters; the call then waits
 * for its work.  With out_stats NULL the call only enqueues kernels on the
 * context's stream and returns (no host synchronisation, no copies).
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind; calls that overlap on one GPU (two streams or two contexts) race
 * and must not be made. */
#define THOR_NOALLOC_MAX_BATCHES 64
#define THOR_NOALLOC_MAX_BINS 4096
#define THOR_NOALLOC_SCRATCH_BYTES 1081344
thor_status thor_transport_noalloc(thor_ctx *ctx, const thor_transport_opts *opt, double *d_spectrum,
                                   float *d_cube, thor_stats *out_stats);

#ifdef __cplusplus
}
#endif
#endif
