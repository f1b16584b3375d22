// thor_engine.hpp -- per-packet transport engine (arXiv 2507.11603,
// Section 3.4): emission, cell march with tau accumulation, interaction
// (dust or resonant scattering), peeling off, escape binning.  Shared by the
// plain and the persistent kernels.  GRID selects the uniform-grid medium at
// compile time; otherwise the meshless sphere/shell/slab.
//
// The FP64 instantiation evaluates the march, interaction and peel formulas
// in the same order as the CPU reference, so same-seed runs follow the same
// histories.  The FP32 (mixed) instantiation keeps positions, distances and
// optical depths in FP64 but derives cell quantities, directions, frequency
// redistribution and the Voigt function in FP32 and marches with the
// reciprocal direction.
#pragma once
#include <type_traits>

#include "thor_device.hpp"

// cells of a grid peel ray whose records are fetched together: inline and
// FP64 rays, and the FP32 rays of the peel pass
#ifndef THOR_PEEL_LOOKAHEAD
#define THOR_PEEL_LOOKAHEAD 2
#endif
// (THOR_PASS_LOOKAHEAD: 12-byte records of grids without dust; the 16-byte
// records with dust take THOR_PASS_LOOKAHEAD_DUST, within the same registers)
#ifndef THOR_PASS_LOOKAHEAD
#define THOR_PASS_LOOKAHEAD 5
#endif
#ifndef THOR_PASS_LOOKAHEAD_DUST
#define THOR_PASS_LOOKAHEAD_DUST 4
#endif
// peel pass, FP32 rays: request the next group's records before summing the
// current group (two groups in flight per lane)
#ifndef THOR_PASS_PREFETCH
#define THOR_PASS_PREFETCH 1
#endif

namespace thor {

template <class R> struct Pkt {
    double p[3];
    int c[3];
    int region;
    R k[3];
    R dv;
    double tau_t, tau_a;
    uint64_t id, q;
    uint32_t event, n_res, n_dust;
    int model;
};

template <class R> struct Fields {
    R vth, a;
    double k0, kd;
    R v[3];
};

__device__ __forceinline__ double dot3d(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
template <class R> __device__ __forceinline__ R dot3(const R a[3], const R b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Opacity of a meshless doublet's second line (Section 2.4: a doublet's
// cross-section is the sum of its lines') at line 0's gas-frame offset x.
template <class R>
__device__ __forceinline__ double second_line_k(const ModelDev& m, double k0, R a, R vth, R x, const float* dtab) {
    const R x1 = R(m.lrho1) * (x - R(m.lc1) / vth);
    const R a1 = a * R(m.lam1);
    if constexpr (sizeof(R) == 4) return (k0 * m.lk1) * double(voigt32(a1, x1, dtab));
    else return (k0 * m.lk1) * double(voigt<R>(a1, x1));
}

// sin and cos of 2 pi u
template <class R> __device__ __forceinline__ R sincos2pi(R u, R* c);
template <> __device__ __forceinline__ double sincos2pi<double>(double u, double* c) {
    double s;
    ::sincos(2.0 * kPi * u, &s, c);
    return s;
}
template <> __device__ __forceinline__ float sincos2pi<float>(float u, float* c) {
    // v_sin_f32 / v_cos_f32 take their argument in revolutions
    *c = __builtin_amdgcn_cosf(u);
    return __builtin_amdgcn_sinf(u);
}

// ----------------------------------------------------------------- grid
template <class R>
__device__ __forceinline__ void fields_from_rec(const GridDev& g, const CellRec& r, Fields<R>& f) {
    f.v[0] = R(r.lo.x); f.v[1] = R(r.lo.y); f.v[2] = R(r.lo.z);
    if constexpr (sizeof(R) == 8) {
        const double n = double(r.lo.w);
        if (n > 0.0) {
            const double T = double(r.hi.x);
            const double vth = sqrt(kVth2PerT * T);
            f.vth = vth;
            f.a = kDampTimesVth / vth;
            f.k0 = n * (kSigma0TimesVth / vth);
            f.kd = g.sigma_d * n;
        } else {
            f.vth = 1.0; f.a = 0.0; f.k0 = 0.0; f.kd = 0.0;
        }
    } else {
        const float n = r.lo.w;
        if (n > 0.0f) {
            f.vth = r.hi.y;
            f.a = r.hi.z;
            f.k0 = double(r.hi.w);
            f.kd = g.sigma_d * double(n);
        } else {
            f.vth = 1.0f; f.a = 0.0f; f.k0 = 0.0; f.kd = 0.0;
        }
    }
}

__device__ __forceinline__ uint64_t cell_index(const GridDev& g, const int c[3]) {
    return (uint64_t(c[2]) * uint64_t(g.ny) + uint64_t(c[1])) * uint64_t(g.nx) + uint64_t(c[0]);
}

template <class R>
__device__ __forceinline__ void grid_fields(const GridDev& g, const int c[3], Fields<R>& f) {
    fields_from_rec<R>(g, g.rec[cell_index(g, c)], f);
}

// Hubble flow of a grid medium: the cross-section is taken in the frame of
// the gas (Section 2.2), which moves with the expansion, v(p) = v_cell +
// H (p - href); along a flight the gas-frame frequency drifts by -H per unit
// length.  Sub-cell stepping (Section 3.4): a cell crossing of length t is
// cut into n equal steps, n the smallest with H t / n <= hstep v_th, each
// with the profile at its midpoint.
__device__ __forceinline__ void hubble_velocity(const GridDev& g, const double p[3], double vh[3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) vh[i] = g.hubble * (p[i] - g.href[i]);
}
__device__ __forceinline__ int hubble_steps(const GridDev& g, double t, double vth) {
    const double r = g.hubble * t / (g.hstep * vth);
    return r > 1.0 ? int(ceil(r)) : 1;
}
// The cell fields with the gas velocity of point p (cell velocity + Hubble flow).
template <class R>
__device__ __forceinline__ Fields<R> with_hubble(const GridDev& g, const Fields<R>& f, const double p[3]) {
    Fields<R> o = f;
    double vh[3];
    hubble_velocity(g, p, vh);
#pragma unroll
    for (int i = 0; i < 3; ++i) o.v[i] = R(double(f.v[i]) + vh[i]);
    return o;
}
// Optical depth of a peel-ray segment of length t along an axis in a Hubble
// flow: u0 is the gas-frame offset (cm/s) at the segment's start.
template <class R>
__device__ __forceinline__ double hubble_segment_tau(const GridDev& g, double u0, double t, R vth, R a, double k0,
                                                     double kd) {
    const int n = hubble_steps(g, t, double(vth));
    const double ds = t / n;
    double tau = 0.0;
    for (int j = 0; j < n; ++j) {
        const R x = R((u0 - g.hubble * ((j + 0.5) * ds)) / double(vth));
        tau += (k0 * double(voigt<R>(a, x)) + kd) * ds;
    }
    return tau;
}

// choose among three values without indexing a private array
template <class T> __device__ __forceinline__ T sel3(int a, T x, T y, T z) {
    return a == 0 ? x : (a == 1 ? y : z);
}

// f(integral_constant<int, i>) for i = 0 .. N-1: per-observer arrays of a
// lane are then indexed by constants and stay in registers
template <int N, class F> __device__ __forceinline__ void static_for(F&& f) {
    if constexpr (N > 0) {
        static_for<N - 1>(f);
        f(std::integral_constant<int, N - 1>{});
    }
}

// distance to the next cell face; *mask = axes whose face is hit first.
// FP64: (face - p) / k as in the reference; FP32 path: (face - p) * (1/k).
template <class R>
__device__ __forceinline__ double grid_step(const GridDev& g, const double p[3], const int c[3], const R k[3],
                                            const double ik[3], int* mask) {
    double tm[3];
    double tmin = __builtin_inf();
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const double kk = double(k[ax]);
        const double face = kk > 0.0 ? g.lo[ax] + double(c[ax] + 1) * g.dx[ax] : g.lo[ax] + double(c[ax]) * g.dx[ax];
        if (kk != 0.0) tm[ax] = sizeof(R) == 8 ? (face - p[ax]) / kk : (face - p[ax]) * ik[ax];
        else tm[ax] = __builtin_inf();
        tmin = tm[ax] < tmin ? tm[ax] : tmin;
    }
    int mk = 0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) mk |= (tm[ax] == tmin) ? (1 << ax) : 0;
    *mask = mk;
    return tmin < 0.0 ? 0.0 : tmin;
}

// apply a full segment; returns true when the packet leaves the grid
template <class R>
__device__ __forceinline__ bool grid_advance(const GridDev& g, double p[3], int c[3], const R k[3], double t, int mask) {
#pragma unroll
    for (int i = 0; i < 3; ++i) p[i] += t * double(k[i]);
    bool out = false;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        if (mask & (1 << ax)) {
            if (k[ax] > R(0)) { c[ax] += 1; p[ax] = g.lo[ax] + double(c[ax]) * g.dx[ax]; }
            else { c[ax] -= 1; p[ax] = g.lo[ax] + double(c[ax] + 1) * g.dx[ax]; }
        }
    }
    const int dims[3] = {g.nx, g.ny, g.nz};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) out |= (c[ax] < 0) | (c[ax] >= dims[ax]);
    return out;
}

// ----------------------------------------------------------------- meshless
// Exit distance from a sphere of radius R0 along k: the far root of
// |p + t k|^2 = R0^2 (a point rounded just outside while moving inwards still
// crosses the sphere; a point outside moving away exits at once).
__device__ __forceinline__ double sphere_exit(const double p[3], const double k[3], double R0) {
    const double b = dot3d(p, k);
    const double c = dot3d(p, p) - R0 * R0;
    const double disc = b * b - c;
    if (disc <= 0.0) return 0.0;
    const double q = sqrt(disc);
    if (b <= 0.0) return q - b;
    return c < 0.0 ? -c / (q + b) : 0.0;
}

template <class R>
__device__ __forceinline__ void meshless_velocity(const ModelDev& m, const double q[3], R v[3]) {
    v[0] = v[1] = v[2] = R(0);
    if (m.v_profile == kVelNone) return;
    if (m.kind == kGeomSlab) { v[2] = R(m.v_max * q[2] / m.r_out); return; }
    if (m.v_profile == kVelConstRadial) {
        const double r = sqrt(dot3d(q, q));
        if (r > 0.0) {
#pragma unroll
            for (int i = 0; i < 3; ++i) v[i] = R(m.v_max * q[i] / r);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 3; ++i) v[i] = R(m.v_max * q[i] / m.r_out);
    }
}

// segment of the meshless medium: boundary distance, limiter sub-step and
// midpoint fields; *cross = 1 when the segment ends on a boundary.
template <class R>
__device__ __forceinline__ double meshless_query(const ModelDev& m, const double p[3], int region, const R kR[3],
                                                 Fields<R>& f, int* next, int* cross) {
    const double k[3] = {double(kR[0]), double(kR[1]), double(kR[2])};
    double t;
    int nxt;
    if (m.kind == kGeomSlab) {
        if (k[2] > 0.0) t = (m.r_out - p[2]) / k[2];
        else if (k[2] < 0.0) t = (-m.r_out - p[2]) / k[2];
        else t = __builtin_inf();
        t = t < 0.0 ? 0.0 : t;
        nxt = kRegOut;
    } else if (region == kRegCavity) {
        t = sphere_exit(p, k, m.r_in);
        nxt = kRegGas;
    } else {
        t = sphere_exit(p, k, m.r_out);
        nxt = kRegOut;
        if (m.r_in > 0.0) {
            const double b = dot3d(p, k);
            const double ci = dot3d(p, p) - m.r_in * m.r_in;
            const double disc = b * b - ci;
            if (b < 0.0 && disc > 0.0) {
                double tin = ci / (-b + sqrt(disc));
                tin = tin < 0.0 ? 0.0 : tin;
                if (tin < t) { t = tin; nxt = kRegCavity; }
            }
        }
    }
    *cross = 1;
    if (region == kRegCavity) {
        f.vth = R(1); f.a = R(0); f.k0 = 0.0; f.kd = 0.0;
        f.v[0] = f.v[1] = f.v[2] = R(0);
        *next = nxt;
        return t;
    }
    f.vth = R(m.vth); f.a = R(m.a); f.k0 = m.k0; f.kd = m.kd;
    if (m.v_profile != kVelNone && m.v_max != 0.0) {
        double scale;
        if (m.kind == kGeomSlab || m.v_profile == kVelLinear) {
            scale = m.r_out;
        } else {
            const double r = sqrt(dot3d(p, p));
            scale = r > 1e-6 * m.r_out ? r : 1e-6 * m.r_out;
        }
        const double lmax = m.step_f * m.vth * scale / fabs(m.v_max);
        if (t > lmax) { t = lmax; *cross = 0; nxt = region; }
        double mid[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) mid[i] = p[i] + 0.5 * t * k[i];
        meshless_velocity<R>(m, mid, f.v);
    } else {
        f.v[0] = f.v[1] = f.v[2] = R(0);
    }
    *next = nxt;
    return t;
}

__device__ __forceinline__ int meshless_locate(const ModelDev& m, const double p[3]) {
    if (m.kind == kGeomSlab) return fabs(p[2]) < m.r_out ? kRegGas : kRegOut;
    const double r = sqrt(dot3d(p, p));
    return r < m.r_in ? kRegCavity : (r < m.r_out ? kRegGas : kRegOut);
}

// ----------------------------------------------------------------- ray location
struct Loc {
    double p[3];
    int c[3];
    int region;
};

// Fields of the cell a grid ray is in, reused while it stays there.
template <class R> struct CellCache {
    int c[3];
    bool valid;
    Fields<R> f;
};

// Peel seeds (the paper's peel-seed buffer, Section 3.4.1).  The transport
// kernel finishes each peel ray's first segment at the event and writes the
// rays that go on to a seed buffer in HBM; a separate kernel with a small
// register footprint (high occupancy) marches them.  Each lane writes into its
// own run of `chunk` consecutive slots, so it never waits for the rest of its
// wave between events; runs are claimed for all lanes of a wave that need one
// with a single atomic.  Slots left unused stay empty (obs < 0) and the pass
// skips them, clearing every slot it reads.
struct alignas(16) PeelSeed {
    int32_t c[3];      // front cell: the cell after the event's cell
    int32_t obs;       // observer index; -1 marks an empty slot
    double tau;        // tau of the first segment
    double dv;         // peeled lab-frame frequency
    double w;          // weight
    uint64_t cube;     // cube element the contribution goes to
};
static_assert(sizeof(PeelSeed) == 48, "seed layout");

struct SeedBuf {
    PeelSeed* s;
    uint64_t cap;                  // slots
    unsigned long long* count;     // slots claimed this step
    unsigned long long* parked;    // waves with a lane stopped by a full buffer
    uint32_t chunk;                // slots a lane claims at a time, >= observers
    const uint32_t* order;         // peel pass: slots in this order (null: buffer order)
    uint32_t* keys;                // sort key of each written slot (null: none kept)
    uint32_t key_blocks;           // pencil blocks of one axis in the keys
};

// observers the seed path serves (more go through the inline march)
constexpr int kMaxSeedObs = 3;

struct SeedLane {                  // a lane's current run of claimed slots
    uint64_t cur;
    uint32_t left;
};

// default slots per claim: about twenty events of three rays
constexpr uint32_t kSeedChunk = 64;

template <class R>
__device__ __forceinline__ void cached_fields(const GridDev& g, const int c[3], CellCache<R>& cc) {
    if (!(cc.valid && cc.c[0] == c[0] && cc.c[1] == c[1] && cc.c[2] == c[2])) {
        grid_fields<R>(g, c, cc.f);
        cc.c[0] = c[0]; cc.c[1] = c[1]; cc.c[2] = c[2];
        cc.valid = true;
    }
}

// ----------------------------------------------------------------- peeling
__device__ __forceinline__ void obs_dir(int axis, double k[3]) {
    const int a = axis % 3;
    const double s = axis < 3 ? 1.0 : -1.0;
    k[0] = a == 0 ? s : 0.0;
    k[1] = a == 1 ? s : 0.0;
    k[2] = a == 2 ? s : 0.0;
}

__device__ __forceinline__ void obs_image(int axis, const double p[3], double* u, double* v) {
    const int a = axis % 3;
    *u = sel3(a, p[1], p[2], p[0]);
    *v = sel3(a, p[2], p[0], p[1]);
}

__device__ __forceinline__ int bin_of(double v, double lo, double w, int nb) {
    const double b = floor((v - lo) / w);
    return (b >= 0.0 && b < double(nb)) ? int(b) : -1;
}

// A peel contribution c >= 0 into cube element idx: a float32 atomic add, or
// in the fixed-point mode an integer add of c rounded to units of
// 1/fx_scale (integer sums do not depend on the order of the additions).
__device__ __forceinline__ unsigned long long to_fixed(const OutDev& o, double c) {
    return (unsigned long long)(c * o.fx_scale + 0.5);
}
__device__ __forceinline__ void cube_add(const OutDev& o, uint64_t idx, double c) {
    if (o.cube_fx) atomicAdd(o.cube_fx + idx, to_fixed(o, c));
    else unsafeAtomicAdd(o.cube + idx, float(c));
}

// Contribution weight * exp(-tau) of a finished ray into its observer cube
// at the pixel of the event position and the bin of the peeled frequency.
__device__ __forceinline__ void peel_deposit(const OutDev& o, int obs, int axis, const double p[3], double dv_peel,
                                             double weight, double tau, Counters& cnt) {
    double u, v;
    obs_image(axis, p, &u, &v);
    const int ix = bin_of(u, o.img_lo[0], o.img_w[0], o.cube_nx);
    const int iy = bin_of(v, o.img_lo[1], o.img_w[1], o.cube_ny);
    const int ib = bin_of(dv_peel, o.v_lo, o.v_w, o.cube_nb);
    if (ix < 0 || iy < 0 || ib < 0) { cnt.peel_dropped++; return; }
    const uint64_t idx = ((uint64_t(obs) * o.cube_ny + iy) * o.cube_nx + ix) * o.cube_nb + ib;
    cube_add(o, idx, weight * exp(-tau));
}

// Peel-off ray (Section 3.4.1): tau along the observer axis from the event,
// at the fixed lab-frame frequency of the peeled photon; contribution
// weight * exp(-tau) into the observer cube.  On a grid the ray is axis
// aligned, so only one axis steps; `f0` holds the fields of the event's
// cell (the first segment).
template <class R, bool GRID>
__device__ void peel(const GridDev& g, const ModelDev& m, const OutDev& o, const Loc& L0, const Fields<R>& f0,
                     int obs, double weight, R dv_peel, Counters& cnt) {
    const int axis = o.obs_axis[obs];
    cnt.peel_contrib++;
    double tau = 0.0;
    bool cut = false;
    if constexpr (GRID) {
        // the ray runs along axis a; its cells are known in advance, so the
        // records of up to kLook cells are fetched together
        constexpr int kLook = THOR_PEEL_LOOKAHEAD;
        const int a = axis % 3;
        const bool pos = axis < 3;
        const int dim = sel3(a, g.nx, g.ny, g.nz);
        const double lo = sel3(a, g.lo[0], g.lo[1], g.lo[2]);
        const double dx = sel3(a, g.dx[0], g.dx[1], g.dx[2]);
        const int64_t stride = (a == 0 ? int64_t(1) : (a == 1 ? int64_t(g.nx) : int64_t(g.nx) * int64_t(g.ny))) *
                               (pos ? 1 : -1);
        int ca = sel3(a, L0.c[0], L0.c[1], L0.c[2]);
        double pa = sel3(a, L0.p[0], L0.p[1], L0.p[2]);
        int64_t idx = int64_t(cell_index(g, L0.c));
        // first segment: from the event to the face, fields of the event's cell
        // (their velocity includes the Hubble flow at the event)
        const double href = sel3(a, g.href[0], g.href[1], g.href[2]);
        {
            const double face = pos ? lo + double(ca + 1) * dx : lo + double(ca) * dx;
            double t = pos ? face - pa : pa - face;
            t = t < 0.0 ? 0.0 : t;
            cnt.peel_visits++;
            if (f0.k0 > 0.0 || f0.kd > 0.0) {
                const R va = sel3(a, f0.v[0], f0.v[1], f0.v[2]);
                if (g.hubble > 0.0) {
                    tau += hubble_segment_tau<R>(g, double(dv_peel) - (pos ? double(va) : -double(va)), t, f0.vth,
                                                 f0.a, f0.k0, f0.kd);
                } else {
                    const R x = fdiv(dv_peel - (pos ? va : -va), f0.vth);
                    tau += (f0.k0 * double(voigt<R>(f0.a, x)) + f0.kd) * t;
                }
                cut = tau > o.tau_cut;
            }
            pa = face;
            ca += pos ? 1 : -1;
            idx += stride;
        }
        while (!cut) {
            const int left = pos ? dim - ca : ca + 1;
            if (left <= 0) break;
            const int m = left < kLook ? left : kLook;
            CellRec r[kLook];
#pragma unroll
            for (int j = 0; j < kLook; ++j)
                if (j < m) r[j] = g.rec[idx + int64_t(j) * stride];
#pragma unroll
            for (int j = 0; j < kLook; ++j) {
                if (j >= m || cut) break;
                const int cj = ca + (pos ? j : -j);
                const double face = pos ? lo + double(cj + 1) * dx : lo + double(cj) * dx;
                const double t = pos ? face - pa : pa - face;
                cnt.peel_visits++;
                Fields<R> f;
                fields_from_rec<R>(g, r[j], f);
                if (f.k0 > 0.0 || f.kd > 0.0) {
                    const R va = sel3(a, f.v[0], f.v[1], f.v[2]);
                    if (g.hubble > 0.0) {
                        // gas-frame offset at the entry face, with the Hubble flow there
                        const double hv = g.hubble * (pa - href);
                        tau += hubble_segment_tau<R>(g, double(dv_peel) - (pos ? double(va) : -double(va)) -
                                                            (pos ? hv : -hv), t, f.vth, f.a, f.k0, f.kd);
                    } else {
                        const R x = fdiv(dv_peel - (pos ? va : -va), f.vth);
                        tau += (f.k0 * double(voigt<R>(f.a, x)) + f.kd) * t;
                    }
                    cut = tau > o.tau_cut;
                }
                pa = face;
            }
            ca += pos ? m : -m;
            idx += int64_t(m) * stride;
        }
    } else {
        double kd[3];
        obs_dir(axis, kd);
        const R k[3] = {R(kd[0]), R(kd[1]), R(kd[2])};
        Loc L = L0;
        for (;;) {
            Fields<R> f;
            int nr, cm;
            const double t = meshless_query<R>(m, L.p, L.region, k, f, &nr, &cm);
            cnt.peel_visits++;
            if (f.k0 > 0.0 || f.kd > 0.0) {
                const R x = fdiv(dv_peel - dot3<R>(f.v, k), f.vth);
                double kh = f.k0 * double(voigt<R>(f.a, x));
                if (m.nl > 1) kh += second_line_k<R>(m, f.k0, f.a, f.vth, x, c_dawson32);
                const double kt = kh + f.kd;
                if (isinf(t)) { cut = true; break; }
                tau += kt * t;
            } else if (isinf(t)) {
                break;
            }
            if (tau > o.tau_cut) { cut = true; break; }
#pragma unroll
            for (int i = 0; i < 3; ++i) L.p[i] += t * kd[i];
            if (cm) L.region = nr;
            if (L.region == kRegOut) break;
        }
    }
    if (cut) { cnt.peel_cut++; return; }
    peel_deposit(o, obs, axis, L0.p, double(dv_peel), weight, tau, cnt);
}

// First segment of a grid peel ray (from the event to the face of its cell,
// fields f0 of that cell), the same arithmetic as in `peel`.  Finishes the
// ray when tau already exceeds the cut or the next cell is outside the grid;
// otherwise returns true with tau so far, and the rest of the ray is marched
// from the next cell by the wave (ring or cooperative groups).
template <class R>
__device__ __forceinline__ bool peel_first(const GridDev& g, const OutDev& o, const Loc& L0, const Fields<R>& f0,
                                           int obs, double weight, R dv_peel, Counters& cnt, double* tau_out) {
    const int axis = o.obs_axis[obs];
    const int a = axis % 3;
    const bool pos = axis < 3;
    cnt.peel_contrib++;
    cnt.peel_visits++;
    const int dim = sel3(a, g.nx, g.ny, g.nz);
    const double lo = sel3(a, g.lo[0], g.lo[1], g.lo[2]);
    const double dx = sel3(a, g.dx[0], g.dx[1], g.dx[2]);
    const int ca = sel3(a, L0.c[0], L0.c[1], L0.c[2]);
    const double pa = sel3(a, L0.p[0], L0.p[1], L0.p[2]);
    const double face = pos ? lo + double(ca + 1) * dx : lo + double(ca) * dx;
    double t = pos ? face - pa : pa - face;
    t = t < 0.0 ? 0.0 : t;
    double tau = 0.0;
    if (f0.k0 > 0.0 || f0.kd > 0.0) {
        const R va = sel3(a, f0.v[0], f0.v[1], f0.v[2]);
        if (g.hubble > 0.0) {
            // f0's velocity includes the Hubble flow at the event
            tau = hubble_segment_tau<R>(g, double(dv_peel) - (pos ? double(va) : -double(va)), t, f0.vth, f0.a,
                                        f0.k0, f0.kd);
        } else {
            const R x = fdiv(dv_peel - (pos ? va : -va), f0.vth);
            // a sure cut needs no profile: the same test on a lower bound of H
            // (each step of the expression is monotone in H)
            if ((f0.k0 * double(voigt_floor(float(f0.a), float(x))) + f0.kd) * t > o.tau_cut) {
                cnt.peel_cut++;
                return false;
            }
            tau = (f0.k0 * double(voigt<R>(f0.a, x)) + f0.kd) * t;
        }
        if (tau > o.tau_cut) { cnt.peel_cut++; return false; }
    }
    const int nxt = ca + (pos ? 1 : -1);
    if (nxt < 0 || nxt >= dim) {
        peel_deposit(o, obs, axis, L0.p, double(dv_peel), weight, tau, cnt);
        return false;
    }
    *tau_out = tau;
    return true;
}

// Cube element of a ray (pixel of the event position, bin of the peeled
// frequency), or -1 when it falls outside the cube.
__device__ __forceinline__ int64_t cube_index(const OutDev& o, int obs, int axis, const double p[3], double dv) {
    double u, v;
    obs_image(axis, p, &u, &v);
    const int ix = bin_of(u, o.img_lo[0], o.img_w[0], o.cube_nx);
    const int iy = bin_of(v, o.img_lo[1], o.img_w[1], o.cube_ny);
    const int ib = bin_of(dv, o.v_lo, o.v_w, o.cube_nb);
    if (ix < 0 || iy < 0 || ib < 0) return -1;
    return int64_t(((uint64_t(obs) * o.cube_ny + iy) * o.cube_nx + ix) * o.cube_nb + ib);
}

// Peel ray `ob` of an event on the seed path: first segment now; a ray that
// goes on becomes a seed (returns true), unless its pixel or bin lies
// outside the cube.
template <class R>
__device__ __forceinline__ bool seed_make(const GridDev& g, const OutDev& o, const Loc& L, const Fields<R>& f, int ob,
                                          double weight, R dv_peel, Counters& cnt, PeelSeed& sd) {
    double tau;
    if (!peel_first<R>(g, o, L, f, ob, weight, dv_peel, cnt, &tau)) return false;
    const int axis = o.obs_axis[ob];
    const int64_t ci = cube_index(o, ob, axis, L.p, double(dv_peel));
    if (ci < 0) { cnt.peel_dropped++; return false; }
    const int a = axis % 3;
    const int nx = sel3(a, L.c[0], L.c[1], L.c[2]) + (axis < 3 ? 1 : -1);
    sd.c[0] = a == 0 ? nx : L.c[0];
    sd.c[1] = a == 1 ? nx : L.c[1];
    sd.c[2] = a == 2 ? nx : L.c[2];
    sd.obs = ob;
    sd.tau = tau;
    sd.dv = double(dv_peel);
    sd.w = weight;
    sd.cube = uint64_t(ci);
    return true;
}

// Sort key of a seed for the peel pass: the ray's axis, the pencil of its
// front cell and the 256-cell block of that pencil it starts in (one 4 KiB
// page of 16-byte pencil records), so that once sorted the rays a wave
// marches together run along the same pencils and pages.
__device__ __forceinline__ uint32_t seed_key(const GridDev& g, const OutDev& o, const PeelSeed& sd,
                                             uint32_t key_blocks) {
    const uint32_t nx = uint32_t(g.nx), ny = uint32_t(g.ny), nz = uint32_t(g.nz);
    const int a = sel3(sd.obs, o.obs_axis[0], o.obs_axis[1], o.obs_axis[2]) % 3;
    const uint32_t x = uint32_t(sd.c[0]), y = uint32_t(sd.c[1]), z = uint32_t(sd.c[2]);
    // pencil index and position along the pencil, as the pencil records are laid out
    const uint32_t pencil = a == 0 ? z * ny + y : (a == 1 ? z * nx + x : y * nx + x);
    const uint32_t pos = a == 0 ? x : (a == 1 ? y : z);
    const uint32_t per = ((a == 0 ? nx : (a == 1 ? ny : nz)) + 255u) >> 8;
    return uint32_t(a) * key_blocks + pencil * per + (pos >> 8);
}

// Marks the rest of a lane's run of slots, which it gives up, empty in the
// sort keys (all ones: after every ray, so the peel pass meets them last).
__device__ __forceinline__ void seed_release(const SeedBuf& sb, SeedLane& sl) {
    if (sb.keys)
        for (uint32_t i = 0; i < sl.left; ++i) sb.keys[sl.cur + i] = ~0u;
    sl.left = 0;
}

// The same, written to the lane's claimed slots (room for it was checked
// before the event), with its sort key.
template <class R>
__device__ __forceinline__ void seed_emit(const GridDev& g, const OutDev& o, const Loc& L, const Fields<R>& f, int ob,
                                          double weight, R dv_peel, Counters& cnt, const SeedBuf& sb, SeedLane& sl) {
    PeelSeed sd;
    if (!seed_make<R>(g, o, L, f, ob, weight, dv_peel, cnt, sd)) return;
    sb.s[sl.cur] = sd;
    if (sb.keys) sb.keys[sl.cur] = seed_key(g, o, sd, sb.key_blocks);
    ++sl.cur;
    --sl.left;
}

// A peel ray recorded by a serial event loop, its first segment marched
// later by whichever lane takes it (seed_make with these arguments).
template <class R> struct PeelJob {
    double p[3];
    int c[3];
    int ob;
    Fields<R> f;
    R pv;          // phase function value; the weight is pv / 2 pi
    R dvp;
};
template <class R> struct JobSink {
    PeelJob<R>* jobs;
    uint32_t n;
};

// ----------------------------------------------------------------- event draws
// Quantities of interaction `event` that depend only on the packet's key and
// the event number (the counter-based draws, Section 3.4.3), not on its
// state: a wave with few live packets evaluates them for the packets' next
// events on its idle lanes.  The inline path and the precomputation call the
// same functions below, so both give the same bits.
template <class R> __device__ __forceinline__ double tau_target(const Uni2<double>& d) {
    return sizeof(R) == 8 ? -log(1.0 - d.a) : double(-__logf(float(1.0 - d.a)));
}
template <class R> __device__ __forceinline__ R sin_of_cos(R mu) { return M<R>::sqrt(fmax(R(0), R(1) - mu * mu)); }
template <class R> __device__ __forceinline__ R uperp_rho2(R u) { return -M<R>::log(R(1) - u); }

template <class R> struct EventDraws {
    Uni2<double> typ;       // interaction choice, albedo
    double tau_t;           // optical depth target of the next flight
    R mu_hg, s_hg;          // dust: Henyey-Greenstein mu, sqrt(1 - mu^2)
    R mu_ph, s_ph;          // resonant: the phase function of the run
    R mu_dp, s_dp;          // resonant, core/wing mix outside the core: dipole
    R cphi, sphi;           // azimuth of the new direction
    R rho2, cps, sps;       // u_perp: radius^2 before core skipping, its angle
    Uni2<R> up[kPreUpar];   // first u_par proposals
};

template <class R>
__device__ __forceinline__ void event_draws(const Key& key, uint32_t event, int phase, R g_hg, EventDraws<R>& d) {
    d.typ = draw<double>(key, kSlotType, event);
    const Uni2<R> dm = draw<R>(key, kSlotMu, event);
    d.mu_hg = sample_mu<R>(kPhaseHG, dm.a, g_hg);
    d.s_hg = sin_of_cos<R>(d.mu_hg);
    d.mu_ph = sample_mu<R>(phase, dm.a, R(0));
    d.s_ph = sin_of_cos<R>(d.mu_ph);
    d.mu_dp = d.mu_ph;
    d.s_dp = d.s_ph;
    if (phase == kPhaseCoreWing) {
        d.mu_dp = sample_mu<R>(kPhaseDipole, dm.a, R(0));
        d.s_dp = sin_of_cos<R>(d.mu_dp);
    }
    d.sphi = sincos2pi<R>(dm.b, &d.cphi);
    const Uni2<R> dp = draw<R>(key, kSlotUperp, event);
    d.rho2 = uperp_rho2<R>(dp.a);
    d.sps = sincos2pi<R>(dp.b, &d.cps);
    d.tau_t = tau_target<R>(draw<double>(key, kSlotTau, event));
#pragma unroll
    for (uint32_t j = 0; j < kPreUpar; ++j) d.up[j] = draw<R>(key, kSlotUpar + j, event);
}

// ----------------------------------------------------------------- emission
// Cell of an n_HI^2-weighted emission (Section 3.4 "Emission"): the first
// index whose inclusive prefix of n_HI^2 exceeds u times the total.
__device__ __forceinline__ uint64_t emission_cell(const GridDev& g, double u) {
    const double target = u * g.cdf_total;
    uint64_t lo = 0, hi = g.ncell - 1;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (g.cdf[mid] > target) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// Generator + photon initialisation (Section 3.4 "Emission").
// Q: peel rays go to the seed buffer (sb, sl) instead of being marched here.
template <class R, bool GRID, bool Q = false>
__device__ void emit(const GridDev& g, const ModelDev& m, const OutDev& o, uint64_t id, uint64_t q, int model,
                     Pkt<R>& pk, Counters& cnt, const SeedBuf* sb = nullptr, SeedLane* sl = nullptr) {
    const Key key{m.seed, m.req, uint32_t(id), uint32_t(id >> 32)};
    pk.id = id; pk.q = q; pk.model = model;
    pk.event = 0; pk.n_res = 0; pk.n_dust = 0;
    {
        const Uni2<R> d = draw<R>(key, kSlotEDir, 0);
        const R mu = R(2) * d.a - R(1);
        R cphi;
        const R sphi = sincos2pi<R>(d.b, &cphi);
        const R st = M<R>::sqrt(fmax(R(0), R(1) - mu * mu));
        pk.k[0] = st * cphi; pk.k[1] = st * sphi; pk.k[2] = mu;
    }
    Loc L;
    if (GRID && m.src_kind == kSrcCellN2) {
        const Uni2<double> d1 = draw<double>(key, kSlotECell, 0);
        const Uni2<double> d2 = draw<double>(key, kSlotEOffs, 0);
        const uint64_t lo = emission_cell(g, d1.a);
        L.c[0] = int(lo % uint64_t(g.nx));
        L.c[1] = int((lo / uint64_t(g.nx)) % uint64_t(g.ny));
        L.c[2] = int(lo / (uint64_t(g.nx) * uint64_t(g.ny)));
        const double off[3] = {d1.b, d2.a, d2.b};
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) L.p[ax] = g.lo[ax] + (double(L.c[ax]) + off[ax]) * g.dx[ax];
        L.region = kRegGas;
    } else {
#pragma unroll
        for (int i = 0; i < 3; ++i) L.p[i] = m.pos[i];
        if constexpr (GRID) {
            const int dims[3] = {g.nx, g.ny, g.nz};
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                int c = int(floor((L.p[ax] - g.lo[ax]) / g.dx[ax]));
                c = c < 0 ? 0 : (c >= dims[ax] ? dims[ax] - 1 : c);
                L.c[ax] = c;
            }
            L.region = kRegGas;
        } else {
            L.region = meshless_locate(m, L.p);
            L.c[0] = L.c[1] = L.c[2] = 0;
        }
    }
    Fields<R> f0;
    if (L.region == kRegOut) {
        f0.vth = R(1); f0.a = R(0); f0.k0 = 0.0; f0.kd = 0.0; f0.v[0] = f0.v[1] = f0.v[2] = R(0);
    } else if constexpr (GRID) {
        grid_fields<R>(g, L.c, f0);
        if (g.hubble > 0.0) f0 = with_hubble<R>(g, f0, L.p);
    } else {
        int nr, cm;
        (void)meshless_query<R>(m, L.p, L.region, pk.k, f0, &nr, &cm);
    }
    R z = R(0), uflat = R(0);
    if (m.spectrum != kSpecDelta) {
        const Uni2<R> d = draw<R>(key, kSlotEGauss, 0);
        if (m.spectrum == kSpecFlat) {
            uflat = d.a;
        } else {
            R cs;
            (void)sincos2pi<R>(d.b, &cs);
            z = M<R>::sqrt(R(-2) * M<R>::log(R(1) - d.a)) * cs;
        }
    }
    // a doublet source emits in line 1 with probability 1 - lw0, at its centre
    R lcen = R(0);
    if (m.lines && m.nl > 1 && draw<double>(key, kSlotELine, 0).a >= m.lw0) lcen = R(m.lc1);
    R dv_loc = R(0);
    if (m.spectrum == kSpecThermal) {
        dv_loc = R(m.dv0) + f0.vth * z / R(1.4142135623730951) + lcen;
        pk.dv = dv_loc + dot3<R>(f0.v, pk.k);
    } else if (m.spectrum == kSpecGauss) {
        pk.dv = R(m.dv0) + R(m.sigma_v) * z + lcen;
    } else if (m.spectrum == kSpecFlat) {
        pk.dv = R(m.dv0) + R(m.sigma_v) * (R(2) * uflat - R(1)) + lcen;   // flat continuum dv0 +- sigma_v
    } else {
        pk.dv = R(m.dv0) + lcen;
    }
    cnt.emitted++;
    if (L.region != kRegOut) {
        if constexpr (GRID && Q) {
            {
                static_for<kMaxSeedObs>([&](auto obc) {
                    constexpr int ob = decltype(obc)::value;
                    if (ob < o.n_obs) {
                        double kd[3];
                        obs_dir(o.obs_axis[ob], kd);
                        const R ko[3] = {R(kd[0]), R(kd[1]), R(kd[2])};
                        const R dvp = (m.spectrum == kSpecThermal) ? dv_loc + dot3<R>(f0.v, ko) : pk.dv;
                        seed_emit<R>(g, o, L, f0, ob, 1.0 / (4.0 * kPi), dvp, cnt, *sb, *sl);
                    }
                });
            }
        }
        if constexpr (!(GRID && Q)) {
            for (int ob = 0; ob < o.n_obs; ++ob) {
                double kd[3];
                obs_dir(o.obs_axis[ob], kd);
                const R ko[3] = {R(kd[0]), R(kd[1]), R(kd[2])};
                const R dvp = (m.spectrum == kSpecThermal) ? dv_loc + dot3<R>(f0.v, ko) : pk.dv;
                peel<R, GRID>(g, m, o, L, f0, ob, 1.0 / (4.0 * kPi), dvp, cnt);
            }
        }
    }
    const Uni2<double> dt = draw<double>(key, kSlotETau, 0);
    pk.tau_t = tau_target<R>(dt);
    pk.tau_a = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) { pk.p[i] = L.p[i]; pk.c[i] = L.c[i]; }
    pk.region = L.region;
}

// ----------------------------------------------------------------- interaction
// Dust (Section 2.3.2) or resonant scattering (Sections 2.3.1, 3.4, 3.4.2)
// at location L in a cell with fields f; kt is the total opacity there.
// Returns kFateAbsorbed or kFateNone; peels off to every observer.  PRE:
// `pre` holds this event's draws evaluated ahead (event_draws).
template <class R, bool GRID, bool Q, bool PRE = false>
__device__ __forceinline__ int interact(const GridDev& g, const ModelDev& m, const OutDev& o, Pkt<R>& pk,
                                        const Loc& L, const Fields<R>& f, double kt, const Key& key,
                                        Counters& cnt, const SeedBuf* sb, SeedLane* sl,
                                        const EventDraws<R>* pre = nullptr, JobSink<R>* js = nullptr) {
    Uni2<double> dtyp;
    if constexpr (PRE) dtyp = pre->typ; else dtyp = draw<double>(key, kSlotType, pk.event);
    R kout[3], e1[3], e2[3];
    if (dtyp.a * kt < f.kd) {
        if (dtyp.b >= m.albedo) return kFateAbsorbed;
        R mu, s_, cphi, sphi;
        if constexpr (PRE) {
            mu = pre->mu_hg; s_ = pre->s_hg; cphi = pre->cphi; sphi = pre->sphi;
        } else {
            const Uni2<R> dm = draw<R>(key, kSlotMu, pk.event);
            mu = sample_mu<R>(kPhaseHG, dm.a, R(m.g_hg));
            s_ = sin_of_cos<R>(mu);
            sphi = sincos2pi<R>(dm.b, &cphi);
        }
        const R dvl = pk.dv - dot3<R>(f.v, pk.k);
        onb<R>(pk.k, e1, e2);
#pragma unroll
        for (int i = 0; i < 3; ++i) kout[i] = mu * pk.k[i] + s_ * (cphi * e1[i] + sphi * e2[i]);
        if constexpr (GRID && Q) {
            static_for<kMaxSeedObs>([&](auto obc) {
                constexpr int ob = decltype(obc)::value;
                if (ob < o.n_obs) {
                    double kd[3];
                    obs_dir(o.obs_axis[ob], kd);
                    const R ko[3] = {R(kd[0]), R(kd[1]), R(kd[2])};
                    const R pv = phase_value<R>(kPhaseHG, dot3<R>(pk.k, ko), R(m.g_hg));
                    if constexpr (PRE) {
                        js->jobs[js->n++] = PeelJob<R>{{L.p[0], L.p[1], L.p[2]}, {L.c[0], L.c[1], L.c[2]}, ob, f, pv,
                                                       R(dvl + dot3<R>(f.v, ko))};
                    } else {
                        seed_emit<R>(g, o, L, f, ob, double(pv) / (2.0 * kPi), dvl + dot3<R>(f.v, ko), cnt, *sb, *sl);
                    }
                }
            });
        } else {
            for (int ob = 0; ob < o.n_obs; ++ob) {
                double kd[3];
                obs_dir(o.obs_axis[ob], kd);
                const R ko[3] = {R(kd[0]), R(kd[1]), R(kd[2])};
                const double c = double(phase_value<R>(kPhaseHG, dot3<R>(pk.k, ko), R(m.g_hg))) / (2.0 * kPi);
                peel<R, GRID>(g, m, o, L, f, ob, c, dvl + dot3<R>(f.v, ko), cnt);
            }
        }
        pk.dv = dvl + dot3<R>(f.v, kout);
        pk.n_dust++;
        cnt.n_dust++;
    } else {
        R x = fdiv(pk.dv - dot3<R>(f.v, pk.k), f.vth);
        R aj = f.a;
        int line = 0;
        if constexpr (!GRID && !PRE) {
            if (m.nl > 1) {
                // a doublet scatters in line 1 with probability k_1 / (k_0 + k_1)
                // at the site (the same uniform rescaled to the resonant share)
                // and re-emits in that line; h (2P1/2) re-emits isotropically
                const double k_first = f.k0 * double(voigt<R>(f.a, x));
                const double kres = k_first + second_line_k<R>(m, f.k0, f.a, f.vth, x, c_dawson32);
                const double u_line = (dtyp.a * kt - f.kd) / (kt - f.kd);
                if (u_line * kres >= k_first) {
                    line = 1;
                    x = R(m.lrho1) * (x - R(m.lc1) / f.vth);
                    aj = f.a * R(m.lam1);
                }
            }
        }
        uint32_t trials = 0;
        const R upar = upar_sample<R>(x, aj, key, pk.event, &trials, PRE ? pre->up : nullptr);
        cnt.upar_trials += trials;
        R rho2, cps, sps;
        if constexpr (PRE) {
            rho2 = pre->rho2; cps = pre->cps; sps = pre->sps;
        } else {
            const Uni2<R> dp = draw<R>(key, kSlotUperp, pk.event);
            rho2 = uperp_rho2<R>(dp.a);
            sps = sincos2pi<R>(dp.b, &cps);
        }
        if (m.xcrit > 0.0 && fabs(x) < R(m.xcrit)) rho2 += R(m.xcrit * m.xcrit);
        const R rho = M<R>::sqrt(rho2);
        const R up1 = rho * cps, up2 = rho * sps;
        onb<R>(pk.k, e1, e2);
        R u[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) u[i] = upar * pk.k[i] + up1 * e1[i] + up2 * e2[i];
        const R x_atom = x - upar;
        int ph = line ? int(kPhaseIso) : o.phase;
        if (ph == kPhaseCoreWing && fabs(x_atom) >= R(0.2)) ph = kPhaseDipole;
        R mu, s_, cphi, sphi;
        if constexpr (PRE) {
            const bool wing = ph != o.phase;
            mu = wing ? pre->mu_dp : pre->mu_ph;
            s_ = wing ? pre->s_dp : pre->s_ph;
            cphi = pre->cphi; sphi = pre->sphi;
        } else {
            const Uni2<R> dm = draw<R>(key, kSlotMu, pk.event);
            mu = sample_mu<R>(ph, dm.a, R(0));
            s_ = sin_of_cos<R>(mu);
            sphi = sincos2pi<R>(dm.b, &cphi);
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) kout[i] = mu * pk.k[i] + s_ * (cphi * e1[i] + sphi * e2[i]);
        if constexpr (GRID && Q) {
            static_for<kMaxSeedObs>([&](auto obc) {
                constexpr int ob = decltype(obc)::value;
                if (ob < o.n_obs) {
                    double kd[3];
                    obs_dir(o.obs_axis[ob], kd);
                    const R ko[3] = {R(kd[0]), R(kd[1]), R(kd[2])};
                    const R pv = phase_value<R>(ph, dot3<R>(pk.k, ko), R(0));
                    const R xo = x_atom + dot3<R>(u, ko);
                    if constexpr (PRE) {
                        js->jobs[js->n++] = PeelJob<R>{{L.p[0], L.p[1], L.p[2]}, {L.c[0], L.c[1], L.c[2]}, ob, f, pv,
                                                       R(xo * f.vth + dot3<R>(f.v, ko))};
                    } else {
                        seed_emit<R>(g, o, L, f, ob, double(pv) / (2.0 * kPi), xo * f.vth + dot3<R>(f.v, ko), cnt,
                                     *sb, *sl);
                    }
                }
            });
        } else {
            for (int ob = 0; ob < o.n_obs; ++ob) {
                double kd[3];
                obs_dir(o.obs_axis[ob], kd);
                const R ko[3] = {R(kd[0]), R(kd[1]), R(kd[2])};
                const double c = double(phase_value<R>(ph, dot3<R>(pk.k, ko), R(0))) / (2.0 * kPi);
                const R xo = x_atom + dot3<R>(u, ko);
                const R dvo = line ? (xo / R(m.lrho1)) * f.vth + R(m.lc1) + dot3<R>(f.v, ko)
                                   : xo * f.vth + dot3<R>(f.v, ko);
                peel<R, GRID>(g, m, o, L, f, ob, c, dvo, cnt);
            }
        }
        const R x_out = x_atom + dot3<R>(u, kout);
        if (line) pk.dv = (x_out / R(m.lrho1)) * f.vth + R(m.lc1) + dot3<R>(f.v, kout);
        else pk.dv = x_out * f.vth + dot3<R>(f.v, kout);
        pk.n_res++;
        cnt.n_res++;
    }
    if constexpr (sizeof(R) == 4) {   // FP32 directions drift: renormalise
        const R inv = rsqrtf(dot3<R>(kout, kout));
#pragma unroll
        for (int i = 0; i < 3; ++i) kout[i] *= inv;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) pk.k[i] = kout[i];
    if constexpr (PRE) pk.tau_t = pre->tau_t; else pk.tau_t = tau_target<R>(draw<double>(key, kSlotTau, pk.event));
    pk.tau_a = 0.0;
    return kFateNone;
}

// ----------------------------------------------------------------- march
// Advance a packet by at most `max_visits` march segments and `max_events`
// interactions (propagation, Section 3.4: piecewise-linear tau integration
// until tau_current = tau_target, then the interaction).  Returns the fate
// (kFateNone while it lives on); the packet state is complete on return, so
// a later call resumes it exactly.  PRE: `pre` holds the draws of events
// pre_event, pre_event + 1, ... evaluated ahead; max_events must not run
// past them; `dtab` is the FP32 Dawson table the march reads (an LDS copy
// in the persistent and tail kernels).
// refill (persistent waves, 1..63): the call also ends once refill/64 of the
// lanes that entered it have left, so that the wave refills them without
// waiting for its longest flight (0 or 64: only at the visit bound).
// park (persistent waves, > 0): a lane that reaches its interaction site
// waits there, its position, opacity and cell fields kept, while the other
// lanes march on; the waiting lanes interact together once `park` of them
// wait, once no lane is marching, or when the call ends.  Each packet's
// arithmetic and its order are unchanged (the same histories); the wave runs
// the long interaction code for many lanes at once instead of for the few
// that happen to interact at the same march step.
template <class R, bool GRID, bool Q = false, bool PRE = false>
__device__ int advance(const GridDev& g, const ModelDev& m, const OutDev& o, Pkt<R>& pk, Counters& cnt,
                       uint32_t max_visits, uint32_t max_events, uint32_t* events_done,
                       const SeedBuf* sb = nullptr, SeedLane* sl = nullptr, CellCache<R>* ccp = nullptr,
                       const EventDraws<R>* pre = nullptr, uint32_t pre_event = 0, JobSink<R>* js = nullptr,
                       const float* dtab = c_dawson32, uint32_t refill = 0, uint32_t park = 0) {
    const Key key{m.seed, m.req, uint32_t(pk.id), uint32_t(pk.id >> 32)};
    Loc L;
#pragma unroll
    for (int i = 0; i < 3; ++i) { L.p[i] = pk.p[i]; L.c[i] = pk.c[i]; }
    L.region = pk.region;
    if (L.region == kRegOut) return kFateEscaped;
    // the seed path keeps the cell cache across calls (one event per call)
    CellCache<R> cc_local;
    cc_local.valid = false;
    CellCache<R>& cc = Q ? *ccp : cc_local;
    double ik[3];
    auto set_inverse = [&]() {
        if constexpr (sizeof(R) == 4) {
#pragma unroll
            for (int i = 0; i < 3; ++i) ik[i] = pk.k[i] != R(0) ? rcp64(double(pk.k[i])) : 0.0;
        }
    };
    set_inverse();
    const uint64_t emax = o.max_events ? o.max_events : 100000000ull;
    int fate = kFateNone;
    uint32_t ev = 0;
    const bool early_end = refill > 0 && refill < 64;
    // lanes that must have left before the turn ends early (at least one)
    const int n_in = early_end ? __popcll(__ballot(1)) : 0;
    const int n_leave = early_end ? max(1, int((uint32_t(n_in) * refill + 63u) >> 6)) : 0;
    // a lane at its interaction site: the opacity there and (meshless media)
    // the fields there; on a grid the cell cache keeps the site's fields
    bool parked = false;
    double kt_site = 0.0;
    Fields<R> f_site;
    if constexpr (!GRID) f_site = Fields<R>{R(1), R(0), 0.0, 0.0, {R(0), R(0), R(0)}};
    uint32_t vis = 0;
    for (;;) {
        // the call ends at the visit or event bound, or once the refill share
        // of the lanes that entered have left (finished packets wait for a refill)
        bool stop = !(vis < max_visits && ev < max_events);
        if (early_end && n_in - __popcll(__ballot(1)) >= n_leave) stop = true;
        if (!stop && !parked) {
            ++vis;
            int nr, cm;
            double t;
            Fields<R> fl;
            if constexpr (GRID) {
                t = grid_step<R>(g, L.p, L.c, pk.k, ik, &cm);
                cached_fields<R>(g, L.c, cc);
                nr = kRegGas;
            } else {
                t = meshless_query<R>(m, L.p, L.region, pk.k, fl, &nr, &cm);
            }
            const Fields<R>& f = GRID ? cc.f : fl;
            cnt.main_visits++;
            double kt = 0.0;
            double s = -1.0;            // interaction site along the segment, if any
            double tau_seg = pk.tau_a;  // tau at the end of the segment (Hubble sub-steps)
            if (GRID && g.hubble > 0.0) {
                double vh[3];
                hubble_velocity(g, L.p, vh);
                const double kd3[3] = {double(pk.k[0]), double(pk.k[1]), double(pk.k[2])};
                // gas-frame offset at the segment start
                const double u0 = double(pk.dv) - double(dot3<R>(f.v, pk.k)) - dot3d(vh, kd3);
                if (g.stop_dv > 0.0 && u0 < -g.stop_dv) { fate = kFateRedshifted; break; }
                if (f.k0 > 0.0 || f.kd > 0.0) {
                    const int n = hubble_steps(g, t, double(f.vth));
                    const double ds = t / n;
                    for (int j = 0; j < n; ++j) {
                        const R x = R((u0 - g.hubble * ((j + 0.5) * ds)) / double(f.vth));
                        double ktj;
                        if constexpr (sizeof(R) == 4) ktj = f.k0 * double(voigt32(f.a, x, dtab)) + f.kd;
                        else ktj = f.k0 * double(voigt<R>(f.a, x)) + f.kd;
                        if (tau_seg + ktj * ds >= pk.tau_t) {
                            s = j * ds + div_tau<R>(pk.tau_t - tau_seg, ktj);
                            kt = ktj;
                            break;
                        }
                        tau_seg += ktj * ds;
                    }
                }
            } else {
                if (f.k0 > 0.0 || f.kd > 0.0) {
                    const R x = fdiv(pk.dv - dot3<R>(f.v, pk.k), f.vth);
                    if constexpr (!GRID) {
                        if (m.nl > 1) {
                            // doublet: both lines' opacities (meshless media)
                            double kh;
                            if constexpr (sizeof(R) == 4) kh = f.k0 * double(voigt32(f.a, x, dtab));
                            else kh = f.k0 * double(voigt<R>(f.a, x));
                            kt = (kh + second_line_k<R>(m, f.k0, f.a, f.vth, x, dtab)) + f.kd;
                        } else {
                            if constexpr (sizeof(R) == 4) kt = f.k0 * double(voigt32(f.a, x, dtab)) + f.kd;
                            else kt = f.k0 * double(voigt<R>(f.a, x)) + f.kd;
                        }
                    } else {
                        if constexpr (sizeof(R) == 4) kt = f.k0 * double(voigt32(f.a, x, dtab)) + f.kd;
                        else kt = f.k0 * double(voigt<R>(f.a, x)) + f.kd;
                    }
                }
                if (kt > 0.0 && pk.tau_a + kt * t >= pk.tau_t) s = div_tau<R>(pk.tau_t - pk.tau_a, kt);
            }
            if (s >= 0.0) {
                if constexpr (Q && !PRE) {
                    // no room for this event's rays: end the turn before it (state
                    // unchanged); the wave claims a new run of slots
                    if (sl->left < uint32_t(o.n_obs)) break;
                }
                // interaction site where tau_current = tau_target along the step
#pragma unroll
                for (int i = 0; i < 3; ++i) L.p[i] += s * double(pk.k[i]);
                pk.event++;
                ++ev;
                if (uint64_t(pk.event) > emax) { fate = kFateCapped; break; }
                parked = true;
                kt_site = kt;
                if constexpr (!GRID) f_site = fl;
            } else {
                if (isinf(t)) { fate = kFateEscaped; break; }
                if (GRID && g.hubble > 0.0) pk.tau_a = tau_seg;
                else pk.tau_a += kt * t;
                bool out;
                if constexpr (GRID) {
                    out = grid_advance<R>(g, L.p, L.c, pk.k, t, cm);
                } else {
#pragma unroll
                    for (int i = 0; i < 3; ++i) L.p[i] += t * double(pk.k[i]);
                    if (cm) L.region = nr;
                    out = L.region == kRegOut;
                }
                if (out) { fate = kFateEscaped; break; }
            }
        }
        // when the parked lanes interact: at once without parking; with
        // parking, once `park` lanes wait, no lane marches, or the call ends
        bool go = parked;
        if (park) {
            const uint64_t pm = __ballot(parked);
            const bool marching = __ballot(!parked && !stop) != 0;
            go = parked && (stop || uint32_t(__popcll(pm)) >= park || !marching);
        }
        if (go) {
            parked = false;
            // the gas at the site moves with the cell and, on a grid in a Hubble
            // flow, with the expansion at the site
            Fields<R> fs = GRID ? cc.f : f_site;
            if (GRID && g.hubble > 0.0) fs = with_hubble<R>(g, fs, L.p);
            fate = interact<R, GRID, Q, PRE>(g, m, o, pk, L, fs, kt_site, key, cnt, sb, sl,
                                             PRE ? pre + (pk.event - pre_event) : nullptr, js);
            if (fate != kFateNone) break;
            set_inverse();
        }
        if (stop) break;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) { pk.p[i] = L.p[i]; pk.c[i] = L.c[i]; }
    pk.region = L.region;
    *events_done += ev;
    return fate;
}

// ----------------------------------------------------------------- waves
__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0u));
}

// ----------------------------------------------------------------- finish
template <class R, bool GRID>
__device__ void finish(const GridDev& g, const ModelDev& m, const OutDev& o, const Pkt<R>& pk, int fate,
                       Counters& cnt) {
    if (fate == kFateEscaped || fate == kFateRedshifted) {
        cnt.escaped++;
        if (fate == kFateRedshifted) cnt.redshifted++;
        else if (GRID && g.handoff) cnt.handed_off++;
        const int b = bin_of(double(pk.dv) * m.spec_scale, m.spec_lo, m.spec_w, m.spec_nb);
        if (b >= 0) unsafeAtomicAdd(m.spec + uint64_t(blockIdx.x % uint32_t(m.spec_rep)) * uint32_t(m.spec_nb) + b, 1.0);
    } else if (fate == kFateAbsorbed) {
        cnt.absorbed++;
    } else if (fate == kFateCapped) {
        cnt.capped++;
    }
    if (o.rec_dv) {
        const uint64_t r = pk.q - o.q_rec0;
        o.rec_dv[r] = double(pk.dv);
        o.rec_nres[r] = pk.n_res;
        o.rec_ndust[r] = pk.n_dust;
        o.rec_fate[r] = fate;
    }
    if (m.done) atomicAdd(m.done, 1ull);
    cnt.max_events = pk.event > cnt.max_events ? pk.event : cnt.max_events;
}

// ----------------------------------------------------------------- counters
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sums of the lanes' counters into g (one atomic per counter and wave); the
// longest history into *gmax when given.
__device__ __forceinline__ void flush_counters(const Counters& c, unsigned long long* g,
                                               unsigned long long* gmax = nullptr) {
    const uint64_t vals[kNumU64Counters] = {c.emitted, c.escaped, c.absorbed, c.capped, c.handed_off,
                                            c.n_res, c.n_dust, c.main_visits, c.peel_visits,
                                            c.peel_contrib, c.peel_dropped, c.peel_cut, c.upar_trials, c.redshifted};
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < kNumU64Counters; ++i) {
        const uint64_t s = wave_sum_u64(vals[i]);
        if (lane == 0 && s) atomicAdd(g + i, (unsigned long long)s);
    }
    if (gmax) {
        uint32_t mx = c.max_events;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const uint32_t o = __shfl_xor(mx, off, 64);
            mx = o > mx ? o : mx;
        }
        if (lane == 0 && mx) atomicMax(gmax, (unsigned long long)mx);
    }
}

}  // namespace thor
