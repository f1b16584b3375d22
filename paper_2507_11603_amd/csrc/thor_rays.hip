// thor_rays.hip -- the raytracing driver of libthor.so (include/thor_rays.h):
// projections and Lyman-alpha absorption spectra along rays parallel to a
// grid axis (arXiv 2507.11603, Section 3.5).
//
// Projection streams each field once from HBM: consecutive lanes take
// consecutive cells of the fastest axis, so every load of a wave is one
// contiguous run.  Absorption spectra are bound by the Voigt evaluations
// (cells x sub-steps x bins per ray): a workgroup stages one ray's cells in
// LDS and each lane owns one spectral bin, so every LDS read is a broadcast.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <string>

#include "../../include/thor_rays.h"

// Device code objects are per translation unit, so this unit carries its own
// device copy of the Dawson coefficient tables behind the Voigt functions.
#define c_dawson64 c_ray_dawson64
#define c_dawson32 c_ray_dawson32
#include "thor_device.hpp"
#undef c_dawson64
#undef c_dawson32

namespace thor {
__constant__ double c_ray_dawson64[kDawsonIntervals * (kDawsonDeg64 + 1)];
__constant__ float c_ray_dawson32[kDawsonIntervals * (kDawsonDeg32 + 1)];
}  // namespace thor

using namespace thor;

namespace {

constexpr int kThreads = 256;
constexpr int kChunk = 512;          // cells of one ray staged in LDS per pass
// Below these workgroup counts a ray is split into segments whose sums are
// added atomically.  Long per-thread column streams beat more, shorter ones:
// at 512^3 the column kernels read 5.5 TB/s unsplit (256 workgroups) and
// 3.6 TB/s split eight ways.
constexpr int kFillRows = 2048;
constexpr int kFillCols = 256;

struct RayGeo {
    int nx, ny, nz, axis;
    double ds;
};

__device__ __forceinline__ size_t ray_cell(const RayGeo& g, int i, int j, int k) {
    const int x = g.axis == 0 ? k : i;
    const int y = g.axis == 1 ? k : (g.axis == 0 ? i : j);
    const int z = g.axis == 2 ? k : j;
    return (size_t(z) * size_t(g.ny) + size_t(y)) * size_t(g.nx) + size_t(x);
}

__global__ void k_zero(double* p, size_t n) {
    const size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0.0;
}

// Rays along y or z.  The grid is [outer][ray][inner] with the inner index
// contiguous; one thread per (outer, inner) column sums its segment of the
// ray (blockIdx.y), the lanes of a wave reading consecutive inner cells.
__global__ __launch_bounds__(kThreads) void k_project_cols(
    const float* __restrict__ q, const float* __restrict__ w, size_t n_inner, size_t n_col,
    int n_ray, int seg, double ds, double* Q, double* W, bool atomic) {
    const size_t col = size_t(blockIdx.x) * kThreads + threadIdx.x;
    if (col >= n_col) return;
    const size_t o = col / n_inner, in = col - o * n_inner;
    const int k0 = int(blockIdx.y) * seg, k1 = min(n_ray, k0 + seg);
    const float* qp = q + (o * size_t(n_ray) + size_t(k0)) * n_inner + in;
    const float* wp = w ? w + (qp - q) : nullptr;
    double aq = 0.0, aw = 0.0;
    if (wp) {
        for (int k = k0; k < k1; ++k, qp += n_inner, wp += n_inner) {
            const double wv = *wp;
            aq += double(*qp) * wv;          // exact product of two floats
            aw += wv;
        }
    } else {
        for (int k = k0; k < k1; ++k, qp += n_inner) aq += double(*qp);
        aw = double(k1 - k0);
    }
    if (atomic) {
        atomicAdd(Q + col, aq * ds);
        if (W) atomicAdd(W + col, aw * ds);
    } else {
        Q[col] = aq * ds;
        if (W) W[col] = aw * ds;
    }
}

// The same with four adjacent columns per thread and 16-byte loads (the
// inner extent a multiple of 4, the fields 16-byte aligned).
__global__ __launch_bounds__(kThreads) void k_project_cols4(
    const float4* __restrict__ q, const float4* __restrict__ w, size_t n_inner4, size_t n_col4,
    int n_ray, int seg, double ds, double* Q, double* W, bool atomic) {
    const size_t c4 = size_t(blockIdx.x) * kThreads + threadIdx.x;
    if (c4 >= n_col4) return;
    const size_t o = c4 / n_inner4, in4 = c4 - o * n_inner4;
    const int k0 = int(blockIdx.y) * seg, k1 = min(n_ray, k0 + seg);
    const size_t first = (o * size_t(n_ray) + size_t(k0)) * n_inner4 + in4;
    double aq[4] = {0.0, 0.0, 0.0, 0.0}, aw[4] = {0.0, 0.0, 0.0, 0.0};
    if (w) {
#pragma unroll 4
        for (int k = k0; k < k1; ++k) {
            const size_t at = first + size_t(k - k0) * n_inner4;
            const float4 qv = q[at], wv = w[at];
            aq[0] += double(qv.x) * double(wv.x); aw[0] += double(wv.x);
            aq[1] += double(qv.y) * double(wv.y); aw[1] += double(wv.y);
            aq[2] += double(qv.z) * double(wv.z); aw[2] += double(wv.z);
            aq[3] += double(qv.w) * double(wv.w); aw[3] += double(wv.w);
        }
    } else {
#pragma unroll 4
        for (int k = k0; k < k1; ++k) {
            const float4 qv = q[first + size_t(k - k0) * n_inner4];
            aq[0] += double(qv.x); aq[1] += double(qv.y); aq[2] += double(qv.z); aq[3] += double(qv.w);
        }
        aw[0] = aw[1] = aw[2] = aw[3] = double(k1 - k0);
    }
    const size_t col = 4 * c4;                  // = o * n_inner + 4 * in4
    for (int c = 0; c < 4; ++c) {
        if (atomic) {
            atomicAdd(Q + col + c, aq[c] * ds);
            if (W) atomicAdd(W + col + c, aw[c] * ds);
        } else {
            Q[col + c] = aq[c] * ds;
            if (W) W[col + c] = aw[c] * ds;
        }
    }
}

// Rays along x: each ray is contiguous.  One wave per (ray, segment); the
// lanes stride the segment and reduce across the wave at the end.
__global__ __launch_bounds__(kThreads) void k_project_rows(
    const float* __restrict__ q, const float* __restrict__ w, size_t n_rows, int n_ray, int seg,
    double ds, double* Q, double* W, bool atomic) {
    const int lane = threadIdx.x & 63;
    const size_t row = size_t(blockIdx.x) * (kThreads / 64) + (threadIdx.x >> 6);
    if (row >= n_rows) return;              // the whole wave leaves together
    const int k0 = int(blockIdx.y) * seg, k1 = min(n_ray, k0 + seg);
    const float* qr = q + row * size_t(n_ray);
    const float* wr = w ? w + row * size_t(n_ray) : nullptr;
    double aq = 0.0, aw = 0.0;
    if (wr) {
        for (int k = k0 + lane; k < k1; k += 64) {
            const double wv = wr[k];
            aq += double(qr[k]) * wv;
            aw += wv;
        }
    } else {
        for (int k = k0 + lane; k < k1; k += 64) aq += double(qr[k]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        aq += __shfl_xor(aq, off);
        aw += __shfl_xor(aw, off);
    }
    if (!wr) aw = double(k1 - k0);
    if (lane == 0) {
        if (atomic) {
            atomicAdd(Q + row, aq * ds);
            if (W) atomicAdd(W + row, aw * ds);
        } else {
            Q[row] = aq * ds;
            if (W) W[row] = aw * ds;
        }
    }
}

// Rays along x with 16-byte loads (ray length a multiple of 4, aligned
// fields): segments are whole multiples of 64 float4 (one per lane).  The
// loop is left rolled: at 512^3 a lane takes two iterations per ray, and
// unrolling it by 4 (or summing 4 or 8 rays per wave) read 4.1, 4.9 and
// 2.6 TB/s against 5.0 TB/s.
__global__ __launch_bounds__(kThreads) void k_project_rows4(
    const float4* __restrict__ q, const float4* __restrict__ w, size_t n_rows, int n_ray4, int seg4,
    double ds, double* Q, double* W, bool atomic) {
    const int lane = threadIdx.x & 63;
    const size_t row = size_t(blockIdx.x) * (kThreads / 64) + (threadIdx.x >> 6);
    if (row >= n_rows) return;              // the whole wave leaves together
    const int k0 = int(blockIdx.y) * seg4, k1 = min(n_ray4, k0 + seg4);
    const float4* qr = q + row * size_t(n_ray4);
    const float4* wr = w ? w + row * size_t(n_ray4) : nullptr;
    double aq = 0.0, aw = 0.0;
    if (wr) {
        for (int k = k0 + lane; k < k1; k += 64) {
            const float4 qv = qr[k], wv = wr[k];
            aq += double(qv.x) * double(wv.x) + double(qv.y) * double(wv.y) +
                  (double(qv.z) * double(wv.z) + double(qv.w) * double(wv.w));
            aw += (double(wv.x) + double(wv.y)) + (double(wv.z) + double(wv.w));
        }
    } else {
        for (int k = k0 + lane; k < k1; k += 64) {
            const float4 qv = qr[k];
            aq += (double(qv.x) + double(qv.y)) + (double(qv.z) + double(qv.w));
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        aq += __shfl_xor(aq, off);
        aw += __shfl_xor(aw, off);
    }
    if (!wr) aw = 4.0 * double(k1 - k0);
    if (lane == 0) {
        if (atomic) {
            atomicAdd(Q + row, aq * ds);
            if (W) atomicAdd(W + row, aw * ds);
        } else {
            Q[row] = aq * ds;
            if (W) W[row] = aw * ds;
        }
    }
}

template <class R>
__device__ __forceinline__ R voigt_forest(R a, R x) {
    const R ax = fabs(x);
    if constexpr (sizeof(R) == 8) {
        if (ax >= 40.0) return voigt_wing<double, 4>(a, x);
        if (ax >= 20.0) return voigt_wing<double, 6>(a, x);
        if (ax >= 12.0) return voigt_wing<double, 9>(a, x);
        return voigt64(a, x);
    } else {
        return ax >= 6.5f ? voigt_wing<float, 4>(a, x) : voigt32(a, x);
    }
}

// eq. (abs): one workgroup per (ray, block of kThreads bins).  Per cell the
// LDS holds the optical depth per unit profile of one sub-step
// (n_HI sigma0 ds / n_sub), the Voigt parameter a, 1/v_th and the velocity
// v + H s of the first sub-step's midpoint; sub-step m adds m H ds / n_sub.
template <class R>
__global__ __launch_bounds__(kThreads) void k_forest(
    RayGeo g, int n_ray, const float* __restrict__ nHI, const float* __restrict__ T,
    const float* __restrict__ v, int i0, int ni, int j0, double hubble, int n_sub, uint32_t nb,
    double u_lo, double du, double* __restrict__ tau) {
    __shared__ double s_k0[kChunk], s_c[kChunk];
    __shared__ R s_a[kChunk], s_iv[kChunk];
    const uint32_t ray = blockIdx.x;
    const int i = i0 + int(ray % uint32_t(ni)), j = j0 + int(ray / uint32_t(ni));
    const uint32_t b = blockIdx.y * kThreads + threadIdx.x;
    const double u = u_lo + (double(b) + 0.5) * du;
    const double step = g.ds / double(n_sub), dc = hubble * step;
    double acc = 0.0;
    for (int kb = 0; kb < n_ray; kb += kChunk) {
        const int nc = min(kChunk, n_ray - kb);
        __syncthreads();                   // the previous chunk has been read
        for (int t = threadIdx.x; t < nc; t += kThreads) {
            const size_t c = ray_cell(g, i, j, kb + t);
            const double n = nHI[c];
            const double vth = sqrt(kVth2PerT * double(T[c]));
            const bool empty = n == 0.0;   // adds exactly zero, whatever T is
            s_k0[t] = empty ? 0.0 : n * (kSigma0TimesVth / vth) * step;
            s_a[t] = empty ? R(0) : R(kDampTimesVth / vth);
            s_iv[t] = empty ? R(0) : R(1.0 / vth);
            s_c[t] = double(v[c]) + hubble * ((double(kb + t) + 0.5 / double(n_sub)) * g.ds);
        }
        __syncthreads();
        if (b < nb) {
            for (int t = 0; t < nc; ++t) {
                const double k0 = s_k0[t];
                if (k0 == 0.0) continue;   // the same cell for every lane
                const R a = s_a[t], iv = s_iv[t];
                const double c0 = s_c[t];
                for (int m = 0; m < n_sub; ++m) {
                    const R x = R(u - fma(double(m), dc, c0)) * iv;
                    acc = fma(k0, double(voigt_forest<R>(a, x)), acc);
                }
            }
        }
    }
    if (b < nb) tau[size_t(ray) * nb + b] = acc;
}

// ----------------------------------------------------------------- host
thread_local std::string g_ray_error;

thor_status fail(thor_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
thor_status fail(thor_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_ray_error = buf;
    return s;
}

// The Dawson tables of this unit, built like the transport library's: at
// each interval centre c, F(c) = exp(-c^2) sum c^(2n+1) / (n! (2n+1)) in long
// double, higher derivatives from F' = 1 - 2xF and
// F^(n+1) = -2x F^(n) - 2n F^(n-1), Taylor coefficients F^(n)(c) h^n / n!
// in s = (x - c)/h with h = 1/16.
void build_tables(double* t64, float* t32) {
    for (int i = 0; i < kDawsonIntervals; ++i) {
        const long double c = ((long double)i + 0.5L) * 0.125L, x2 = c * c;
        long double term = c, sum = 0.0L;
        for (int n = 0; n < 4000; ++n) {
            const long double add = term / (long double)(2 * n + 1);
            sum += add;
            if (add <= sum * 1e-22L) break;
            term *= x2 / (long double)(n + 1);
        }
        long double d[kDawsonDeg64 + 1];
        d[0] = expl(-x2) * sum;
        d[1] = 1.0L - 2.0L * c * d[0];
        for (int n = 1; n < kDawsonDeg64; ++n) d[n + 1] = -2.0L * c * d[n] - 2.0L * (long double)n * d[n - 1];
        long double hp = 1.0L, fact = 1.0L;
        for (int n = 0; n <= kDawsonDeg64; ++n) {
            if (n > 0) { hp *= 0.0625L; fact *= (long double)n; }
            const long double coef = d[n] * hp / fact;
            t64[i * (kDawsonDeg64 + 1) + n] = (double)coef;
            if (n <= kDawsonDeg32) t32[i * (kDawsonDeg32 + 1) + n] = (float)coef;
        }
    }
}

// uploads the tables once per device (synchronously, on first use)
thor_status ensure_tables() {
    static std::mutex mu;
    static bool built = false, loaded[64] = {};
    static double t64[kDawsonIntervals * (kDawsonDeg64 + 1)];
    static float t32[kDawsonIntervals * (kDawsonDeg32 + 1)];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return fail(THOR_E_DEVICE, "no usable current HIP device");
    std::lock_guard<std::mutex> lk(mu);
    if (loaded[dev]) return THOR_OK;
    if (!built) { build_tables(t64, t32); built = true; }
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_ray_dawson64), t64, sizeof t64) != hipSuccess ||
        hipMemcpyToSymbol(HIP_SYMBOL(c_ray_dawson32), t32, sizeof t32) != hipSuccess)
        return fail(THOR_E_DEVICE, "Dawson table upload failed");
    loaded[dev] = true;
    return THOR_OK;
}

thor_status check_grid(const thor_ray_grid* g) {
    if (!g) return fail(THOR_E_INVAL, "grid is NULL");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1)
        return fail(THOR_E_INVAL, "grid dims must be >= 1 (got %d %d %d)", g->nx, g->ny, g->nz);
    if (g->axis < 0 || g->axis > 2) return fail(THOR_E_INVAL, "axis must be 0, 1 or 2 (got %d)", g->axis);
    if (!(g->ds > 0.0) || !std::isfinite(g->ds)) return fail(THOR_E_INVAL, "ds must be finite and > 0");
    return THOR_OK;
}

// (n_i, n_j, n_ray) of the rays along the grid's axis
void ray_dims(const thor_ray_grid* g, int* ni, int* nj, int* nk) {
    const int n[3] = {g->nx, g->ny, g->nz};
    *nk = n[g->axis];
    *ni = g->axis == 0 ? g->ny : g->nx;
    *nj = g->axis == 2 ? g->ny : g->nz;
}

thor_status launched(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(THOR_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
    return THOR_OK;
}

// segments per ray: enough workgroups to fill the chip, each segment at
// least `min_len` cells
int segments(size_t blocks, int n_ray, int min_len, int fill) {
    if (blocks >= size_t(fill)) return 1;
    const int want = int((size_t(fill) + blocks - 1) / blocks);
    return std::max(1, std::min(want, n_ray / min_len));
}

}  // namespace

extern "C" {

const char* thor_ray_last_error(void) { return g_ray_error.c_str(); }

thor_status thor_ray_project(const thor_ray_grid* g, const float* q, const float* w, double* Q,
                             double* W, void* hip_stream) {
    if (thor_status s = check_grid(g)) return s;
    if (!q || !Q) return fail(THOR_E_INVAL, "q and Q must be device pointers");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    int ni, nj, nk;
    ray_dims(g, &ni, &nj, &nk);
    const size_t n_img = size_t(ni) * size_t(nj);
    const double ds = g->ds;
    const bool aligned = (reinterpret_cast<uintptr_t>(q) % 16 == 0) &&
                         (!w || reinterpret_cast<uintptr_t>(w) % 16 == 0);
    if (g->axis == 0 && aligned && nk % 4 == 0) {
        const size_t blocks = (n_img + kThreads / 64 - 1) / (kThreads / 64);
        const int nk4 = nk / 4;
        const int nseg = segments(blocks, nk4, 256, kFillRows);
        const int seg4 = ((nk4 + nseg - 1) / nseg + 63) / 64 * 64;
        const int nseg_used = (nk4 + seg4 - 1) / seg4;
        if (nseg_used > 1) {
            const unsigned zb = unsigned((n_img + kThreads - 1) / kThreads);
            k_zero<<<zb, kThreads, 0, st>>>(Q, n_img);
            if (W) k_zero<<<zb, kThreads, 0, st>>>(W, n_img);
        }
        k_project_rows4<<<dim3(unsigned(blocks), unsigned(nseg_used)), kThreads, 0, st>>>(
            reinterpret_cast<const float4*>(q), reinterpret_cast<const float4*>(w), n_img, nk4, seg4, ds, Q, W,
            nseg_used > 1);
    } else if (g->axis == 0) {
        const size_t blocks = (n_img + kThreads / 64 - 1) / (kThreads / 64);
        const int nseg = segments(blocks, nk, 1024, kFillRows);
        const int seg = (nk + nseg - 1) / nseg;
        const int nseg_used = (nk + seg - 1) / seg;
        if (nseg_used > 1) {
            const unsigned zb = unsigned((n_img + kThreads - 1) / kThreads);
            k_zero<<<zb, kThreads, 0, st>>>(Q, n_img);
            if (W) k_zero<<<zb, kThreads, 0, st>>>(W, n_img);
        }
        k_project_rows<<<dim3(unsigned(blocks), unsigned(nseg_used)), kThreads, 0, st>>>(
            q, w, n_img, nk, seg, ds, Q, W, nseg_used > 1);
    } else {
        // [outer][ray][inner]: axis y -> outer z, inner x; axis z -> outer 1, inner y*x
        const size_t n_inner = g->axis == 1 ? size_t(g->nx) : size_t(g->nx) * size_t(g->ny);
        if (aligned && n_inner % 4 == 0) {
            const size_t n_col4 = n_img / 4;
            const size_t blocks = (n_col4 + kThreads - 1) / kThreads;
            const int nseg = segments(blocks, nk, 32, kFillCols);
            const int seg = (nk + nseg - 1) / nseg;
            const int nseg_used = (nk + seg - 1) / seg;
            if (nseg_used > 1) {
                const unsigned zb = unsigned((n_img + kThreads - 1) / kThreads);
                k_zero<<<zb, kThreads, 0, st>>>(Q, n_img);
                if (W) k_zero<<<zb, kThreads, 0, st>>>(W, n_img);
            }
            k_project_cols4<<<dim3(unsigned(blocks), unsigned(nseg_used)), kThreads, 0, st>>>(
                reinterpret_cast<const float4*>(q), reinterpret_cast<const float4*>(w), n_inner / 4, n_col4,
                nk, seg, ds, Q, W, nseg_used > 1);
            return launched("thor_ray_project");
        }
        const size_t blocks = (n_img + kThreads - 1) / kThreads;
        const int nseg = segments(blocks, nk, 64, kFillCols);
        const int seg = (nk + nseg - 1) / nseg;
        const int nseg_used = (nk + seg - 1) / seg;
        if (nseg_used > 1) {
            k_zero<<<unsigned(blocks), kThreads, 0, st>>>(Q, n_img);
            if (W) k_zero<<<unsigned(blocks), kThreads, 0, st>>>(W, n_img);
        }
        k_project_cols<<<dim3(unsigned(blocks), unsigned(nseg_used)), kThreads, 0, st>>>(
            q, w, n_inner, n_img, nk, seg, ds, Q, W, nseg_used > 1);
    }
    return launched("thor_ray_project");
}

thor_status thor_ray_forest(const thor_ray_grid* g, const thor_forest_opts* o, const float* n_HI,
                            const float* T, const float* v_los, double* tau, void* hip_stream) {
    if (thor_status s = check_grid(g)) return s;
    if (!o) return fail(THOR_E_INVAL, "opts is NULL");
    int ni, nj, nk;
    ray_dims(g, &ni, &nj, &nk);
    if (o->ni < 0 || o->nj < 0 || o->i0 < 0 || o->j0 < 0 || int64_t(o->i0) + o->ni > ni ||
        int64_t(o->j0) + o->nj > nj)
        return fail(THOR_E_INVAL, "rays [%d, %d) x [%d, %d) outside the %d x %d rays of the axis",
                    o->i0, o->i0 + o->ni, o->j0, o->j0 + o->nj, ni, nj);
    if (o->n_sub < 1 || o->n_sub > 65536) return fail(THOR_E_INVAL, "n_sub must be in 1..65536");
    if (o->nb < 1 || o->nb > (1u << 22)) return fail(THOR_E_INVAL, "nb must be in 1..2^22");
    if (!(o->u_hi > o->u_lo) || !std::isfinite(o->u_lo) || !std::isfinite(o->u_hi))
        return fail(THOR_E_INVAL, "need finite u_lo < u_hi");
    if (!std::isfinite(o->hubble)) return fail(THOR_E_INVAL, "hubble must be finite");
    if (o->precision != THOR_PREC_FP64 && o->precision != THOR_PREC_MIXED)
        return fail(THOR_E_INVAL, "precision must be THOR_PREC_FP64 or THOR_PREC_MIXED");
    const int64_t n_rays = int64_t(o->ni) * int64_t(o->nj);
    if (n_rays == 0) return THOR_OK;
    if (n_rays > INT32_MAX) return fail(THOR_E_INVAL, "too many rays in one call");
    if (!n_HI || !T || !v_los || !tau) return fail(THOR_E_INVAL, "fields and tau must be device pointers");
    if (thor_status s = ensure_tables()) return s;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const RayGeo rg{g->nx, g->ny, g->nz, g->axis, g->ds};
    const double du = (o->u_hi - o->u_lo) / double(o->nb);
    const dim3 grid(unsigned(n_rays), (o->nb + kThreads - 1) / kThreads);
    if (o->precision == THOR_PREC_FP64)
        k_forest<double><<<grid, kThreads, 0, st>>>(rg, nk, n_HI, T, v_los, o->i0, o->ni, o->j0, o->hubble,
                                                     o->n_sub, o->nb, o->u_lo, du, tau);
    else
        k_forest<float><<<grid, kThreads, 0, st>>>(rg, nk, n_HI, T, v_los, o->i0, o->ni, o->j0, o->hubble,
                                                    o->n_sub, o->nb, o->u_lo, du, tau);
    return launched("thor_ray_forest");
}

}  // extern "C"
