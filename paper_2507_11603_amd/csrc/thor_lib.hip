// thor_lib.hip -- kernels and the C ABI (include/thor.h) of the MI355X
// resonant-line Monte Carlo transport library (arXiv 2507.11603, Section 3.4).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/thor.h"
#include "thor_engine.hpp"

namespace thor {

__constant__ double c_dawson64[kDawsonIntervals * (kDawsonDeg64 + 1)];
__constant__ float c_dawson32[kDawsonIntervals * (kDawsonDeg32 + 1)];

// ===========================================================================
// Kernels
// ===========================================================================

// Plain path: one thread per packet, the whole history in one launch.
template <class R, bool GRID>
__global__ __launch_bounds__(256) void k_plain(GridDev g, const ModelDev* __restrict__ models, BatchDev b, OutDev o,
                                               unsigned long long* gstats, unsigned long long* gmax) {
    const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    Counters cnt = {};
    if (i < b.n) {
        const ModelDev& m = models[b.model];
        Pkt<R> pk;
        emit<R, GRID>(g, m, o, b.first_id + i, b.q0 + i, b.model, pk, cnt);
        uint32_t ev = 0;
        int fate = pk.region == kRegOut ? kFateEscaped : kFateNone;
        while (fate == kFateNone) fate = advance<R, GRID>(g, m, o, pk, cnt, ~0u, ~0u, &ev);
        finish<R, GRID>(g, m, o, pk, fate, cnt);
    }
    flush_counters(cnt, gstats, gmax);
}

// Pool of packets parked between bounded persistent steps (one slot per lane).
template <class R> struct PoolDev {
    Pkt<R>* pk;
    int* alive;
};

// Packets handed from the persistent kernel to the tail kernel: the packet,
// its home pool slot (the lane that held it), the count and a claim cursor;
// `gone` counts the persistent waves that have left their loop, and waves
// hand off only once at most `max_waves` are still running (the tail).
template <class R> struct TailDev {
    Pkt<R>* pk;
    uint32_t* home;
    unsigned long long* count;
    unsigned long long* cursor;
    unsigned long long* gone;
    uint64_t max_waves;
};

__device__ __forceinline__ int find_batch(const BatchDev* b, int nb, uint64_t q) {
    int lo = 0, hi = nb - 1;   // last batch with q0 <= q
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b[mid].q0 <= q) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Persistent path: resident waves; each lane keeps one packet in registers
// and refills from the global queue (one atomic per wave, ballot + mbcnt
// prefix for the lane offsets) when its packet finishes.  Each turn a lane
// advances its packet by at most `turn_visits` march segments, so lanes with
// short flights (packets trapped near line centre) make progress at the
// pace of their neighbours' long flights.  A bounded step (step_events > 0)
// parks live packets in the pool for the next launch.
//
// Tail hand-off (desc->wide > 0, unbounded calls): once the queue is drained,
// at most tail.max_waves waves (four per CU) are still running and a wave
// holds at most desc->wide live packets, it appends them to the tail list and
// exits; k_tail then runs each of them in a wave of its own.
//
// Queue order (perm, may be null): slot q of the queue holds packet perm[q]
// (spatially sorted emission, see k_emit_keys); every packet's history
// depends only on its photon id, so the order changes no result.
template <class R, bool GRID, bool SEEDS>
__global__ __launch_bounds__(256) void k_persistent(GridDev g, const ModelDev* __restrict__ models,
                                                    const BatchDev* __restrict__ batches,
                                                    const StepDesc* __restrict__ desc,
                                                    unsigned long long* cursor, OutDev o, PoolDev<R> pool,
                                                    TailDev<R> tail, SeedBuf sb, unsigned long long* gstats,
                                                    unsigned long long* gmax, const uint64_t* __restrict__ perm) {
    const uint64_t gid = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint64_t q_end = desc->q_end;
    const int nbatch = desc->nbatch;
    const uint32_t step_events = desc->step_events;
    const uint32_t turn_visits = desc->turn_visits;
    const uint32_t park = desc->park;
    const uint32_t refill = desc->refill;
    const int hand_off = tail.pk ? int(desc->wide) : 0;
    const uint64_t waves_total = uint64_t(gridDim.x) * (blockDim.x >> 6);
    // peel rays of grid media: first segment at the event, the rest written to
    // the seed buffer for the peel pass (SEEDS: 1..kMaxSeedObs observers)
    constexpr bool useq = GRID && SEEDS;
    // the FP32 Dawson table in LDS for the march's Voigt evaluations
    constexpr int kDaw = kDawsonIntervals * (kDawsonDeg32 + 1);
    __shared__ float daw[kDaw];
    for (int k = threadIdx.x; k < kDaw; k += blockDim.x) daw[k] = c_dawson32[k];
    __syncthreads();
    SeedLane sl{0, 0};
    bool stalled = false;          // the seed buffer is full: park and stop
    Counters cnt = {};
    Pkt<R> pk;
    CellCache<R> cc;
    cc.valid = false;
    bool active = false;
    if (pool.alive && pool.alive[gid]) {
        pk = pool.pk[gid];
        active = true;
    }
    bool exhausted = false;
    const uint32_t budget = step_events ? step_events : ~0u;
    uint32_t used = 0;
    for (;;) {
        bool need = !active && !exhausted && !stalled && used < budget;
        if constexpr (useq) {
            // once the buffer is full every lane stops at its next turn, so the
            // launch ends promptly and the peel pass can empty the buffer
            if (__hip_atomic_load(sb.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= sb.cap) {
                stalled = true;
                need = false;
            }
            // lanes without room for one more event's rays get a new run of
            // slots, one atomic for the wave; with the buffer full they stop
            const bool low = (need || (active && !stalled && used < budget)) && sl.left < uint32_t(o.n_obs);
            const uint64_t lm = __ballot(low);
            if (lm) {
                const int leader = __ffsll((unsigned long long)lm) - 1;
                unsigned long long base = 0;
                if (int(threadIdx.x & 63) == leader)
                    base = atomicAdd(sb.count, (unsigned long long)__popcll(lm) * sb.chunk);
                base = __shfl(base, leader, 64);
                if (low) {
                    const uint64_t mine = base + uint64_t(lane_rank(lm)) * sb.chunk;
                    seed_release(sb, sl);
                    if (mine + sb.chunk <= sb.cap) {
                        sl.cur = mine;
                        sl.left = sb.chunk;
                    } else {
                        stalled = true;
                        need = false;
                    }
                }
            }
        }
        const uint64_t mask = __ballot(need);
        if (mask) {
            const int leader = __ffsll((unsigned long long)mask) - 1;
            const int lane = threadIdx.x & 63;
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(cursor, (unsigned long long)__popcll(mask));
            base = __shfl(base, leader, 64);
            const uint32_t rank = lane_rank(mask);
            if (need) {
                const uint64_t qs = base + rank;
                if (qs < q_end) {
                    const uint64_t q = perm ? perm[qs] : qs;
                    const int bi = find_batch(batches, nbatch, q);
                    const BatchDev b = batches[bi];
                    emit<R, GRID, useq>(g, models[b.model], o, b.first_id + (q - b.q0), q, b.model, pk, cnt, &sb,
                                        &sl);
                    cc.valid = false;
                    active = true;
                    if (pk.region == kRegOut) {
                        finish<R, GRID>(g, models[b.model], o, pk, kFateEscaped, cnt);
                        active = false;
                    }
                } else {
                    exhausted = true;
                }
            }
        }
        const bool work = active && !stalled && used < budget;
        const uint64_t wm = __ballot(work);
        if (wm == 0) break;
        if (hand_off && __popcll(wm) <= hand_off && __ballot(exhausted) != 0 &&
            waves_total - __hip_atomic_load(tail.gone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <=
                tail.max_waves) {
            // queue drained, few packets left: the tail kernel takes them
            const int leader = __ffsll((unsigned long long)wm) - 1;
            unsigned long long base = 0;
            if (int(threadIdx.x & 63) == leader) base = atomicAdd(tail.count, (unsigned long long)__popcll(wm));
            base = __shfl(base, leader, 64);
            if (work) {
                const uint64_t t = base + lane_rank(wm);
                tail.pk[t] = pk;
                tail.home[t] = uint32_t(gid);
                active = false;
            }
            break;
        }
        if (work) {
            const ModelDev& m = models[pk.model];
            const int fate = advance<R, GRID, useq>(g, m, o, pk, cnt, turn_visits, budget - used, &used, &sb, &sl,
                                                    &cc, nullptr, 0u, nullptr, daw, refill, park);
            if (fate != kFateNone) {
                finish<R, GRID>(g, m, o, pk, fate, cnt);
                active = false;
            }
        }
    }
    if constexpr (useq) seed_release(sb, sl);
    if (useq && __ballot(stalled) && (threadIdx.x & 63) == 0) atomicAdd(sb.parked, 1ull);
    if (hand_off && (threadIdx.x & 63) == 0) atomicAdd(tail.gone, 1ull);
    if (pool.alive) {
        pool.alive[gid] = active ? 1 : 0;
        if (active) pool.pk[gid] = pk;
    }
    flush_counters(cnt, gstats, gmax);
}

// Tail of a persistent launch: the packets handed off by waves whose queue
// was drained (typically a few trapped near line centre that scatter 1e4-1e6
// times and would set the launch time alone), one packet per wave (one wave
// per workgroup).  Each turn, all 64 lanes first evaluate the
// state-independent draws of the packet's next events (event_draws, the same
// functions as the inline path, so the histories are the same bits) into
// LDS; lane 0 then runs those events, its serial chain reduced to what
// depends on the packet's state (march, Voigt, u_parallel, basis).  On the
// seed path lane 0 only records each event's peel rays, and all lanes then
// march their first segments (seed_make), one ray per lane, into a run of
// slots claimed for the turn.  When the seed buffer is full, packets go back
// to their home pool slots for the next round.
template <class R, bool GRID, bool SEEDS>
__global__ __launch_bounds__(64) void k_tail(GridDev g, const ModelDev* __restrict__ models,
                                             const StepDesc* __restrict__ desc, OutDev o, PoolDev<R> pool,
                                             TailDev<R> tail, SeedBuf sb, unsigned long long* gstats,
                                             unsigned long long* gmax) {
    constexpr bool useq = GRID && SEEDS;
    constexpr int kDaw = kDawsonIntervals * (kDawsonDeg32 + 1);
    __shared__ EventDraws<R> wd[64];
    __shared__ PeelJob<R> wj[useq ? 64 : 1];
    __shared__ float daw[kDaw];          // the FP32 Dawson table, read on the serial chain
    const int lane = int(threadIdx.x);
    for (int k = lane; k < kDaw; k += 64) daw[k] = c_dawson32[k];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint64_t n = *tail.count;
    const uint32_t turn_visits = desc->turn_visits;
    // events per turn: at most one peel ray per lane
    const uint32_t per = useq ? uint32_t(64 / o.n_obs) : 64u;
    Counters cnt = {};
    SeedLane sl{0, 0};
    bool stalled = false;          // wave-uniform
    for (;;) {
        unsigned long long i = 0;
        if (lane == 0) i = atomicAdd(tail.cursor, 1ull);
        i = __shfl(i, 0, 64);
        if (i >= n) break;
        Pkt<R> pk = tail.pk[i];
        const uint32_t home = tail.home[i];
        const ModelDev& m = models[pk.model];
        const Key key{m.seed, m.req, uint32_t(pk.id), uint32_t(pk.id >> 32)};
        CellCache<R> cc;
        cc.valid = false;
        int fate = kFateNone;
        while (!stalled) {
            unsigned long long base = 0;
            if constexpr (useq) {
                // slots for every ray of the turn, claimed before its events
                const uint64_t need = uint64_t(per) * uint64_t(o.n_obs);
                int st = 0;
                if (lane == 0) {
                    if (__hip_atomic_load(sb.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= sb.cap) {
                        st = 1;
                    } else {
                        base = atomicAdd(sb.count, (unsigned long long)need);
                        if (base + need > sb.cap) st = 1;
                    }
                }
                stalled = __shfl(st, 0, 64) != 0;
                if (stalled) break;
                base = __shfl(base, 0, 64);
            }
            event_draws<R>(key, pk.event + 1u + uint32_t(lane), o.phase, R(m.g_hg), wd[lane]);
            // the wave's own LDS stores, read back by lane 0
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            JobSink<R> js{wj, 0u};
            if (lane == 0) {
                uint32_t used = 0;
                fate = advance<R, GRID, useq, true>(g, m, o, pk, cnt, turn_visits, per, &used, &sb, &sl, &cc, wd,
                                                    pk.event + 1u, &js, daw);
            }
            fate = __shfl(fate, 0, 64);
            pk.event = __shfl(pk.event, 0, 64);
            if constexpr (useq) {
                const uint32_t nj = __shfl(js.n, 0, 64);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                bool keep = false;
                PeelSeed sd;
                if (uint32_t(lane) < nj) {
                    const PeelJob<R> j = wj[lane];
                    Loc L;
#pragma unroll
                    for (int k = 0; k < 3; ++k) { L.p[k] = j.p[k]; L.c[k] = j.c[k]; }
                    L.region = kRegGas;
                    keep = seed_make<R>(g, o, L, j.f, j.ob, double(j.pv) / (2.0 * kPi), j.dvp, cnt, sd);
                }
                const uint64_t km = __ballot(keep);
                if (keep) {
                    const uint64_t slot = base + lane_rank(km);
                    sb.s[slot] = sd;
                    if (sb.keys) sb.keys[slot] = seed_key(g, o, sd, sb.key_blocks);
                }
                // the turn's slots past its kept rays stay empty
                const uint64_t need = uint64_t(per) * uint64_t(o.n_obs);
                if (sb.keys)
                    for (uint64_t i = uint64_t(__popcll(km)) + uint64_t(lane); i < need; i += 64)
                        sb.keys[base + i] = ~0u;
            }
            // every read of this turn's draws and jobs precedes the next turn's stores
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (fate != kFateNone) break;
        }
        if (lane == 0) {
            if (fate != kFateNone) {
                finish<R, GRID>(g, m, o, pk, fate, cnt);
            } else {            // seed buffer full: the next round resumes it
                pool.pk[home] = pk;
                pool.alive[home] = 1;
            }
        }
    }
    if (useq && stalled && lane == 0) atomicAdd(sb.parked, 1ull);
    flush_counters(cnt, gstats, gmax);
}

// Peel pass: marches the rays appended by the transport kernel.  Each wave
// takes chunks of kPassChunk slots from per-XCD counters; a lane whose ray is
// finished takes the next slot of the chunk (ballot + mbcnt), so lanes keep
// marching while their neighbours' rays are long.  A ray advances
// THOR_PASS_LOOKAHEAD cells (FP32 pencil records; THOR_PEEL_LOOKAHEAD in
// FP64) per round with their records fetched together;
// segment lengths and the order of the tau sum are those of the serial march.
// Contributions are summed per cube element in an LDS table of the workgroup
// first and reach the cube once per element at the end (a point source
// sends every emission ray to the same few elements).
constexpr uint32_t kPassChunk = 1024;
constexpr uint32_t kSpecCopies = 32;    // escape spectrum copies of a transport call
constexpr uint32_t kXcds = 8;           // accelerator complex dies of an MI355X
constexpr uint32_t kAggSlots = 512;     // LDS sums per workgroup (power of two)
constexpr int kAggProbes = 4;

// Adds contribution c to cube element ci through the workgroup's LDS table
// (keys: element + 1, 0 = free; short linear probing); a crowded table
// passes c straight to the cube.  The table holds float32 sums, or integer
// sums in the fixed-point mode (V = unsigned long long).
template <class V> __device__ __forceinline__ V agg_value(const OutDev& o, double c);
template <> __device__ __forceinline__ float agg_value<float>(const OutDev&, double c) { return float(c); }
template <> __device__ __forceinline__ unsigned long long agg_value<unsigned long long>(const OutDev& o, double c) {
    return to_fixed(o, c);
}
template <class V> __device__ __forceinline__ void agg_flush(const OutDev& o, uint64_t ci, V v);
template <> __device__ __forceinline__ void agg_flush<float>(const OutDev& o, uint64_t ci, float v) {
    unsafeAtomicAdd(o.cube + ci, v);
}
template <> __device__ __forceinline__ void agg_flush<unsigned long long>(const OutDev& o, uint64_t ci,
                                                                         unsigned long long v) {
    atomicAdd(o.cube_fx + ci, v);
}

template <class V>
__device__ __forceinline__ void deposit_lds(uint32_t* keys, V* vals, const OutDev& o, uint64_t ci, double c) {
    const V v = agg_value<V>(o, c);
    if (ci < 0xFFFFFFFFull) {
        const uint32_t k = uint32_t(ci) + 1u;
        uint32_t h = (k * 2654435761u) & (kAggSlots - 1u);
        for (int p = 0; p < kAggProbes; ++p) {
            uint32_t cur = __hip_atomic_load(keys + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (cur == 0u) cur = atomicCAS(keys + h, 0u, k);
            if (cur == 0u || cur == k) {
                __hip_atomic_fetch_add(vals + h, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                return;
            }
            h = (h + 1u) & (kAggSlots - 1u);
        }
    }
    agg_flush<V>(o, ci, v);
}

template <class R, class V, class AR>
__device__ __forceinline__ void peel_pass(const GridDev& g, const OutDev& o, const SeedBuf& sb,
                                          unsigned long long* work, unsigned long long* gstats) {
    // FP32 (mixed) rays read the pencil records of their axis: consecutive
    // cells of a ray are consecutive 16-byte records
    constexpr bool kAxis = sizeof(R) == 4;
    const uint64_t claimed = *sb.count;
    const uint64_t n = claimed < sb.cap ? claimed : sb.cap;
    const int lane = int(threadIdx.x & 63);
    Counters cnt = {};
    bool have = false, drained = false;
    // FP32 rays with THOR_PASS_PREFETCH: the records of a ray's next group of
    // cells are requested before the current group is summed, so their latency
    // overlaps that work
    constexpr bool kPre = kAxis && THOR_PASS_PREFETCH;
    constexpr int kPassLook = sizeof(AR) == sizeof(AxisRec3) ? THOR_PASS_LOOKAHEAD : THOR_PASS_LOOKAHEAD_DUST;
    AR nx[kPre ? kPassLook : 1] = {};
    bool pre = false;                      // nx holds the current ray's next group
    int a = 0, ca = 0, dim = 0;
    bool pos = true;
    double lo = 0.0, dx = 0.0, pa = 0.0, tau = 0.0, w = 0.0;
    int64_t stride = 0, idx = 0;
    const AR* axr = nullptr;
    uint64_t ci = 0;
    R dvp = R(0);
    uint64_t cur = 0, end = 0;             // the wave's chunk, [cur, end)
    const uint32_t xcd = blockIdx.x % kXcds; // workgroups are dealt round-robin over the XCDs
    __shared__ uint32_t agg_key[kAggSlots];
    __shared__ V agg_val[kAggSlots];
    // the FP32 Dawson table in LDS: its lookups are per-lane gathers
    constexpr int kDaw = kDawsonIntervals * (kDawsonDeg32 + 1);
    __shared__ float daw[kAxis ? kDaw : 1];
    for (uint32_t i = threadIdx.x; i < kAggSlots; i += blockDim.x) {
        agg_key[i] = 0u;
        agg_val[i] = V(0);
    }
    if constexpr (kAxis)
        for (uint32_t i = threadIdx.x; i < uint32_t(kDaw); i += blockDim.x) daw[i] = c_dawson32[i];
    __syncthreads();
    uint32_t part = 0;
    for (;;) {
        uint64_t m = __ballot(!have);
        while (m && !drained) {
            if (cur >= end) {
                // the buffer is split in kXcds contiguous parts; waves take chunks
                // of their own XCD's part first (seeds written by one lane are
                // consecutive, so its rays' cells stay in that XCD's L2), then
                // help the other parts
                for (;;) {
                    const uint32_t x = (xcd + part) % kXcds;
                    const uint64_t p_lo = n * x / kXcds, p_hi = n * (x + 1) / kXcds;
                    unsigned long long base = 0;
                    if (lane == 0) base = atomicAdd(work + x, (unsigned long long)kPassChunk);
                    base = __shfl(base, 0, 64) + p_lo;
                    if (base < p_hi) {
                        cur = base;
                        end = base + kPassChunk < p_hi ? base + kPassChunk : p_hi;
                        break;
                    }
                    if (++part == kXcds) { drained = true; break; }
                }
                if (drained) break;
            }
            const bool mine = (m >> lane) & 1ull;
            const uint32_t r = lane_rank(m);
            const uint64_t room = end - cur;
            const uint32_t take = uint64_t(__popcll(m)) < room ? uint32_t(__popcll(m)) : uint32_t(room);
            if (mine && r < take) {
                PeelSeed* slot = sb.s + (sb.order ? uint64_t(sb.order[cur + r]) : (cur + r));
                const PeelSeed sd = *slot;
                if (sd.obs >= 0) {
                    slot->obs = -1;          // the slot is free for the next step
                    const int axis = sel3(sd.obs, o.obs_axis[0], o.obs_axis[1], o.obs_axis[2]);
                    a = axis % 3;
                    pos = axis < 3;
                    dim = sel3(a, g.nx, g.ny, g.nz);
                    lo = sel3(a, g.lo[0], g.lo[1], g.lo[2]);
                    dx = sel3(a, g.dx[0], g.dx[1], g.dx[2]);
                    ca = sel3(a, sd.c[0], sd.c[1], sd.c[2]);
                    if constexpr (kAxis) {
                        const uint64_t x = uint64_t(sd.c[0]), y = uint64_t(sd.c[1]), z = uint64_t(sd.c[2]);
                        idx = int64_t(a == 0 ? (z * g.ny + y) * g.nx + x
                                             : (a == 1 ? (z * g.nx + x) * g.ny + y : (y * g.nx + x) * g.nz + z));
                        stride = pos ? 1 : -1;
                        if constexpr (sizeof(AR) == sizeof(AxisRec3)) axr = sel3(a, g.axc[0], g.axc[1], g.axc[2]);
                        else axr = sel3(a, g.axr[0], g.axr[1], g.axr[2]);
                    } else {
                        idx = int64_t(cell_index(g, sd.c));
                        stride = (a == 0 ? int64_t(1) : (a == 1 ? int64_t(g.nx) : int64_t(g.nx) * int64_t(g.ny))) *
                                 (pos ? 1 : -1);
                    }
                    pa = pos ? lo + double(ca) * dx : lo + double(ca + 1) * dx;   // face shared with the event cell
                    tau = sd.tau;
                    w = sd.w;
                    dvp = R(sd.dv);
                    ci = sd.cube;
                    pre = false;
                    have = true;
                }
            }
            cur += take;
            m = __ballot(mine && r >= take);
        }
        if (__ballot(have) == 0) {
            if (drained) break;
            continue;
        }
        if (have) {
            constexpr int kLook = kAxis ? kPassLook : THOR_PEEL_LOOKAHEAD;
            const int left = pos ? dim - ca : ca + 1;       // >= 1
            const int mm = left < kLook ? left : kLook;
            bool cut = false;
            const double href = sel3(a, g.href[0], g.href[1], g.href[2]);
            if constexpr (kAxis) {
                AR rc[kLook];
                if (kPre && pre) {
#pragma unroll
                    for (int j = 0; j < kLook; ++j) rc[j] = nx[kPre ? j : 0];
                } else {
#pragma unroll
                    for (int j = 0; j < kLook; ++j)
                        if (j < mm) rc[j] = axr[idx + int64_t(j) * stride];
                }
                if constexpr (kPre) {
                    // the group after this one, when the ray goes on past it
                    const int mm2 = left - mm < kLook ? left - mm : kLook;
#pragma unroll
                    for (int j = 0; j < kLook; ++j)
                        if (j < mm2) nx[j] = axr[idx + int64_t(mm + j) * stride];
                    pre = mm2 > 0;
                }
#pragma unroll
                for (int j = 0; j < kLook; ++j) {
                    if (j >= mm || cut) break;
                    // every cell after the event's is crossed whole: segment = cell width
                    cnt.peel_visits++;
                    if (rc[j].k0 > 0.0f || rec_kd(rc[j]) > 0.0f) {
                        const float av = float(kDampTimesVth) * rc[j].ivth;
                        if (g.hubble > 0.0) {
                            // entry face of cell j, the Hubble flow there, sub-steps
                            const int cj = ca + (pos ? j : -j);
                            const double entry = pos ? lo + double(cj) * dx : lo + double(cj + 1) * dx;
                            const double hv = g.hubble * (entry - href);
                            const double u0 = double(dvp) - (pos ? double(rc[j].v) : -double(rc[j].v)) -
                                              (pos ? hv : -hv);
                            const double vth = 1.0 / double(rc[j].ivth);
                            const int n = hubble_steps(g, dx, vth);
                            const double ds = dx / n;
                            for (int q = 0; q < n; ++q) {
                                const float x = float(u0 - g.hubble * ((q + 0.5) * ds)) * rc[j].ivth;
                                tau += (double(rc[j].k0) * double(voigt32(av, x, daw)) + double(rec_kd(rc[j]))) * ds;
                            }
                        } else {
                            const float x = (dvp - (pos ? rc[j].v : -rc[j].v)) * rc[j].ivth;
                            tau += (double(rc[j].k0) * double(voigt32(av, x, daw)) + double(rec_kd(rc[j]))) * dx;
                        }
                        cut = tau > o.tau_cut;
                    }
                }
            } else {
                CellRec rc[kLook];
#pragma unroll
                for (int j = 0; j < kLook; ++j)
                    if (j < mm) rc[j] = g.rec[idx + int64_t(j) * stride];
#pragma unroll
                for (int j = 0; j < kLook; ++j) {
                    if (j >= mm || cut) break;
                    const int cj = ca + (pos ? j : -j);
                    const double face = pos ? lo + double(cj + 1) * dx : lo + double(cj) * dx;
                    double t = pos ? face - pa : pa - face;
                    t = t < 0.0 ? 0.0 : t;
                    cnt.peel_visits++;
                    Fields<R> f;
                    fields_from_rec<R>(g, rc[j], f);
                    if (f.k0 > 0.0 || f.kd > 0.0) {
                        const R va = sel3(a, f.v[0], f.v[1], f.v[2]);
                        if (g.hubble > 0.0) {
                            const double hv = g.hubble * (pa - href);
                            tau += hubble_segment_tau<R>(g, double(dvp) - (pos ? double(va) : -double(va)) -
                                                                (pos ? hv : -hv), t, f.vth, f.a, f.k0, f.kd);
                        } else {
                            const R x = fdiv(dvp - (pos ? va : -va), f.vth);
                            tau += (f.k0 * double(voigt<R>(f.a, x)) + f.kd) * t;
                        }
                        cut = tau > o.tau_cut;
                    }
                    pa = face;
                }
            }
            ca += pos ? mm : -mm;
            idx += int64_t(mm) * stride;
            if (cut) {
                cnt.peel_cut++;
                have = false;
            } else if (mm == left) {
                deposit_lds<V>(agg_key, agg_val, o, ci, w * exp(-tau));
                have = false;
            }
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < kAggSlots; i += blockDim.x)
        if (agg_key[i]) agg_flush<V>(o, agg_key[i] - 1u, agg_val[i]);
    flush_counters(cnt, gstats);
}

// FP32 pass: four waves per SIMD (at most 128 VGPRs).  A lane sums a ray's
// cells in groups of THOR_PASS_LOOKAHEAD and requests the next group's records
// before summing the current one, so two groups are in flight while it
// works: a wave's gathers are latency-bound, and on the 1024^3 web box this
// beat one group of eight cells at a time by 15 % (and three waves with
// larger groups by 9-13 %).
// V: float32 cube, or unsigned long long for the fixed-point cube.
#ifndef THOR_PEEL_WAVES
#define THOR_PEEL_WAVES 4
#endif
// AR: the pencil record (AxisRec, or AxisRec3 on grids without dust).
template <class V, class AR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(THOR_PEEL_WAVES)))
void k_peel_pass_f32(GridDev g, OutDev o, SeedBuf sb, unsigned long long* work, unsigned long long* gstats) {
    peel_pass<float, V, AR>(g, o, sb, work, gstats);
}

template <class V>
__global__ __launch_bounds__(256) void k_peel_pass_f64(GridDev g, OutDev o, SeedBuf sb, unsigned long long* work,
                                                       unsigned long long* gstats) {
    peel_pass<double, V, AxisRec>(g, o, sb, work, gstats);
}

// The fixed-point cube as float32 (units of 1/scale).
__global__ void k_fx_to_f32(const unsigned long long* __restrict__ src, float* __restrict__ dst, uint64_t n,
                            double inv_scale) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
        dst[i] = float(double(src[i]) * inv_scale);
}

// Sort keys of the queue.  mode 1 (spatial): the Morton code (x, y, z bits
// interleaved) of each n_HI^2-weighted packet's emission cell, drawn exactly
// as the generator draws it; other sources sort first.  mode 2 (frequency):
// the packet's emitted offset in the source frame (line centre, Gaussian or
// flat draw, the doublet line chosen; the thermal draw without its cell's
// width), its IEEE bits mapped to an order-preserving integer.
__device__ __forceinline__ uint64_t spread3(uint64_t v) {   // bit i -> bit 3i (21 bits)
    v &= 0x1FFFFFull;
    v = (v | (v << 32)) & 0x1F00000000FFFFull;
    v = (v | (v << 16)) & 0x1F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}
__global__ void k_emit_keys(GridDev g, const ModelDev* __restrict__ models, const BatchDev* __restrict__ batches,
                            int nbatch, uint64_t q_end, uint64_t* __restrict__ keys, uint64_t* __restrict__ vals,
                            int mode) {
    for (uint64_t q = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < q_end;
         q += uint64_t(gridDim.x) * blockDim.x) {
        const BatchDev b = batches[find_batch(batches, nbatch, q)];
        const ModelDev& m = models[b.model];
        uint64_t key = 0;
        const uint64_t id = b.first_id + (q - b.q0);
        const Key k{m.seed, m.req, uint32_t(id), uint32_t(id >> 32)};
        if (mode == 2) {
            double off = m.dv0;
            if (m.spectrum != kSpecDelta) {
                const Uni2<double> d = draw<double>(k, kSlotEGauss, 0);
                if (m.spectrum == kSpecFlat) {
                    off += m.sigma_v * (2.0 * d.a - 1.0);
                } else {
                    const double z = sqrt(-2.0 * log(1.0 - d.a)) * cospi(2.0 * d.b);
                    off += (m.spectrum == kSpecGauss ? m.sigma_v : 1.0) * z;
                }
            }
            if (m.lines && m.nl > 1 && draw<double>(k, kSlotELine, 0).a >= m.lw0) off += m.lc1;
            const uint64_t bits = uint64_t(__double_as_longlong(off));
            key = (bits >> 63) ? ~bits : (bits | (1ull << 63));
        } else if (m.src_kind == kSrcCellN2) {
            const uint64_t c = emission_cell(g, draw<double>(k, kSlotECell, 0).a);
            const uint64_t x = c % uint64_t(g.nx), y = (c / uint64_t(g.nx)) % uint64_t(g.ny);
            const uint64_t z = c / (uint64_t(g.nx) * uint64_t(g.ny));
            key = spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
        }
        keys[q] = key;
        vals[q] = q;
    }
}

// Slot indices 0..n-1 (the values the seed sort permutes).
__global__ void k_iota_u32(uint32_t* __restrict__ v, uint64_t n) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
        v[i] = uint32_t(i);
}

// Keys for photon fusing (Section 3.4.1): observer, the pencil-order index
// of the front cell and the peeled frequency's 1/m sub-bin of a cube
// frequency bin (m = fuse_bins).  Rays of one key start in the same cell
// towards the same observer and end in the same cube element; they are
// merged into one ray (k_seed_fuse).  Empty slots sort last.
__global__ void k_fuse_keys(GridDev g, OutDev o, SeedBuf sb, uint64_t n, int m, uint64_t* __restrict__ keys,
                            uint32_t* __restrict__ vals) {
    const uint64_t nx = uint64_t(g.nx), ny = uint64_t(g.ny), nz = uint64_t(g.nz);
    const uint64_t nc = nx * ny * nz;
    const uint64_t nsub = uint64_t(o.cube_nb) * uint64_t(m);
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
        const PeelSeed sd = sb.s[i];
        uint64_t key = uint64_t(o.n_obs) * nc * nsub;      // empty: past every ray's key
        if (sd.obs >= 0) {
            const int a = sel3(sd.obs, o.obs_axis[0], o.obs_axis[1], o.obs_axis[2]) % 3;
            const uint64_t x = uint64_t(sd.c[0]), y = uint64_t(sd.c[1]), z = uint64_t(sd.c[2]);
            const uint64_t idx = a == 0 ? (z * ny + y) * nx + x : (a == 1 ? (z * nx + x) * ny + y : (y * nx + x) * nz + z);
            const double u = (sd.dv - o.v_lo) / o.v_w * double(m);
            uint64_t sub = u > 0.0 ? uint64_t(u) : 0;
            sub = sub < nsub ? sub : nsub - 1;
            key = (uint64_t(sd.obs) * nc + idx) * nsub + sub;
        }
        keys[i] = key;
        vals[i] = uint32_t(i);
    }
}

// Merges each run of equal fusing keys (and equal cube elements) in the
// sorted order into its first seed: weight sum_j w_j exp(-tau_j) with the
// first segments' optical depths folded in (tau 0), the first seed's
// frequency for the rest of the ray; the others are emptied.  *fused counts
// the rays merged away.
__global__ void k_seed_fuse(SeedBuf sb, const uint64_t* __restrict__ keys, const uint32_t* __restrict__ order,
                            uint64_t n, uint64_t empty, unsigned long long* fused) {
    unsigned long long merged = 0;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
        if (keys[i] >= empty) continue;
        PeelSeed* head = sb.s + order[i];
        if (i > 0 && keys[i - 1] == keys[i] && sb.s[order[i - 1]].cube == head->cube) continue;   // not a run head
        double w = head->w * exp(-head->tau);
        uint64_t j = i + 1;
        for (; j < n && keys[j] == keys[i]; ++j) {
            PeelSeed* t = sb.s + order[j];
            if (t->cube != head->cube) break;
            w += t->w * exp(-t->tau);
            t->obs = -1;
            ++merged;
        }
        if (j > i + 1) {
            head->w = w;
            head->tau = 0.0;
        }
    }
    if (merged) atomicAdd(fused, merged);
}

// Marks every slot of a fresh seed buffer empty.
__global__ void k_seed_clear(PeelSeed* s, uint64_t n) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
        s[i].obs = -1;
}

// Re-layout of the grid fields into 32-byte cell records (see CellRec), with
// the FP32 line quantities derived in FP64 and rounded once; counts cells
// that are not finite, have n_HI < 0, or hold gas at T <= 0.
__global__ void k_pack_grid(const float* __restrict__ n, const float* __restrict__ vx, const float* __restrict__ vy,
                            const float* __restrict__ vz, const float* __restrict__ T, CellRec* __restrict__ out,
                            uint64_t count, unsigned long long* bad) {
    unsigned long long nbad = 0;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += uint64_t(gridDim.x) * blockDim.x) {
        const float4 r = make_float4(vx[i], vy[i], vz[i], n[i]);
        const float t = T[i];
        const bool ok = isfinite(r.x) && isfinite(r.y) && isfinite(r.z) && isfinite(r.w) && r.w >= 0.0f &&
                        (r.w == 0.0f || (isfinite(t) && t > 0.0f));
        nbad += ok ? 0ull : 1ull;
        float4 h = make_float4(t, 1.0f, 0.0f, 0.0f);
        if (ok && r.w > 0.0f) {
            const double vth = sqrt(kVth2PerT * double(t));
            h = make_float4(t, float(vth), float(kDampTimesVth / vth), float(double(r.w) * (kSigma0TimesVth / vth)));
        }
        CellRec c;
        c.lo = r;
        c.hi = h;
        out[i] = c;
    }
    if (nbad) atomicAdd(bad, nbad);
}

// Pencil-order copy of the cell records for rays along `axis`: index with
// that axis fastest ([z][y][x] for x, [z][x][y] for y, [y][x][z] for z).
template <class AR>
__global__ void k_pack_axis(const CellRec* __restrict__ rec, AR* __restrict__ out, int axis, int nx, int ny,
                            int nz, double sigma_d, uint64_t count) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += uint64_t(gridDim.x) * blockDim.x) {
        const uint64_t x = i % uint64_t(nx), y = (i / uint64_t(nx)) % uint64_t(ny), z = i / (uint64_t(nx) * ny);
        const CellRec r = rec[i];
        AR o;
        o.v = axis == 0 ? r.lo.x : (axis == 1 ? r.lo.y : r.lo.z);
        if (r.lo.w > 0.0f) {
            o.ivth = float(1.0 / sqrt(kVth2PerT * double(r.hi.x)));
            o.k0 = r.hi.w;
            if constexpr (sizeof(AR) == sizeof(AxisRec)) o.kd = float(sigma_d * double(r.lo.w));
        } else {
            o.ivth = 0.0f; o.k0 = 0.0f;
            if constexpr (sizeof(AR) == sizeof(AxisRec)) o.kd = 0.0f;
        }
        const uint64_t j = axis == 0 ? i : (axis == 1 ? (z * nx + x) * ny + y : (y * nx + x) * nz + z);
        out[j] = o;
    }
}

struct NSquared {
    __host__ __device__ double operator()(const CellRec& r) const { return double(r.lo.w) * double(r.lo.w); }
};

// Device-function harnesses (tests of the kernels' own device code).
template <class R>
__global__ void k_eval_voigt(const double* a, const double* x, double* out, uint64_t n) {
    const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = double(voigt<R>(R(a[i]), R(x[i])));
}

template <class R>
__global__ void k_eval_xcw(const double* a, double* out, uint64_t n) {
    const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = double(xcw_b25<R>(R(a[i])));
}

template <class R>
__global__ void k_sample_upar(double x, double a, uint32_t seed, uint32_t event, double* u, uint32_t* tr, uint64_t n) {
    const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) {
        const Key key{seed, 0u, uint32_t(i), uint32_t(i >> 32)};
        uint32_t t = 0;
        u[i] = double(upar_sample<R>(R(x), R(a), key, event, &t));
        tr[i] = t;
    }
}

__global__ void k_clamp_cursor(unsigned long long* cursor, const StepDesc* desc) {
    if (threadIdx.x == 0 && *cursor > desc->q_end) *cursor = desc->q_end;
}

// Adds copies 1..copies-1 of the escape spectrum into copy 0 and clears them
// (sums of unit weights: exact in FP64, in any order).
__global__ void k_spec_fold(double* spec, int nb, int copies) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += gridDim.x * blockDim.x) {
        double s = spec[i];
        for (int c = 1; c < copies; ++c) {
            s += spec[uint64_t(c) * nb + i];
            spec[uint64_t(c) * nb + i] = 0.0;
        }
        spec[i] = s;
    }
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
    if (int(threadIdx.x) < n) p[threadIdx.x] = 0ull;
}

__global__ void k_zero_u32(unsigned* p, uint64_t n) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
        p[i] = 0u;
}

// ---------------------------------------------------- no-allocation scratch
// Layout of the static array that thor_transport_noalloc uses instead of
// allocated buffers (byte offsets, each 256-aligned): counters and queue
// cursor, longest history, step descriptor, batch table, model table, the
// escape spectrum's partial copies.
constexpr uint64_t na_align(uint64_t b) { return (b + 255) & ~uint64_t(255); }
constexpr uint64_t kNaMaxBatches = THOR_NOALLOC_MAX_BATCHES;
constexpr uint64_t kNaMaxBins = THOR_NOALLOC_MAX_BINS;
constexpr uint64_t kNaCounters = 0;                                      // kNumU64Counters + cursor
constexpr uint64_t kNaMax = na_align(kNaCounters + (kNumU64Counters + 1) * 8);
constexpr uint64_t kNaDesc = na_align(kNaMax + 8);
constexpr uint64_t kNaBatches = na_align(kNaDesc + sizeof(StepDesc));
constexpr uint64_t kNaModels = na_align(kNaBatches + kNaMaxBatches * sizeof(BatchDev));
constexpr uint64_t kNaSpec = na_align(kNaModels + kNaMaxBatches * sizeof(ModelDev));
constexpr uint64_t kNaEnd = kNaSpec + uint64_t(kSpecCopies) * kNaMaxBins * 8;
static_assert(kNaEnd <= THOR_NOALLOC_SCRATCH_BYTES, "no-allocation scratch too small for its layout");

// Clears the counters, cursor, longest history and the first `spec_words`
// doubles of the spectrum copies, and writes the step descriptor.
__global__ void k_na_setup(unsigned char* s, StepDesc d, uint64_t spec_words) {
    const uint64_t tid = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (tid < kNumU64Counters + 1) reinterpret_cast<unsigned long long*>(s + kNaCounters)[tid] = 0ull;
    if (tid == 0) {
        *reinterpret_cast<unsigned long long*>(s + kNaMax) = 0ull;
        *reinterpret_cast<StepDesc*>(s + kNaDesc) = d;
    }
    double* spec = reinterpret_cast<double*>(s + kNaSpec);
    for (uint64_t i = tid; i < spec_words; i += uint64_t(gridDim.x) * blockDim.x) spec[i] = 0.0;
}

// Writes entry i of the batch and model tables.
__global__ void k_na_put(unsigned char* s, uint32_t i, ModelDev m, BatchDev b) {
    if (threadIdx.x == 0) {
        reinterpret_cast<ModelDev*>(s + kNaModels)[i] = m;
        reinterpret_cast<BatchDev*>(s + kNaBatches)[i] = b;
    }
}

// Adds the spectrum copies of the scratch into the caller's spectrum.
__global__ void k_na_fold(const unsigned char* s, double* dst, int nb, int copies) {
    const double* spec = reinterpret_cast<const double*>(s + kNaSpec);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int c = 0; c < copies; ++c) v += spec[uint64_t(c) * nb + i];
        dst[i] += v;
    }
}

}  // namespace thor

// The scratch of thor_transport_noalloc: one copy per GPU, held until the
// process ends.  Host code never passes this name to a kernel or a copy (on
// the host it is only a stand-in for the symbol); it uses the device address
// that thor_create looks up with hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[THOR_NOALLOC_SCRATCH_BYTES];

using namespace thor;

// ===========================================================================
// Host side
// ===========================================================================
namespace {

thread_local std::string g_last_error;

thor_status fail(thor_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
thor_status fail(thor_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

// Host-side table of Dawson's integral F(x) = exp(-x^2) int_0^x exp(t^2) dt
// for the device Voigt function: at each interval centre c, F(c) from the
// positive power series sum x^(2n+1)/(n!(2n+1)) (long double), the higher
// derivatives from F' = 1 - 2xF, F^(n+1) = -2x F^(n) - 2n F^(n-1), and the
// Taylor coefficients F^(n)(c) h^n / n! in s = (x - c)/h, h = 1/16.
void build_dawson_tables(double* t64, float* t32) {
    for (int i = 0; i < kDawsonIntervals; ++i) {
        const long double c = ((long double)i + 0.5L) * 0.125L;
        long double x2 = c * c, term = c, sum = 0.0L;
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

struct BatchHost {
    thor_source src;
    uint64_t n, first_id, q0;
};

struct ServingReq {
    int model;             // slot in the serving model table
    uint64_t n_packets;
    double* d_spec;
    int spec_nb;
    uint64_t reserved;     // packet-state bytes reserved against the budget
    bool finished;
};

constexpr uint32_t kDefaultParkLanes = 32;  // lanes that wait before interacting together
constexpr int kServingMaxModels = 1 << 16;
constexpr int kServingMaxBatches = 1 << 14;

// Device address of the no-allocation scratch, per device, looked up once
// (with that device current) by the first thor_create on it.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

struct thor_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    uint64_t budget = 0, used = 0;
    bool poisoned = false;
    int num_cu = 256;

    // medium
    bool has_geom = false;
    thor_geometry geom{};
    GridDev grid{};
    CellRec* d_rec = nullptr;
    double* d_cdf = nullptr;
    uint64_t grid_bytes = 0, cdf_bytes = 0;

    // queued batches
    std::vector<BatchHost> pending;

    // outputs
    double* d_spec = nullptr;
    int spec_nb = 0;
    float* d_cube = nullptr;
    unsigned long long* d_cube_fx = nullptr;   // the cube in the fixed-point mode (instead of d_cube)
    uint64_t cube_elems = 0;
    int cube_shape[5] = {0, 0, 0, 0, 0};       // observers, ny, nx, bins, accumulation mode
    double cube_fx_scale = 0.0;
    unsigned long long* d_stats = nullptr;   // kNumU64Counters counters, then cursor
    unsigned long long* d_xstats = nullptr;  // longest history, then the tail kernel's counters
    ModelDev* d_models = nullptr;
    size_t models_cap = 0;
    BatchDev* d_batches = nullptr;
    size_t batches_cap = 0;

    // records of the last call
    double* d_rec_dv = nullptr;
    uint32_t* d_rec_nres = nullptr;
    uint32_t* d_rec_ndust = nullptr;
    int32_t* d_rec_fate = nullptr;
    uint64_t rec_cap = 0, rec_n = 0;

    // persistent pool (bounded steps)
    void* d_pool_pk = nullptr;
    int* d_pool_alive = nullptr;
    uint64_t pool_slots = 0;
    int pool_prec = -1;
    uint64_t q_total = 0;        // queue indices handed out so far
    uint64_t pool_bytes = 0;

    // tail list (packets handed to k_tail), one slot per persistent lane
    void* d_tail_pk = nullptr;
    uint32_t* d_tail_home = nullptr;
    unsigned long long* d_tailctl = nullptr;   // count, cursor
    uint64_t tail_slots = 0;

    thor_stats last{};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    StepDesc* d_desc = nullptr;            // step descriptor of the transport path
    StepDesc* h_desc = nullptr;            // pinned
    StepDesc* d_s_desc = nullptr;          // step descriptor of the serving path
    StepDesc* h_s_desc = nullptr;          // pinned
    BatchDev* h_s_batches = nullptr;       // pinned mirror, kServingMaxBatches entries
    unsigned long long* h_s_done = nullptr;    // pinned mirror of d_done
    unsigned long long* h_s_misc = nullptr;    // pinned: counters then cursor
    hipStream_t cap_stream = nullptr;      // private stream for graph capture
    void* d_axr[3] = {nullptr, nullptr, nullptr};      // pencil records per axis (mixed peel pass)
    uint64_t axr_bytes[3] = {0, 0, 0};
    PeelSeed* d_seeds = nullptr;           // peel seed buffer of the grid persistent path
    uint64_t seed_cap = 0;                 // slots
    unsigned long long* d_seedctl = nullptr;   // claimed slots, parked waves, then kXcds pass work counters
    hipEvent_t ev_a = nullptr, ev_b = nullptr;  // per-step split of transport and peel-pass time
    hipEvent_t ev_c = nullptr;                  // end of the persistent kernel (the tail kernel follows)
    double split_tr = 0.0, split_pp = 0.0;     // ms of the last call's transport and peel-pass kernels
    double split_tail = 0.0;                   // ms of the last call's tail kernels (part of split_tr)
    uint64_t split_passes = 0;
    hipGraphExec_t s_graph = nullptr;
    int s_graph_prec = -1, s_graph_grid = 0, s_graph_block = 0;
    unsigned char* d_scratch = nullptr;    // this device's no-allocation scratch (device address)
    // spatial presort of the queue: keys and values, their sorted copies, hipCUB scratch
    uint64_t* d_sort = nullptr;            // 4 arrays of sort_cap entries
    uint64_t sort_cap = 0;
    void* d_sort_tmp = nullptr;
    size_t sort_tmp_bytes = 0;
    double split_presort = 0.0;
    // sort of the seed buffer before each peel pass: keys and slot indices,
    // their sorted copies, hipCUB scratch
    uint32_t* d_skeys = nullptr;           // 2 arrays of ssort_cap
    uint32_t* d_svals = nullptr;           // 2 arrays of ssort_cap
    uint64_t ssort_cap = 0;
    void* d_ssort_tmp = nullptr;
    size_t ssort_tmp_bytes = 0;
    double split_ssort = 0.0;
    uint64_t* d_fkeys = nullptr;           // photon fusing: 2 arrays of 64-bit keys of ssort_cap
    uint64_t fkeys_cap = 0;
    unsigned long long* d_fused = nullptr; // rays merged away by fusing in the last call
    hipEvent_t ev_s = nullptr;             // end of the seed sort of a round

    // serving (continuous batching of shell-model requests)
    bool s_init = false;
    std::vector<ModelDev> s_models;        // host copy of the model table
    std::vector<int> s_free;               // recycled model slots
    int s_next_slot = 0;
    std::vector<BatchDev> s_batches;       // queue ranges of live requests, by q0
    std::map<uint64_t, ServingReq> s_reqs;
    ModelDev* d_s_models = nullptr;
    BatchDev* d_s_batches = nullptr;
    size_t s_batches_cap = 0;
    unsigned long long* d_done = nullptr;  // finished packets per model slot
    unsigned long long* d_s_cursor = nullptr;
    void* d_s_pool = nullptr;
    int* d_s_alive = nullptr;
    uint64_t s_pool_slots = 0, s_pool_bytes = 0;
    int s_pool_prec = -1;
    uint64_t s_next_handle = 1;
    uint64_t s_q_total = 0, s_cursor = 0;
    uint64_t s_reserved = 0;
    bool s_dirty = false;
};

namespace {

bool hip_ok(thor_ctx* ctx, hipError_t e, const char* what) {
    if (e == hipSuccess) return true;
    ctx->poisoned = true;
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return false;
}

thor_status dalloc(thor_ctx* ctx, void** p, uint64_t bytes, const char* what) {
    if (bytes == 0) bytes = 8;
    if (ctx->budget && ctx->used + bytes > ctx->budget)
        return fail(THOR_E_BUDGET, "%s: %llu bytes exceed the HBM budget (%llu of %llu used)", what,
                    (unsigned long long)bytes, (unsigned long long)ctx->used, (unsigned long long)ctx->budget);
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();   // a caller may fall back to a smaller size: leave no error behind
        return fail(THOR_E_NOMEM, "%s: hipMalloc(%llu) failed: %s", what, (unsigned long long)bytes,
                    hipGetErrorString(e));
    }
    ctx->used += bytes;
    return THOR_OK;
}

void dfree(thor_ctx* ctx, void* p, uint64_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    if (bytes == 0) bytes = 8;
    ctx->used -= std::min(ctx->used, bytes);
}

#define CHECK_CTX(ctx)                                                              \
    do {                                                                            \
        if (!(ctx)) return fail(THOR_E_INVAL, "null context");                     \
        if ((ctx)->poisoned) return fail(THOR_E_DEVICE, "context poisoned by an earlier device error"); \
        if (hipSetDevice((ctx)->device) != hipSuccess) return fail(THOR_E_DEVICE, "hipSetDevice failed"); \
    } while (0)

#define HIPCHK(ctx, call)                                                           \
    do {                                                                            \
        if (!hip_ok((ctx), (call), #call)) return THOR_E_DEVICE;                    \
    } while (0)

void line_params(double T, double* vth, double* a, double* sig0) {
    const double v = std::sqrt(kVth2PerT * T);
    *vth = v;
    *a = kDampTimesVth / v;
    *sig0 = kSigma0TimesVth / v;
}

// Line 0 of the medium's species at temperature T (v_th, a, sigma0).
void species_params(int line, double T, double* vth, double* a, double* sig0) {
    if (line == THOR_LINE_LYA) {
        line_params(T, vth, a, sig0);
        return;
    }
    const double v = std::sqrt(2.0 * kBoltzmann * T / kMassMg);
    const double dnu = v / kMgKLambda;
    *vth = v;
    *a = kMgKA21 / (4.0 * kPi * dnu);
    *sig0 = kMgKF12 * kSqrtPi * kCharge * kCharge / (kMassE * kClight * dnu);
}

// Model constants of a batch (meshless medium constants, source, outputs).
thor_status make_model(thor_ctx* ctx, const thor_source& s, const thor_transport_opts& o, ModelDev& m) {
    const thor_geometry& g = ctx->geom;
    std::memset(&m, 0, sizeof m);
    m.kind = g.kind;
    m.v_profile = g.v_profile;
    m.src_kind = s.kind;
    m.spectrum = s.spectrum;
    m.albedo = g.albedo;
    m.g_hg = g.g_hg;
    for (int i = 0; i < 3; ++i) m.pos[i] = s.pos[i];
    m.dv0 = s.dv0;
    m.sigma_v = s.sigma_v;
    m.seed = s.seed;
    m.req = s.request_id;
    m.nl = 1;
    m.lines = s.lines;
    if (g.line == THOR_LINE_MG2) {
        m.nl = 2;
        m.lc1 = kClight * (kMgKLambda / kMgHLambda - 1.0);
        m.lrho1 = kMgHLambda / kMgKLambda;
        m.lam1 = (kMgHA21 * kMgHLambda) / (kMgKA21 * kMgKLambda);
        m.lk1 = (kMgHF12 * kMgHLambda) / (kMgKF12 * kMgKLambda);
        m.lw0 = kMgKF12 / (kMgKF12 + kMgHF12);
    }
    if (g.kind != THOR_GEOM_GRID) {
        const double L = g.r_outer - g.r_inner;
        double sig0;
        species_params(g.line, g.T, &m.vth, &m.a, &sig0);
        m.r_in = g.r_inner;
        m.r_out = g.r_outer;
        m.n = g.tau0 > 0.0 ? g.tau0 / (sig0 * L) : g.n_HI;
        m.k0 = m.n * sig0;
        const double sigd = g.tau_d > 0.0 ? g.tau_d / (m.n * L) : g.sigma_d;
        m.kd = sigd * m.n;
        m.v_max = g.v_max;
        m.step_f = g.step_f > 0.0 ? g.step_f : 0.01;
        if (o.core_skip == THOR_CS_FIXED) m.xcrit = o.x_crit;
        else if (o.core_skip == THOR_CS_ADAPTIVE) {
            const double atau = m.a * m.k0 * L;
            m.xcrit = atau >= 1.0 ? 0.2 * std::cbrt(atau) : 0.0;
        }
    } else {
        if (o.core_skip == THOR_CS_FIXED) m.xcrit = o.x_crit;
        else if (o.core_skip == THOR_CS_ADAPTIVE)
            return fail(THOR_E_UNSUPPORTED, "adaptive core skipping needs a meshless medium");
    }
    m.spec = ctx->d_spec;
    m.spec_nb = o.spec_nb;
    m.spec_rep = int(kSpecCopies);
    m.spec_lo = o.spec_lo;
    m.spec_w = (o.spec_hi - o.spec_lo) / o.spec_nb;
    m.spec_scale = 1.0;
    if (o.spec_T_ref > 0.0) {
        double vth, a, s0;
        species_params(g.line, o.spec_T_ref, &vth, &a, &s0);
        m.spec_scale = 1.0 / vth;
    }
    m.done = nullptr;
    return THOR_OK;
}

thor_status check_opts(const thor_transport_opts* o) {
    if (!o) return fail(THOR_E_INVAL, "null options");
    if (o->precision != THOR_PREC_FP64 && o->precision != THOR_PREC_MIXED) return fail(THOR_E_INVAL, "bad precision");
    if (o->path != THOR_PATH_PLAIN && o->path != THOR_PATH_PERSISTENT) return fail(THOR_E_INVAL, "bad path");
    if (o->phase < 0 || o->phase > 2) return fail(THOR_E_INVAL, "bad phase function");
    if (o->core_skip < 0 || o->core_skip > 2) return fail(THOR_E_INVAL, "bad core_skip");
    if (o->n_obs < 0 || o->n_obs > 6) return fail(THOR_E_INVAL, "n_obs must be 0..6");
    if (o->presort < -1 || o->presort > 2) return fail(THOR_E_INVAL, "presort must be -1, 0, 1 or 2");
    if (o->seed_sort < -1 || o->seed_sort > 1) return fail(THOR_E_INVAL, "seed_sort must be -1, 0 or 1");
    if (o->fuse_bins < 0 || o->fuse_bins > 4096) return fail(THOR_E_INVAL, "fuse_bins must be in 0..4096");
    for (int i = 0; i < o->n_obs; ++i)
        if (o->obs_axis[i] < 0 || o->obs_axis[i] > 5) return fail(THOR_E_INVAL, "bad observer axis");
    if (o->n_obs > 0) {
        if (o->cube_nx <= 0 || o->cube_ny <= 0 || o->cube_nb <= 0) return fail(THOR_E_INVAL, "bad cube shape");
        if (!(o->img_hi[0] > o->img_lo[0]) || !(o->img_hi[1] > o->img_lo[1]) || !(o->cube_v_hi > o->cube_v_lo))
            return fail(THOR_E_INVAL, "bad cube ranges");
    }
    if (o->spec_nb <= 0 || !(o->spec_hi > o->spec_lo)) return fail(THOR_E_INVAL, "bad spectrum bins");
    if (o->step_events && o->path != THOR_PATH_PERSISTENT)
        return fail(THOR_E_INVAL, "bounded steps need the persistent path");
    if (o->block && (o->block % 64 || o->block > 256)) return fail(THOR_E_INVAL, "block must be 64..256, multiple of 64");
    if (o->accum != THOR_ACCUM_F32_ATOMIC && o->accum != THOR_ACCUM_FIXED64) return fail(THOR_E_INVAL, "bad accum mode");
    if (o->fixed_bits < 0 || o->fixed_bits > 60) return fail(THOR_E_INVAL, "fixed_bits must be 0..60");
    return THOR_OK;
}

double fixed_scale(const thor_transport_opts* o) {
    return std::ldexp(1.0, o->fixed_bits > 0 ? o->fixed_bits : 40);
}

thor_status ensure_outputs(thor_ctx* ctx, const thor_transport_opts* o) {
    if (o->spec_nb != ctx->spec_nb) {
        dfree(ctx, ctx->d_spec, uint64_t(ctx->spec_nb) * 8 * kSpecCopies);
        ctx->d_spec = nullptr;
        ctx->spec_nb = 0;
        thor_status s = dalloc(ctx, (void**)&ctx->d_spec, uint64_t(o->spec_nb) * 8 * kSpecCopies, "spectrum");
        if (s) return s;
        ctx->spec_nb = o->spec_nb;
        HIPCHK(ctx, hipMemsetAsync(ctx->d_spec, 0, uint64_t(o->spec_nb) * 8 * kSpecCopies, ctx->stream));
    }
    const int fx = o->n_obs > 0 && o->accum == THOR_ACCUM_FIXED64;
    const int shape[5] = {o->n_obs, o->cube_ny, o->cube_nx, o->cube_nb, fx};
    if (std::memcmp(shape, ctx->cube_shape, sizeof shape) != 0 ||
        (fx && ctx->cube_fx_scale != fixed_scale(o))) {
        dfree(ctx, ctx->d_cube, ctx->cube_elems * 4);
        dfree(ctx, ctx->d_cube_fx, ctx->cube_elems * 8);
        ctx->d_cube = nullptr;
        ctx->d_cube_fx = nullptr;
        ctx->cube_elems = 0;
        ctx->cube_fx_scale = 0.0;
        std::memset(ctx->cube_shape, 0, sizeof ctx->cube_shape);
        if (o->n_obs > 0) {
            const uint64_t elems = uint64_t(o->n_obs) * o->cube_ny * o->cube_nx * o->cube_nb;
            if (fx) {
                thor_status s = dalloc(ctx, (void**)&ctx->d_cube_fx, elems * 8, "fixed-point cube");
                if (s) return s;
                HIPCHK(ctx, hipMemsetAsync(ctx->d_cube_fx, 0, elems * 8, ctx->stream));
                ctx->cube_fx_scale = fixed_scale(o);
            } else {
                thor_status s = dalloc(ctx, (void**)&ctx->d_cube, elems * 4, "cube");
                if (s) return s;
                HIPCHK(ctx, hipMemsetAsync(ctx->d_cube, 0, elems * 4, ctx->stream));
            }
            ctx->cube_elems = elems;
        }
        std::memcpy(ctx->cube_shape, shape, sizeof shape);
    }
    return THOR_OK;
}

template <class T>
thor_status ensure_array(thor_ctx* ctx, T** p, size_t* cap, size_t need, const char* what) {
    if (need <= *cap) return THOR_OK;
    size_t n = std::max(need, *cap * 2 + 16);
    dfree(ctx, *p, *cap * sizeof(T));
    *p = nullptr;
    *cap = 0;
    thor_status s = dalloc(ctx, (void**)p, n * sizeof(T), what);
    if (s) return s;
    *cap = n;
    return THOR_OK;
}

OutDev make_out(thor_ctx* ctx, const thor_transport_opts* o) {
    OutDev out;
    std::memset(&out, 0, sizeof out);
    out.phase = o->phase;
    out.n_obs = o->n_obs;
    for (int i = 0; i < 6; ++i) out.obs_axis[i] = o->obs_axis[i];
    out.cube_nx = o->cube_nx;
    out.cube_ny = o->cube_ny;
    out.cube_nb = o->cube_nb;
    for (int i = 0; i < 2; ++i) {
        out.img_lo[i] = o->img_lo[i];
        out.img_w[i] = o->n_obs ? (o->img_hi[i] - o->img_lo[i]) / (i == 0 ? o->cube_nx : o->cube_ny) : 1.0;
    }
    out.v_lo = o->cube_v_lo;
    out.v_w = o->n_obs ? (o->cube_v_hi - o->cube_v_lo) / o->cube_nb : 1.0;
    out.cube = ctx->d_cube;
    out.cube_fx = ctx->d_cube_fx;
    out.fx_scale = ctx->d_cube_fx ? ctx->cube_fx_scale : 0.0;
    out.tau_cut = o->tau_cut > 0.0 ? o->tau_cut : 40.0;
    out.max_events = o->max_events;
    return out;
}

// The presort of a call: 0 none, 1 spatial, 2 frequency.  The library
// default is spatial for grids with n_HI^2-weighted sources, by frequency
// for meshless media whose sources spread in frequency (Gaussian, flat,
// doublet lines), none otherwise.
int presort_mode(const thor_transport_opts* o, bool grid, bool any_cell, bool any_spread) {
    if (o->presort < 0) return 0;
    if (o->presort == 2) return 2;
    if (grid) return any_cell ? 1 : 0;
    return o->presort == 0 && any_spread ? 2 : 0;
}

// Lanes of a persistent wave that wait at their interaction sites before
// they interact together (0: each interacts when it gets there).
uint32_t park_lanes(const thor_transport_opts* o) {
    if (o->park_lanes < 0) return 0u;
    if (o->park_lanes == 0) return kDefaultParkLanes;
    return o->park_lanes > 64 ? 64u : uint32_t(o->park_lanes);
}

// Share (in 64ths) of a turn's lanes that must have finished before the turn
// ends early so that the wave refills them (64: only at the visit bound).
uint32_t refill_64ths(const thor_transport_opts* o) {
    if (o->refill_64ths <= 0) return 16u;
    return o->refill_64ths > 64 ? 64u : uint32_t(o->refill_64ths);
}

// Live lanes at or below which a persistent wave takes wide turns.
uint32_t wide_lanes(const thor_transport_opts* o) {
    if (o->wide_lanes < 0) return 0u;
    if (o->wide_lanes == 0) return 8u;
    return o->wide_lanes > 16 ? 16u : uint32_t(o->wide_lanes);
}

int launch_grid_size(thor_ctx* ctx, const thor_transport_opts* o, int block) {
    const int waves = o->waves_per_cu > 0 ? o->waves_per_cu : 8;
    const int wpb = block / 64;
    return std::max(1, ctx->num_cu * waves / wpb);
}

template <class R, bool GRID>
void launch_plain(thor_ctx* ctx, const BatchDev& b, const OutDev& out) {
    const unsigned blocks = unsigned((b.n + 255) / 256);
    hipLaunchKernelGGL((k_plain<R, GRID>), dim3(blocks), dim3(256), 0, ctx->stream, ctx->grid, ctx->d_models, b,
                       out, ctx->d_stats, ctx->d_xstats);
}

template <class R>
TailDev<R> tail_dev(thor_ctx* ctx, bool on) {
    if (!on) return TailDev<R>{nullptr, nullptr, nullptr, nullptr, nullptr, 0};
    return TailDev<R>{reinterpret_cast<Pkt<R>*>(ctx->d_tail_pk), ctx->d_tail_home, ctx->d_tailctl,
                      ctx->d_tailctl + 1, ctx->d_tailctl + 2, uint64_t(ctx->num_cu) * 4};
}

template <class R, bool GRID>
void launch_persistent(thor_ctx* ctx, hipStream_t stream, int grid, int block, const BatchDev* d_b,
                       const StepDesc* d_desc, unsigned long long* cursor, const OutDev& out,
                       const ModelDev* d_models, void* pool_pk, int* pool_alive, const SeedBuf& sb,
                       bool hand_off = false, unsigned long long* gmax = nullptr,
                       unsigned long long* gstats = nullptr, const uint64_t* perm = nullptr) {
    PoolDev<R> pool{reinterpret_cast<Pkt<R>*>(pool_pk), pool_alive};
    const TailDev<R> tail = tail_dev<R>(ctx, hand_off);
    if (!gstats) gstats = ctx->d_stats;
    bool seeds = false;
    if constexpr (GRID) seeds = sb.s != nullptr;
    if (seeds)
        hipLaunchKernelGGL((k_persistent<R, GRID, GRID>), dim3(grid), dim3(block), 0, stream, ctx->grid, d_models,
                           d_b, d_desc, cursor, out, pool, tail, sb, gstats, gmax, perm);
    else
        hipLaunchKernelGGL((k_persistent<R, GRID, false>), dim3(grid), dim3(block), 0, stream, ctx->grid, d_models,
                           d_b, d_desc, cursor, out, pool, tail, sb, gstats, gmax, perm);
}

// The tail kernel over what the preceding persistent launch handed off (its
// waves exit at once when nothing was).
template <class R, bool GRID>
void launch_tail(thor_ctx* ctx, const StepDesc* d_desc, const OutDev& out, void* pool_pk, int* pool_alive,
                 const SeedBuf& sb) {
    PoolDev<R> pool{reinterpret_cast<Pkt<R>*>(pool_pk), pool_alive};
    const TailDev<R> tail = tail_dev<R>(ctx, true);
    bool seeds = false;
    if constexpr (GRID) seeds = sb.s != nullptr;
    if (seeds)
        hipLaunchKernelGGL((k_tail<R, GRID, GRID>), dim3(ctx->num_cu * 4), dim3(64), 0, ctx->stream, ctx->grid,
                           ctx->d_models, d_desc, out, pool, tail, sb, ctx->d_xstats + 1, ctx->d_xstats);
    else
        hipLaunchKernelGGL((k_tail<R, GRID, false>), dim3(ctx->num_cu * 4), dim3(64), 0, ctx->stream, ctx->grid,
                           ctx->d_models, d_desc, out, pool, tail, sb, ctx->d_xstats + 1, ctx->d_xstats);
}

// Whether the peel pass takes its rays in sorted order (library default: yes).
bool seed_sort_on(const thor_transport_opts* o) { return o->seed_sort >= 0; }

// Arrays of the seed sort: keys (written by the transport kernels with each
// seed) and slot indices (0..cap-1, never changed), each with a second copy
// the sort writes.  Sets sb->keys when 32-bit keys suffice.
thor_status ensure_seed_sort(thor_ctx* ctx, SeedBuf* sb) {
    if (ctx->ssort_cap < ctx->seed_cap) {
        dfree(ctx, ctx->d_skeys, ctx->ssort_cap * 8);
        dfree(ctx, ctx->d_svals, ctx->ssort_cap * 8);
        ctx->d_skeys = nullptr;
        ctx->d_svals = nullptr;
        ctx->ssort_cap = 0;
        thor_status s = dalloc(ctx, (void**)&ctx->d_skeys, ctx->seed_cap * 8, "seed sort keys");
        if (s) return s;
        s = dalloc(ctx, (void**)&ctx->d_svals, ctx->seed_cap * 8, "seed sort slots");
        if (s) return s;
        ctx->ssort_cap = ctx->seed_cap;
        hipLaunchKernelGGL(k_iota_u32, dim3(ctx->num_cu * 8), dim3(256), 0, ctx->stream, ctx->d_svals, ctx->ssort_cap);
        HIPCHK(ctx, hipGetLastError());
    }
    const uint64_t nx = uint64_t(ctx->grid.nx), ny = uint64_t(ctx->grid.ny), nz = uint64_t(ctx->grid.nz);
    const uint64_t blocks = std::max(ny * nz * ((nx + 255) / 256),
                                     std::max(nz * nx * ((ny + 255) / 256), ny * nx * ((nz + 255) / 256)));
    sb->keys = nullptr;
    sb->key_blocks = 0;
    if (3 * blocks < (uint64_t(1) << 32)) {          // else: too many pencils for 32-bit keys, buffer order
        sb->keys = ctx->d_skeys;
        sb->key_blocks = uint32_t(blocks);
    }
    return THOR_OK;
}

thor_status fuse_seeds(thor_ctx* ctx, const OutDev& out, SeedBuf* sb, uint64_t n, int m);

// Sorts the first n slots of the seed buffer by the keys the transport
// kernels wrote (seed_key) into sb->order; photon fusing sorts by its own keys.
thor_status sort_seeds(thor_ctx* ctx, const OutDev& out, SeedBuf* sb, uint64_t n, int fuse_bins) {
    if (fuse_bins > 0) return fuse_seeds(ctx, out, sb, n, fuse_bins);
    if (!sb->keys) return THOR_OK;
    uint32_t* keys = ctx->d_skeys;
    uint32_t* keys2 = ctx->d_skeys + ctx->ssort_cap;
    uint32_t* vals = ctx->d_svals;
    uint32_t* vals2 = ctx->d_svals + ctx->ssort_cap;
    // slots claimed but left empty keep stale keys: they sort anywhere and the
    // pass skips them
    const uint64_t top = 3 * uint64_t(sb->key_blocks);
    int end_bit = 1;
    while (end_bit < 32 && (uint64_t(1) << end_bit) < top) ++end_bit;
    size_t need = 0;
    HIPCHK(ctx, hipcub::DeviceRadixSort::SortPairs(nullptr, need, keys, keys2, vals, vals2, (int64_t)n, 0, end_bit,
                                                   ctx->stream));
    if (need > ctx->ssort_tmp_bytes) {
        dfree(ctx, ctx->d_ssort_tmp, ctx->ssort_tmp_bytes);
        ctx->d_ssort_tmp = nullptr;
        ctx->ssort_tmp_bytes = 0;
        thor_status s = dalloc(ctx, &ctx->d_ssort_tmp, need, "seed sort scratch");
        if (s) return s;
        ctx->ssort_tmp_bytes = need;
    }
    size_t tmp = ctx->ssort_tmp_bytes;
    HIPCHK(ctx, hipcub::DeviceRadixSort::SortPairs(ctx->d_ssort_tmp, tmp, keys, keys2, vals, vals2, (int64_t)n, 0,
                                                   end_bit, ctx->stream));
    sb->order = vals2;
    return THOR_OK;
}

// Photon fusing (Section 3.4.1): the round's seeds sorted by the fusing key
// (k_fuse_keys), runs merged (k_seed_fuse); sb->order is the sorted order.
thor_status fuse_seeds(thor_ctx* ctx, const OutDev& out, SeedBuf* sb, uint64_t n, int m) {
    sb->keys = nullptr;                 // the transport's keys are not used here
    if (ctx->fkeys_cap < ctx->ssort_cap) {
        dfree(ctx, ctx->d_fkeys, ctx->fkeys_cap * 16);
        ctx->d_fkeys = nullptr;
        ctx->fkeys_cap = 0;
        thor_status s = dalloc(ctx, (void**)&ctx->d_fkeys, ctx->ssort_cap * 16, "fusing keys");
        if (s) return s;
        ctx->fkeys_cap = ctx->ssort_cap;
    }
    uint64_t* keys = ctx->d_fkeys;
    uint64_t* keys2 = ctx->d_fkeys + ctx->fkeys_cap;
    uint32_t* vals = ctx->d_svals;
    uint32_t* vals2 = ctx->d_svals + ctx->ssort_cap;
    const uint64_t top = uint64_t(out.n_obs) * ctx->grid.ncell * uint64_t(out.cube_nb) * uint64_t(m);   // empty key
    if (top == 0 || top / uint64_t(out.n_obs) / uint64_t(out.cube_nb) / uint64_t(m) != ctx->grid.ncell)
        return fail(THOR_E_INVAL, "fusing keys overflow 64 bits (grid x bins x fuse_bins too large)");
    int end_bit = 1;
    while (end_bit < 64 && (uint64_t(1) << end_bit) <= top) ++end_bit;
    size_t need = 0;
    HIPCHK(ctx, hipcub::DeviceRadixSort::SortPairs(nullptr, need, keys, keys2, vals, vals2, (int64_t)n, 0, end_bit,
                                                   ctx->stream));
    if (need > ctx->ssort_tmp_bytes) {
        dfree(ctx, ctx->d_ssort_tmp, ctx->ssort_tmp_bytes);
        ctx->d_ssort_tmp = nullptr;
        ctx->ssort_tmp_bytes = 0;
        thor_status s = dalloc(ctx, &ctx->d_ssort_tmp, need, "seed sort scratch");
        if (s) return s;
        ctx->ssort_tmp_bytes = need;
    }
    hipLaunchKernelGGL(k_fuse_keys, dim3(ctx->num_cu * 8), dim3(256), 0, ctx->stream, ctx->grid, out, *sb, n, m, keys,
                       vals);
    HIPCHK(ctx, hipGetLastError());
    size_t tmp = ctx->ssort_tmp_bytes;
    HIPCHK(ctx, hipcub::DeviceRadixSort::SortPairs(ctx->d_ssort_tmp, tmp, keys, keys2, vals, vals2, (int64_t)n, 0,
                                                   end_bit, ctx->stream));
    hipLaunchKernelGGL(k_seed_fuse, dim3(ctx->num_cu * 8), dim3(256), 0, ctx->stream, *sb, keys2, vals2, n, top,
                       ctx->d_fused);
    HIPCHK(ctx, hipGetLastError());
    sb->order = vals2;
    return THOR_OK;
}

// Tail list of `slots` packets of either precision.
thor_status ensure_tail(thor_ctx* ctx, uint64_t slots) {
    if (ctx->d_tail_pk && ctx->tail_slots >= slots) return THOR_OK;
    dfree(ctx, ctx->d_tail_pk, ctx->tail_slots * sizeof(Pkt<double>));
    dfree(ctx, ctx->d_tail_home, ctx->tail_slots * 4);
    ctx->d_tail_pk = nullptr;
    ctx->d_tail_home = nullptr;
    ctx->tail_slots = 0;
    static_assert(sizeof(Pkt<double>) >= sizeof(Pkt<float>), "tail slots sized for FP64 packets");
    thor_status s = dalloc(ctx, &ctx->d_tail_pk, slots * sizeof(Pkt<double>), "tail list");
    if (s) return s;
    s = dalloc(ctx, (void**)&ctx->d_tail_home, slots * 4, "tail list homes");
    if (s) return s;
    if (!ctx->d_tailctl) {
        s = dalloc(ctx, (void**)&ctx->d_tailctl, 3 * 8, "tail list counters");
        if (s) return s;
    }
    ctx->tail_slots = slots;
    return THOR_OK;
}

// Peel seed buffer of the grid persistent path (slots of 48 B, all empty).
thor_status ensure_seeds(thor_ctx* ctx, uint64_t slots, SeedBuf* sb) {
    if (ctx->seed_cap != slots) {
        dfree(ctx, ctx->d_seeds, ctx->seed_cap * sizeof(PeelSeed));
        ctx->d_seeds = nullptr;
        ctx->seed_cap = 0;
        thor_status s = dalloc(ctx, (void**)&ctx->d_seeds, slots * sizeof(PeelSeed), "peel seed buffer");
        if (s) return s;
        ctx->seed_cap = slots;
        hipLaunchKernelGGL(k_seed_clear, dim3(ctx->num_cu * 8), dim3(256), 0, ctx->stream, ctx->d_seeds, slots);
    }
    if (!ctx->d_seedctl) {
        thor_status s = dalloc(ctx, (void**)&ctx->d_seedctl, (2 + kXcds) * 8, "peel seed counters");
        if (s) return s;
    }
    sb->s = ctx->d_seeds;
    sb->order = nullptr;
    sb->cap = ctx->seed_cap;
    sb->count = ctx->d_seedctl;
    sb->parked = ctx->d_seedctl + 1;
    return THOR_OK;
}

template <class R, class V>
void launch_peel_pass_v(thor_ctx* ctx, const OutDev& out, const SeedBuf& sb) {
    const bool compact = !(ctx->grid.sigma_d > 0.0);     // the records ensure_axis_records built
    if constexpr (sizeof(R) == 4) {
        if (compact)
            hipLaunchKernelGGL((k_peel_pass_f32<V, AxisRec3>), dim3(ctx->num_cu * 6), dim3(256), 0, ctx->stream,
                               ctx->grid, out, sb, ctx->d_seedctl + 2, ctx->d_stats);
        else
            hipLaunchKernelGGL((k_peel_pass_f32<V, AxisRec>), dim3(ctx->num_cu * 6), dim3(256), 0, ctx->stream,
                               ctx->grid, out, sb, ctx->d_seedctl + 2, ctx->d_stats);
    }
    else
        hipLaunchKernelGGL(k_peel_pass_f64<V>, dim3(ctx->num_cu * 4), dim3(256), 0, ctx->stream, ctx->grid, out, sb,
                           ctx->d_seedctl + 2, ctx->d_stats);
}

template <class R>
void launch_peel_pass(thor_ctx* ctx, const OutDev& out, const SeedBuf& sb) {
    if (out.cube_fx) launch_peel_pass_v<R, unsigned long long>(ctx, out, sb);
    else launch_peel_pass_v<R, float>(ctx, out, sb);
}

thor_status ensure_pool(thor_ctx* ctx, uint64_t slots, int prec) {
    const uint64_t pk_bytes = prec == THOR_PREC_FP64 ? sizeof(Pkt<double>) : sizeof(Pkt<float>);
    if (ctx->d_pool_pk && ctx->pool_slots == slots && ctx->pool_prec == prec) return THOR_OK;
    dfree(ctx, ctx->d_pool_pk, ctx->pool_bytes);
    dfree(ctx, ctx->d_pool_alive, ctx->pool_slots * 4);
    ctx->d_pool_pk = nullptr;
    ctx->d_pool_alive = nullptr;
    ctx->pool_slots = 0;
    thor_status s = dalloc(ctx, &ctx->d_pool_pk, slots * pk_bytes, "packet pool");
    if (s) return s;
    ctx->pool_bytes = slots * pk_bytes;
    s = dalloc(ctx, (void**)&ctx->d_pool_alive, slots * 4, "packet pool flags");
    if (s) return s;
    ctx->pool_slots = slots;
    ctx->pool_prec = prec;
    HIPCHK(ctx, hipMemsetAsync(ctx->d_pool_alive, 0, slots * 4, ctx->stream));
    return THOR_OK;
}

void collect_stats(thor_ctx* ctx, const unsigned long long* h, float ms, thor_stats* st) {
    std::memset(st, 0, sizeof *st);
    uint64_t* dst[kNumU64Counters] = {&st->emitted, &st->escaped, &st->absorbed, &st->capped, &st->handed_off,
                                      &st->n_res, &st->n_dust, &st->main_visits, &st->peel_visits,
                                      &st->peel_contrib, &st->peel_dropped, &st->peel_cut, &st->upar_trials,
                                      &st->redshifted};
    for (int i = 0; i < kNumU64Counters; ++i) *dst[i] = h[i];
    st->w_escaped = double(st->escaped);     // packet weights are 1
    st->w_absorbed = double(st->absorbed);
    st->kernel_ms = ms;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* thor_last_error(void) { return g_last_error.c_str(); }

thor_status thor_create(thor_ctx** out, int hip_device, void* hip_stream, uint64_t hbm_budget_bytes) {
    if (!out) return fail(THOR_E_INVAL, "null output pointer");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(THOR_E_DEVICE, "no HIP device");
    if (hip_device < 0 || hip_device >= ndev) return fail(THOR_E_INVAL, "device %d out of range", hip_device);
    if (hipSetDevice(hip_device) != hipSuccess) return fail(THOR_E_DEVICE, "hipSetDevice failed");
    thor_ctx* ctx = new thor_ctx();
    ctx->device = hip_device;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    ctx->budget = hbm_budget_bytes;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, hip_device) == hipSuccess && ncu > 0)
        ctx->num_cu = ncu;
    static double t64[kDawsonIntervals * (kDawsonDeg64 + 1)];
    static float t32[kDawsonIntervals * (kDawsonDeg32 + 1)];
    static bool built = false;
    if (!built) { build_dawson_tables(t64, t32); built = true; }
    thor_status s = THOR_OK;
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_dawson64), t64, sizeof t64) != hipSuccess ||
        hipMemcpyToSymbol(HIP_SYMBOL(c_dawson32), t32, sizeof t32) != hipSuccess)
        s = fail(THOR_E_DEVICE, "Dawson table upload failed");
    if (!s) s = dalloc(ctx, (void**)&ctx->d_stats, (kNumU64Counters + 1) * 8, "counters");
    if (!s) s = dalloc(ctx, (void**)&ctx->d_xstats, (kNumU64Counters + 1) * 8, "tail counters");
    if (!s && (hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess ||
               hipEventCreate(&ctx->ev_a) != hipSuccess || hipEventCreate(&ctx->ev_b) != hipSuccess ||
               hipEventCreate(&ctx->ev_c) != hipSuccess || hipEventCreate(&ctx->ev_s) != hipSuccess))
        s = fail(THOR_E_DEVICE, "hipEventCreate failed");
    if (!s) {
        // the no-allocation scratch of this device (hipSetDevice above made it current)
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (hip_device < kMaxDevices && !g_scratch_ptr[hip_device]) {
            void* p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
                s = fail(THOR_E_DEVICE, "hipGetSymbolAddress of the no-allocation scratch failed");
            else
                g_scratch_ptr[hip_device] = static_cast<unsigned char*>(p);
        }
        if (hip_device < kMaxDevices) ctx->d_scratch = g_scratch_ptr[hip_device];
    }
    if (!s) s = dalloc(ctx, (void**)&ctx->d_desc, sizeof(StepDesc), "step descriptor");
    if (!s && hipHostMalloc((void**)&ctx->h_desc, sizeof(StepDesc)) != hipSuccess)
        s = fail(THOR_E_NOMEM, "pinned host allocation failed");
    if (s) {
        thor_destroy(ctx);
        return s;
    }
    *out = ctx;
    return THOR_OK;
}

void thor_destroy(thor_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    void* ptrs[] = {ctx->d_rec, ctx->d_cdf, ctx->d_spec, ctx->d_cube, ctx->d_cube_fx, ctx->d_stats,
                    ctx->d_models, ctx->d_batches, ctx->d_rec_dv, ctx->d_rec_nres, ctx->d_rec_ndust,
                    ctx->d_rec_fate, ctx->d_pool_pk, ctx->d_pool_alive, ctx->d_done,
                    ctx->d_s_models, ctx->d_s_batches, ctx->d_s_cursor, ctx->d_s_pool, ctx->d_s_alive,
                    ctx->d_seeds, ctx->d_seedctl, ctx->d_axr[0], ctx->d_axr[1], ctx->d_axr[2],
                    ctx->d_tail_pk, ctx->d_tail_home, ctx->d_tailctl, ctx->d_xstats, ctx->d_sort,
                    ctx->d_sort_tmp, ctx->d_skeys, ctx->d_svals, ctx->d_ssort_tmp, ctx->d_fkeys, ctx->d_fused};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (auto& kv : ctx->s_reqs)
        if (kv.second.d_spec) (void)hipFree(kv.second.d_spec);
    void* dev2[] = {ctx->d_desc, ctx->d_s_desc};
    for (void* p : dev2)
        if (p) (void)hipFree(p);
    void* pinned[] = {ctx->h_desc, ctx->h_s_desc, ctx->h_s_batches, ctx->h_s_done, ctx->h_s_misc};
    for (void* p : pinned)
        if (p) (void)hipHostFree(p);
    if (ctx->s_graph) (void)hipGraphExecDestroy(ctx->s_graph);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    if (ctx->ev_a) (void)hipEventDestroy(ctx->ev_a);
    if (ctx->ev_b) (void)hipEventDestroy(ctx->ev_b);
    if (ctx->ev_c) (void)hipEventDestroy(ctx->ev_c);
    if (ctx->ev_s) (void)hipEventDestroy(ctx->ev_s);
    delete ctx;
}

void free_axis_records(thor_ctx* ctx) {
    for (int a = 0; a < 3; ++a) {
        dfree(ctx, ctx->d_axr[a], ctx->axr_bytes[a]);
        ctx->d_axr[a] = nullptr;
        ctx->axr_bytes[a] = 0;
        ctx->grid.axr[a] = nullptr;
        ctx->grid.axc[a] = nullptr;
    }
}

// Pencil records for peel rays along axis a (mixed precision), built once per
// grid from the cell records; staging, outside the timed transport.  Compact
// (12 B) when the grid has no dust.
thor_status ensure_axis_records(thor_ctx* ctx, int a) {
    if (ctx->d_axr[a]) return THOR_OK;
    const uint64_t cells = ctx->grid.ncell;
    const bool compact = !(ctx->grid.sigma_d > 0.0);
    const uint64_t bytes = cells * (compact ? sizeof(AxisRec3) : sizeof(AxisRec));
    thor_status s = dalloc(ctx, &ctx->d_axr[a], bytes, "axis records");
    if (s) return s;
    ctx->axr_bytes[a] = bytes;
    if (compact) {
        hipLaunchKernelGGL(k_pack_axis<AxisRec3>, dim3(ctx->num_cu * 8), dim3(256), 0, ctx->stream, ctx->d_rec,
                           static_cast<AxisRec3*>(ctx->d_axr[a]), a, ctx->grid.nx, ctx->grid.ny, ctx->grid.nz,
                           ctx->grid.sigma_d, cells);
        ctx->grid.axc[a] = static_cast<const AxisRec3*>(ctx->d_axr[a]);
    } else {
        hipLaunchKernelGGL(k_pack_axis<AxisRec>, dim3(ctx->num_cu * 8), dim3(256), 0, ctx->stream, ctx->d_rec,
                           static_cast<AxisRec*>(ctx->d_axr[a]), a, ctx->grid.nx, ctx->grid.ny, ctx->grid.nz,
                           ctx->grid.sigma_d, cells);
        ctx->grid.axr[a] = static_cast<const AxisRec*>(ctx->d_axr[a]);
    }
    HIPCHK(ctx, hipGetLastError());
    return THOR_OK;
}

thor_status thor_load_grid(thor_ctx* ctx, const thor_geometry* g) {
    CHECK_CTX(ctx);
    if (!g) return fail(THOR_E_INVAL, "null geometry");
    if (g->kind < 0 || g->kind > 2) return fail(THOR_E_INVAL, "bad geometry kind %d", g->kind);
    if (g->albedo < 0.0 || g->albedo > 1.0) return fail(THOR_E_INVAL, "albedo must be in [0, 1]");
    if (g->g_hg <= -1.0 || g->g_hg >= 1.0) return fail(THOR_E_INVAL, "g_hg must be in (-1, 1)");
    if (g->line < THOR_LINE_LYA || g->line > THOR_LINE_MG2K) return fail(THOR_E_INVAL, "bad line %d", g->line);
    if (g->line != THOR_LINE_LYA && g->kind == THOR_GEOM_GRID)
        return fail(THOR_E_UNSUPPORTED, "the Mg II lines need a meshless medium");
    if (g->kind != THOR_GEOM_GRID) {
        if (!(g->r_outer > g->r_inner) || g->r_inner < 0.0) return fail(THOR_E_INVAL, "need 0 <= r_inner < r_outer");
        if (!(g->T > 0.0)) return fail(THOR_E_INVAL, "T must be positive");
        if (g->n_HI < 0.0 || g->tau0 < 0.0 || (g->n_HI == 0.0 && g->tau0 == 0.0))
            return fail(THOR_E_INVAL, "need n_HI > 0 or tau0 > 0");
        if (g->v_profile < 0 || g->v_profile > 2) return fail(THOR_E_INVAL, "bad velocity profile");
        if (g->kind == THOR_GEOM_SLAB && g->v_profile == THOR_VEL_CONST_RADIAL)
            return fail(THOR_E_UNSUPPORTED, "slab supports NONE or LINEAR velocity");
        if (g->tau_d > 0.0 && g->n_HI == 0.0 && g->tau0 == 0.0) return fail(THOR_E_INVAL, "dust needs gas");
        // release a previous grid
        free_axis_records(ctx);
        dfree(ctx, ctx->d_rec, ctx->grid_bytes);
        dfree(ctx, ctx->d_cdf, ctx->cdf_bytes);
        ctx->d_rec = nullptr; ctx->d_cdf = nullptr;
        ctx->grid_bytes = ctx->cdf_bytes = 0;
        std::memset(&ctx->grid, 0, sizeof ctx->grid);
        ctx->geom = *g;
        ctx->geom.n_HI_field = ctx->geom.T_field = ctx->geom.vx = ctx->geom.vy = ctx->geom.vz = nullptr;
        ctx->has_geom = true;
        ctx->pending.clear();
        return THOR_OK;
    }
    if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0) return fail(THOR_E_INVAL, "bad grid dimensions");
    if (!(g->hubble >= 0.0) || !(g->hubble_step >= 0.0) || !(g->stop_dv >= 0.0))
        return fail(THOR_E_INVAL, "hubble, hubble_step and stop_dv must be >= 0");
    for (int i = 0; i < 3; ++i)
        if (!(g->hi[i] > g->lo[i])) return fail(THOR_E_INVAL, "grid needs lo < hi");
    if (!g->n_HI_field || !g->T_field || !g->vx || !g->vy || !g->vz) return fail(THOR_E_INVAL, "null grid field");
    if (g->mem != THOR_MEM_HOST && g->mem != THOR_MEM_DEVICE) return fail(THOR_E_INVAL, "bad memory kind");
    const uint64_t cells = uint64_t(g->nx) * g->ny * g->nz;
    const uint64_t need = cells * sizeof(CellRec);
    const uint64_t staging = g->mem == THOR_MEM_HOST ? cells * 20 : 0;
    const uint64_t freed = ctx->grid_bytes + ctx->cdf_bytes;
    if (ctx->budget && ctx->used - std::min(ctx->used, freed) + need + staging > ctx->budget)
        return fail(THOR_E_BUDGET, "grid of %llu cells exceeds the HBM budget", (unsigned long long)cells);
    free_axis_records(ctx);
    dfree(ctx, ctx->d_rec, ctx->grid_bytes);
    dfree(ctx, ctx->d_cdf, ctx->cdf_bytes);
    ctx->d_rec = nullptr; ctx->d_cdf = nullptr;
    ctx->grid_bytes = ctx->cdf_bytes = 0;
    ctx->has_geom = false;
    ctx->pending.clear();
    thor_status s = dalloc(ctx, (void**)&ctx->d_rec, need, "grid records");
    if (s) return s;
    ctx->grid_bytes = need;
    const float *n = g->n_HI_field, *vx = g->vx, *vy = g->vy, *vz = g->vz, *T = g->T_field;
    float* stage = nullptr;
    if (g->mem == THOR_MEM_HOST) {
        s = dalloc(ctx, (void**)&stage, cells * 20, "grid staging");
        if (s) return s;
        const hipMemcpyKind kind = hipMemcpyHostToDevice;
        HIPCHK(ctx, hipMemcpyAsync(stage, g->n_HI_field, cells * 4, kind, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(stage + cells, g->vx, cells * 4, kind, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(stage + 2 * cells, g->vy, cells * 4, kind, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(stage + 3 * cells, g->vz, cells * 4, kind, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(stage + 4 * cells, g->T_field, cells * 4, kind, ctx->stream));
        n = stage; vx = stage + cells; vy = stage + 2 * cells; vz = stage + 3 * cells; T = stage + 4 * cells;
    }
    HIPCHK(ctx, hipMemsetAsync(ctx->d_stats, 0, 8, ctx->stream));
    hipLaunchKernelGGL(k_pack_grid, dim3(4096), dim3(256), 0, ctx->stream, n, vx, vy, vz, T, ctx->d_rec, cells,
                       ctx->d_stats);
    HIPCHK(ctx, hipGetLastError());
    unsigned long long nbad = 0;
    HIPCHK(ctx, hipMemcpyAsync(&nbad, ctx->d_stats, 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (stage) dfree(ctx, stage, cells * 20);
    if (nbad) {
        dfree(ctx, ctx->d_rec, ctx->grid_bytes);
        ctx->d_rec = nullptr; ctx->grid_bytes = 0;
        return fail(THOR_E_INVAL, "%llu grid cells are not finite, have n_HI < 0 or gas at T <= 0", nbad);
    }
    ctx->geom = *g;
    ctx->geom.n_HI_field = ctx->geom.T_field = ctx->geom.vx = ctx->geom.vy = ctx->geom.vz = nullptr;
    GridDev& gd = ctx->grid;
    std::memset(&gd, 0, sizeof gd);
    gd.nx = g->nx; gd.ny = g->ny; gd.nz = g->nz;
    gd.handoff = g->boundary_handoff;
    const int dims[3] = {g->nx, g->ny, g->nz};
    for (int i = 0; i < 3; ++i) {
        gd.lo[i] = g->lo[i];
        gd.dx[i] = (g->hi[i] - g->lo[i]) / dims[i];
    }
    gd.rec = ctx->d_rec;
    gd.ncell = cells;
    gd.sigma_d = g->sigma_d;
    gd.hubble = g->hubble;
    for (int i = 0; i < 3; ++i) gd.href[i] = g->hubble_ref[i];
    gd.hstep = g->hubble_step > 0.0 ? g->hubble_step : 0.1;
    gd.stop_dv = g->stop_dv;
    ctx->has_geom = true;
    return THOR_OK;
}

thor_status thor_emit(thor_ctx* ctx, const thor_source* src, uint64_t n_packets, uint64_t first_photon_id) {
    CHECK_CTX(ctx);
    if (!src) return fail(THOR_E_INVAL, "null source");
    if (!ctx->has_geom) return fail(THOR_E_STATE, "thor_load_grid first");
    if (src->kind != THOR_SRC_POINT && src->kind != THOR_SRC_CELL_N2) return fail(THOR_E_INVAL, "bad source kind");
    if (src->spectrum < 0 || src->spectrum > 3) return fail(THOR_E_INVAL, "bad source spectrum");
    if ((src->spectrum == THOR_SPEC_GAUSS || src->spectrum == THOR_SPEC_FLAT) && src->sigma_v < 0.0)
        return fail(THOR_E_INVAL, "sigma_v < 0");
    if (src->lines != 0 && src->lines != 1) return fail(THOR_E_INVAL, "lines must be 0 or 1");
    if (src->kind == THOR_SRC_CELL_N2 && ctx->geom.kind != THOR_GEOM_GRID)
        return fail(THOR_E_INVAL, "CELL_N2 sources need a grid");
    if (src->spectrum == THOR_SPEC_THERMAL && ctx->geom.kind != THOR_GEOM_GRID)
        return fail(THOR_E_UNSUPPORTED, "THERMAL sources need a grid");
    if (n_packets == 0) return THOR_OK;
    if (src->kind == THOR_SRC_CELL_N2 && !ctx->d_cdf) {
        // inclusive prefix sum of n_HI^2 (FP64) over cells in x-fastest order
        const uint64_t cells = ctx->grid.ncell;
        thor_status s = dalloc(ctx, (void**)&ctx->d_cdf, cells * 8, "emission CDF");
        if (s) return s;
        ctx->cdf_bytes = cells * 8;
        hipcub::TransformInputIterator<double, NSquared, const CellRec*> it(ctx->d_rec, NSquared());
        size_t tmp_bytes = 0;
        HIPCHK(ctx, hipcub::DeviceScan::InclusiveSum(nullptr, tmp_bytes, it, ctx->d_cdf, (int64_t)cells, ctx->stream));
        void* tmp = nullptr;
        s = dalloc(ctx, &tmp, tmp_bytes, "scan scratch");
        if (s) return s;
        HIPCHK(ctx, hipcub::DeviceScan::InclusiveSum(tmp, tmp_bytes, it, ctx->d_cdf, (int64_t)cells, ctx->stream));
        double total = 0.0;
        HIPCHK(ctx, hipMemcpyAsync(&total, ctx->d_cdf + cells - 1, 8, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        dfree(ctx, tmp, tmp_bytes);
        if (!(total > 0.0)) return fail(THOR_E_INVAL, "grid has no gas to emit from");
        ctx->grid.cdf = ctx->d_cdf;
        ctx->grid.cdf_total = total;
    }
    BatchHost b;
    b.src = *src;
    b.n = n_packets;
    b.first_id = first_photon_id;
    b.q0 = 0;
    ctx->pending.push_back(b);
    return THOR_OK;
}

thor_status thor_reset_outputs(thor_ctx* ctx) {
    CHECK_CTX(ctx);
    if (ctx->d_spec)
        HIPCHK(ctx, hipMemsetAsync(ctx->d_spec, 0, uint64_t(ctx->spec_nb) * 8 * kSpecCopies, ctx->stream));
    if (ctx->d_cube) HIPCHK(ctx, hipMemsetAsync(ctx->d_cube, 0, ctx->cube_elems * 4, ctx->stream));
    if (ctx->d_cube_fx) HIPCHK(ctx, hipMemsetAsync(ctx->d_cube_fx, 0, ctx->cube_elems * 8, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return THOR_OK;
}

thor_status thor_transport(thor_ctx* ctx, const thor_transport_opts* opt, thor_stats* out_stats) {
    CHECK_CTX(ctx);
    thor_status s = check_opts(opt);
    if (s) return s;
    if (!ctx->has_geom) return fail(THOR_E_STATE, "thor_load_grid first");
    const bool grid = ctx->geom.kind == THOR_GEOM_GRID;
    const bool fp64 = opt->precision == THOR_PREC_FP64;
    const bool bounded = opt->step_events > 0;
    // a bounded persistent run in progress continues without new batches
    const bool resuming = bounded && ctx->q_total > 0;
    if (ctx->pending.empty() && !resuming) {
        if (out_stats) std::memset(out_stats, 0, sizeof *out_stats);
        return THOR_OK;
    }
    s = ensure_outputs(ctx, opt);
    if (s) return s;
    // models and queue layout of the pending batches
    const size_t nb = ctx->pending.size();
    std::vector<ModelDev> models(nb);
    std::vector<BatchDev> batches(nb);
    uint64_t q = 0;
    for (size_t i = 0; i < nb; ++i) {
        s = make_model(ctx, ctx->pending[i].src, *opt, models[i]);
        if (s) return s;
        batches[i].q0 = q;
        batches[i].first_id = ctx->pending[i].first_id;
        batches[i].n = ctx->pending[i].n;
        batches[i].model = int(i);
        batches[i].pad = 0;
        q += ctx->pending[i].n;
    }
    const uint64_t q_end = q;
    s = ensure_array(ctx, &ctx->d_models, &ctx->models_cap, nb, "models");
    if (s) return s;
    s = ensure_array(ctx, &ctx->d_batches, &ctx->batches_cap, nb, "batches");
    if (s) return s;
    OutDev out = make_out(ctx, opt);
    if (opt->records) {
        if (q_end > ctx->rec_cap) {
            dfree(ctx, ctx->d_rec_dv, ctx->rec_cap * 8);
            dfree(ctx, ctx->d_rec_nres, ctx->rec_cap * 4);
            dfree(ctx, ctx->d_rec_ndust, ctx->rec_cap * 4);
            dfree(ctx, ctx->d_rec_fate, ctx->rec_cap * 4);
            ctx->d_rec_dv = nullptr; ctx->d_rec_nres = nullptr; ctx->d_rec_ndust = nullptr; ctx->d_rec_fate = nullptr;
            ctx->rec_cap = 0;
            s = dalloc(ctx, (void**)&ctx->d_rec_dv, q_end * 8, "records");
            if (!s) s = dalloc(ctx, (void**)&ctx->d_rec_nres, q_end * 4, "records");
            if (!s) s = dalloc(ctx, (void**)&ctx->d_rec_ndust, q_end * 4, "records");
            if (!s) s = dalloc(ctx, (void**)&ctx->d_rec_fate, q_end * 4, "records");
            if (s) return s;
            ctx->rec_cap = q_end;
        }
        out.rec_dv = ctx->d_rec_dv;
        out.rec_nres = ctx->d_rec_nres;
        out.rec_ndust = ctx->d_rec_ndust;
        out.rec_fate = ctx->d_rec_fate;
        out.q_rec0 = 0;
        ctx->rec_n = q_end;
    } else {
        ctx->rec_n = 0;
    }
    HIPCHK(ctx, hipMemcpyAsync(ctx->d_models, models.data(), nb * sizeof(ModelDev), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(ctx->d_batches, batches.data(), nb * sizeof(BatchDev), hipMemcpyHostToDevice, ctx->stream));
    if (!resuming) {
        HIPCHK(ctx, hipMemsetAsync(ctx->d_stats, 0, (kNumU64Counters + 1) * 8, ctx->stream));
    } else {
        HIPCHK(ctx, hipMemsetAsync(ctx->d_stats, 0, kNumU64Counters * 8, ctx->stream));
    }
    HIPCHK(ctx, hipMemsetAsync(ctx->d_xstats, 0, (kNumU64Counters + 1) * 8, ctx->stream));
    if (grid && opt->path == THOR_PATH_PERSISTENT && !fp64 && opt->n_obs > 0 && opt->n_obs <= kMaxSeedObs &&
        !opt->inline_peel) {
        for (int i = 0; i < opt->n_obs; ++i) {
            s = ensure_axis_records(ctx, opt->obs_axis[i] % 3);
            if (s) return s;
        }
    }
    HIPCHK(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    ctx->split_passes = 0;
    ctx->split_tail = 0.0;
    if (opt->path == THOR_PATH_PLAIN) {
        for (size_t i = 0; i < nb; ++i) {
            if (fp64) grid ? launch_plain<double, true>(ctx, batches[i], out) : launch_plain<double, false>(ctx, batches[i], out);
            else grid ? launch_plain<float, true>(ctx, batches[i], out) : launch_plain<float, false>(ctx, batches[i], out);
        }
    } else {
        const int block = opt->block > 0 ? opt->block : 256;
        const int gsize = launch_grid_size(ctx, opt, block);
        const uint32_t turn = opt->visits_per_turn > 0 ? uint32_t(opt->visits_per_turn) : 256u;
        if (opt->step_events > 0xFFFFFFFFull) return fail(THOR_E_INVAL, "step_events must fit 32 bits");
        // unbounded calls hand the last packets of drained waves to k_tail
        // the tail kernel's events run on draws evaluated ahead for one line;
        // doublet packets stay in the persistent kernel
        const bool hand_off = !bounded && wide_lanes(opt) > 0 && ctx->geom.line == THOR_LINE_LYA;
        *ctx->h_desc = StepDesc{q_end, int(nb), uint32_t(opt->step_events), turn, hand_off ? wide_lanes(opt) : 0u,
                                park_lanes(opt), refill_64ths(opt), 0u};
        HIPCHK(ctx, hipMemcpyAsync(ctx->d_desc, ctx->h_desc, sizeof(StepDesc), hipMemcpyHostToDevice, ctx->stream));
        if (bounded) {
            s = ensure_pool(ctx, uint64_t(gsize) * block, opt->precision);
            if (s) return s;
        }
        SeedBuf sb;
        std::memset(&sb, 0, sizeof sb);
        const bool seeds = grid && opt->n_obs > 0 && opt->n_obs <= kMaxSeedObs && !opt->inline_peel;
        if (seeds) {
            // default: the largest power of two from 2^28 to 2^30 slots whose
            // seeds and sort arrays (64 B a slot) take at most half of the device
            // memory free (and of the budget left); else 2^28 (12.9 GB), else
            // 2^26 (3.2 GB) or two runs of kSeedChunk per lane when that much
            // cannot be had; a smaller buffer shrinks the runs, down to one
            // event's rays.  More seeds per round put more rays on each pencil,
            // so the rays a peel-pass wave marches share more cache lines.
            const uint64_t lanes = uint64_t(gsize) * block;
            const uint64_t ev_rays = uint64_t(opt->n_obs);
            const uint64_t small = std::max<uint64_t>(uint64_t(1) << 26, lanes * 2 * kSeedChunk);
            const uint64_t base = std::max<uint64_t>(uint64_t(1) << 28, small);
            uint64_t slots = opt->seed_slots;
            if (!slots) {
                size_t free_b = 0, total_b = 0;
                HIPCHK(ctx, hipMemGetInfo(&free_b, &total_b));
                // what this context already holds for seeds counts as free
                uint64_t avail = uint64_t(free_b) + ctx->seed_cap * sizeof(PeelSeed) + ctx->ssort_cap * 16;
                if (ctx->budget)
                    avail = std::min<uint64_t>(avail, ctx->budget - std::min(ctx->used, ctx->budget) +
                                                          ctx->seed_cap * sizeof(PeelSeed) + ctx->ssort_cap * 16);
                slots = base;
                while (slots < (uint64_t(1) << 30) && 2 * slots * (sizeof(PeelSeed) + 16) <= avail / 2) slots *= 2;
            }
            if (slots < lanes * ev_rays)
                return fail(THOR_E_INVAL, "seed_slots must be at least %llu (observers per lane)",
                            (unsigned long long)(lanes * ev_rays));
            s = ensure_seeds(ctx, slots, &sb);
            if (s && !opt->seed_slots && slots > base) {
                slots = base;
                s = ensure_seeds(ctx, slots, &sb);
            }
            if (s && !opt->seed_slots && slots != small) {
                slots = small;
                s = ensure_seeds(ctx, slots, &sb);
            }
            if (s) return s;
            sb.chunk = uint32_t(std::max<uint64_t>(ev_rays, std::min<uint64_t>(kSeedChunk, slots / (2 * lanes))));
            if (seed_sort_on(opt) || opt->fuse_bins > 0) {
                s = ensure_seed_sort(ctx, &sb);
                if (s) return s;
                if (opt->fuse_bins > 0) { sb.keys = nullptr; sb.key_blocks = 0; }
            }
            if (!bounded) {
                // packets wait in the pool while the buffer is full
                s = ensure_pool(ctx, uint64_t(gsize) * block, opt->precision);
                if (s) return s;
            }
        }
        if (hand_off) {
            s = ensure_tail(ctx, uint64_t(gsize) * block);
            if (s) return s;
        }
        const bool use_pool = bounded || seeds;
        void* ppk = use_pool ? ctx->d_pool_pk : nullptr;
        int* pal = use_pool ? ctx->d_pool_alive : nullptr;
        if (use_pool && !resuming)    // nothing may be left over from an abandoned bounded run
            hipLaunchKernelGGL(k_zero_u32, dim3(ctx->num_cu), dim3(256), 0, ctx->stream,
                               reinterpret_cast<unsigned*>(ctx->d_pool_alive), ctx->pool_slots);
        unsigned long long* cur = ctx->d_stats + kNumU64Counters;
        double t_tr = 0.0, t_pp = 0.0, t_tail = 0.0, t_ss = 0.0;
        uint64_t passes = 0;
        // spatial order of the queue: emission cells drawn by a pre-pass, Morton
        // keys radix-sorted; the persistent kernel takes packets through the
        // sorted permutation
        const uint64_t* perm = nullptr;
        ctx->split_presort = 0.0;
        ctx->split_ssort = 0.0;
        if (opt->fuse_bins > 0 && !ctx->d_fused) {
            s = dalloc(ctx, (void**)&ctx->d_fused, 8, "fusing counter");
            if (s) return s;
        }
        if (ctx->d_fused) hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, ctx->stream, ctx->d_fused, 1);
        bool any_cell = false, any_spread = false;
        for (size_t i = 0; i < nb; ++i) {
            const thor_source& src = ctx->pending[i].src;
            any_cell |= src.kind == THOR_SRC_CELL_N2;
            any_spread |= src.spectrum != THOR_SPEC_DELTA || (src.lines && ctx->geom.line == THOR_LINE_MG2);
        }
        const int sort_mode = bounded ? 0 : presort_mode(opt, grid, any_cell, any_spread);
        if (sort_mode && q_end > 1) {
            if (q_end > ctx->sort_cap) {
                dfree(ctx, ctx->d_sort, ctx->sort_cap * 32);
                ctx->d_sort = nullptr;
                ctx->sort_cap = 0;
                s = dalloc(ctx, (void**)&ctx->d_sort, q_end * 32, "presort keys");
                if (s) return s;
                ctx->sort_cap = q_end;
            }
            uint64_t* keys = ctx->d_sort;
            uint64_t* vals = ctx->d_sort + ctx->sort_cap;
            uint64_t* keys2 = ctx->d_sort + 2 * ctx->sort_cap;
            uint64_t* vals2 = ctx->d_sort + 3 * ctx->sort_cap;
            int bits = 1;
            if (grid)
                while ((1 << bits) < std::max(ctx->grid.nx, std::max(ctx->grid.ny, ctx->grid.nz))) ++bits;
            const int end_bit = sort_mode == 2 ? 64 : std::min(64, 3 * bits);
            size_t need = 0;
            HIPCHK(ctx, hipcub::DeviceRadixSort::SortPairs(nullptr, need, keys, keys2, vals, vals2, (int64_t)q_end, 0,
                                                           end_bit, ctx->stream));
            if (need > ctx->sort_tmp_bytes) {
                dfree(ctx, ctx->d_sort_tmp, ctx->sort_tmp_bytes);
                ctx->d_sort_tmp = nullptr;
                ctx->sort_tmp_bytes = 0;
                s = dalloc(ctx, &ctx->d_sort_tmp, need, "presort scratch");
                if (s) return s;
                ctx->sort_tmp_bytes = need;
            }
            HIPCHK(ctx, hipEventRecord(ctx->ev_a, ctx->stream));
            hipLaunchKernelGGL(k_emit_keys, dim3(ctx->num_cu * 8), dim3(256), 0, ctx->stream, ctx->grid,
                               ctx->d_models, ctx->d_batches, int(nb), q_end, keys, vals, sort_mode);
            HIPCHK(ctx, hipGetLastError());
            size_t tmp = ctx->sort_tmp_bytes;
            HIPCHK(ctx, hipcub::DeviceRadixSort::SortPairs(ctx->d_sort_tmp, tmp, keys, keys2, vals, vals2,
                                                           (int64_t)q_end, 0, end_bit, ctx->stream));
            HIPCHK(ctx, hipEventRecord(ctx->ev_b, ctx->stream));
            HIPCHK(ctx, hipEventSynchronize(ctx->ev_b));
            float ms = 0.0f;
            HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->ev_a, ctx->ev_b));
            ctx->split_presort = ms;
            perm = vals2;
        }
        for (;;) {
            if (seeds)
                hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, ctx->stream, ctx->d_seedctl, 2 + kXcds);
            if (hand_off)
                hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, ctx->stream, ctx->d_tailctl, 3);
            if (seeds || hand_off) HIPCHK(ctx, hipEventRecord(ctx->ev_a, ctx->stream));
            if (fp64) grid ? launch_persistent<double, true>(ctx, ctx->stream, gsize, block, ctx->d_batches, ctx->d_desc, cur, out, ctx->d_models, ppk, pal, sb, hand_off, ctx->d_xstats, nullptr, perm)
                           : launch_persistent<double, false>(ctx, ctx->stream, gsize, block, ctx->d_batches, ctx->d_desc, cur, out, ctx->d_models, ppk, pal, sb, hand_off, ctx->d_xstats, nullptr, perm);
            else grid ? launch_persistent<float, true>(ctx, ctx->stream, gsize, block, ctx->d_batches, ctx->d_desc, cur, out, ctx->d_models, ppk, pal, sb, hand_off, ctx->d_xstats, nullptr, perm)
                      : launch_persistent<float, false>(ctx, ctx->stream, gsize, block, ctx->d_batches, ctx->d_desc, cur, out, ctx->d_models, ppk, pal, sb, hand_off, ctx->d_xstats, nullptr, perm);
            if (hand_off) {
                HIPCHK(ctx, hipEventRecord(ctx->ev_c, ctx->stream));
                if (fp64) grid ? launch_tail<double, true>(ctx, ctx->d_desc, out, ppk, pal, sb)
                               : launch_tail<double, false>(ctx, ctx->d_desc, out, ppk, pal, sb);
                else grid ? launch_tail<float, true>(ctx, ctx->d_desc, out, ppk, pal, sb)
                          : launch_tail<float, false>(ctx, ctx->d_desc, out, ppk, pal, sb);
            }
            hipLaunchKernelGGL(k_clamp_cursor, dim3(1), dim3(64), 0, ctx->stream, cur, ctx->d_desc);
            if (seeds || hand_off) HIPCHK(ctx, hipEventRecord(ctx->ev_b, ctx->stream));
            if (!seeds) {
                if (hand_off) {
                    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
                    float ms_tl = 0.0f, ms_tr = 0.0f;
                    HIPCHK(ctx, hipEventElapsedTime(&ms_tr, ctx->ev_a, ctx->ev_b));
                    HIPCHK(ctx, hipEventElapsedTime(&ms_tl, ctx->ev_c, ctx->ev_b));
                    ctx->split_tr = ms_tr;
                    ctx->split_tail = ms_tl;
                    ctx->split_passes = 1;
                }
                break;
            }
            SeedBuf sbp = sb;
            if (seed_sort_on(opt) || opt->fuse_bins > 0) {
                unsigned long long claimed = 0;
                HIPCHK(ctx, hipMemcpyAsync(&claimed, ctx->d_seedctl, 8, hipMemcpyDeviceToHost, ctx->stream));
                HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
                const uint64_t nseeds = std::min<uint64_t>(claimed, sb.cap);
                if (nseeds > 1) {
                    s = sort_seeds(ctx, out, &sbp, nseeds, opt->fuse_bins);
                    if (s) return s;
                }
            }
            HIPCHK(ctx, hipEventRecord(ctx->ev_s, ctx->stream));
            if (fp64) launch_peel_pass<double>(ctx, out, sbp);
            else launch_peel_pass<float>(ctx, out, sbp);
            HIPCHK(ctx, hipGetLastError());
            HIPCHK(ctx, hipEventRecord(ctx->ev1, ctx->stream));
            unsigned long long ctl[4];
            HIPCHK(ctx, hipMemcpyAsync(ctl, ctx->d_seedctl, sizeof ctl, hipMemcpyDeviceToHost, ctx->stream));
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
            float ms_tr = 0.0f, ms_pp = 0.0f, ms_ss = 0.0f;
            HIPCHK(ctx, hipEventElapsedTime(&ms_tr, ctx->ev_a, ctx->ev_b));
            HIPCHK(ctx, hipEventElapsedTime(&ms_ss, ctx->ev_b, ctx->ev_s));
            HIPCHK(ctx, hipEventElapsedTime(&ms_pp, ctx->ev_s, ctx->ev1));
            t_tr += ms_tr;
            t_pp += ms_pp;
            t_ss += ms_ss;
            if (hand_off) {
                float ms_tl = 0.0f;
                HIPCHK(ctx, hipEventElapsedTime(&ms_tl, ctx->ev_c, ctx->ev_b));
                t_tail += ms_tl;
            }
            ++passes;
            if (ctl[1] == 0) break;     // no wave stopped on a full buffer
        }
        if (seeds) {
            ctx->split_tr = t_tr;
            ctx->split_pp = t_pp;
            ctx->split_tail = t_tail;
            ctx->split_ssort = t_ss;
            ctx->split_passes = passes;
        }
    }
    hipLaunchKernelGGL(k_spec_fold, dim3(std::max(1, std::min(ctx->num_cu, (ctx->spec_nb + 255) / 256))), dim3(256),
                       0, ctx->stream, ctx->d_spec, ctx->spec_nb, int(kSpecCopies));
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipEventRecord(ctx->ev1, ctx->stream));
    unsigned long long h[kNumU64Counters + 1], hx[kNumU64Counters + 1];
    HIPCHK(ctx, hipMemcpyAsync(h, ctx->d_stats, sizeof h, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(hx, ctx->d_xstats, sizeof hx, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < kNumU64Counters; ++i) h[i] += hx[1 + i];      // the tail kernel's share
    float ms = 0.0f;
    HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    if (!ctx->split_passes) {       // one kernel type: all device time is transport
        ctx->split_tr = ms;
        ctx->split_pp = 0.0;
        ctx->split_passes = 1;
    }
    collect_stats(ctx, h, ms, &ctx->last);
    ctx->last.transport_ms = ctx->split_tr;
    ctx->last.peel_ms = ctx->split_pp;
    ctx->last.passes = ctx->split_passes;
    ctx->last.tail_ms = ctx->split_tail;
    ctx->last.max_events = hx[0];
    ctx->last.tail_events = hx[1 + 5] + hx[1 + 6];          // n_res + n_dust
    ctx->last.tail_main_visits = hx[1 + 7];
    ctx->last.tail_peel_visits = hx[1 + 8];
    ctx->last.presort_ms = ctx->split_presort;
    ctx->last.seedsort_ms = ctx->split_ssort;
    if (ctx->d_fused) {
        unsigned long long f = 0;
        HIPCHK(ctx, hipMemcpy(&f, ctx->d_fused, 8, hipMemcpyDeviceToHost));
        ctx->last.peel_fused = f;
    }
    if (out_stats) *out_stats = ctx->last;
    if (bounded) {
        // work left: queue not drained or packets parked in the pool
        bool left = h[kNumU64Counters] < q_end;
        if (!left) {
            std::vector<int> alive(ctx->pool_slots);
            HIPCHK(ctx, hipMemcpy(alive.data(), ctx->d_pool_alive, ctx->pool_slots * 4, hipMemcpyDeviceToHost));
            for (int a : alive) if (a) { left = true; break; }
        }
        ctx->q_total = left ? q_end : 0;
        if (left) return THOR_INCOMPLETE;
    }
    ctx->pending.clear();
    return THOR_OK;
}

thor_status thor_transport_noalloc(thor_ctx* ctx, const thor_transport_opts* opt, double* d_spectrum,
                                   float* d_cube, thor_stats* out_stats) {
    CHECK_CTX(ctx);
    thor_status s = check_opts(opt);
    if (s) return s;
    if (!ctx->has_geom) return fail(THOR_E_STATE, "thor_load_grid first");
    if (opt->path != THOR_PATH_PERSISTENT) return fail(THOR_E_UNSUPPORTED, "no-allocation transport: PERSISTENT path only");
    if (opt->step_events) return fail(THOR_E_UNSUPPORTED, "no-allocation transport: no bounded steps");
    if (opt->records) return fail(THOR_E_UNSUPPORTED, "no-allocation transport: no per-packet records");
    if (opt->accum != THOR_ACCUM_F32_ATOMIC)
        return fail(THOR_E_UNSUPPORTED, "no-allocation transport: float32 cube accumulation only");
    if (uint64_t(opt->spec_nb) > kNaMaxBins)
        return fail(THOR_E_INVAL, "no-allocation transport: %d spectrum bins exceed the maximum of %d", opt->spec_nb,
                    int(kNaMaxBins));
    if (ctx->pending.size() > kNaMaxBatches)
        return fail(THOR_E_INVAL, "no-allocation transport: %zu queued batches exceed the maximum of %d",
                    ctx->pending.size(), int(kNaMaxBatches));
    if (!d_spectrum) return fail(THOR_E_INVAL, "null spectrum output");
    if (opt->n_obs > 0 && !d_cube) return fail(THOR_E_INVAL, "null cube output (observers given)");
    if (!ctx->d_scratch) return fail(THOR_E_UNSUPPORTED, "no scratch address for device %d", ctx->device);
    if (out_stats) std::memset(out_stats, 0, sizeof *out_stats);
    if (ctx->pending.empty()) return THOR_OK;
    const bool grid = ctx->geom.kind == THOR_GEOM_GRID;
    const bool fp64 = opt->precision == THOR_PREC_FP64;
    const size_t nb = ctx->pending.size();
    unsigned char* sc = ctx->d_scratch;
    std::vector<ModelDev> models(nb);
    std::vector<BatchDev> batches(nb);
    uint64_t q = 0;
    for (size_t i = 0; i < nb; ++i) {
        s = make_model(ctx, ctx->pending[i].src, *opt, models[i]);
        if (s) return s;
        models[i].spec = reinterpret_cast<double*>(sc + kNaSpec);
        models[i].spec_rep = int(kSpecCopies);
        batches[i] = BatchDev{q, ctx->pending[i].first_id, ctx->pending[i].n, int(i), 0};
        q += ctx->pending[i].n;
    }
    OutDev out = make_out(ctx, opt);
    out.cube = d_cube;
    out.cube_fx = nullptr;
    out.fx_scale = 0.0;
    const int block = opt->block > 0 ? opt->block : 256;
    const int gsize = launch_grid_size(ctx, opt, block);
    const uint32_t turn = opt->visits_per_turn > 0 ? uint32_t(opt->visits_per_turn) : 256u;
    const StepDesc desc{q, int(nb), 0u, turn, 0u, park_lanes(opt), refill_64ths(opt), 0u};
    if (out_stats) HIPCHK(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    const uint64_t spec_words = uint64_t(kSpecCopies) * uint64_t(opt->spec_nb);
    hipLaunchKernelGGL(k_na_setup, dim3(std::max<uint64_t>(1, std::min<uint64_t>(1024, (spec_words + 255) / 256))),
                       dim3(256), 0, ctx->stream, sc, desc, spec_words);
    for (size_t i = 0; i < nb; ++i)
        hipLaunchKernelGGL(k_na_put, dim3(1), dim3(64), 0, ctx->stream, sc, uint32_t(i), models[i], batches[i]);
    const BatchDev* d_b = reinterpret_cast<const BatchDev*>(sc + kNaBatches);
    const StepDesc* d_desc = reinterpret_cast<const StepDesc*>(sc + kNaDesc);
    const ModelDev* d_m = reinterpret_cast<const ModelDev*>(sc + kNaModels);
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(sc + kNaCounters);
    unsigned long long* gmax = reinterpret_cast<unsigned long long*>(sc + kNaMax);
    SeedBuf sb;
    std::memset(&sb, 0, sizeof sb);    // no seed buffer: grid peel rays are marched inline
    unsigned long long* cur = cnt + kNumU64Counters;
    if (fp64) grid ? launch_persistent<double, true>(ctx, ctx->stream, gsize, block, d_b, d_desc, cur, out, d_m, nullptr, nullptr, sb, false, gmax, cnt)
                   : launch_persistent<double, false>(ctx, ctx->stream, gsize, block, d_b, d_desc, cur, out, d_m, nullptr, nullptr, sb, false, gmax, cnt);
    else grid ? launch_persistent<float, true>(ctx, ctx->stream, gsize, block, d_b, d_desc, cur, out, d_m, nullptr, nullptr, sb, false, gmax, cnt)
              : launch_persistent<float, false>(ctx, ctx->stream, gsize, block, d_b, d_desc, cur, out, d_m, nullptr, nullptr, sb, false, gmax, cnt);
    hipLaunchKernelGGL(k_na_fold, dim3(std::max(1, std::min(ctx->num_cu, (opt->spec_nb + 255) / 256))), dim3(256), 0,
                       ctx->stream, sc, d_spectrum, opt->spec_nb, int(kSpecCopies));
    HIPCHK(ctx, hipGetLastError());
    ctx->pending.clear();
    if (!out_stats) return THOR_OK;
    HIPCHK(ctx, hipEventRecord(ctx->ev1, ctx->stream));
    unsigned long long h[kNumU64Counters + 1], hmax = 0;
    HIPCHK(ctx, hipMemcpyAsync(h, cnt, sizeof h, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(&hmax, gmax, 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    float ms = 0.0f;
    HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    collect_stats(ctx, h, ms, out_stats);
    out_stats->transport_ms = ms;
    out_stats->passes = 1;
    out_stats->max_events = hmax;
    return THOR_OK;
}

uint64_t thor_output_bytes(thor_ctx* ctx, thor_output which) {
    if (!ctx) return 0;
    switch (which) {
    case THOR_OUT_SPECTRUM: return uint64_t(ctx->spec_nb) * 8;
    case THOR_OUT_CUBE: return ctx->cube_elems * 4;
    case THOR_OUT_CUBE_FIXED: return ctx->d_cube_fx ? ctx->cube_elems * 8 : 0;
    case THOR_OUT_RECORDS: return ctx->rec_n * sizeof(thor_record);
    case THOR_OUT_STATS: return sizeof(thor_stats);
    }
    return 0;
}

thor_status thor_read_spectra(thor_ctx* ctx, thor_output which, uint32_t index, void* dst, uint64_t dst_bytes,
                              int dst_on_device) {
    CHECK_CTX(ctx);
    if (!dst) return fail(THOR_E_INVAL, "null destination");
    if (index != 0) return fail(THOR_E_INVAL, "index must be 0");
    const uint64_t need = thor_output_bytes(ctx, which);
    if (dst_bytes < need) return fail(THOR_E_INVAL, "destination too small (%llu < %llu bytes)",
                                      (unsigned long long)dst_bytes, (unsigned long long)need);
    const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    switch (which) {
    case THOR_OUT_SPECTRUM:
        if (!need) return fail(THOR_E_STATE, "no spectrum yet");
        HIPCHK(ctx, hipMemcpyAsync(dst, ctx->d_spec, need, kind, ctx->stream));
        break;
    case THOR_OUT_CUBE:
        if (!need) return fail(THOR_E_STATE, "no cube (no observers)");
        if (ctx->d_cube_fx) {
            const double inv = 1.0 / ctx->cube_fx_scale;
            if (dst_on_device) {
                hipLaunchKernelGGL(k_fx_to_f32, dim3(ctx->num_cu * 4), dim3(256), 0, ctx->stream, ctx->d_cube_fx,
                                   static_cast<float*>(dst), ctx->cube_elems, inv);
                HIPCHK(ctx, hipGetLastError());
            } else {
                std::vector<unsigned long long> raw(ctx->cube_elems);
                HIPCHK(ctx, hipMemcpyAsync(raw.data(), ctx->d_cube_fx, ctx->cube_elems * 8, hipMemcpyDeviceToHost,
                                           ctx->stream));
                HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
                float* d = static_cast<float*>(dst);
                for (uint64_t i = 0; i < ctx->cube_elems; ++i) d[i] = float(double(raw[i]) * inv);
                return THOR_OK;
            }
        } else {
            HIPCHK(ctx, hipMemcpyAsync(dst, ctx->d_cube, need, kind, ctx->stream));
        }
        break;
    case THOR_OUT_CUBE_FIXED:
        if (!need) return fail(THOR_E_STATE, "no fixed-point cube (accum FIXED64 with observers)");
        HIPCHK(ctx, hipMemcpyAsync(dst, ctx->d_cube_fx, need, kind, ctx->stream));
        break;
    case THOR_OUT_RECORDS: {
        if (!need) return fail(THOR_E_STATE, "no records (set opts.records)");
        if (dst_on_device) return fail(THOR_E_UNSUPPORTED, "records are copied to host memory only");
        const uint64_t n = ctx->rec_n;
        std::vector<double> dv(n);
        std::vector<uint32_t> nr(n), nd(n);
        std::vector<int32_t> fa(n);
        HIPCHK(ctx, hipMemcpyAsync(dv.data(), ctx->d_rec_dv, n * 8, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(nr.data(), ctx->d_rec_nres, n * 4, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(nd.data(), ctx->d_rec_ndust, n * 4, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(fa.data(), ctx->d_rec_fate, n * 4, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        thor_record* r = static_cast<thor_record*>(dst);
        for (uint64_t i = 0; i < n; ++i) r[i] = thor_record{dv[i], nr[i], nd[i], fa[i], 0u};
        return THOR_OK;
    }
    case THOR_OUT_STATS:
        if (dst_on_device) return fail(THOR_E_UNSUPPORTED, "stats are copied to host memory only");
        std::memcpy(dst, &ctx->last, sizeof ctx->last);
        return THOR_OK;
    default:
        return fail(THOR_E_INVAL, "bad output kind");
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return THOR_OK;
}

thor_status thor_eval_voigt(thor_ctx* ctx, const double* a, const double* x, double* out, uint64_t n,
                            int32_t precision) {
    CHECK_CTX(ctx);
    if (!a || !x || !out) return fail(THOR_E_INVAL, "null array");
    if (n == 0) return THOR_OK;
    const unsigned blocks = unsigned((n + 255) / 256);
    if (precision == THOR_PREC_FP64)
        hipLaunchKernelGGL(k_eval_voigt<double>, dim3(blocks), dim3(256), 0, ctx->stream, a, x, out, n);
    else if (precision == THOR_PREC_MIXED)
        hipLaunchKernelGGL(k_eval_voigt<float>, dim3(blocks), dim3(256), 0, ctx->stream, a, x, out, n);
    else
        return fail(THOR_E_INVAL, "bad precision");
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return THOR_OK;
}

thor_status thor_eval_xcw(thor_ctx* ctx, const double* a, double* out, uint64_t n, int32_t precision) {
    CHECK_CTX(ctx);
    if (!a || !out) return fail(THOR_E_INVAL, "null array");
    if (n == 0) return THOR_OK;
    const unsigned blocks = unsigned((n + 255) / 256);
    if (precision == THOR_PREC_FP64)
        hipLaunchKernelGGL(k_eval_xcw<double>, dim3(blocks), dim3(256), 0, ctx->stream, a, out, n);
    else if (precision == THOR_PREC_MIXED)
        hipLaunchKernelGGL(k_eval_xcw<float>, dim3(blocks), dim3(256), 0, ctx->stream, a, out, n);
    else
        return fail(THOR_E_INVAL, "bad precision");
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return THOR_OK;
}

thor_status thor_sample_upar(thor_ctx* ctx, double x, double a, uint32_t seed, uint32_t event, double* out_u,
                             uint32_t* out_trials, uint64_t n, int32_t precision) {
    CHECK_CTX(ctx);
    if (!out_u || !out_trials) return fail(THOR_E_INVAL, "null array");
    if (!(a > 0.0)) return fail(THOR_E_INVAL, "a must be positive");
    if (n == 0) return THOR_OK;
    const unsigned blocks = unsigned((n + 255) / 256);
    if (precision == THOR_PREC_FP64)
        hipLaunchKernelGGL(k_sample_upar<double>, dim3(blocks), dim3(256), 0, ctx->stream, x, a, seed, event, out_u, out_trials, n);
    else if (precision == THOR_PREC_MIXED)
        hipLaunchKernelGGL(k_sample_upar<float>, dim3(blocks), dim3(256), 0, ctx->stream, x, a, seed, event, out_u, out_trials, n);
    else
        return fail(THOR_E_INVAL, "bad precision");
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return THOR_OK;
}

// ------------------------------------------------------------- serving
// Continuous batching of shell-model solves: each admitted request owns a
// model slot (medium constants, source key, spectrum) and a contiguous range
// of the serving queue; thor_step runs one bounded persistent launch over
// every live request, parking unfinished packets in the serving pool.

static thor_status serving_init(thor_ctx* ctx) {
    if (ctx->s_init) return THOR_OK;
    thor_status s = dalloc(ctx, (void**)&ctx->d_s_models, sizeof(ModelDev) * kServingMaxModels, "serving models");
    if (!s) s = dalloc(ctx, (void**)&ctx->d_done, 8ull * kServingMaxModels, "serving counters");
    if (!s) s = dalloc(ctx, (void**)&ctx->d_s_cursor, 8, "serving cursor");
    if (s) return s;
    if (!s) s = dalloc(ctx, (void**)&ctx->d_s_desc, sizeof(StepDesc), "serving step descriptor");
    if (!s) s = dalloc(ctx, (void**)&ctx->d_s_batches, sizeof(BatchDev) * kServingMaxBatches, "serving batches");
    if (s) return s;
    if (hipHostMalloc((void**)&ctx->h_s_desc, sizeof(StepDesc)) != hipSuccess ||
        hipHostMalloc((void**)&ctx->h_s_batches, sizeof(BatchDev) * kServingMaxBatches) != hipSuccess ||
        hipHostMalloc((void**)&ctx->h_s_done, 8ull * kServingMaxModels) != hipSuccess ||
        hipHostMalloc((void**)&ctx->h_s_misc, 8ull * (kNumU64Counters + 1)) != hipSuccess)
        return fail(THOR_E_NOMEM, "pinned host allocation failed");
    std::memset(ctx->h_s_done, 0, 8ull * kServingMaxModels);
    HIPCHK(ctx, hipMemsetAsync(ctx->d_done, 0, 8ull * kServingMaxModels, ctx->stream));
    HIPCHK(ctx, hipMemsetAsync(ctx->d_s_cursor, 0, 8, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->s_models.assign(kServingMaxModels, ModelDev{});
    ctx->s_init = true;
    return THOR_OK;
}

thor_status thor_submit(thor_ctx* ctx, const thor_shell_request* r, uint64_t* req_id) {
    CHECK_CTX(ctx);
    if (!r || !req_id) return fail(THOR_E_INVAL, "null argument");
    if (!(r->N_HI > 0.0) || !(r->T > 0.0) || r->tau_d < 0.0 || !(r->r_outer > r->r_inner) || r->r_inner < 0.0)
        return fail(THOR_E_INVAL, "bad shell parameters");
    if (r->albedo < 0.0 || r->albedo > 1.0 || r->g_hg <= -1.0 || r->g_hg >= 1.0 || r->sigma_v < 0.0)
        return fail(THOR_E_INVAL, "bad dust or source parameters");
    if (r->n_packets == 0 || r->spec_nb <= 0 || !(r->spec_hi > r->spec_lo))
        return fail(THOR_E_INVAL, "bad packet count or spectrum bins");
    thor_status s = serving_init(ctx);
    if (s) return s;
    // admission: the request's spectrum and the state of all its packets
    // (as if every packet were resident at once) must fit the budget
    const uint64_t spec_bytes = uint64_t(r->spec_nb) * 8;
    const uint64_t reserve = r->n_packets * uint64_t(sizeof(Pkt<double>));
    if (ctx->budget && ctx->used + ctx->s_reserved + spec_bytes + reserve > ctx->budget)
        return fail(THOR_E_BUDGET, "request of %llu packets does not fit the HBM budget now",
                    (unsigned long long)r->n_packets);
    if (ctx->s_batches.size() >= size_t(kServingMaxBatches))
        return fail(THOR_E_BUDGET, "too many queued requests");
    int slot;
    if (!ctx->s_free.empty()) slot = ctx->s_free.back();
    else if (ctx->s_next_slot < kServingMaxModels) slot = ctx->s_next_slot;
    else return fail(THOR_E_BUDGET, "too many live requests");
    double* d_spec = nullptr;
    s = dalloc(ctx, (void**)&d_spec, spec_bytes, "request spectrum");
    if (s) return s;
    HIPCHK(ctx, hipMemsetAsync(d_spec, 0, spec_bytes, ctx->stream));
    HIPCHK(ctx, hipMemsetAsync(ctx->d_done + slot, 0, 8, ctx->stream));
    if (!ctx->s_free.empty()) ctx->s_free.pop_back(); else ctx->s_next_slot++;
    ModelDev m;
    std::memset(&m, 0, sizeof m);
    m.kind = kGeomShell;
    m.v_profile = r->v_exp != 0.0 ? kVelConstRadial : kVelNone;
    m.src_kind = kSrcPoint;
    m.spectrum = kSpecGauss;
    const double L = r->r_outer - r->r_inner;
    double sig0;
    line_params(r->T, &m.vth, &m.a, &sig0);
    m.r_in = r->r_inner;
    m.r_out = r->r_outer;
    m.n = r->N_HI / L;
    m.k0 = m.n * sig0;
    m.kd = r->tau_d / L;
    m.v_max = r->v_exp;
    m.step_f = r->step_f > 0.0 ? r->step_f : 0.01;
    const double atau = m.a * m.k0 * L;     // Section 3.4.2 adaptive x_crit
    m.xcrit = atau >= 1.0 ? 0.2 * std::cbrt(atau) : 0.0;
    m.albedo = r->albedo;
    m.g_hg = r->g_hg;
    m.dv0 = 0.0;
    m.sigma_v = r->sigma_v;
    m.seed = r->seed;
    m.req = r->request_id;
    m.spec = d_spec;
    m.spec_nb = r->spec_nb;
    m.spec_rep = 1;
    m.spec_lo = r->spec_lo;
    m.spec_w = (r->spec_hi - r->spec_lo) / r->spec_nb;
    m.spec_scale = 1.0;
    m.done = ctx->d_done + slot;
    ctx->s_models[slot] = m;
    ctx->h_s_done[slot] = 0;
    BatchDev b;
    b.q0 = ctx->s_q_total;
    b.first_id = 0;
    b.n = r->n_packets;
    b.model = slot;
    b.pad = 0;
    ctx->s_batches.push_back(b);
    ctx->s_q_total += r->n_packets;
    ctx->s_reserved += reserve;
    ctx->s_dirty = true;
    const uint64_t h = ctx->s_next_handle++;
    ctx->s_reqs[h] = ServingReq{slot, r->n_packets, d_spec, r->spec_nb, reserve, false};
    *req_id = h;
    return THOR_OK;
}

// Enqueue one serving step on `stream`: descriptor and batch table from the
// pinned mirrors, counters cleared by a kernel, the bounded persistent launch,
// the cursor clamp, and the done counters / cursor / counters back into the
// pinned mirrors.  The same sequence is captured once into a hipGraph.
static void enqueue_serving_step(thor_ctx* ctx, hipStream_t st, int prec, int gsize, int block) {
    (void)hipMemcpyAsync(ctx->d_s_desc, ctx->h_s_desc, sizeof(StepDesc), hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(ctx->d_s_batches, ctx->h_s_batches, sizeof(BatchDev) * kServingMaxBatches,
                         hipMemcpyHostToDevice, st);
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, ctx->d_stats, kNumU64Counters);
    OutDev out;
    std::memset(&out, 0, sizeof out);
    out.phase = THOR_PHASE_DIPOLE;
    out.tau_cut = 40.0;
    out.img_w[0] = out.img_w[1] = out.v_w = 1.0;
    SeedBuf sb;
    std::memset(&sb, 0, sizeof sb);
    if (prec == THOR_PREC_FP64)
        launch_persistent<double, false>(ctx, st, gsize, block, ctx->d_s_batches, ctx->d_s_desc, ctx->d_s_cursor, out,
                                         ctx->d_s_models, ctx->d_s_pool, ctx->d_s_alive, sb);
    else
        launch_persistent<float, false>(ctx, st, gsize, block, ctx->d_s_batches, ctx->d_s_desc, ctx->d_s_cursor, out,
                                        ctx->d_s_models, ctx->d_s_pool, ctx->d_s_alive, sb);
    hipLaunchKernelGGL(k_clamp_cursor, dim3(1), dim3(64), 0, st, ctx->d_s_cursor, ctx->d_s_desc);
    (void)hipMemcpyAsync(ctx->h_s_done, ctx->d_done, 8ull * kServingMaxModels, hipMemcpyDeviceToHost, st);
    (void)hipMemcpyAsync(ctx->h_s_misc, ctx->d_stats, 8ull * kNumU64Counters, hipMemcpyDeviceToHost, st);
    (void)hipMemcpyAsync(ctx->h_s_misc + kNumU64Counters, ctx->d_s_cursor, 8, hipMemcpyDeviceToHost, st);
}

thor_status thor_step(thor_ctx* ctx, uint32_t max_events_per_packet, const thor_transport_opts* opt) {
    CHECK_CTX(ctx);
    if (!opt) return fail(THOR_E_INVAL, "null options");
    if (opt->precision != THOR_PREC_FP64 && opt->precision != THOR_PREC_MIXED) return fail(THOR_E_INVAL, "bad precision");
    if (opt->block && (opt->block % 64 || opt->block > 256)) return fail(THOR_E_INVAL, "bad block");
    if (!ctx->s_init) return THOR_OK;
    const int block = opt->block > 0 ? opt->block : 256;
    const int gsize = launch_grid_size(ctx, opt, block);
    const uint64_t slots = uint64_t(gsize) * block;
    const uint64_t pk_bytes = opt->precision == THOR_PREC_FP64 ? sizeof(Pkt<double>) : sizeof(Pkt<float>);
    if (!ctx->d_s_pool || ctx->s_pool_slots != slots || ctx->s_pool_prec != opt->precision) {
        // the pool can change shape only while no packet is parked in it
        if (ctx->d_s_pool && ctx->s_cursor > 0) {
            bool parked = false;
            std::vector<int> alive(ctx->s_pool_slots);
            HIPCHK(ctx, hipMemcpy(alive.data(), ctx->d_s_alive, ctx->s_pool_slots * 4, hipMemcpyDeviceToHost));
            for (int a : alive) if (a) { parked = true; break; }
            if (parked) return fail(THOR_E_STATE, "launch shape or precision changed while packets are parked");
        }
        dfree(ctx, ctx->d_s_pool, ctx->s_pool_bytes);
        dfree(ctx, ctx->d_s_alive, ctx->s_pool_slots * 4);
        ctx->d_s_pool = nullptr; ctx->d_s_alive = nullptr; ctx->s_pool_slots = 0;
        thor_status s = dalloc(ctx, &ctx->d_s_pool, slots * pk_bytes, "serving pool");
        if (!s) s = dalloc(ctx, (void**)&ctx->d_s_alive, slots * 4, "serving pool flags");
        if (s) return s;
        ctx->s_pool_slots = slots;
        ctx->s_pool_bytes = slots * pk_bytes;
        ctx->s_pool_prec = opt->precision;
        HIPCHK(ctx, hipMemsetAsync(ctx->d_s_alive, 0, slots * 4, ctx->stream));
        if (ctx->s_graph) { (void)hipGraphExecDestroy(ctx->s_graph); ctx->s_graph = nullptr; }
    }
    // drop queue ranges the cursor has passed (their packets were all taken;
    // parked ones carry their model slot, so the range is no longer needed)
    {
        size_t keep = 0;
        while (keep < ctx->s_batches.size()) {
            const BatchDev& b = ctx->s_batches[keep];
            if (b.q0 + b.n <= ctx->s_cursor) ++keep; else break;
        }
        if (keep) ctx->s_batches.erase(ctx->s_batches.begin(), ctx->s_batches.begin() + keep);
    }
    bool any_live = false;
    for (auto& kv : ctx->s_reqs) any_live |= !kv.second.finished;
    if (!any_live) return THOR_OK;
    const size_t nb = ctx->s_batches.size();
    if (nb) std::memcpy(ctx->h_s_batches, ctx->s_batches.data(), nb * sizeof(BatchDev));
    const uint32_t turn = opt->visits_per_turn > 0 ? uint32_t(opt->visits_per_turn) : 256u;
    // nb == 0: only parked packets are left; no lane can take a new index
    *ctx->h_s_desc = StepDesc{ctx->s_q_total, int(nb), max_events_per_packet, turn, 0u, park_lanes(opt),
                              refill_64ths(opt), 0u};
    if (ctx->s_dirty) {
        const int hi = ctx->s_next_slot;
        HIPCHK(ctx, hipMemcpyAsync(ctx->d_s_models, ctx->s_models.data(), sizeof(ModelDev) * hi,
                                   hipMemcpyHostToDevice, ctx->stream));
        ctx->s_dirty = false;
    }
    if (opt->use_graph) {
        if (ctx->s_graph && (ctx->s_graph_prec != opt->precision || ctx->s_graph_grid != gsize ||
                             ctx->s_graph_block != block)) {
            (void)hipGraphExecDestroy(ctx->s_graph);
            ctx->s_graph = nullptr;
        }
        if (!ctx->s_graph) {
            if (!ctx->cap_stream) HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
            hipGraph_t graph = nullptr;
            HIPCHK(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed));
            enqueue_serving_step(ctx, ctx->cap_stream, opt->precision, gsize, block);
            HIPCHK(ctx, hipStreamEndCapture(ctx->cap_stream, &graph));
            hipError_t e = hipGraphInstantiate(&ctx->s_graph, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (!hip_ok(ctx, e, "hipGraphInstantiate")) return THOR_E_DEVICE;
            ctx->s_graph_prec = opt->precision;
            ctx->s_graph_grid = gsize;
            ctx->s_graph_block = block;
        }
        HIPCHK(ctx, hipEventRecord(ctx->ev0, ctx->stream));
        HIPCHK(ctx, hipGraphLaunch(ctx->s_graph, ctx->stream));
    } else {
        HIPCHK(ctx, hipEventRecord(ctx->ev0, ctx->stream));
        enqueue_serving_step(ctx, ctx->stream, opt->precision, gsize, block);
    }
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipEventRecord(ctx->ev1, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    float ms = 0.0f;
    HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    collect_stats(ctx, ctx->h_s_misc, ms, &ctx->last);
    ctx->s_cursor = ctx->h_s_misc[kNumU64Counters];
    bool left = false;
    for (auto& kv : ctx->s_reqs) {
        ServingReq& q = kv.second;
        if (!q.finished && ctx->h_s_done[q.model] >= q.n_packets) q.finished = true;
        left |= !q.finished;
    }
    return left ? THOR_INCOMPLETE : THOR_OK;
}

thor_status thor_poll(thor_ctx* ctx, uint64_t req_id, double* spectrum, thor_stats* st, int* done) {
    CHECK_CTX(ctx);
    if (!done) return fail(THOR_E_INVAL, "null done pointer");
    auto it = ctx->s_reqs.find(req_id);
    if (it == ctx->s_reqs.end()) return fail(THOR_E_INVAL, "unknown request %llu", (unsigned long long)req_id);
    ServingReq& q = it->second;
    *done = q.finished ? 1 : 0;
    if (!q.finished) return THOR_OK;
    if (spectrum)
        HIPCHK(ctx, hipMemcpyAsync(spectrum, q.d_spec, uint64_t(q.spec_nb) * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (st) {
        std::memset(st, 0, sizeof *st);
        st->emitted = q.n_packets;
    }
    dfree(ctx, q.d_spec, uint64_t(q.spec_nb) * 8);
    ctx->s_reserved -= std::min(ctx->s_reserved, q.reserved);
    ctx->s_free.push_back(q.model);
    ctx->s_reqs.erase(it);
    return THOR_OK;
}

}  // extern "C"
