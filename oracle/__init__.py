"""Serial FP64 CPU oracle of the resonant-line Monte Carlo transport.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product library
(``paper_2507_11603_amd``) never imports, links or calls it, and the two share
no code: the oracle is plain C (``thor_oracle.c``) bound here with ctypes.

Parity status of each exported function (what pins it) is listed in
``thor_oracle.c``'s header comments and in the tests under ``tests/``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "thor_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GEOMETRY = {"shell": 0, "sphere": 0, "slab": 1, "grid": 2}
VELOCITY = {"none": 0, "const_radial": 1, "linear": 2}
SOURCE = {"point": 0, "cell_n2": 1}
SPECTRUM = {"delta": 0, "gauss": 1, "thermal": 2, "flat": 3}
LINE = {"lya": 0, "mg2": 1, "mg2k": 2}
PHASE = {"iso": 0, "dipole": 1, "core_wing": 2, "hg": 3}
CORE_SKIP = {"off": 0, "fixed": 1, "adaptive": 2}
OBS_AXIS = {"+x": 0, "+y": 1, "+z": 2, "-x": 3, "-y": 4, "-z": 5}
FATE = {0: "none", 1: "escaped", 2: "absorbed", 3: "capped"}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Geometry(C.Structure):
    _fields_ = [("kind", C.c_int32), ("r_inner", C.c_double), ("r_outer", C.c_double),
                ("n_HI", C.c_double), ("tau0", C.c_double), ("T", C.c_double),
                ("v_profile", C.c_int32), ("v_max", C.c_double), ("step_f", C.c_double),
                ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("f_n", C.c_void_p), ("f_T", C.c_void_p), ("f_vx", C.c_void_p),
                ("f_vy", C.c_void_p), ("f_vz", C.c_void_p),
                ("boundary_handoff", C.c_int32),
                ("sigma_d", C.c_double), ("tau_d", C.c_double),
                ("albedo", C.c_double), ("g_hg", C.c_double),
                ("hubble", C.c_double), ("hubble_ref", C.c_double * 3), ("hubble_step", C.c_double),
                ("stop_dv", C.c_double), ("line", C.c_int32)]


class Source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pos", C.c_double * 3), ("spectrum", C.c_int32),
                ("dv0", C.c_double), ("sigma_v", C.c_double),
                ("seed", C.c_uint32), ("request_id", C.c_uint32), ("lines", C.c_int32)]


class Opts(C.Structure):
    _fields_ = [("phase", C.c_int32), ("core_skip", C.c_int32), ("x_crit", C.c_double),
                ("n_obs", C.c_int32), ("obs_axis", C.c_int32 * 6),
                ("cube_nx", C.c_int32), ("cube_ny", C.c_int32), ("cube_nb", C.c_int32),
                ("img_lo", C.c_double * 2), ("img_hi", C.c_double * 2),
                ("cube_v_lo", C.c_double), ("cube_v_hi", C.c_double),
                ("spec_nb", C.c_int32), ("spec_lo", C.c_double), ("spec_hi", C.c_double),
                ("spec_T_ref", C.c_double), ("tau_cut", C.c_double),
                ("max_events", C.c_uint64)]


class Stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in (
        "emitted", "escaped", "absorbed", "capped", "handed_off", "n_res", "n_dust",
        "main_visits", "peel_visits", "peel_contrib", "peel_dropped", "peel_cut",
        "upar_trials")] + [("w_escaped", C.c_double), ("w_absorbed", C.c_double), ("redshifted", C.c_uint64)]


RECORD_DTYPE = np.dtype([("dv", "<f8"), ("n_res", "<u4"), ("n_dust", "<u4"),
                         ("fate", "<i4"), ("pad", "<u4")])

_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        d, u32, u64 = C.c_double, C.c_uint32, C.c_uint64
        L.or_voigt.restype = d
        L.or_voigt.argtypes = [d, d]
        L.or_dawson.restype = d
        L.or_dawson.argtypes = [d]
        L.or_species_params.argtypes = [C.c_int, d, C.POINTER(d), C.POINTER(d), C.POINTER(d)]
        for fn in ("or_lambert_wm1", "or_xcw_exact", "or_xcw_b25"):
            getattr(L, fn).restype = d
            getattr(L, fn).argtypes = [d]
        L.or_line_params.argtypes = [d, C.POINTER(d), C.POINTER(d), C.POINTER(d)]
        L.or_philox4x32_10.argtypes = [C.POINTER(u32), C.POINTER(u32), C.POINTER(u32)]
        L.or_draw.argtypes = [u32, u32, u32, u32, u64, C.POINTER(d)]
        L.or_sample_upar.restype = d
        L.or_sample_upar.argtypes = [d, d, u32, u32, u64, C.POINTER(u64)]
        L.or_upar_expected_trials.restype = d
        L.or_upar_expected_trials.argtypes = [d, d]
        L.or_sample_mu.restype = d
        L.or_sample_mu.argtypes = [C.c_int, d, d]
        L.or_basis.argtypes = [C.POINTER(d)] * 3
        L.or_transport.restype = C.c_int
        L.or_transport.argtypes = [C.POINTER(Geometry), C.POINTER(Source), C.POINTER(Opts),
                                   u64, u64, C.c_void_p, C.c_void_p, C.POINTER(Stats),
                                   C.c_void_p]
        L.or_prepare.restype = C.c_void_p
        L.or_prepare.argtypes = [C.POINTER(Geometry), C.POINTER(Source), C.POINTER(Opts)]
        L.or_transport_prepared.restype = C.c_int
        L.or_transport_prepared.argtypes = [C.c_void_p, u64, u64, C.c_void_p, C.c_void_p,
                                            C.POINTER(Stats), C.c_void_p]
        L.or_release.restype = None
        L.or_release.argtypes = [C.c_void_p]
        L.or_emit.restype = C.c_int
        L.or_emit.argtypes = [C.POINTER(Geometry), C.POINTER(Source), u64, u64, C.c_void_p]
        L.or_scatter_resonant.restype = C.c_int
        L.or_scatter_resonant.argtypes = [d, d, C.POINTER(d), d, C.c_int, u32, u32, u64, C.c_void_p]
        i32 = C.c_int32
        L.or_project.restype = C.c_int
        L.or_project.argtypes = [C.c_void_p, C.c_void_p, i32, i32, i32, i32, d,
                                 C.c_void_p, C.c_void_p]
        L.or_forest.restype = C.c_int
        L.or_forest.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, i32, i32, i32, i32, d, d,
                                i32, C.c_void_p, u32, u32, d, d, C.c_void_p]
        _lib = L
    return _lib


# ----------------------------------------------------------------- scalars
def species_params(line: str, T: float):
    """(v_th, a, sigma0) of the reference line of a species ("lya", or "mg2":
    the Mg II k line, with the Mg mass)."""
    v, a, s = C.c_double(), C.c_double(), C.c_double()
    lib().or_species_params(LINE[line], float(T), C.byref(v), C.byref(a), C.byref(s))
    return v.value, a.value, s.value


def line_params(T: float):
    """(v_th [cm/s], a, sigma0 [cm^2]) at temperature T (Section 2.3.1)."""
    v, a, s = C.c_double(), C.c_double(), C.c_double()
    lib().or_line_params(float(T), C.byref(v), C.byref(a), C.byref(s))
    return v.value, a.value, s.value


def voigt(a, x):
    """H(a, x) = Re w(x + i a), elementwise (Section 3.4, Appendix A.3)."""
    a_b, x_b = np.broadcast_arrays(np.asarray(a, float), np.asarray(x, float))
    f = lib().or_voigt
    return np.array([f(float(ai), float(xi)) for ai, xi in zip(a_b.ravel(), x_b.ravel())]
                    ).reshape(a_b.shape)


def dawson(x):
    f = lib().or_dawson
    return np.array([f(float(v)) for v in np.ravel(x)]).reshape(np.shape(x))


def lambert_wm1(z):
    """Lower real branch of Lambert's W on [-1/e, 0), elementwise."""
    f = lib().or_lambert_wm1
    return np.array([f(float(v)) for v in np.ravel(z)]).reshape(np.shape(z))


def xcw(a, method="exact"):
    """Core-to-wing transition x_cw(a) (Appendix A.2): "exact" by Lambert W,
    "b25" by the quartic in ln a."""
    f = {"exact": lib().or_xcw_exact, "b25": lib().or_xcw_b25}[method]
    return np.array([f(float(v)) for v in np.ravel(a)]).reshape(np.shape(a))


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return list(o)


def draw(seed, request_id, slot, event, pid):
    out = (C.c_double * 2)()
    lib().or_draw(seed, request_id, slot, event, pid, out)
    return out[0], out[1]


def sample_upar(x: float, a: float, n: int, seed: int = 7, event: int = 1):
    """n samples of u_parallel at fixed (x, a), photon ids 0..n-1; returns (u, trials)."""
    f = lib().or_sample_upar
    u = np.empty(n)
    tr = np.empty(n, dtype=np.uint64)
    t = C.c_uint64()
    for i in range(n):
        u[i] = f(float(x), float(a), seed, event, i, C.byref(t))
        tr[i] = t.value
    return u, tr


def upar_expected_trials(x: float, a: float) -> float:
    return lib().or_upar_expected_trials(float(x), float(a))


def sample_mu(phase: str, U, g: float = 0.0):
    f = lib().or_sample_mu
    ph = PHASE[phase]
    return np.array([f(ph, float(u), float(g)) for u in np.ravel(U)])


def basis(n):
    nn = (C.c_double * 3)(*map(float, n))
    e1, e2 = (C.c_double * 3)(), (C.c_double * 3)()
    lib().or_basis(nn, e1, e2)
    return np.array(list(e1)), np.array(list(e2))


# ----------------------------------------------------------------- transport
def _f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


def make_structs(geom: dict, src: dict, opts: dict):
    """Build (Geometry, Source, Opts, keepalive) from the plain-dict description
    used by the tests and the benchmark (see ``workloads``)."""
    g = Geometry()
    g.kind = GEOMETRY[geom["kind"]]
    g.r_inner = geom.get("r_inner", 0.0)
    g.r_outer = geom.get("r_outer", 0.0)
    g.n_HI = geom.get("n_HI", 0.0)
    g.tau0 = geom.get("tau0", 0.0)
    g.T = geom.get("T", 1e4)
    g.v_profile = VELOCITY[geom.get("v_profile", "none")]
    g.v_max = geom.get("v_max", 0.0)
    g.step_f = geom.get("step_f", 0.01)
    keep = []
    if g.kind == 2:
        fields = [_f32(geom[k]) for k in ("n_HI_field", "T_field", "vx", "vy", "vz")]
        keep += fields
        nz, ny, nx = fields[0].shape
        g.nx, g.ny, g.nz = nx, ny, nz
        g.lo[:] = list(map(float, geom["lo"]))
        g.hi[:] = list(map(float, geom["hi"]))
        g.f_n, g.f_T, g.f_vx, g.f_vy, g.f_vz = [f.ctypes.data for f in fields]
    g.boundary_handoff = int(geom.get("boundary_handoff", 0))
    g.sigma_d = geom.get("sigma_d", 0.0)
    g.tau_d = geom.get("tau_d", 0.0)
    g.albedo = geom.get("albedo", 0.0)
    g.g_hg = geom.get("g_hg", 0.73)
    g.hubble = geom.get("hubble", 0.0)
    g.hubble_ref[:] = list(map(float, geom.get("hubble_ref", (0.0, 0.0, 0.0))))
    g.hubble_step = geom.get("hubble_step", 0.0)
    g.stop_dv = geom.get("stop_dv", 0.0)
    g.line = LINE[geom.get("line", "lya")]

    s = Source()
    s.kind = SOURCE[src.get("kind", "point")]
    s.pos[:] = list(map(float, src.get("pos", (0.0, 0.0, 0.0))))
    s.spectrum = SPECTRUM[src.get("spectrum", "delta")]
    s.dv0 = src.get("dv0", 0.0)
    s.sigma_v = src.get("sigma_v", 0.0)
    s.seed = src.get("seed", 1)
    s.request_id = src.get("request_id", 0)
    s.lines = int(src.get("lines", 0))

    o = Opts()
    o.phase = PHASE[opts.get("phase", "iso")]
    o.core_skip = CORE_SKIP[opts.get("core_skip", "off")]
    o.x_crit = opts.get("x_crit", 0.0)
    obs = opts.get("observers", [])
    o.n_obs = len(obs)
    for i, ax in enumerate(obs):
        o.obs_axis[i] = OBS_AXIS[ax]
    cube = opts.get("cube", None)
    if cube:
        o.cube_nx, o.cube_ny, o.cube_nb = cube["nx"], cube["ny"], cube["nb"]
        o.img_lo[:] = list(map(float, cube["img_lo"]))
        o.img_hi[:] = list(map(float, cube["img_hi"]))
        o.cube_v_lo, o.cube_v_hi = cube["v_lo"], cube["v_hi"]
    sp = opts["spectrum"]
    o.spec_nb, o.spec_lo, o.spec_hi = sp["nb"], sp["lo"], sp["hi"]
    o.spec_T_ref = sp.get("T_ref", 0.0)
    o.tau_cut = opts.get("tau_cut", 40.0)
    o.max_events = opts.get("max_events", 0)
    return g, s, o, keep


def run(geom: dict, src: dict, opts: dict, first_id: int, n: int, records: bool = False):
    """Transport packets [first_id, first_id + n) serially.  Returns a dict with
    'spectrum' (f64), 'cube' (f64 [n_obs, ny, nx, nb] or None), 'stats' (dict)
    and optionally 'records' (structured array)."""
    g, s, o, keep = make_structs(geom, src, opts)
    spec = np.zeros(o.spec_nb)
    cube = None
    if o.n_obs > 0:
        cube = np.zeros((o.n_obs, o.cube_ny, o.cube_nx, o.cube_nb))
    st = Stats()
    rec = np.zeros(n, dtype=RECORD_DTYPE) if records else None
    rc = lib().or_transport(C.byref(g), C.byref(s), C.byref(o), first_id, n,
                            spec.ctypes.data, None if cube is None else cube.ctypes.data,
                            C.byref(st), None if rec is None else rec.ctypes.data)
    if rc != 0:
        raise RuntimeError("oracle transport failed with code %d" % rc)
    del keep
    stats = {name: getattr(st, name) for name, _ in Stats._fields_}
    out = {"spectrum": spec, "cube": cube, "stats": stats}
    if records:
        out["records"] = rec
    return out


def emit(geom: dict, src: dict, first_id: int, n: int):
    """The generator alone (Section 3.4 "Emission") for photon ids
    [first_id, first_id + n): position, direction, lab-frame dv, gas-frame dv
    (THERMAL spectra) and the emitting cell of every packet."""
    g, s, _, keep = make_structs(geom, src, {"spectrum": {"nb": 1, "lo": 0.0, "hi": 1.0}})
    out = np.zeros((n, 11))
    rc = lib().or_emit(C.byref(g), C.byref(s), int(first_id), int(n), out.ctypes.data)
    if rc != 0:
        raise RuntimeError("or_emit failed with code %d" % rc)
    del keep
    return {"pos": out[:, 0:3], "dir": out[:, 3:6], "dv": out[:, 6], "dv_loc": out[:, 7],
            "cell": out[:, 8:11].astype(np.int64)}


def scatter_resonant(x: float, a: float, k, n: int, x_crit: float = 0.0, phase: str = "iso",
                     seed: int = 11, event: int = 1):
    """n resonant scatterings of a photon at gas-frame x along unit k (photon
    ids 0..n-1): u_par, u_perp (n, 2), x_atom, x_out, k_out (n, 3), trials and
    the phase function used."""
    kk = (C.c_double * 3)(*map(float, k))
    out = np.zeros((n, 10))
    rc = lib().or_scatter_resonant(float(x), float(a), kk, float(x_crit), PHASE[phase], seed, event,
                                   int(n), out.ctypes.data)
    if rc != 0:
        raise ValueError("or_scatter_resonant: invalid arguments")
    return {"upar": out[:, 0], "uperp": out[:, 1:3], "x_atom": out[:, 3], "x_out": out[:, 4],
            "kout": out[:, 5:8], "trials": out[:, 8].astype(np.int64), "phase": out[:, 9].astype(int)}


def run_threaded(geom: dict, src: dict, opts: dict, first_id: int, n: int, threads: int,
                 records: bool = False, reduce: bool = True):
    """Same result as ``run`` (up to summation order of the FP64 accumulators)
    with the id range split over `threads` host threads that share one prepared
    medium (one emission CDF, the caller's field arrays); each thread has its
    own outputs.  ctypes releases the GIL for the duration of each call.
    'transport_seconds' is the wall time of the threads' transport calls
    alone (no preparation, no reduction); with reduce=False only the summed
    counters and that time are returned."""
    import time
    from concurrent.futures import ThreadPoolExecutor
    g, s, o, keep = make_structs(geom, src, opts)
    L = lib()
    prep = L.or_prepare(C.byref(g), C.byref(s), C.byref(o))
    if not prep:
        raise RuntimeError("or_prepare failed")
    threads = max(1, min(int(threads), n))
    bounds = np.linspace(0, n, threads + 1).astype(np.int64)

    def part(i):
        lo, hi = int(bounds[i]), int(bounds[i + 1])
        spec = np.zeros(o.spec_nb)
        cube = np.zeros((o.n_obs, o.cube_ny, o.cube_nx, o.cube_nb)) if o.n_obs > 0 else None
        st = Stats()
        rec = np.zeros(hi - lo, dtype=RECORD_DTYPE) if records else None
        rc = L.or_transport_prepared(prep, first_id + lo, hi - lo, spec.ctypes.data,
                                     None if cube is None else cube.ctypes.data, C.byref(st),
                                     None if rec is None else rec.ctypes.data)
        if rc != 0:
            raise RuntimeError("oracle transport failed with code %d" % rc)
        return spec, cube, {name: getattr(st, name) for name, _ in Stats._fields_}, rec

    try:
        with ThreadPoolExecutor(threads) as ex:
            t0 = time.perf_counter()
            parts = list(ex.map(part, range(threads)))
            seconds = time.perf_counter() - t0
    finally:
        L.or_release(prep)
    del keep
    stats = {k: sum(p[2][k] for p in parts) for k in parts[0][2]}
    if not reduce:
        return {"stats": stats, "transport_seconds": seconds}
    out = {"spectrum": sum(p[0] for p in parts), "transport_seconds": seconds,
           "cube": None if parts[0][1] is None else sum(p[1] for p in parts), "stats": stats}
    if records:
        out["records"] = np.concatenate([p[3] for p in parts])
    return out


_JOB = None


def _run_chunk(bounds):
    geom, src, opts, records = _JOB
    return run(geom, src, opts, bounds[0], bounds[1], records)


def run_parallel(geom, src, opts, first_id, n, workers=None, records=False):
    """Same result as ``run`` (up to summation order of the FP64 accumulators),
    split into contiguous id ranges over ``workers`` forked processes (which
    inherit the inputs instead of receiving copies)."""
    import multiprocessing as mp
    global _JOB
    workers = workers or min(8, os.cpu_count() or 1)
    if workers <= 1 or n < 2 * workers:
        return run(geom, src, opts, first_id, n, records)
    bounds = np.linspace(0, n, workers + 1).astype(np.int64)
    jobs = [(first_id + int(bounds[i]), int(bounds[i + 1] - bounds[i])) for i in range(workers)]
    build()
    lib()
    _JOB = (geom, src, opts, records)
    try:
        with mp.get_context("fork").Pool(workers) as pool:
            parts = pool.map(_run_chunk, jobs)
    finally:
        _JOB = None
    out = {"spectrum": sum(p["spectrum"] for p in parts),
           "cube": None if parts[0]["cube"] is None else sum(p["cube"] for p in parts),
           "stats": {k: sum(p["stats"][k] for p in parts) for k in parts[0]["stats"]}}
    if records:
        out["records"] = np.concatenate([p["records"] for p in parts])
    return out


# ------------------------------------------------------------- raytracing
def _grid32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.ndim != 3:
        raise ValueError("fields are [z][y][x] arrays")
    return a


def ray_image_shape(shape, axis: int):
    """(n_j, n_i) of the image of rays along `axis` through a [z][y][x] grid."""
    nz, ny, nx = shape
    if axis not in (0, 1, 2):
        raise ValueError("axis must be 0 (x), 1 (y) or 2 (z)")
    return {0: (nz, ny), 1: (nz, nx), 2: (ny, nx)}[axis]


def project(q, w=None, axis: int = 2, ds: float = 1.0):
    """Projection Q = int q w ds and Q_hat = int w ds along `axis` (Section 3.5.1).
    Returns (Q, Q_hat) as [j][i] float64 images."""
    q = _grid32(q)
    w = None if w is None else _grid32(w)
    Q = np.zeros(ray_image_shape(q.shape, axis))
    W = np.zeros_like(Q)
    nz, ny, nx = q.shape
    rc = lib().or_project(q.ctypes.data, None if w is None else w.ctypes.data, nx, ny, nz,
                          int(axis), float(ds), Q.ctypes.data, W.ctypes.data)
    if rc != 0:
        raise ValueError("or_project: invalid arguments")
    return Q, W


def forest(n_HI, T, v_los, axis: int, ds: float, hubble: float, n_sub: int, los,
           nb: int, u_lo: float, u_hi: float):
    """Lyman-alpha optical depth tau[n_los][nb] along axis-parallel rays
    (Section 3.5.2, eq. abs); `los` is an (n_los, 2) array of (i, j)."""
    n_HI, T, v_los = _grid32(n_HI), _grid32(T), _grid32(v_los)
    if not (n_HI.shape == T.shape == v_los.shape):
        raise ValueError("field shapes differ")
    los = np.ascontiguousarray(np.asarray(los, dtype=np.int32).reshape(-1, 2))
    tau = np.zeros((los.shape[0], int(nb)))
    nz, ny, nx = n_HI.shape
    rc = lib().or_forest(n_HI.ctypes.data, T.ctypes.data, v_los.ctypes.data, nx, ny, nz,
                         int(axis), float(ds), float(hubble), int(n_sub), los.ctypes.data,
                         los.shape[0], int(nb), float(u_lo), float(u_hi), tau.ctypes.data)
    if rc != 0:
        raise ValueError("or_forest: invalid arguments")
    return tau
