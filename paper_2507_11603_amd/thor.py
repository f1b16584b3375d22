"""ctypes binding of libthor.so (include/thor.h: the transport; include/thor_rays.h:
the raytracing driver's projections and absorption spectra).

Argument marshalling only: every step of the transport and of the raytracing
runs in the HIP kernels of libthor.so.  PyTorch supplies device memory and the stream.
Importing works without a GPU; any call that needs the library raises if
libthor.so has not been built (``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("THOR_LIB") or os.path.join(HERE, "libthor.so")

OK, INCOMPLETE = 0, 1
STATUS = {0: "THOR_OK", 1: "THOR_INCOMPLETE", -1: "THOR_E_INVAL", -2: "THOR_E_NOMEM",
          -3: "THOR_E_BUDGET", -4: "THOR_E_DEVICE", -5: "THOR_E_STATE", -6: "THOR_E_UNSUPPORTED"}
GEOM = {"shell": 0, "sphere": 0, "slab": 1, "grid": 2}
VEL = {"none": 0, "const_radial": 1, "linear": 2}
SRC = {"point": 0, "cell_n2": 1}
SPEC = {"delta": 0, "gauss": 1, "thermal": 2, "flat": 3}
LINE = {"lya": 0, "mg2": 1, "mg2k": 2}
PREC = {"fp64": 0, "mixed": 1}
PATH = {"plain": 0, "persistent": 1}
PHASE = {"iso": 0, "dipole": 1, "core_wing": 2}
CORE_SKIP = {"off": 0, "fixed": 1, "adaptive": 2}
OBS = {"+x": 0, "+y": 1, "+z": 2, "-x": 3, "-y": 4, "-z": 5}
OUT = {"spectrum": 0, "cube": 1, "records": 2, "stats": 3, "cube_fixed": 4}
ACCUM = {"f32": 0, "fixed64": 1}
SYMBOLS = ["thor_create", "thor_destroy", "thor_load_grid", "thor_emit", "thor_transport",
           "thor_reset_outputs", "thor_read_spectra", "thor_output_bytes", "thor_last_error",
           "thor_eval_voigt", "thor_eval_xcw", "thor_sample_upar", "thor_submit", "thor_step", "thor_poll",
           "thor_ray_project", "thor_ray_forest", "thor_ray_last_error", "thor_transport_noalloc"]


class ThorError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


class thor_geometry(C.Structure):
    _fields_ = [("kind", C.c_int32), ("r_inner", C.c_double), ("r_outer", C.c_double),
                ("n_HI", C.c_double), ("tau0", C.c_double), ("T", C.c_double),
                ("v_profile", C.c_int32), ("v_max", C.c_double), ("step_f", C.c_double),
                ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("n_HI_field", C.c_void_p), ("T_field", C.c_void_p), ("vx", C.c_void_p),
                ("vy", C.c_void_p), ("vz", C.c_void_p), ("mem", C.c_int32),
                ("boundary_handoff", C.c_int32), ("sigma_d", C.c_double), ("tau_d", C.c_double),
                ("albedo", C.c_double), ("g_hg", C.c_double),
                ("hubble", C.c_double), ("hubble_ref", C.c_double * 3), ("hubble_step", C.c_double),
                ("stop_dv", C.c_double), ("line", C.c_int32)]


class thor_source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pos", C.c_double * 3), ("spectrum", C.c_int32),
                ("dv0", C.c_double), ("sigma_v", C.c_double),
                ("seed", C.c_uint32), ("request_id", C.c_uint32), ("lines", C.c_int32)]


class thor_transport_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("path", C.c_int32), ("phase", C.c_int32),
                ("core_skip", C.c_int32), ("x_crit", C.c_double), ("n_obs", C.c_int32),
                ("obs_axis", C.c_int32 * 6), ("cube_nx", C.c_int32), ("cube_ny", C.c_int32),
                ("cube_nb", C.c_int32), ("img_lo", C.c_double * 2), ("img_hi", C.c_double * 2),
                ("cube_v_lo", C.c_double), ("cube_v_hi", C.c_double), ("spec_nb", C.c_int32),
                ("spec_lo", C.c_double), ("spec_hi", C.c_double), ("spec_T_ref", C.c_double),
                ("tau_cut", C.c_double), ("max_events", C.c_uint64), ("step_events", C.c_uint64),
                ("waves_per_cu", C.c_int32), ("block", C.c_int32), ("visits_per_turn", C.c_int32),
                ("use_graph", C.c_int32), ("inline_peel", C.c_int32), ("records", C.c_int32),
                ("seed_slots", C.c_uint64),
                ("wide_lanes", C.c_int32), ("park_lanes", C.c_int32), ("refill_64ths", C.c_int32),
                ("accum", C.c_int32), ("fixed_bits", C.c_int32), ("presort", C.c_int32),
                ("seed_sort", C.c_int32), ("fuse_bins", C.c_int32)]


STAT_U64 = ("emitted", "escaped", "absorbed", "capped", "handed_off", "n_res", "n_dust",
            "main_visits", "peel_visits", "peel_contrib", "peel_dropped", "peel_cut", "upar_trials")


class thor_stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in STAT_U64] + [
        ("w_escaped", C.c_double), ("w_absorbed", C.c_double), ("kernel_ms", C.c_double),
        ("transport_ms", C.c_double), ("peel_ms", C.c_double), ("passes", C.c_uint64),
        ("tail_ms", C.c_double), ("max_events", C.c_uint64), ("tail_events", C.c_uint64),
        ("tail_main_visits", C.c_uint64), ("tail_peel_visits", C.c_uint64), ("redshifted", C.c_uint64),
        ("presort_ms", C.c_double), ("seedsort_ms", C.c_double), ("peel_fused", C.c_uint64)]

    def to_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class thor_record(C.Structure):
    _fields_ = [("dv", C.c_double), ("n_res", C.c_uint32), ("n_dust", C.c_uint32),
                ("fate", C.c_int32), ("pad", C.c_uint32)]


RECORD_DTYPE = np.dtype([("dv", "<f8"), ("n_res", "<u4"), ("n_dust", "<u4"),
                         ("fate", "<i4"), ("pad", "<u4")])


class thor_shell_request(C.Structure):
    _fields_ = [("N_HI", C.c_double), ("v_exp", C.c_double), ("T", C.c_double),
                ("tau_d", C.c_double), ("albedo", C.c_double), ("g_hg", C.c_double),
                ("r_inner", C.c_double), ("r_outer", C.c_double), ("sigma_v", C.c_double),
                ("step_f", C.c_double), ("n_packets", C.c_uint64), ("seed", C.c_uint32),
                ("request_id", C.c_uint32), ("spec_nb", C.c_int32), ("spec_lo", C.c_double),
                ("spec_hi", C.c_double)]


class thor_ray_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("axis", C.c_int32),
                ("ds", C.c_double)]


class thor_forest_opts(C.Structure):
    _fields_ = [("i0", C.c_int32), ("ni", C.c_int32), ("j0", C.c_int32), ("nj", C.c_int32),
                ("hubble", C.c_double), ("n_sub", C.c_int32), ("nb", C.c_uint32),
                ("u_lo", C.c_double), ("u_hi", C.c_double), ("precision", C.c_int32)]


_lib = None


def lib():
    """Load libthor.so; raises when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libthor.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        vp, u64, i32, u32, d = C.c_void_p, C.c_uint64, C.c_int32, C.c_uint32, C.c_double
        sig = {
            "thor_create": ([C.POINTER(vp), C.c_int, vp, u64], C.c_int),
            "thor_destroy": ([vp], None),
            "thor_load_grid": ([vp, C.POINTER(thor_geometry)], C.c_int),
            "thor_emit": ([vp, C.POINTER(thor_source), u64, u64], C.c_int),
            "thor_transport": ([vp, C.POINTER(thor_transport_opts), C.POINTER(thor_stats)], C.c_int),
            "thor_reset_outputs": ([vp], C.c_int),
            "thor_read_spectra": ([vp, C.c_int, u32, vp, u64, C.c_int], C.c_int),
            "thor_output_bytes": ([vp, C.c_int], u64),
            "thor_last_error": ([], C.c_char_p),
            "thor_eval_voigt": ([vp, vp, vp, vp, u64, i32], C.c_int),
            "thor_eval_xcw": ([vp, vp, vp, u64, i32], C.c_int),
            "thor_sample_upar": ([vp, d, d, u32, u32, vp, vp, u64, i32], C.c_int),
            "thor_submit": ([vp, C.POINTER(thor_shell_request), C.POINTER(u64)], C.c_int),
            "thor_step": ([vp, u32, C.POINTER(thor_transport_opts)], C.c_int),
            "thor_poll": ([vp, u64, vp, C.POINTER(thor_stats), C.POINTER(C.c_int)], C.c_int),
            "thor_ray_project": ([C.POINTER(thor_ray_grid), vp, vp, vp, vp, vp], C.c_int),
            "thor_ray_forest": ([C.POINTER(thor_ray_grid), C.POINTER(thor_forest_opts), vp, vp, vp,
                                 vp, vp], C.c_int),
            "thor_ray_last_error": ([], C.c_char_p),
            "thor_transport_noalloc": ([vp, C.POINTER(thor_transport_opts), vp, vp, C.POINTER(thor_stats)],
                                       C.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(code, allow_incomplete=False):
    if code == OK or (allow_incomplete and code == INCOMPLETE):
        return code
    raise ThorError(code, lib().thor_last_error().decode())


# ------------------------------------------------------------------ C-ABI names
def thor_create(device: int = 0, stream: int | None = None, hbm_budget_bytes: int = 0):
    h = C.c_void_p()
    _check(lib().thor_create(C.byref(h), device, stream, hbm_budget_bytes))
    return h


def thor_destroy(ctx):
    lib().thor_destroy(ctx)


def thor_load_grid(ctx, geom: thor_geometry):
    _check(lib().thor_load_grid(ctx, C.byref(geom)))


def thor_emit(ctx, src: thor_source, n_packets: int, first_photon_id: int):
    _check(lib().thor_emit(ctx, C.byref(src), n_packets, first_photon_id))


def thor_transport(ctx, opts: thor_transport_opts):
    st = thor_stats()
    code = _check(lib().thor_transport(ctx, C.byref(opts), C.byref(st)), allow_incomplete=True)
    return code, st


def thor_transport_noalloc(ctx, opts: thor_transport_opts, spec_ptr, cube_ptr, want_stats: bool = True):
    st = thor_stats() if want_stats else None
    _check(lib().thor_transport_noalloc(ctx, C.byref(opts), spec_ptr, cube_ptr,
                                        C.byref(st) if want_stats else None))
    return st


def thor_reset_outputs(ctx):
    _check(lib().thor_reset_outputs(ctx))


def thor_read_spectra(ctx, which: str, dst_ptr: int, dst_bytes: int, on_device: bool):
    _check(lib().thor_read_spectra(ctx, OUT[which], 0, dst_ptr, dst_bytes, int(on_device)))


def thor_output_bytes(ctx, which: str) -> int:
    return lib().thor_output_bytes(ctx, OUT[which])


def thor_eval_voigt(ctx, a_ptr, x_ptr, out_ptr, n, precision):
    _check(lib().thor_eval_voigt(ctx, a_ptr, x_ptr, out_ptr, n, PREC[precision]))


def thor_eval_xcw(ctx, a_ptr, out_ptr, n, precision):
    _check(lib().thor_eval_xcw(ctx, a_ptr, out_ptr, n, PREC[precision]))


def thor_sample_upar(ctx, x, a, seed, event, u_ptr, tr_ptr, n, precision):
    _check(lib().thor_sample_upar(ctx, x, a, seed, event, u_ptr, tr_ptr, n, PREC[precision]))


def thor_submit(ctx, req: thor_shell_request):
    rid = C.c_uint64()
    code = lib().thor_submit(ctx, C.byref(req), C.byref(rid))
    return code, rid.value


def thor_step(ctx, max_events_per_packet: int, opts: thor_transport_opts):
    return _check(lib().thor_step(ctx, max_events_per_packet, C.byref(opts)), allow_incomplete=True)


def thor_poll(ctx, req_id: int, spectrum: np.ndarray | None):
    st = thor_stats()
    done = C.c_int()
    ptr = None if spectrum is None else spectrum.ctypes.data
    _check(lib().thor_poll(ctx, req_id, ptr, C.byref(st), C.byref(done)))
    return bool(done.value), st


# ------------------------------------------------------------------ struct builders
def _check_ray(code):
    if code != OK:
        raise ThorError(code, lib().thor_ray_last_error().decode())


def thor_ray_project(grid: thor_ray_grid, q_ptr, w_ptr, Q_ptr, W_ptr, stream):
    _check_ray(lib().thor_ray_project(C.byref(grid), q_ptr, w_ptr, Q_ptr, W_ptr, stream))


def thor_ray_forest(grid: thor_ray_grid, opts: thor_forest_opts, n_ptr, T_ptr, v_ptr, tau_ptr, stream):
    _check_ray(lib().thor_ray_forest(C.byref(grid), C.byref(opts), n_ptr, T_ptr, v_ptr, tau_ptr, stream))


def make_geometry(geom: dict, device_fields=None) -> thor_geometry:
    """Plain-dict medium description (see ``workloads``) -> thor_geometry.
    For grids, ``device_fields`` holds the five float32 device tensors
    (n_HI, T, vx, vy, vz) whose pointers are passed; they are copied in."""
    g = thor_geometry()
    g.kind = GEOM[geom["kind"]]
    g.r_inner = geom.get("r_inner", 0.0)
    g.r_outer = geom.get("r_outer", 0.0)
    g.n_HI = geom.get("n_HI", 0.0)
    g.tau0 = geom.get("tau0", 0.0)
    g.T = geom.get("T", 1e4)
    g.v_profile = VEL[geom.get("v_profile", "none")]
    g.v_max = geom.get("v_max", 0.0)
    g.step_f = geom.get("step_f", 0.01)
    if g.kind == 2:
        nz, ny, nx = tuple(device_fields[0].shape)
        g.nx, g.ny, g.nz = nx, ny, nz
        g.lo[:] = list(map(float, geom["lo"]))
        g.hi[:] = list(map(float, geom["hi"]))
        g.n_HI_field, g.T_field, g.vx, g.vy, g.vz = [int(t.data_ptr()) for t in device_fields]
        g.mem = 1
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
    return g


def make_source(src: dict) -> thor_source:
    s = thor_source()
    s.kind = SRC[src.get("kind", "point")]
    s.pos[:] = list(map(float, src.get("pos", (0.0, 0.0, 0.0))))
    s.spectrum = SPEC[src.get("spectrum", "delta")]
    s.dv0 = src.get("dv0", 0.0)
    s.sigma_v = src.get("sigma_v", 0.0)
    s.seed = src.get("seed", 1)
    s.request_id = src.get("request_id", 0)
    s.lines = int(src.get("lines", 0))
    return s


def make_opts(opts: dict, precision="fp64", path="plain", records=False, step_events=0,
              waves_per_cu=0, block=0, visits_per_turn=0, use_graph=False,
              inline_peel=False, seed_slots=0, wide_lanes=0, park_lanes=0,
              refill_64ths=0, accum="f32", fixed_bits=0, presort=0, seed_sort=0,
              fuse_bins=0) -> thor_transport_opts:
    o = thor_transport_opts()
    o.precision = PREC[precision]
    o.path = PATH[path]
    o.phase = PHASE[opts.get("phase", "iso")]
    o.core_skip = CORE_SKIP[opts.get("core_skip", "off")]
    o.x_crit = opts.get("x_crit", 0.0)
    obs = opts.get("observers", [])
    o.n_obs = len(obs)
    for i, ax in enumerate(obs):
        o.obs_axis[i] = OBS[ax]
    cube = opts.get("cube")
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
    o.step_events = step_events
    o.waves_per_cu = waves_per_cu
    o.block = block
    o.visits_per_turn = visits_per_turn
    o.use_graph = int(use_graph)
    o.inline_peel = int(inline_peel)
    o.records = int(records)
    o.seed_slots = int(seed_slots)
    o.wide_lanes = int(wide_lanes)
    o.park_lanes = int(park_lanes)
    o.refill_64ths = int(refill_64ths)
    o.accum = ACCUM[accum]
    o.fixed_bits = int(fixed_bits)
    o.presort = int(presort)
    o.seed_sort = int(seed_sort)
    o.fuse_bins = int(fuse_bins)
    return o


# ------------------------------------------------------------------ convenience
class Transport:
    """One context bound to torch's current stream on ``device``."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = thor_create(device, self.stream.cuda_stream, hbm_budget_bytes)
        self._keep = []

    def close(self):
        if self.ctx is not None:
            thor_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self, geom: dict):
        fields = None
        if geom["kind"] == "grid":
            t = self.torch
            fields = [t.as_tensor(np.ascontiguousarray(geom[k], dtype=np.float32)).to(self.device)
                      if not (isinstance(geom[k], t.Tensor) and geom[k].is_cuda) else geom[k].contiguous()
                      for k in ("n_HI_field", "T_field", "vx", "vy", "vz")]
        thor_load_grid(self.ctx, make_geometry(geom, fields))
        del fields
        self.torch.cuda.synchronize(self.device)

    def emit(self, src: dict, n: int, first_id: int = 0):
        thor_emit(self.ctx, make_source(src), n, first_id)

    def transport(self, opts: dict, **kw):
        code, st = thor_transport(self.ctx, make_opts(opts, **kw))
        return code, st.to_dict()

    def transport_noalloc(self, opts: dict, spectrum, cube=None, want_stats=True, **kw):
        """thor_transport_noalloc into the caller's device tensors `spectrum`
        (float64[spec_nb]) and `cube` (float32[n_obs][ny][nx][nb] or None),
        which it adds to; returns the counters (None without want_stats)."""
        t = self.torch
        sp = opts["spectrum"]
        if not (isinstance(spectrum, t.Tensor) and spectrum.is_cuda and spectrum.dtype == t.float64
                and spectrum.is_contiguous() and spectrum.numel() == sp["nb"]):
            raise ValueError("spectrum must be a contiguous float64 CUDA tensor of %d bins" % sp["nb"])
        obs = opts.get("observers", [])
        if obs:
            c = opts["cube"]
            shape = (len(obs), c["ny"], c["nx"], c["nb"])
            if not (isinstance(cube, t.Tensor) and cube.is_cuda and cube.dtype == t.float32
                    and cube.is_contiguous() and tuple(cube.shape) == shape):
                raise ValueError("cube must be a contiguous float32 CUDA tensor of shape %s" % (shape,))
        st = thor_transport_noalloc(self.ctx, make_opts(opts, path="persistent", **kw), spectrum.data_ptr(),
                                    cube.data_ptr() if obs else None, want_stats)
        return st.to_dict() if st is not None else None

    def reset(self):
        thor_reset_outputs(self.ctx)

    def spectrum(self) -> np.ndarray:
        nb = thor_output_bytes(self.ctx, "spectrum") // 8
        out = np.zeros(nb)
        thor_read_spectra(self.ctx, "spectrum", out.ctypes.data, out.nbytes, False)
        return out

    def cube(self, shape) -> np.ndarray:
        out = np.zeros(shape, dtype=np.float32)
        thor_read_spectra(self.ctx, "cube", out.ctypes.data, out.nbytes, False)
        return out

    def cube_fixed(self, shape) -> np.ndarray:
        """The FIXED64 cube's integer sums (units of 2^-fixed_bits)."""
        out = np.zeros(shape, dtype=np.uint64)
        thor_read_spectra(self.ctx, "cube_fixed", out.ctypes.data, out.nbytes, False)
        return out

    def records(self) -> np.ndarray:
        n = thor_output_bytes(self.ctx, "records") // RECORD_DTYPE.itemsize
        out = np.zeros(n, dtype=RECORD_DTYPE)
        thor_read_spectra(self.ctx, "records", out.ctypes.data, out.nbytes, False)
        return out

    def voigt(self, a, x, precision="fp64") -> np.ndarray:
        t = self.torch
        a_t = t.as_tensor(np.ascontiguousarray(a, dtype=np.float64).ravel(), device=self.device)
        x_t = t.as_tensor(np.ascontiguousarray(x, dtype=np.float64).ravel(), device=self.device)
        out = t.empty_like(x_t)
        thor_eval_voigt(self.ctx, a_t.data_ptr(), x_t.data_ptr(), out.data_ptr(), x_t.numel(), precision)
        return out.cpu().numpy().reshape(np.shape(x))

    def xcw(self, a, precision="fp64") -> np.ndarray:
        """Core-to-wing transition x_cw(a) by the Appendix A.2 quartic."""
        t = self.torch
        a_t = t.as_tensor(np.ascontiguousarray(a, dtype=np.float64).ravel(), device=self.device)
        out = t.empty_like(a_t)
        thor_eval_xcw(self.ctx, a_t.data_ptr(), out.data_ptr(), a_t.numel(), precision)
        return out.cpu().numpy().reshape(np.shape(a))

    def sample_upar(self, x, a, n, seed=7, event=1, precision="fp64"):
        t = self.torch
        u = t.empty(n, dtype=t.float64, device=self.device)
        tr = t.empty(n, dtype=t.int32, device=self.device)
        thor_sample_upar(self.ctx, float(x), float(a), seed, event, u.data_ptr(), tr.data_ptr(), n,
                         precision)
        return u.cpu().numpy(), tr.cpu().numpy().astype(np.uint32)


def run(wl: dict, n: int | None = None, first_id: int = 0, precision="fp64", path="plain",
        records=False, device: int = 0, **kw):
    """Load, emit and transport one workload; returns spectrum, cube, stats (and records)."""
    T = Transport(device)
    try:
        T.load(wl["geom"])
        T.emit(wl["src"], n if n is not None else wl["n_packets"], first_id)
        code, st = T.transport(wl["opts"], precision=precision, path=path, records=records, **kw)
        out = {"spectrum": T.spectrum(), "stats": st, "code": code}
        o = wl["opts"]
        if o.get("observers"):
            c = o["cube"]
            out["cube"] = T.cube((len(o["observers"]), c["ny"], c["nx"], c["nb"]))
        if records:
            out["records"] = T.records()
        return out
    finally:
        T.close()


# ------------------------------------------------------------- raytracing
def ray_image_shape(shape, axis: int):
    """(n_j, n_i) of the image of rays along `axis` through a [z][y][x] grid."""
    nz, ny, nx = shape
    return {0: (nz, ny), 1: (nz, nx), 2: (ny, nx)}[axis]


def _field(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.dim() == 3
            and t.is_contiguous()):
        raise ValueError("%s must be a contiguous float32 [z][y][x] CUDA tensor" % name)
    return t


def _check_out(t, name, shape, device):
    """A caller-supplied output: contiguous float64 of the expected shape on
    the fields' device (a wrong one would be written out of bounds)."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.is_contiguous()
            and tuple(t.shape) == tuple(shape) and t.device == device):
        raise ValueError("%s must be a contiguous float64 tensor of shape %s on %s" % (name, tuple(shape), device))
    return t


def ray_project(q, w=None, axis: int = 2, ds: float = 1.0, out=None):
    """Projection along `axis` (Section 3.5.1): returns device float64 images
    (Q, W) = (int q w ds, int w ds), each [j][i].  `out` may pass both images."""
    import torch
    q = _field(q, "q")
    if w is not None:
        w = _field(w, "w")
        if w.shape != q.shape or w.device != q.device:
            raise ValueError("w must match q")
    nz, ny, nx = q.shape
    g = thor_ray_grid(nx, ny, nz, int(axis), float(ds))
    shape = ray_image_shape(q.shape, axis) if axis in (0, 1, 2) else (1, 1)
    if out is None:
        out = (torch.empty(shape, dtype=torch.float64, device=q.device),
               torch.empty(shape, dtype=torch.float64, device=q.device))
    Q, W = (_check_out(t, n, shape, q.device) for t, n in zip(out, ("out[0]", "out[1]")))
    with torch.cuda.device(q.device):
        thor_ray_project(g, q.data_ptr(), None if w is None else w.data_ptr(), Q.data_ptr(),
                         W.data_ptr(), torch.cuda.current_stream(q.device).cuda_stream)
    return Q, W


def ray_forest(n_HI, T, v_los, axis: int, ds: float, hubble: float, n_sub: int,
               rays, nb: int, u_lo: float, u_hi: float, precision: str = "fp64", out=None):
    """Lyman-alpha optical depth along rays parallel to `axis` (Section 3.5.2,
    eq. abs).  `rays` = (i0, ni, j0, nj); returns a device float64 tensor
    tau[nj][ni][nb]."""
    import torch
    n_HI, T, v_los = _field(n_HI, "n_HI"), _field(T, "T"), _field(v_los, "v_los")
    if not (n_HI.shape == T.shape == v_los.shape):
        raise ValueError("field shapes differ")
    nz, ny, nx = n_HI.shape
    i0, ni, j0, nj = (int(r) for r in rays)
    g = thor_ray_grid(nx, ny, nz, int(axis), float(ds))
    o = thor_forest_opts(i0, ni, j0, nj, float(hubble), int(n_sub), int(nb), float(u_lo),
                         float(u_hi), PREC[precision])
    shape = (max(nj, 0), max(ni, 0), int(nb))
    tau = (_check_out(out, "out", shape, n_HI.device) if out is not None
           else torch.empty(shape, dtype=torch.float64, device=n_HI.device))
    with torch.cuda.device(n_HI.device):
        thor_ray_forest(g, o, n_HI.data_ptr(), T.data_ptr(), v_los.data_ptr(), tau.data_ptr(),
                        torch.cuda.current_stream(n_HI.device).cuda_stream)
    return tau
