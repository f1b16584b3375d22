"""The no-allocation transport (thor_transport_noalloc) against thor_transport
through the C ABI: two calls in a row, the second with fewer packets, must
give the same spectra and counters (bit for bit: both run the same kernels,
so the same histories, and FP64 sums of unit weights are exact in any
order) and, with observers, the same cube up to the order of float atomics."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

EXACT = ("emitted", "escaped", "absorbed", "capped", "n_res", "n_dust", "main_visits", "peel_visits",
         "peel_contrib", "peel_dropped", "peel_cut", "upar_trials", "max_events")


def _say(msg):
    print("[gpu-test] " + msg, flush=True)


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _pair(torch, wl, sizes, precision, **kw):
    """Per call: thor_transport on context A (outputs reset first) and
    thor_transport_noalloc on context B into fresh zeroed tensors."""
    from paper_2507_11603_amd import thor
    A, B = thor.Transport(0), thor.Transport(0)
    out = []
    try:
        A.load(wl["geom"])
        B.load(wl["geom"])
        o = wl["opts"]
        obs = o.get("observers", [])
        first = 0
        for n in sizes:
            _say("%s %s: %d packets" % (wl["name"], precision, n))
            A.reset()
            A.emit(wl["src"], n, first)
            _, sa = A.transport(o, precision=precision, path="persistent", **kw)
            spec_a = A.spectrum()
            spec_b = torch.zeros(o["spectrum"]["nb"], dtype=torch.float64, device="cuda")
            cube_b = None
            if obs:
                c = o["cube"]
                cube_b = torch.zeros((len(obs), c["ny"], c["nx"], c["nb"]), dtype=torch.float32, device="cuda")
            B.emit(wl["src"], n, first)
            sb = B.transport_noalloc(o, spec_b, cube_b, precision=precision, **kw)
            rec = {"spec_a": spec_a, "spec_b": spec_b.cpu().numpy(), "st_a": sa, "st_b": sb}
            if obs:
                c = o["cube"]
                rec["cube_a"] = A.cube((len(obs), c["ny"], c["nx"], c["nb"]))
                rec["cube_b"] = cube_b.cpu().numpy()
            out.append(rec)
            first += n
    finally:
        A.close()
        B.close()
    return out


def _same(rec):
    assert np.array_equal(rec["spec_a"], rec["spec_b"])
    for k in EXACT:
        assert rec["st_a"][k] == rec["st_b"][k], k


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_sphere_matches_transport(torch_mod, precision):
    wl = W.sphere(tau0=1e4, n_packets=3000)
    recs = _pair(torch_mod, wl, [3000, 1100], precision)
    for r in recs:
        _same(r)
        assert r["st_b"]["emitted"] in (3000, 1100) and r["st_b"]["escaped"] == r["st_b"]["emitted"]


def test_noalloc_shell_grid_cube_matches_transport(torch_mod):
    """Grid medium with one observer (peel rays marched inline on both sides)."""
    wl = W.shell(n_grid=32, n_packets=20000)
    recs = _pair(torch_mod, wl, [20000, 6000], "mixed", inline_peel=True)
    for r in recs:
        _same(r)
        a, b = r["cube_a"], r["cube_b"]
        assert a.sum() > 0
        assert abs(b.sum() / a.sum() - 1) < 1e-5
        np.testing.assert_allclose(b, a, rtol=2e-3, atol=1e-6 * a.max())


def test_noalloc_async_call_and_limits(torch_mod):
    """Without stats the call only enqueues; the result is the same after a
    synchronisation.  Sizes beyond the scratch's limits are refused."""
    torch = torch_mod
    from paper_2507_11603_amd import thor
    wl = W.sphere(tau0=1e4, n_packets=800)
    T = thor.Transport(0)
    try:
        T.load(wl["geom"])
        T.emit(wl["src"], 800, 0)
        _, st = T.transport(wl["opts"], precision="fp64", path="persistent")
        ref = T.spectrum()
        spec = torch.zeros(wl["opts"]["spectrum"]["nb"], dtype=torch.float64, device="cuda")
        T.emit(wl["src"], 800, 0)
        assert T.transport_noalloc(wl["opts"], spec, want_stats=False, precision="fp64") is None
        torch.cuda.synchronize()
        assert np.array_equal(spec.cpu().numpy(), ref)
        big = dict(wl["opts"], spectrum=dict(nb=4097, lo=-40.0, hi=40.0))
        T.emit(wl["src"], 10, 0)
        with pytest.raises(thor.ThorError, match="4096"):
            T.transport_noalloc(big, torch.zeros(4097, dtype=torch.float64, device="cuda"), precision="fp64")
        with pytest.raises(thor.ThorError, match="records"):
            T.transport_noalloc(wl["opts"], spec, precision="fp64", records=True)
    finally:
        T.close()
