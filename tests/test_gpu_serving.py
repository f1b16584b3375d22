"""Serving form on the GPU: continuous batching of shell-model requests.
Each result must be the same alone and in a mix; results follow the oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
from stats_util import chi2_two_sample

pytestmark = pytest.mark.gpu

KMS = W.KMS


def _say(msg):
    print("[gpu-test] " + msg, flush=True)


@pytest.fixture(scope="module")
def serve_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2507_11603_amd import serve
    return serve


REQS = [dict(N_HI=3e19, v_exp_kms=150.0, tau_d=0.5, n=3000, rid=11),
        dict(N_HI=1e20, v_exp_kms=300.0, tau_d=1.0, n=500, rid=12),
        dict(N_HI=1e18, v_exp_kms=50.0, tau_d=0.2, n=1500, rid=13),
        dict(N_HI=5e20, v_exp_kms=400.0, tau_d=0.0, n=2000, rid=14)]


def _req(serve, d):
    return serve.make_request(d["N_HI"], d["v_exp_kms"], d["tau_d"], d["n"], d["rid"])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_same_alone_and_in_mix(serve_mod, precision):
    """Each request solved alone with eager steps equals the same request in a
    mix served by replaying one captured hipGraph per step."""
    _say("serving alone vs mix %s" % precision)
    alone = []
    for d in REQS:
        s = serve_mod.ShellServer(precision=precision, step_events=16, use_graph=False)
        try:
            alone.append(s.solve_all([_req(serve_mod, d)])[0])
        finally:
            s.close()
    s = serve_mod.ShellServer(precision=precision, step_events=16, use_graph=True)
    try:
        mix = s.solve_all([_req(serve_mod, d) for d in REQS[::-1]])[::-1]
        assert s.steps > 1
    finally:
        s.close()
    for a, b, d in zip(alone, mix, REQS):
        # escape weights are 1, so the per-bin sums are exact integers
        assert np.array_equal(a, b), d
        assert 0 < a.sum() <= d["n"]


def test_serving_fp64_matches_oracle_same_seed(serve_mod):
    _say("serving vs oracle")
    d = REQS[0]
    s = serve_mod.ShellServer(precision="fp64", step_events=8)
    try:
        gpu = s.solve_all([_req(serve_mod, d)])[0]
    finally:
        s.close()
    wl = W.shell_request(d["N_HI"], d["v_exp_kms"], d["tau_d"], d["n"], d["rid"])
    ref = oracle.run_parallel(wl["geom"], wl["src"], wl["opts"], 0, d["n"])
    diff = np.abs(gpu - ref["spectrum"]).sum()
    _say("same-seed spectrum L1 difference %.0f of %.0f" % (diff, ref["spectrum"].sum()))
    assert diff <= 0.02 * ref["spectrum"].sum() + 4


def test_serving_mixed_chi2_vs_oracle(serve_mod):
    _say("serving mixed chi2")
    d = dict(REQS[2], n=20000, rid=21)
    s = serve_mod.ShellServer(precision="mixed", step_events=64)
    try:
        gpu = s.solve_all([_req(serve_mod, d)])[0]
    finally:
        s.close()
    wl = W.shell_request(d["N_HI"], d["v_exp_kms"], d["tau_d"], 4000, 99)
    ref = oracle.run_parallel(wl["geom"], wl["src"], wl["opts"], 0, 4000)
    chi2, dof, p = chi2_two_sample(gpu, ref["spectrum"])
    _say("chi2 %.1f dof %d p %.3f" % (chi2, dof, p))
    assert p > 0.01


def test_admission_by_budget(serve_mod):
    """A small HBM budget defers a request until an earlier one finishes."""
    from paper_2507_11603_amd import thor
    _say("admission")
    s = serve_mod.ShellServer(precision="mixed", step_events=32, hbm_budget_bytes=200 << 20)
    try:
        big = serve_mod.make_request(1e20, 300.0, 1.0, 1_000_000, 31)
        h1 = s.submit(big)
        assert h1 is not None
        h2 = s.submit(serve_mod.make_request(1e20, 300.0, 1.0, 1_000_000, 32))
        assert h2 is None            # would exceed the budget while h1 is live
        while s.poll(h1) is None:
            s.step()
        h2 = s.submit(serve_mod.make_request(1e20, 300.0, 1.0, 1_000, 33))
        assert h2 is not None
        while s.poll(h2) is None:
            s.step()
        with pytest.raises(thor.ThorError):
            thor.thor_poll(s.ctx, h2, None)   # handle released after completion
    finally:
        s.close()
