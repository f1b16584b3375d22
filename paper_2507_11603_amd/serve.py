"""Continuous-batching request loop for shell-model solves (the serving form).

Requests (N_HI, v_exp, T, tau_d, photon count) arrive over time; each is
admitted by `thor_submit` when its state fits the context's HBM budget,
shares the device with every other live request through bounded persistent
steps (`thor_step`), and is collected with `thor_poll` once all its packets
are done.  The loop itself is host-side bookkeeping; all transport runs in
libthor.so.
"""
from __future__ import annotations

import ctypes as C
import sys
import time

import numpy as np

from . import thor

KPC = 3.0856775814913673e21
KMS = 1.0e5


def make_request(N_HI: float, v_exp_kms: float, tau_d: float, n_packets: int, request_id: int,
                 T: float = 1e4, seed: int = 5, spec_nb: int = 400, spec_kms: float = 2500.0,
                 albedo: float = 0.3, g_hg: float = 0.73, sigma_v_kms: float = 20.0,
                 step_f: float = 0.01) -> thor.thor_shell_request:
    r = thor.thor_shell_request()
    r.N_HI, r.v_exp, r.T, r.tau_d = N_HI, v_exp_kms * KMS, T, tau_d
    r.albedo, r.g_hg = albedo, g_hg
    r.r_inner, r.r_outer = 0.8 * KPC, 1.0 * KPC
    r.sigma_v, r.step_f = sigma_v_kms * KMS, step_f
    r.n_packets, r.seed, r.request_id = n_packets, seed, request_id
    r.spec_nb, r.spec_lo, r.spec_hi = spec_nb, -spec_kms * KMS, spec_kms * KMS
    return r


class ShellServer:
    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, precision: str = "mixed",
                 step_events: int = 4096, waves_per_cu: int = 0, visits_per_turn: int = 0,
                 use_graph: bool = True):
        import torch
        self.stream = torch.cuda.current_stream(torch.device("cuda", device))
        self.ctx = thor.thor_create(device, self.stream.cuda_stream, hbm_budget_bytes)
        self.opts = thor.make_opts(dict(spectrum=dict(nb=1, lo=0.0, hi=1.0)), precision=precision,
                                   path="persistent", waves_per_cu=waves_per_cu,
                                   visits_per_turn=visits_per_turn, use_graph=use_graph)
        self.step_events = step_events
        self.live = {}          # handle -> spec_nb
        self.steps = 0
        self.scatterings = 0
        self.kernel_ms = 0.0

    def close(self):
        if self.ctx is not None:
            thor.thor_destroy(self.ctx)
            self.ctx = None

    def submit(self, req: thor.thor_shell_request):
        """Handle, or None when the budget defers the request."""
        code, h = thor.thor_submit(self.ctx, req)
        if code == -3:
            return None
        thor._check(code)
        self.live[h] = req.spec_nb
        return h

    def step(self) -> int:
        code = thor.thor_step(self.ctx, self.step_events, self.opts)
        st = thor.thor_stats()
        thor._check(thor.lib().thor_read_spectra(self.ctx, thor.OUT["stats"], 0, C.addressof(st),
                                                C.sizeof(st), 0))
        self.steps += 1
        self.scatterings += st.n_res + st.n_dust
        self.kernel_ms += st.kernel_ms
        return code

    def poll(self, h):
        spec = np.zeros(self.live[h])
        done, _ = thor.thor_poll(self.ctx, h, spec)
        if done:
            del self.live[h]
            return spec
        return None

    def solve_all(self, reqs):
        """Submit every request, step until all are done; spectra by handle order."""
        hs = []
        for r in reqs:
            h = self.submit(r)
            assert h is not None, "request deferred by the budget"
            hs.append(h)
        out = {}
        while len(out) < len(hs):
            self.step()
            for h in hs:
                if h not in out:
                    s = self.poll(h)
                    if s is not None:
                        out[h] = s
        return [out[h] for h in hs]

    def run_stream(self, stream, warmup: int = 0, time_scale: float = 1.0, max_wall_s: float = 600.0,
                   progress_s: float = 0.0):
        """Open-loop arrivals: request i becomes available at t_arrival[i] *
        time_scale after the start.  Returns per-request latencies (completion -
        arrival) of the requests after `warmup`, deferral count and throughput.
        progress_s > 0: a line on stderr every that many seconds."""
        t0 = time.monotonic()
        t_said = 0.0
        arrivals = [r["t_arrival"] * time_scale for r in stream]
        nxt = 0
        waiting = []          # arrived, not yet admitted
        live = {}             # handle -> index
        done_at = {}
        deferrals = 0
        scat0, k0 = self.scatterings, self.kernel_ms
        while len(done_at) < len(stream):
            now = time.monotonic() - t0
            if now > max_wall_s:
                raise TimeoutError("stream did not finish within %.0f s" % max_wall_s)
            if progress_s > 0.0 and now - t_said >= progress_s:
                t_said = now
                print("[serve] %.0f s: %d of %d requests done, %d live, %d waiting"
                      % (now, len(done_at), len(stream), len(live), len(waiting)), file=sys.stderr, flush=True)
            while nxt < len(stream) and arrivals[nxt] <= now:
                waiting.append(nxt)
                nxt += 1
            while waiting:
                i = waiting[0]
                r = stream[i]
                h = self.submit(make_request(r["N_HI"], r["v_exp_kms"], r["tau_d"], r["n_packets"],
                                             r["request_id"]))
                if h is None:
                    deferrals += 1
                    break
                live[h] = i
                waiting.pop(0)
            if live:
                self.step()
                t = time.monotonic() - t0
                for h in list(live):
                    if self.poll(h) is not None:
                        done_at[live.pop(h)] = t
            elif nxt < len(stream):
                time.sleep(max(0.0, min(0.01, arrivals[nxt] - (time.monotonic() - t0))))
        wall = time.monotonic() - t0
        lat = np.array([done_at[i] - arrivals[i] for i in range(warmup, len(stream))])
        return dict(latency_s=lat, p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                    deferrals=deferrals, wall_s=wall, scatterings=self.scatterings - scat0,
                    kernel_ms=self.kernel_ms - k0, steps=self.steps)
