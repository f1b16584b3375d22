"""Write the stored oracle spectra that the GPU parity tests compare against.

    python tests/golden/make_oracle_spectra.py [--threads N]

Every value comes from the CPU oracle (oracle/, serial FP64 transport per
packet, host threads over disjoint photon-id ranges); nothing here touches
the HIP path.  Files (text, one header line of '#' comments, then the
escape spectrum's bin counts, one per line):

  oracle_sphere_tau1e5_n1e4.txt     static sphere, tau0 = 1e5, T = 1e4 K,
                                    10000 packets at x = 0, seed 1, isotropic
                                    (200 bins of x over [-40, 40))
  oracle_corewing_tau1e4_n2e4.txt   the same sphere at tau0 = 1e4 with the
                                    core/wing phase-function mix, 20000 packets
  oracle_slab_dust_tau1e6.txt       dusty slab (T = 20 K, tau0 = 1e6, albedo 0,
                                    Section 4's dust test): per line
                                    b = (a tau0)^(1/3) tau_d, tau_d, packets,
                                    escaped (photon ids 0.., seed 1)
"""
from __future__ import annotations

import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

CASES = {
    "oracle_sphere_tau1e5_n1e4.txt": (dict(tau0=1e5, phase="iso"), 10000),
    "oracle_corewing_tau1e4_n2e4.txt": (dict(tau0=1e4, phase="core_wing"), 20000),
}


def write(name, threads):
    kw, n = CASES[name]
    wl = W.sphere(n_packets=n, **kw)
    t0 = time.time()
    r = oracle.run_threaded(wl["geom"], wl["src"], wl["opts"], 0, n, threads)
    st = r["stats"]
    with open(os.path.join(HERE, name), "w") as f:
        f.write("# oracle escape spectrum: sphere tau0=%g T=1e4 K phase=%s seed=%d ids 0..%d; "
                "escaped=%d n_res=%d upar_trials=%d; written by tests/golden/make_oracle_spectra.py\n"
                % (kw["tau0"], kw["phase"], wl["src"]["seed"], n - 1, st["escaped"], st["n_res"], st["upar_trials"]))
        for v in r["spectrum"]:
            f.write("%d\n" % round(v))
    print("%s: %.0f s, mean scatterings %.1f" % (name, time.time() - t0, st["n_res"] / n), flush=True)


SLAB_B = (0.5, 1.0)
SLAB_N = 300


def write_slab(threads):
    name = "oracle_slab_dust_tau1e6.txt"
    T, tau0 = 20.0, 1e6
    _, a, _ = oracle.line_params(T)
    t0 = time.time()
    rows = []
    for b in SLAB_B:
        tau_d = b / (a * tau0) ** (1.0 / 3.0)
        wl = W.dusty_slab(tau0=tau0, T=T, tau_d=tau_d, n_packets=SLAB_N)
        r = oracle.run_threaded(wl["geom"], wl["src"], wl["opts"], 0, SLAB_N, threads)
        rows.append((b, tau_d, SLAB_N, r["stats"]["escaped"]))
    with open(os.path.join(HERE, name), "w") as f:
        f.write("# oracle escape from a dusty slab: T=20 K tau0=1e6 albedo 0 isotropic, line-centre source, "
                "seed 1; columns b tau_d packets escaped; written by tests/golden/make_oracle_spectra.py\n")
        for row in rows:
            f.write("%.3f %.10g %d %d\n" % row)
    print("%s: %.0f s" % (name, time.time() - t0), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", default="")
    a = ap.parse_args()
    oracle.build()
    for name in CASES:
        if not a.only or a.only == name:
            write(name, a.threads)
    if not a.only or a.only == "oracle_slab_dust_tau1e6.txt":
        write_slab(a.threads)


if __name__ == "__main__":
    main()
