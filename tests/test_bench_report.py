"""bench.py's split of a call's device time and cell visits among its kernels
(host logic, no GPU)."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_split_with_tail_kernel():
    b = _bench()
    st = {"transport_ms": 2500.0, "tail_ms": 2000.0, "peel_ms": 80.0, "passes": 1,
          "main_visits": 1_000_000, "peel_visits": 3_000_000, "peel_contrib": 500_000,
          "tail_main_visits": 100_000, "tail_peel_visits": 20_000, "tail_events": 90_000}
    s = b.kernel_split(st)
    assert set(s) == {"transport", "tail", "peel_pass"}
    # first segments of every ray are marched by the transport kernels, the rest by the pass
    assert s["peel_pass"]["visits"] == 3_000_000 - 500_000
    assert s["tail"]["visits"] == 120_000 and s["tail"]["events"] == 90_000
    assert s["transport"]["visits"] == 1_000_000 + 500_000 - 120_000
    assert s["transport"]["ms"] == 500.0 and s["tail"]["ms"] == 2000.0
    assert max(s, key=lambda k: s[k]["ms"]) == "tail"
    # achieved bytes: 20 B per visit over the kernel's own time
    assert abs(s["peel_pass"]["achieved_GBps"] - 20 * 2_500_000 / 0.080 / 1e9) < 1e-9


def test_split_without_tail_or_seeds():
    b = _bench()
    st = {"transport_ms": 100.0, "tail_ms": 0.0, "peel_ms": 0.0, "passes": 1,
          "main_visits": 10, "peel_visits": 30, "peel_contrib": 5,
          "tail_main_visits": 0, "tail_peel_visits": 0, "tail_events": 0}
    s = b.kernel_split(st)
    assert "tail" not in s
    assert s["transport"]["visits"] == 40 and s["peel_pass"]["visits"] == 0


def test_totals_over_calls_and_headline_roofline():
    """Per-call stats add up over the timed calls (the longest history is a
    maximum); the roofline takes the kernel with the most device time, its
    average launch time and algorithmic bytes per launch."""
    b = _bench()
    st = {"transport_ms": 40.0, "tail_ms": 1.0, "peel_ms": 60.0, "passes": 2, "kernel_ms": 101.0,
          "main_visits": 100, "peel_visits": 1000, "peel_contrib": 50, "tail_main_visits": 1,
          "tail_peel_visits": 1, "tail_events": 3, "max_events": 7}
    tot = b.add_stats(None, st)
    tot = b.add_stats(tot, dict(st, max_events=5))
    assert tot["passes"] == 4 and tot["peel_visits"] == 2000 and tot["max_events"] == 7
    roof, split, dom = b.roofline_web(tot)
    assert dom == "peel_pass" and roof["kernel"] == "k_peel_pass_f32" and roof["bound"] == "hbm"
    assert roof["launches"] == 4 and abs(roof["avg_launch_ms"] - 30.0) < 1e-12
    assert abs(roof["algorithmic_bytes_per_launch"] - 20 * (2000 - 100) / 4) < 1e-9
    assert abs(roof["achieved"] - roof["algorithmic_bytes_per_launch"] / 0.030 / 1e9) < 1e-6
    assert abs(roof["frac"] - roof["achieved"] / 8000.0) < 1e-12


def test_alu_bound_dominant_kernel_and_counter_record():
    """When the transport kernel has the most device time the headline
    roofline is its VALU issue rate (bound "alu"), taken from the counter
    record scaled to this run's packets; without a record it stays None.  The
    peel pass's HBM-gather block is reported beside it."""
    b = _bench()
    st = {"transport_ms": 700.0, "tail_ms": 10.0, "peel_ms": 600.0, "passes": 7, "kernel_ms": 1310.0,
          "main_visits": 1000, "peel_visits": 30000, "peel_contrib": 500, "tail_main_visits": 10,
          "tail_peel_visits": 10, "tail_events": 5, "max_events": 9}
    tot = b.add_stats(None, st)
    roof, split, dom = b.roofline_web(tot)
    assert dom == "transport" and roof["bound"] == "alu" and roof["kernel"].startswith("k_persistent")
    assert roof["achieved"] is None and roof["frac"] is None
    assert roof["peak"] == 256 * 4 * 2.4e9 / 4 and roof["unit"] == "wave64 VALU instructions/s"
    gather = b.kernel_roofline(split, "peel_pass")
    assert gather["bound"] == "hbm" and gather["frac"] == split["peel_pass"]["hbm_frac"]
    # a record taken at 100 packets; this run had 1000: everything scales by 10
    rec = {"packets": 100, "path": "profiles/x.json",
           "kernels": {"k_persistent": {"read_bytes_per_batch": 3.0e6, "write_bytes_per_batch": 1.0e6,
                                        "valu_insts_per_batch": 2.0e9, "valu_busy_pct": 70.0,
                                        "valu_lane_util_pct": 24.0},
                       "k_peel_pass": {"read_bytes_per_batch": 5.0e6, "write_bytes_per_batch": 1.0e6}}}
    b.attach_counters(roof, split, "transport", rec, 1000)
    b.attach_counters(gather, split, "peel_pass", rec, 1000)
    # the transport kernel alone: the call's transport time less the tail kernel's
    assert abs(roof["achieved"] - 2.0e10 / 0.69) < 1e-9 * 2.0e10 / 0.69
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-15
    assert abs(roof["traffic"] - 4.0e7 / 7) < 1e-6 and roof["counters"] == "profiles/x.json"
    assert abs(gather["traffic"] - 6.0e7 / 7) < 1e-6 and gather["achieved"] == split["peel_pass"]["achieved_GBps"]
