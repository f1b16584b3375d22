"""The autotuner (host logic, no GPU: a stand-in transport): coordinate-wise
search over the knobs, scored by the median total device time of repeated
runs over the same sample."""
import pytest

from paper_2507_11603_amd import autotune


class FakeTransport:
    """Total device time depends on the knobs, with one slow outlier run out
    of every three (the median ignores it)."""
    device = 0

    def __init__(self):
        self.calls = 0
        self.samples = set()

    def reset(self):
        pass

    def emit(self, src, n, first):
        self.samples.add((n, first))

    def transport(self, opts, precision, path, waves_per_cu, block, park_lanes, refill_64ths, wide_lanes,
                  visits_per_turn, presort):
        self.calls += 1
        ms = (10.0 + abs(waves_per_cu - 4) + abs(park_lanes - 24) / 8.0 + (block != 128)
              + abs(refill_64ths - 32) / 16.0 + abs(wide_lanes - 16) / 4.0 + abs(visits_per_turn - 1024) / 512.0
              + (presort != 2))
        if self.calls % 3 == 0:
            ms += 1000.0
        return 0, {"kernel_ms": ms}


def test_tune_coordinate_search_with_median(monkeypatch, tmp_path):
    torch = pytest.importorskip("torch")
    monkeypatch.setattr(torch.cuda, "get_device_name", lambda d=0: "fake")
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "cache.json"))
    T = FakeTransport()
    wl = {"src": {}, "opts": {}}
    best, table = autotune.tune(T, wl, "fake-web", sample=10, repeats=3)
    assert best == {"waves_per_cu": 4, "block": 128, "park_lanes": 24, "refill_64ths": 32, "wide_lanes": 16,
                    "visits_per_turn": 1024, "presort": 2}
    # every candidate ran on the same packets
    assert T.samples == {(10, 7 * 10**12)}
    assert len(table) <= sum(len(v) for v in autotune.SPACE.values())
    # cached per device, workload, precision and sample
    calls = T.calls
    again, _ = autotune.tune(T, wl, "fake-web", sample=10, repeats=3)
    assert again == best and T.calls == calls
