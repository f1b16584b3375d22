"""The autotuner scores launch knobs by the device time without the tail
kernel (host logic, no GPU: a stand-in transport)."""
import types

import pytest

from paper_2507_11603_amd import autotune


class FakeTransport:
    """Persistent-kernel time depends on the knobs; the tail kernel's time is
    large and unrelated to them (it follows the longest history)."""
    device = 0

    def __init__(self):
        self.calls = 0

    def reset(self):
        pass

    def emit(self, src, n, first):
        pass

    def transport(self, opts, precision, path, waves_per_cu, block, visits_per_turn):
        self.calls += 1
        dense = 10.0 + abs(waves_per_cu - 8) + abs(visits_per_turn - 256) / 64.0
        tail = 1000.0 * ((self.calls * 7919) % 13)        # noise far above the knob effect
        return 0, {"kernel_ms": dense + tail, "tail_ms": tail}


def test_tune_ignores_the_tail(monkeypatch, tmp_path):
    torch = pytest.importorskip("torch")
    monkeypatch.setattr(torch.cuda, "get_device_name", lambda d=0: "fake")
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "cache.json"))
    T = FakeTransport()
    wl = {"src": {}, "opts": {}}
    best, table = autotune.tune(T, wl, "fake-shell", sample=10, batches=1)
    assert best == {"waves_per_cu": 8, "block": 256, "visits_per_turn": 256}
    assert len(table) == len(autotune.DEFAULT_SPACE["waves_per_cu"]) * len(autotune.DEFAULT_SPACE["visits_per_turn"])
    # the choice is cached per device, workload and precision
    again, _ = autotune.tune(T, wl, "fake-shell", sample=10, batches=1)
    assert again == best and T.calls == len(table)
