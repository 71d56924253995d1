"""Host checks of the request server's scheduling helpers (no GPU): the
Poisson arrival times, and the guard that keeps every context the server
drives from several streams on the unsplit layer (the split layer shares
one internal stream and its events across calls)."""
import numpy as np

from paper_2506_11586_amd import serving


class FakeTuning:
    def __init__(self, split):
        self.layer_split = split


class FakeCtx:
    def __init__(self, split):
        self.split = split

    def get_tuning(self):
        return FakeTuning(self.split)

    def set_tuning(self, **kw):
        self.split = kw.get("layer_split", self.split)


def test_single_stream_tunings_resets_split():
    a, b, c = FakeCtx(1), FakeCtx(2), FakeCtx(4)
    changed = serving.single_stream_tunings([a, b, c])
    assert changed == [b, c]
    assert a.split == b.split == c.split == 1
    assert serving.single_stream_tunings([a, b, c]) == []


def test_poisson_arrivals():
    u = np.linspace(0.0, 0.999, 1000)
    t = serving.poisson_arrivals(100.0, 1000, u)
    assert np.all(np.diff(t) >= 0) and t[0] == 0.0
    gaps = -np.log1p(-u) / 100.0
    assert np.allclose(t, np.cumsum(gaps))
