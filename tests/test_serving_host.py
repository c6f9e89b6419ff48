"""Host-side scheduling logic of the session server (no GPU): event steps,
edit application order, weighted percentiles, footprints, trace recipe."""
import numpy as np

from paper_1611_05984_amd import serving as sv
from paper_1611_05984_amd import workloads as wl


class FakeDom:
    def __init__(self):
        self.edits = []

    def apply_edit(self, kind, x0, y0, amp, sigma):
        self.edits.append((kind, x0, y0, amp, sigma))
        return 0


def test_event_steps_walk_edits_then_end():
    spec = wl.Session(0.0, 64, 1.0, 0.05, 130, [(50, 0, 1, 1, .1, .3), (100, 1, 2, 2, .2, .4)])
    assert sv._next_stop(spec, 0, 0) == (50, 0)
    assert sv._next_stop(spec, 49, 0) == (50, 0)
    d, log = FakeDom(), []
    k = sv._apply_due(d, spec, 50, 0, log)
    assert k == 1 and len(d.edits) == 1 and log == [0]
    assert sv._next_stop(spec, 50, k) == (100, 1)
    k = sv._apply_due(d, spec, 100, k, log)
    assert sv._next_stop(spec, 100, k) == (130, 2)
    # an edit due exactly at the last step is never applied: the session ends there
    spec2 = wl.Session(0.0, 64, 1.0, 0.05, 100, [(50, 0, 1, 1, .1, .3), (100, 0, 1, 1, .1, .3)])
    assert sv._next_stop(spec2, 50, 1) == (100, 1)


def test_weighted_percentile():
    lat = [1.0, 2.0, 10.0]
    w = [98, 1, 1]
    assert sv._pct(lat, w, 50) == 1.0
    assert sv._pct(lat, w, 99) == 2.0
    assert sv._pct(lat, w, 100) == 10.0
    assert sv._pct(list(np.arange(100.0)), [1] * 100, 50) == 49.0


def test_footprint_grows_with_area_and_trace_recipe():
    f = [sv.footprint(wl.Session(0, n, 1.0, 0.05, 10, [])) for n in (512, 1024, 2048)]
    assert f[0] < f[1] < f[2]
    assert 3.5 < f[1] / f[0] < 4.5 and 3.5 < f[2] / f[1] < 4.5
    tr = wl.config5_trace()
    assert 2200 < len(tr) < 2600                      # Poisson 4/s over 600 s
    assert all(s.nx in (512, 1024, 2048) for s in tr)
    assert all(500 <= s.steps <= 2000 for s in tr)
    assert all([e[0] for e in s.edits] == list(range(50, s.steps + 1, 50)) for s in tr[:50])
    gaps = np.diff([0.0] + [s.arrival for s in tr])
    assert abs(gaps.mean() - 0.25) < 0.02
