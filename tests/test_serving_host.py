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


# ------------------------------------------------ recovery bookkeeping (fakes)
class SimDom:
    """Stand-in domain: its 'state' is the list of edits applied, with the
    session step each was applied at.  It counts steps since its last
    (re)start, as the library does (a time-step change restarts the count),
    and turns non-finite once its session step passes fail[level], level
    being the number of time-step halvings (None: never)."""

    def __init__(self, fail, dt):
        self.fail, self.model, self.dt, self.dt0 = fail, 0, dt, dt
        self.step, self.abs, self.health, self.stop, self.edits = 0, 0, 0, None, []

    def level(self):
        return round(np.log2(self.dt0 / self.dt))

    def run_to(self, stop):
        while self.step < stop:
            self.step += 1
            self.abs += 1
            f = self.fail[self.level()] if self.level() < len(self.fail) else None
            if f is not None and self.abs >= f:
                self.health = 1

    def advance(self, n):
        self.run_to(self.step + n)

    def query(self):
        return self.step, self.abs * self.dt, self.health

    def snapshot(self, out=None):
        return (self.step, self.abs, self.model, list(self.edits))

    def restore(self, snap):
        assert snap[2] == self.model            # the library checks the model too
        self.step, self.abs, self.health, self.edits = snap[0], snap[1], 0, list(snap[3])

    def update(self, model=None, dt=None):
        assert model == 1
        self.model = model
        if dt is not None and dt != self.dt:
            self.dt, self.step = dt, 0          # the step counter restarts

    def apply_edit(self, kind, x0, y0, amp, sigma):
        self.edits.append((self.abs, kind, x0))
        return 1 if kind == 1 and x0 > 5 else 0  # some terrain edits rejected

    def state_numpy(self):
        return (tuple(self.edits), self.abs, (self.model, self.level()))

    def close(self):
        pass


class SimBatch:
    def __init__(self, max_domains, device=None):
        self.slots = {}

    def attach(self, dom):
        k = len(self.slots) + 100
        self.slots[k] = dom
        return k

    def detach(self, slot):
        del self.slots[slot]

    def set_stop(self, slot, stop):
        self.slots[slot].stop = stop

    def advance(self, n):
        for d in self.slots.values():
            d.run_to(min(d.step + n, d.stop))

    def sync(self):
        pass

    def status(self, slot):
        return self.slots[slot].query()

    def close(self):
        pass


def test_recovery_rolls_back_to_the_last_pause_and_halves_the_step(monkeypatch):
    """With recovery on, a session that fails is restored to its checkpoint
    of the last edit pause before the failure, switched to NLSW with half the
    time step, and re-applies the edits of that pause; in the end every edit
    was applied exactly once, at its own step, with one status each.  The
    domain's step counter restarts with each time-step change, and the
    server's step limits follow it.  After max_recoveries rollbacks a failure
    retires the session.  The single-domain replay follows the same policy
    and ends in the same state."""
    import torch
    fails = {64: (137,), 80: (40, 55, 61, 70), 96: (), 112: (60, 75), 128: (20, 130, None)}
    monkeypatch.setattr(sv.ws, "Domain", lambda nx, ny, dx, dy, dt, *a, **k: SimDom(fails[nx], dt))
    monkeypatch.setattr(sv.ws, "Batch", SimBatch)
    monkeypatch.setattr(sv.ws, "NLSW", 1, raising=False)
    monkeypatch.setattr(sv, "footprint", lambda spec, recover=False: 1 + recover)
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    rng = np.random.default_rng(7)
    trace = []
    for n in fails:
        edits = [(s, int(rng.integers(0, 2)), float(rng.uniform(0, 10)), 1.0, 0.1, 0.3)
                 for s in range(20, 200, 20)]
        trace.append(wl.Session(0.0, n, 1.0, 0.05, 200, edits))
    srv = sv.Server(budget_bytes=100, max_sessions=5, tick_steps=7, keep_results=True, recover=True,
                    max_recoveries=3)
    rep = srv.run(trace, time_scale=0.0)
    assert srv.recovered == {0: 1, 1: 3, 3: 2, 4: 2} and set(srv.failures) == {1}
    assert rep["sessions_recovered"] == 4 and rep["rollbacks"] == 8
    assert rep["sessions_failed"] == 1 and rep["sessions_done"] == 4
    for rid, spec in enumerate(trace):
        alone = sv.replay_alone(spec, max_recoveries=3)
        if rid == 1:
            assert alone[-1] != 0                # fails a fourth time, alone as well
            continue
        edits, step, model = srv.results[rid][:3]
        log = srv.results[rid][3]
        assert step == 200 and model == ((0, 0) if rid == 2 else (1, srv.recovered[rid]))
        assert [(e[0], e[1], e[2]) for e in edits] == [(e[0], e[1], e[2]) for e in spec.edits]
        assert log == [1 if e[1] == 1 and e[2] > 5 else 0 for e in spec.edits]
        assert alone[:4] == srv.results[rid] and alone[4] == 0
    # recovery off: the failing sessions are retired at their first failure
    srv = sv.Server(budget_bytes=100, max_sessions=5, tick_steps=7, keep_results=True)
    rep = srv.run(trace, time_scale=0.0)
    assert set(srv.failures) == {0, 1, 3, 4} and rep["sessions_recovered"] == 0
