"""Runs at the stated lengths of the workloads: the beach basin for 10 000
steps beside the oracle, the 256-domain ensemble for 2000 steps, and the
session-serving trace for its 600 s (plus a shorter run whose memory budget
binds).  Minutes of GPU and host time each, so they run only with
WAVESTEP_LONG=1 (their summaries are kept with the profiles)."""
import json
import math
import os
import sys
import time

import numpy as np
import pytest

import oracle as o
from paper_1611_05984_amd import workloads as wl

pytestmark = [pytest.mark.gpu, pytest.mark.slow,
              pytest.mark.skipif(os.environ.get("WAVESTEP_LONG") != "1",
                                 reason="long runs: set WAVESTEP_LONG=1")]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _ws():
    from paper_1611_05984_amd import wavestep as ws
    return ws


def _pair(w):
    ws = _ws()
    z = w.z.astype(np.float32).astype(np.float64)
    gpu = ws.Domain(w.nx, w.ny, w.dx, w.dy, w.dt, z)
    ora = o.Domain(w.nx, w.ny, w.dx, w.dy, w.dt, z)
    for s, side in enumerate(w.sides):
        if side.kind != wl.SOLID:
            ph = side.phase or None
            gpu.set_boundary(s, side.kind, side.width, side.amp, side.period, side.theta, ph)
            ora.set_boundary(s, side.kind, side.width, side.amp, side.period, side.theta, ph)
    return gpu, ora


def test_config2_10000_steps_beside_the_oracle():
    """Config 2 (1024 x 512 beach, bumps, sine maker) for its 10 000 steps
    (43 s simulated).  Every 1000 steps: the GPU state is finite and
    w >= B in every cell, and its water volume (FP64 sum of the FP32 depths)
    follows the oracle's (the oracle conserves volume in closed basins to
    1e-13; here the maker's inflow changes it, identically on both sides up
    to FP32 rounding).  The surface difference over the cells wet in both
    runs is reported at every checkpoint and bounded at the end."""
    ws = _ws()
    w = wl.config2()
    a = 0.03
    gpu, ora = _pair(w)
    b, _ = ora.bathy()
    area = w.dx * w.dy
    v0 = float(np.sum(np.maximum(ora.state()[0] - b, 0.0))) * area
    say("case: config2 1024x512, 10000 steps; initial volume %.6f m^3" % v0)
    worst_dv = 0.0
    for chunk in range(10):
        t = time.perf_counter()
        gpu.advance(1000)
        step, _, health = gpu.query()
        tg = time.perf_counter() - t
        t = time.perf_counter()
        ora.advance(1000)
        to = time.perf_counter() - t
        ge = gpu.state_numpy()[0].astype(np.float64)
        gh = gpu.state_numpy(ws.READ_H)[0].astype(np.float64)
        oe = ora.state()[0]
        vg, vo = float(gh.sum()) * area, float(np.sum(oe - b)) * area
        wet = ((oe - b) > 1e-4) & ((ge - b) > 1e-4)
        de = float(np.abs(ge - oe)[wet].max())
        below = float((b.astype(np.float32) - ge).max())
        worst_dv = max(worst_dv, abs(vg - vo) / vo)
        say("  step %5d: health %d, max(B - w) %.2e, volume gpu %.6f oracle %.6f (rel %.2e, "
            "change from start %.3e), max|d eta| wet %.3e (%.2e a)  [gpu %.1f s, oracle %.1f s]"
            % (step, health, below, vg, vo, (vg - vo) / vo, (vo - v0) / v0, de, de / a, tg, to))
        assert health == 0 and step == ora.step == 1000 * (chunk + 1)
        assert below <= 1e-6
    assert worst_dv <= 1e-6
    assert de <= 0.02 * a


def test_config4_ensemble_2000_steps():
    """The 256-domain ensemble (nx, ny ~ U{256..1024}, flat or beach,
    solitary waves) for its 2000 steps with the batch autotuner's shapes, as
    the benchmark runs it: every domain stays finite at every checkpoint,
    and the smallest, the largest and a beach domain equal their runs alone
    (same launch shapes) bit for bit at the end."""
    ws = _ws()
    ens = wl.config4()
    cells = [x.cells for x in ens]
    say("case: config4 ensemble, %d domains, %.4g cells, 2000 steps" % (len(ens), sum(cells)))

    def make(x):
        d = ws.Domain(x.nx, x.ny, x.dx, x.dy, x.dt, x.z.astype(np.float32).astype(np.float64))
        for (H, th, x0, y0) in x.solitary:
            d.add_solitary(H, th, x0, y0)
        return d

    doms = [make(x) for x in ens]
    pick = sorted({int(np.argmin(cells)), int(np.argmax(cells)),
                   next(k for k, x in enumerate(ens) if x.z.max() > -0.99)})
    alone = {k: make(ens[k]) for k in pick}
    B = ws.Batch(len(doms))
    for d in doms:
        B.attach(d)
    B.advance(4)                      # the start-up steps on the default shapes, as alone
    tuning = B.tune()
    say("  batch tuning %s" % (tuning,))
    for k in pick:
        alone[k].advance(4)
        alone[k].set_tuning(*tuning)
    t_all, timed = 0.0, 0
    for chunk in range(8):
        n = 246 if chunk == 0 else 250
        t = time.perf_counter()
        B.advance(n)
        B.sync()
        t_all += time.perf_counter() - t
        timed += n
        for k in pick:
            alone[k].advance(n)
        st = [B.status(s) for s in range(len(doms))]
        bad = [k for k, s in enumerate(st) if s[2] != 0]
        say("  step %d: unhealthy %d, batched rate %.3g cell-updates/s"
            % (st[0][0], len(bad), sum(cells) * timed / t_all))
        assert not bad, bad
    steps = {s[0] for s in st}
    assert steps == {2000}, steps
    B.close()
    for k in pick:
        ae, aP, aQ = alone[k].state_numpy()
        be, bP, bQ = doms[k].state_numpy()
        assert np.array_equal(ae, be) and np.array_equal(aP, bP) and np.array_equal(aQ, bQ), k
        say("  domain %d (%s, %dx%d): batch = alone bit for bit" % (k, ens[k].name, ens[k].nx, ens[k].ny))


def _serve(seconds, budget_gb, recover=True):
    from paper_1611_05984_amd import serving as sv
    srv = sv.Server(budget_bytes=int(budget_gb * 2 ** 30), max_sessions=256, tick_steps=10, recover=recover)
    rep = srv.run(wl.config5_trace(), wall_limit=seconds, log=say)
    say("  report: " + json.dumps(rep))
    return rep


def test_serving_600_s():
    """The serving trace (Poisson arrivals at 4/s, 512^2..2048^2 beach
    sessions, an edit every 50 steps) for its full 600 s with recovery on
    and the default 64 GB budget."""
    say("case: serving 600 s, 64 GB budget, recovery on")
    rep = _serve(600.0, 64.0)
    assert rep["sessions_done"] > 1000
    assert rep["wall_s"] >= 600.0
    assert rep["budget_used_max_bytes"] <= rep["budget_bytes"]


def test_serving_budget_binds():
    """The same trace with a 4 GB budget for 120 s (about ten sessions are
    resident at a time, 4 GB of workspaces and checkpoints on average): the
    budget binds -- sessions wait in the queue for memory, the footprint in
    use stays within it."""
    say("case: serving 120 s, 4 GB budget, recovery on")
    rep = _serve(120.0, 4.0)
    assert rep["sessions_queued_max"] > 0 and rep["queue_wait_s_p99"] > 0.0
    assert rep["budget_used_max_bytes"] <= rep["budget_bytes"]
    assert rep["sessions_done"] > 0
