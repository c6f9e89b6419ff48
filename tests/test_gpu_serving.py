"""Serving with continuous batching: sessions arrive while others run, are
admitted by HBM footprint, receive edits while paused at their step limits,
and retire.  Every session's result in the mix equals the same session run
alone with the single-domain path, bit for bit (same kernels, same edits at
the same steps), and the edit outcomes (accepted / rejected terrain) agree."""
import sys

import numpy as np
import pytest

from paper_1611_05984_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_sessions_same_alone_and_in_the_mix():
    from paper_1611_05984_amd import serving as sv
    # small grids, so the edits are scaled down with them (sigma 3..8 cells,
    # humps 2..10 cm, terrain 5..20 cm): the recipe's 10..40-cell edits would
    # cover a whole 48-cell basin
    trace = wl.config5_trace(rate=40.0, duration=0.75, seed=51, sizes=(48, 64, 96, 130),
                             edit_every=20, steps=(40, 160), sigma_cells=(3, 8),
                             water_amp=(0.02, 0.1), terrain_amp=(0.05, 0.2))
    big = max(sv.footprint(s) for s in trace)
    srv = sv.Server(budget_bytes=3 * big, max_sessions=6, tick_steps=7, keep_results=True)
    say("case: %d sessions, budget %d B, 6 slots, tick 7 steps" % (len(trace), 3 * big))
    rep = srv.run(trace)
    say("  report: %s" % rep)
    assert rep["sessions_done"] == len(trace) and rep["sessions_rejected"] == 0
    assert rep["sessions_failed"] == 0
    assert rep["queue_wait_s_p99"] > 0.0
    n_rej = 0
    for rid, spec in enumerate(trace):
        mw, mP, mQ, mlog = srv.results[rid]
        aw, aP, aQ, alog, ahealth = sv.replay_alone(spec)
        assert ahealth == 0 and mlog == alog, (rid, mlog, alog)
        n_rej += sum(1 for s in alog if s != 0)
        for m, a, f in ((mw, aw, "w"), (mP, aP, "P"), (mQ, aQ, "Q")):
            assert np.isfinite(m).all()
            assert np.array_equal(m, a), (rid, f, float(np.abs(m - a).max()))
    say("  %d sessions equal alone and in the mix; %d terrain edits rejected" % (len(trace), n_rej))


def test_failed_session_is_retired_and_isolated():
    """Two sessions of the trace get a time step far beyond the stability
    limit (Courant 3), so their state turns non-finite within a few steps.
    Each is retired with an error at the tick where the batch reports its
    health word, and every other session still equals its run alone."""
    import dataclasses
    from paper_1611_05984_amd import serving as sv
    trace = wl.config5_trace(rate=40.0, duration=0.5, seed=52, sizes=(48, 64, 96),
                             edit_every=20, steps=(40, 120))
    bad = {3, 7}
    trace = [dataclasses.replace(s, courant=3.0) if k in bad else s for k, s in enumerate(trace)]
    srv = sv.Server(budget_bytes=1 << 34, max_sessions=8, tick_steps=5, keep_results=True)
    rep = srv.run(trace)
    say("  report: %s" % rep)
    assert set(srv.failures) == bad and rep["sessions_failed"] == 2
    assert rep["sessions_done"] == len(trace) - 2
    for rid, spec in enumerate(trace):
        aw, aP, aQ, alog, ahealth = sv.replay_alone(spec)
        if rid in bad:
            assert ahealth != 0, rid               # fails alone too
            continue
        mw, mP, mQ, mlog = srv.results[rid]
        assert ahealth == 0 and mlog == alog
        assert np.array_equal(mw, aw) and np.array_equal(mP, aP) and np.array_equal(mQ, aQ), rid


def test_failed_session_recovers_in_nlsw():
    """Recovery on: session 16 of the seed-5 serving trace (512 x 512 cells,
    depth 0.57 m, an edit every 50 steps) goes non-finite in the dispersive
    model (step 760) once its edits have built steep terrain with thin, fast
    flow.  The server rolls it back to its checkpoint of the last edit pause,
    continues it in NLSW with half the time step and runs it to its end.  A
    session at Courant 20 fails again after every rollback and is retired
    after the third.  Every finished session equals its run alone under the
    same policy, bit for bit, edit statuses included."""
    import dataclasses
    from paper_1611_05984_amd import serving as sv
    s16 = wl.config5_trace(seed=5, duration=20.0)[16]
    s16 = dataclasses.replace(s16, arrival=0.0, steps=1000, edits=[e for e in s16.edits if e[0] <= 1000])
    small = wl.config5_trace(rate=40.0, duration=0.2, seed=53, sizes=(48, 64), edit_every=20, steps=(40, 120),
                             sigma_cells=(3, 8), water_amp=(0.02, 0.1), terrain_amp=(0.05, 0.2))[:3]
    c20 = dataclasses.replace(small[0], courant=20.0)
    trace = [s16, c20] + small[1:]
    say("case: session 16 of seed 5 (512^2, 1000 steps), one Courant-20 session, %d small" % (len(trace) - 2))
    base = sv.replay_alone(s16)
    say("  alone without recovery: health %d" % base[4])
    assert base[4] != 0                        # the dispersive run does fail
    srv = sv.Server(budget_bytes=1 << 34, max_sessions=4, tick_steps=10, keep_results=True, recover=True,
                    max_recoveries=3)
    rep = srv.run(trace)
    say("  report: %s" % rep)
    say("  rollbacks: %s" % srv.recovered)
    assert set(srv.recovered) == {0, 1} and srv.recovered[1] == 3 and set(srv.failures) == {1}
    assert rep["sessions_done"] == len(trace) - 1
    for rid, spec in enumerate(trace):
        aw, aP, aQ, alog, ahealth = sv.replay_alone(spec, max_recoveries=3)
        if rid == 1:
            assert ahealth != 0
            continue
        mw, mP, mQ, mlog = srv.results[rid]
        assert ahealth == 0 and mlog == alog and len(mlog) == len(spec.edits) - (spec.edits[-1][0] == spec.steps)
        for m, a, f in ((mw, aw, "w"), (mP, aP, "P"), (mQ, aQ, "Q")):
            assert np.isfinite(m).all()
            assert np.array_equal(m, a), (rid, f, float(np.abs(m - a).max()))
    say("  recovered session finished in NLSW; all finished sessions equal alone")
