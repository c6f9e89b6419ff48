"""Interactive-session serving on one GPU with continuous batching.

Sessions (a domain each) arrive over time.  The server admits them, first
come first served, while the HBM footprint of the resident sessions (their
workspaces) stays within a budget and a batch slot is free; admitted sessions
join the running batch at the next tick, so their steps overlap on the device
with everyone else's.  Each tick advances the batch by up to `tick_steps`
steps; a session pauses at its next event (a user edit, or its last step) by
the batch's per-domain step limit while the others run on.  Between ticks the
server applies due edits (add a Gaussian water hump, raise terrain), retires
finished sessions (freeing their memory for the queue) and admits arrivals.
A session whose state turns non-finite (the batch reports each domain's
health word at every sync) is retired with an error; the others run on.
With recovery on, the server instead keeps a device checkpoint of every
session (taken at admission and at each edit pause, before the edits).  A
session that fails is rolled back to its last checkpoint and continued in
the NLSW model (no dispersion) with half the time step, re-applying the
edits of that pause; a further failure halves the step again, up to
`max_recoveries` times, after which it is retired.  The failures this
answers are Courant-number failures: the edits build steep terrain with
thin, fast sheets of water whose speed far exceeds the sqrt(g d) the fixed
time step was sized for, and the dispersive terms amplify the velocities
there; neither a smaller step alone nor NLSW alone at the original step
cured them, both together did.  The checkpoint counts towards the
session's footprint.  A time-step change restarts the domain's multistep
history and its step counter, so a session counts its steps from the
checkpoint it was rolled back to (`base`).

Reported: throughput (all steps, and the steps run in the paper's BSNQ model
only), the share of steps run degraded (NLSW after a rollback) and of steps
undone by rollbacks, per-step latency seen by a session (tick wall time over
the steps it made in that tick) at p50/p99, real-time ratio (simulated time
over wall time while resident; sessions still resident at the end count with
their time so far), queueing delay, the largest footprint in use and queue
length, and session counts (done, failed, recovered, rollbacks).
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import wavestep as ws
from . import workloads as wl


@dataclass
class _Live:
    rid: int
    spec: wl.Session
    work: wl.Workload
    dom: object
    slot: int
    arrived: float
    admitted: float
    bytes: int
    step: int = 0
    stop: int = 0
    next_edit: int = 0
    edit_status: list = field(default_factory=list)
    snap: object = None       # device checkpoint (recovery on)
    snap_step: int = 0        # session step, edit index and log length at the checkpoint
    snap_edit: int = 0
    snap_log: int = 0
    recoveries: int = 0
    base: int = 0             # session step at which the domain's step counter restarted
    dt: float = 0.0
    t: float = 0.0            # simulated time (s)


def footprint(spec: wl.Session, recover: bool = False) -> int:
    """Device bytes a session holds while resident (its workspace, and its
    checkpoint when the server recovers failed sessions)."""
    w = _grid_of(spec)
    g = ws.grid(w[0], w[0], w[1], w[1], w[2])
    return ws.workspace_bytes(g) + (ws.snapshot_bytes(g) if recover else 0)


def _grid_of(spec):
    dx = 0.1
    return spec.nx, dx, wl.courant_dt(spec.courant, dx, spec.depth)


def _next_stop(spec, step, k):
    """Next event step: the next edit after `step` (index k), else the end."""
    while k < len(spec.edits) and spec.edits[k][0] <= step:
        k += 1
    stop = spec.edits[k][0] if k < len(spec.edits) else spec.steps
    return min(stop, spec.steps), k


def _apply_due(dom, spec, step, k, log):
    while k < len(spec.edits) and spec.edits[k][0] == step:
        _, kind, x0, y0, amp, sigma = spec.edits[k]
        log.append(dom.apply_edit(kind, x0, y0, amp, sigma))
        k += 1
    return k


def _checkpoint(s, dom, step, k, log):
    """Checkpoint before the edits due at `step` (edit index k); the buffer
    is reused from one pause to the next."""
    s.snap = dom.snapshot(out=s.snap)
    s.snap_step, s.snap_edit, s.snap_log = step, k, len(log)


def _recover(s, dom, log):
    """Roll back to the checkpoint, go on in NLSW with half the time step,
    checkpoint that state (so the checkpoint is always in the domain's
    current model, as a restore requires) and re-apply the edits due at the
    checkpoint's step.  Returns (step, next edit index)."""
    dom.restore(s.snap)
    s.recoveries += 1
    s.dt *= 0.5
    dom.update(model=ws.NLSW, dt=s.dt)    # restarts the multistep history and the step counter
    s.base = s.snap_step
    del log[s.snap_log:]
    _checkpoint(s, dom, s.snap_step, s.snap_edit, log)
    k = _apply_due(dom, s.spec, s.snap_step, s.snap_edit, log)
    return s.snap_step, k


def replay_alone(spec: wl.Session, device="cuda:0", max_recoveries=0):
    """The session run by itself with the single-domain path: same edits at
    the same steps, and with `max_recoveries` > 0 the same rollbacks as the
    server's.  Returns (w, P, Q, edit statuses, health word)."""
    work = wl.session_workload(spec)
    dom = ws.Domain(work.nx, work.ny, work.dx, work.dy, work.dt, work.z, device=device, eps=spec.eps)
    s = _Live(0, spec, work, dom, -1, 0.0, 0.0, 0, dt=work.dt)
    step, k, log = 0, 0, []
    if max_recoveries:
        _checkpoint(s, dom, 0, 0, log)
    while step < spec.steps:
        stop, k = _next_stop(spec, step, k)
        dom.advance(stop - step)
        step = stop
        if max_recoveries and dom.query()[2]:
            if s.recoveries >= max_recoveries:
                break
            step, k = _recover(s, dom, log)
            continue
        if step < spec.steps:
            if max_recoveries:
                _checkpoint(s, dom, step, k, log)
            k = _apply_due(dom, spec, step, k, log)
    out = dom.state_numpy()
    health = dom.query()[2]
    dom.close()
    return out + (log, health)


def _pct(samples, weights, q):
    if not len(samples):
        return None
    order = np.argsort(samples)
    s, w = np.asarray(samples)[order], np.asarray(weights, dtype=np.float64)[order]
    c = np.cumsum(w)
    return float(s[np.searchsorted(c, q / 100.0 * c[-1])])


class Server:
    def __init__(self, budget_bytes=64 << 30, max_sessions=256, tick_steps=10, device="cuda:0",
                 keep_results=False, recover=False, max_recoveries=3):
        self.budget = int(budget_bytes)
        self.max_sessions = int(max_sessions)
        self.tick = int(tick_steps)
        self.device = device
        self.keep = keep_results
        self.recover = bool(recover)
        self.max_recoveries = int(max_recoveries) if recover else 0
        self.recovered = {}                  # rid -> rollbacks made
        self.results = {}
        self.failures = {}                   # rid -> step at which a non-finite state was seen

    def run(self, trace, time_scale=1.0, wall_limit=None, log=None):
        """Serve `trace` (workloads.Session list, arrival times in seconds,
        multiplied by `time_scale`).  Ends when every session finished, or at
        `wall_limit` seconds.  Returns the report dict."""
        import torch
        B = ws.Batch(self.max_sessions, device=self.device)
        pending = deque(sorted(enumerate(trace), key=lambda p: p[1].arrival))
        queue = deque()                      # (rid, spec, arrival wall time)
        live = {}                            # slot -> _Live
        used = 0
        lat, lat_w, waits, rt_ratios = [], [], [], []
        cell_steps = 0
        cell_steps_nlsw = 0                  # steps run degraded (NLSW at a reduced dt) after a rollback
        session_steps = session_steps_nlsw = 0
        cell_steps_discarded = 0             # steps undone by rollbacks
        used_max = queue_max = 0
        done = rejected = admitted = ticks = failed = 0
        t0 = time.perf_counter()
        def arrivals():
            now = time.perf_counter() - t0
            while pending and pending[0][1].arrival * time_scale <= now:
                rid, spec = pending.popleft()
                queue.append((rid, spec, spec.arrival * time_scale))

        def admit():
            nonlocal used, admitted, rejected
            while queue and len(live) < self.max_sessions:
                rid, spec, arr = queue[0]
                need = footprint(spec, self.recover)
                if need > self.budget:       # can never fit
                    queue.popleft()
                    rejected += 1
                    continue
                if used + need > self.budget:
                    break
                queue.popleft()
                work = wl.session_workload(spec)
                dom = ws.Domain(work.nx, work.ny, work.dx, work.dy, work.dt, work.z, device=self.device,
                                eps=spec.eps)
                slot = B.attach(dom)         # joins the batch at its next advance
                t_adm = time.perf_counter() - t0
                s = _Live(rid, spec, work, dom, slot, arr, t_adm, need, dt=work.dt)
                if self.recover:
                    _checkpoint(s, dom, 0, 0, s.edit_status)
                s.stop, s.next_edit = _next_stop(spec, 0, 0)
                B.set_stop(slot, s.stop)
                live[slot] = s
                used += need
                admitted += 1
                waits.append(t_adm - arr)
            nonlocal_max(used, len(queue))

        def nonlocal_max(u, q):
            nonlocal used_max, queue_max
            used_max = max(used_max, u)
            queue_max = max(queue_max, q)

        while True:
            if wall_limit is not None and time.perf_counter() - t0 >= wall_limit:
                break
            arrivals()
            if not live:
                admit()
                if not live:
                    if not pending and not queue:
                        break
                    if pending:
                        now = time.perf_counter() - t0
                        time.sleep(max(0.0, min(0.002, pending[0][1].arrival * time_scale - now)))
                    continue
            t_a = time.perf_counter()
            B.advance(self.tick)
            arrivals()                       # host work overlapping the tick:
            admit()                          # new sessions join at the next tick
            B.sync()
            t_b = time.perf_counter()
            ticks += 1
            T = t_b - t_a
            for slot in list(live):
                s = live[slot]
                step, s.t, health = B.status(slot)
                step += s.base
                k = step - s.step
                if k > 0:
                    lat.append(T / k)
                    lat_w.append(k)
                    cell_steps += k * s.work.cells
                    session_steps += k
                    if s.recoveries:
                        cell_steps_nlsw += k * s.work.cells
                        session_steps_nlsw += k
                s.step = step
                if health and s.recoveries < self.max_recoveries:   # roll back, go on in NLSW at dt/2
                    cell_steps_discarded += (step - s.snap_step) * s.work.cells
                    s.step, s.next_edit = _recover(s, s.dom, s.edit_status)
                    self.recovered[s.rid] = s.recoveries
                    s.stop, s.next_edit = _next_stop(s.spec, s.step, s.next_edit)
                    B.set_stop(slot, s.stop - s.base)
                    continue
                if health or step >= s.spec.steps:   # finished or failed: retire, free its memory
                    if health:                       # non-finite state: the session ends with an error
                        self.failures[s.rid] = step
                        failed += 1
                    else:
                        wall = t_b - t0 - s.admitted
                        rt_ratios.append(s.t / wall)
                        done += 1
                    B.detach(slot)
                    if self.keep:
                        self.results[s.rid] = s.dom.state_numpy() + (s.edit_status,)
                    s.dom.close()
                    del live[slot]
                    used -= s.bytes
                elif step == s.stop:                 # paused at an edit
                    if self.recover:
                        _checkpoint(s, s.dom, step, s.next_edit, s.edit_status)
                    s.next_edit = _apply_due(s.dom, s.spec, step, s.next_edit, s.edit_status)
                    s.stop, s.next_edit = _next_stop(s.spec, step, s.next_edit)
                    B.set_stop(slot, s.stop - s.base)
            if log and ticks % 50 == 0:
                log("serve: t=%.1fs ticks %d resident %d queued %d done %d"
                    % (time.perf_counter() - t0, ticks, len(live), len(queue), done))
        wall = time.perf_counter() - t0
        for s in live.values():                      # still resident: ratio so far
            if s.step > 0:
                rt_ratios.append(s.t / max(1e-9, wall - s.admitted))
        torch.cuda.synchronize()
        B.close()
        for s in live.values():
            s.dom.close()
        return {
            "wall_s": wall, "ticks": ticks, "tick_steps": self.tick,
            "sessions_arrived": admitted + len(queue) + rejected,
            "sessions_admitted": admitted, "sessions_done": done, "sessions_rejected": rejected,
            "sessions_failed": failed, "sessions_recovered": len(self.recovered),
            "rollbacks": sum(self.recovered.values()),
            "sessions_resident_at_end": len(live), "sessions_queued_at_end": len(queue),
            "budget_bytes": self.budget,
            "budget_used_max_bytes": used_max, "sessions_queued_max": queue_max,
            "throughput_cell_updates_per_s": cell_steps / wall if wall > 0 else 0.0,
            "throughput_bsnq_cell_updates_per_s": (cell_steps - cell_steps_nlsw) / wall if wall > 0 else 0.0,
            "degraded_share_of_session_steps": session_steps_nlsw / session_steps if session_steps else 0.0,
            "degraded_share_of_cell_steps": cell_steps_nlsw / cell_steps if cell_steps else 0.0,
            "discarded_share_of_cell_steps": cell_steps_discarded / cell_steps if cell_steps else 0.0,
            "step_latency_ms_p50": None if not lat else 1e3 * _pct(lat, lat_w, 50),
            "step_latency_ms_p99": None if not lat else 1e3 * _pct(lat, lat_w, 99),
            "queue_wait_s_p50": None if not waits else float(np.percentile(waits, 50)),
            "queue_wait_s_p99": None if not waits else float(np.percentile(waits, 99)),
            "real_time_ratio_p50": None if not rt_ratios else float(np.percentile(rt_ratios, 50)),
            "real_time_ratio_min": None if not rt_ratios else float(np.min(rt_ratios)),
        }
