"""Batched stepping (many independent domains, one launch per phase for all
of them, the step replayed as a HIP graph) through the C ABI.

The batched kernels run the same per-cell arithmetic as the single-domain
kernels, so a domain advanced in a batch must equal, bit for bit, the same
domain advanced alone (which the single-domain parity tests tie to the FP64
oracle); a few batched domains are also compared with the oracle directly.
"""
import math
import sys

import numpy as np
import pytest

import oracle as o
from paper_1611_05984_amd import workloads as wl

pytestmark = pytest.mark.gpu
G = 9.81


def _ws():
    from paper_1611_05984_amd import wavestep as ws
    return ws


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def make(w, **params):
    ws = _ws()
    z = w.z.astype(np.float32).astype(np.float64)
    d = ws.Domain(w.nx, w.ny, w.dx, w.dy, w.dt, z, **params)
    for s, side in enumerate(w.sides):
        if side.kind != wl.SOLID:
            d.set_boundary(s, side.kind, side.width, side.amp, side.period, side.theta,
                           side.phase or None)
    for (H, th, x0, y0) in w.solitary:
        d.add_solitary(H, th, x0, y0)
    return d


def mixed_cases():
    """Uneven ensemble members plus domains with wave makers, sponges and other
    corrector counts / models, so one batch mixes every pass count."""
    cases = [(w, {}) for w in wl.config4(n_domains=5, lo=64, hi=200, seed=41)]
    c2 = wl.config2(nx=200, ny=72, seed=7)
    cases.append((c2, {}))
    cases.append((c2, {"n_corr": 1}))
    cases.append((wl.config1(nx=130, ny=40), {"n_corr": 3}))
    cases.append((wl.config1(nx=96, ny=66), {"model": 1}))
    cases.append((wl.config1(nx=70, ny=70), {"n_corr": 0}))
    return cases


def same(a, b, what):
    ae, aP, aQ = a.state_numpy()
    be, bP, bQ = b.state_numpy()
    for x, y, f in ((ae, be, "w"), (aP, bP, "P"), (aQ, bQ, "Q")):
        if not np.array_equal(x, y):
            k = np.unravel_index(np.argmax(np.abs(x - y)), x.shape)
            raise AssertionError("%s %s differs: max |d| = %.3e at %s" % (what, f, np.abs(x - y).max(), k))
    sa, sb = a.query(), b.query()
    assert sa[0] == sb[0] and sa[1] == sb[1] and sa[2] == 0 and sb[2] == 0, (what, sa, sb)


def test_batch_equals_single_domains_bitwise():
    ws = _ws()
    cases = mixed_cases()
    say("case: batch of %d mixed domains vs the same domains alone" % len(cases))
    alone = [make(w, **p) for w, p in cases]
    inb = [make(w, **p) for w, p in cases]
    for k, (a, b) in enumerate(zip(alone, inb)):   # mixed step indices, Euler start-ups in the batch
        a.advance(k % 4)
        b.advance(k % 4)
    B = ws.Batch(16)
    for b in inb:
        B.attach(b)
    done = 0
    for chunk in (1, 1, 3, 7, 20):
        B.advance(chunk)
        for a in alone:
            a.advance(chunk)
        done += chunk
        B.sync()
        say("  after %d batched steps" % done)
        for k, (a, b) in enumerate(zip(alone, inb)):
            same(a, b, "domain %d (%s)" % (k, cases[k][0].name))
    B.close()


def test_batch_edits_attach_detach_and_busy():
    ws = _ws()
    cases = [(w, {}) for w in wl.config4(n_domains=4, lo=80, hi=160, seed=42)]
    say("case: batch edits / detach / attach, %d domains" % len(cases))
    alone = [make(w, **p) for w, p in cases]
    inb = [make(w, **p) for w, p in cases]
    B = ws.Batch(4)
    slots = [B.attach(b) for b in inb[:3]]
    B.advance(10)
    for a in alone[:3]:
        a.advance(10)
    with pytest.raises(ws.WaveStepError) as e:       # stale until synced
        inb[0].read()
    assert e.value.status == ws.EBUSY
    B.sync()
    with pytest.raises(ws.WaveStepError) as e:       # attached: advanced only by the batch
        inb[0].advance(1)
    assert e.value.status == ws.EBUSY
    w0, w1 = cases[0][0], cases[1][0]
    for d in (alone[0], inb[0]):
        assert d.apply_edit(ws.EDIT_WATER, 0.4 * w0.nx * w0.dx, 0.5 * w0.ny * w0.dy, 0.2, 4 * w0.dx) == 0
    for d in (alone[1], inb[1]):
        assert d.apply_edit(ws.EDIT_TERRAIN, 0.85 * w1.nx * w1.dx, 0.3 * w1.ny * w1.dy, 0.3,
                            6 * w1.dx) == 0
    B.advance(5)
    for a in alone[:3]:
        a.advance(5)
    B.sync()
    B.detach(slots[2])
    inb[2].advance(4)                               # usable alone again
    alone[2].advance(4)
    alone[3].advance(2)
    inb[3].advance(2)
    B.attach(inb[3])
    for step in range(3):                           # repeated graph replays with eager work between
        B.advance(4)
        for k in (0, 1, 3):
            alone[k].advance(4)
        B.sync()
        for k in (0, 1, 3):
            same(alone[k], inb[k], "domain %d replay %d" % (k, step))
    same(alone[2], inb[2], "detached domain")
    # runtime parameter changes of attached domains: friction on one, a new
    # time step (history restart) on another; the batch follows them
    for d in (alone[0], inb[0]):
        d.update(friction=1, friction_coef=0.02)
    for d in (alone[1], inb[1]):
        d.update(dt=0.75 * cases[1][0].dt)
    B.advance(6)
    for k in (0, 1, 3):
        alone[k].advance(6)
    B.sync()
    for k in (0, 1, 3):
        same(alone[k], inb[k], "domain %d after parameter changes" % k)
    assert inb[1].query()[0] == 6
    B.close()


def test_batch_vs_oracle():
    ws = _ws()
    cases = wl.config4(n_domains=3, lo=96, hi=144, seed=43)
    say("case: batched config-4 members vs oracle, 60 steps")
    gpus = [make(w) for w in cases]
    oras = []
    for w in cases:
        z = w.z.astype(np.float32).astype(np.float64)
        d = o.Domain(w.nx, w.ny, w.dx, w.dy, w.dt, z)
        for (H, th, x0, y0) in w.solitary:
            d.add_solitary(H, th, x0, y0)
        oras.append(d)
    B = ws.Batch(3)
    for g in gpus:
        B.attach(g)
    B.advance(60)
    for d in oras:
        d.advance(60)
    B.sync()
    for w, g, d in zip(cases, gpus, oras):
        H = w.solitary[0][0]
        ge, gP, gQ = g.state_numpy()
        oe, oP, oQ = d.state()
        de, dP, dQ = np.abs(ge - oe).max(), np.abs(gP - oP).max(), np.abs(gQ - oQ).max()
        say("  %s: max|d eta| %.3e  |dP| %.3e  |dQ| %.3e (H %.3f)" % (w.name, de, dP, dQ, H))
        assert de <= 1e-4 * H and max(dP, dQ) <= 1e-4 * H * math.sqrt(G * 1.0), w.name
        assert g.query()[0] == d.step
    B.close()


def test_config4_full_size_batch_sampled_vs_alone():
    """The full 256-domain ensemble (nx, ny ~ U{256..1024}) as the benchmark
    runs it: every domain stays finite, and the smallest, the largest and a
    beach domain equal their single-domain runs bit for bit."""
    ws = _ws()
    ens = wl.config4()
    say("case: config4 full size, %d domains, %.3g cells" % (len(ens), sum(w.cells for w in ens)))
    doms = [make(w) for w in ens]
    cells = [w.cells for w in ens]
    pick = sorted({int(np.argmin(cells)), int(np.argmax(cells)),
                   next(k for k, w in enumerate(ens) if w.z.max() > -0.99)})
    alone = {k: make(ens[k]) for k in pick}
    B = ws.Batch(len(ens))
    for d in doms:
        B.attach(d)
    B.advance(12)
    for k in pick:
        alone[k].advance(12)
    B.sync()
    for k in pick:
        same(alone[k], doms[k], "ensemble domain %d (%s)" % (k, ens[k].name))
    bad = [k for k, d in enumerate(doms) if d.query()[2] != 0]
    assert not bad, bad
    B.close()


def test_snapshot_restore_continues_exactly():
    """A snapshot (state, history, edited bathymetry, step, time) restored
    into a fresh domain of the same grid continues bit for bit as the
    original run; a snapshot of another grid is refused; the snapshot's
    size equals the one ws_snapshot_bytes_grid gives for the grid."""
    ws = _ws()
    w = wl.config2(nx=160, ny=72, seed=9)
    say("case: snapshot / restore on %s" % w.name)
    a = make(w)
    a.advance(25)
    assert a.apply_edit(ws.EDIT_TERRAIN, 0.6 * w.nx * w.dx, 0.5 * w.ny * w.dy, 0.2, 5 * w.dx) == 0
    a.advance(5)
    snap = a.snapshot()
    assert snap.numel() == ws.snapshot_bytes(a.g)   # the size a caller can budget before the domain exists
    a.advance(20)
    b = make(w)                                    # same grid and boundaries, fresh state
    b.advance(3)
    b.restore(snap)
    assert b.query()[0] == 30
    b.advance(20)
    same(a, b, "restored run")
    a.restore(snap)                                # rewind the original in place
    a.advance(20)
    same(a, b, "rewound run")
    other = make(wl.config1(nx=64, ny=32))
    with pytest.raises(ws.WaveStepError) as e:
        other.restore(snap)
    assert e.value.status == ws.EINVAL


def test_tunings_identical_results_and_autotuner(tmp_path):
    """Every launch-shape choice gives the same bits; the autotuner leaves
    the state untouched, picks a valid shape and reuses its cache."""
    ws = _ws()
    w = wl.config2(nx=300, ny=150, seed=11)
    say("case: tunings on %s" % w.name)
    ref = make(w)
    ref.advance(30)
    for sy, pn, syc in [(8, 64, 0), (16, 128, 0), (24, 256, 8), (48, 64, 0), (64, 128, 16), (32, 256, 64)]:
        d = make(w)
        d.set_tuning(sy, pn, ws.SOLVE_PCR, syc)
        assert d.tuning() == (sy, pn, ws.SOLVE_PCR, syc)
        d.advance(30)
        same(ref, d, "tuning %s" % ((sy, pn, syc),))
    # the lane-per-system Thomas solve of the reduced systems rounds
    # differently from PCR: equal within the parity tolerance of the solve
    th = make(w)
    th.set_tuning(16, 128, ws.SOLVE_THOMAS)
    th.advance(30)
    for x, y in zip(ref.state_numpy(), th.state_numpy()):
        assert np.abs(x - y).max() <= 1e-6 * max(1.0, np.abs(x).max())
    # the factored solve repeats the Thomas arithmetic with stored factors:
    # the same bits, also across a terrain edit and a boundary change (both
    # refactor) and a restore
    lu = make(w)
    lu.set_tuning(8, 128, ws.SOLVE_LU)
    lu.advance(30)
    same(th, lu, "factored solve vs Thomas")
    snap = lu.snapshot()
    for dd in (th, lu):
        assert dd.apply_edit(ws.EDIT_TERRAIN, 0.7 * w.nx * w.dx, 0.6 * w.ny * w.dy, 0.15, 6 * w.dx) == 0
        dd.set_boundary(ws.EAST, ws.SPONGE, 12)
        dd.advance(15)
    same(th, lu, "factored solve after edit and boundary change")
    for dd in (th, lu):
        dd.restore(snap)
        dd.advance(5)
    same(th, lu, "factored solve after restore")
    d = make(w)
    d.advance(30)
    before = d.state_numpy()
    cache = str(tmp_path / "tune.txt")
    t = d.tune(cache)
    assert t[0] in (8, 16, 24, 32, 48, 64) and t[1] in (64, 128, 256) and t[2] in (0, 1, 2, 3, 4)
    assert t[3] in (0, 8, 16, 24, 32, 48, 64) and t[3] != t[0]
    assert d.tuning() == t
    after = d.state_numpy()
    assert all(np.array_equal(x, y) for x, y in zip(before, after)) and d.query()[0] == 30
    line = open(cache).read().split()
    assert [int(v) for v in line] == [w.nx, w.ny, 2, 0, t[0], t[1], t[2], t[3]]
    d2 = make(w)
    assert d2.tune(cache) == t                     # read from the cache
    old = str(tmp_path / "old.txt")                # a line without corrector rows
    open(old, "w").write("%d %d 2 0 16 64 1\n" % (w.nx, w.ny))
    assert make(w).tune(old) == (16, 64, ws.SOLVE_THOMAS, 0)
    d.set_tuning(t[0], t[1], ws.SOLVE_PCR, t[3])  # bitwise comparable with the reference
    d.advance(10)
    ref.advance(10)
    same(ref, d, "after tuning")
    with pytest.raises(ws.WaveStepError):
        d.set_tuning(40, 128)
    with pytest.raises(ws.WaveStepError):
        d.set_tuning(8, 128, ws.SOLVE_PCR, 12)
    B = ws.Batch(4)
    b = make(w)
    B.set_tuning(24, 64)
    B.attach(b)
    B.advance(20)
    tb = B.tune()                                  # leaves the states alone
    assert tb[0] in (8, 16, 24, 32, 48, 64) and tb[1] in (64, 128, 256) and tb[2] in (0, 1, 2, 3, 4)
    assert tb[3] in (0, 8, 16, 24, 32, 48, 64)
    B.set_tuning(tb[0], tb[1], ws.SOLVE_PCR, tb[3])
    B.advance(20)
    B.sync()
    same(ref, b, "batch tuned 24/64, then autotuned %s" % (tb,))
    th2 = make(w)                                  # batched Thomas equals single-domain Thomas
    th2b = make(w)
    th2.set_tuning(16, 128, ws.SOLVE_THOMAS)
    B.detach(0)
    B.set_tuning(16, 128, ws.SOLVE_THOMAS)
    B.attach(th2b)
    B.advance(30)
    th2.advance(30)
    B.sync()
    same(th2, th2b, "batched Thomas")
    lu2 = make(w)                                  # batched factored solve equals single-domain
    lu2b = make(w)
    lu2.set_tuning(16, 128, ws.SOLVE_LU)
    B.set_tuning(16, 128, ws.SOLVE_LU)
    B.attach(lu2b)
    B.advance(25)
    lu2.advance(25)
    B.sync()
    same(lu2, lu2b, "batched factored solve")
    # two-ended factored solve: rounds differently from the one-ended sweep;
    # batched equals single-domain bit for bit
    tw = make(w)
    twb = make(w)
    tw.set_tuning(16, 128, ws.SOLVE_LU2)
    B.set_tuning(16, 128, ws.SOLVE_LU2)
    B.attach(twb)
    B.advance(25)
    tw.advance(25)
    B.sync()
    same(tw, twb, "batched two-ended factored solve")
    for x, y in zip(lu2.state_numpy(), tw.state_numpy()):
        assert np.abs(x - y).max() <= 1e-6 * max(1.0, np.abs(x).max())
    B.close()


@pytest.mark.parametrize("nx,ny", [(300, 150), (90, 40), (1000, 100), (1030, 520), (2050, 300), (4096, 64)])
def test_wave_pcr_equals_lds_pcr(nx, ny):
    """PCR on one wave per system (lane shuffles, no LDS array, no barrier)
    gives the bits of the workgroup PCR: reduced systems of 2 x 19 .. 512
    unknowns (every equations-per-lane variant, ragged against the wave),
    over Euler, predictor and corrector passes, alone and in a batch.
    Longer systems are refused for a single domain."""
    ws = _ws()
    w = wl.config2(nx=nx, ny=ny, seed=13)
    say("case: wave PCR vs workgroup PCR on %s" % w.name)
    a, b = make(w), make(w)
    a.set_tuning(16, 128, ws.SOLVE_PCR)
    b.set_tuning(16, 128, ws.SOLVE_PCR_WAVE)
    assert b.tuning()[2] == ws.SOLVE_PCR_WAVE
    for n in (2, 1, 9):
        a.advance(n)
        b.advance(n)
        same(a, b, "wave PCR after %d steps" % a.query()[0])
    big = make(wl.config1(nx=4100, ny=16))          # row systems of 2 x 257 unknowns
    with pytest.raises(ws.WaveStepError) as e:
        big.set_tuning(16, 128, ws.SOLVE_PCR_WAVE)
    assert e.value.status == ws.EINVAL
    c = make(w)                                     # the same domain in a batch with a small one
    small = make(wl.config1(nx=70, ny=40))
    B = ws.Batch(2)
    B.set_tuning(16, 128, ws.SOLVE_PCR_WAVE)
    B.attach(c)
    B.attach(small)
    B.advance(12)
    B.sync()
    B.close()
    same(a, c, "wave PCR in a batch")


def test_factored_solve_workgroup_form_and_long_systems():
    """The factored solve runs systems of up to 512 unknowns as one
    workgroup per 64 systems (a wave per 32 unknowns, the chain handed from
    wave to wave), longer ones lane per system.  Every shape must give the
    Thomas solve's bits: row- and column-dominated domains on both paths,
    alone and batched (a batch takes the workgroup form only when all its
    systems fit)."""
    ws = _ws()
    shapes = [(1100, 24), (24, 1100), (4096, 20), (20, 4096), (5000, 20), (20, 16384)]
    lus = []
    for nx, ny in shapes:
        w = wl.config2(nx=nx, ny=ny, seed=5)
        say("case: factored vs Thomas %dx%d" % (nx, ny))
        th, lu = make(w), make(w)
        th.set_tuning(16, 128, ws.SOLVE_THOMAS)
        lu.set_tuning(16, 128, ws.SOLVE_LU)
        th.advance(12)
        lu.advance(12)
        same(th, lu, "factored vs Thomas %dx%d" % (nx, ny))
        th.close()
        lus.append((w, lu))
    small = wl.config2(nx=300, ny=150, seed=11)
    for members in ((0, 1, 3), (0, 4, 5)):
        say("case: batched factored solve over %s + 300x150" % ([shapes[m] for m in members],))
        B = ws.Batch(4)
        B.set_tuning(16, 128, ws.SOLVE_LU)
        pairs = []
        for m in members:
            w, lu = lus[m]
            b = make(w)
            B.attach(b)
            pairs.append((lu, b))
        alone = make(small)
        alone.set_tuning(16, 128, ws.SOLVE_LU)
        sb = make(small)
        B.attach(sb)
        pairs.append((alone, sb))
        B.advance(12)
        alone.advance(12)
        B.sync()
        for a_, b_ in pairs:
            same(a_, b_, "batched factored solve, mixed lengths")
        B.close()
        for _, b_ in pairs:
            b_.close()
        alone.close()
