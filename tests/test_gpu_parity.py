"""GPU (FP32, HIP on gfx950) vs FP64 oracle, element by element, through the
C ABI.

Tolerance (stated with the method): after a run, max |d eta| <= 1e-4 a0 and
max |dP|, |dQ| <= 1e-4 a0 sqrt(g d), with a0 the wave amplitude scale of the
case and d its depth scale; short runs use tighter bounds.  Inputs are the
same seeded arrays on both sides (bathymetry rounded to float32 first).
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


def build_pair(w: wl.Workload, **params):
    ws = _ws()
    z = w.z.astype(np.float32).astype(np.float64)
    gpu = ws.Domain(w.nx, w.ny, w.dx, w.dy, w.dt, z, **params)
    oparams = {k: v for k, v in params.items()}
    if "friction_coef" in oparams:
        oparams["fcoef"] = oparams.pop("friction_coef")
    ora = o.Domain(w.nx, w.ny, w.dx, w.dy, w.dt, z, **oparams)
    for s, side in enumerate(w.sides):
        if side.kind == wl.SOLID:
            continue
        ph = side.phase if side.phase else None
        gpu.set_boundary(s, side.kind, side.width, side.amp, side.period, side.theta, ph)
        ora.set_boundary(s, side.kind, side.width, side.amp, side.period, side.theta, ph)
    for (H, th, x0, y0) in w.solitary:
        gpu.add_solitary(H, th, x0, y0)
        ora.add_solitary(H, th, x0, y0)
    return gpu, ora


def compare(gpu, ora, a0, depth, what=""):
    ge, gP, gQ = gpu.state_numpy()
    oe, oP, oQ = ora.state()
    de, dP, dQ = (np.abs(ge - oe).max(), np.abs(gP - oP).max(), np.abs(gQ - oQ).max())
    say("  %s: max|d eta| = %.3e (a0 %.3g)  max|dP| = %.3e  max|dQ| = %.3e"
        % (what, de, a0, dP, dQ))
    return de, dP, dQ


def check(gpu, ora, a0, depth, rel=1e-4, what=""):
    de, dP, dQ = compare(gpu, ora, a0, depth, what)
    c = math.sqrt(G * depth)
    assert de <= rel * a0, (what, de)
    assert dP <= rel * a0 * c and dQ <= rel * a0 * c, (what, dP, dQ)
    step, t, health = gpu.query()
    assert health == 0 and step == ora.step and abs(t - ora.t) < 1e-12


# ------------------------------------------------------------------ config 1
def test_config1_500_steps_parity_and_invariants():
    """Config 1 as specified: 128x64, flat 1 m, solitary H = 0.1 m, walls,
    Courant 0.2, 500 steps."""
    say("case: config1 128x64, 500 steps")
    w = wl.config1()
    gpu, ora = build_pair(w)
    for n in (1, 2, 3, 500 - 6):
        gpu.advance(n)
        ora.advance(n)
        check(gpu, ora, 0.1, 1.0, rel=1e-4, what="step %d" % ora.step)
    ge, gP, gQ = gpu.state_numpy()
    assert np.all(gQ == 0.0)                       # y-invariance exact in FP32 too
    assert np.all(ge == ge[0:1]) and np.all(gP == gP[0:1])
    gh = gpu.state_numpy(_ws().READ_H)[0].astype(np.float64)
    oe, _, _ = ora.state()
    b, _ = ora.bathy()
    vol_o = np.sum(oe - b)
    assert abs(gh.sum() - vol_o) <= 1e-6 * vol_o   # volume to FP32 round-off


# --------------------------------------------- all boundary types, ragged tiles
def _mixed_case(nx, ny, seed=21, dx=0.05):
    rng = np.random.default_rng(seed)
    X = np.arange(nx + 1)[None, :] * dx
    Lx = nx * dx
    z = np.maximum(-0.5, (X - 0.8 * Lx) / 10.0) * np.ones((ny + 1, 1))
    z = wl.gaussian_bumps(z, dx, dx, rng, n=10, amp=(-0.05, 0.05), sigma=(0.1, 0.4))
    sides = wl.walls()
    sides[wl.WEST] = wl.Side(wl.WAVES, 2, [0.02, 0.01], [1.5, 0.9], [0.3, -0.2], [0.0, 1.0])
    sides[wl.SOUTH] = wl.Side(wl.SPONGE, 8)
    w = wl.Workload("mixed_%dx%d" % (nx, ny), nx, ny, dx, dx, wl.courant_dt(0.2, dx, 0.55), z,
                    sides, solitary=[(0.03, 0.6, 0.3 * Lx, 0.5 * ny * dx)])
    return w


@pytest.mark.parametrize("nx,ny", [(150, 70), (64, 16), (130, 33)])
def test_mixed_boundaries_ragged_tiles(nx, ny):
    """Wave maker (2 components, oblique), sponge, walls, beach with a moving
    shoreline, bumps, an oblique solitary wave; grids that are not whole tiles
    (64 x 16) and a single-tile grid."""
    say("case: mixed boundaries %dx%d" % (nx, ny))
    w = _mixed_case(nx, ny)
    gpu, ora = build_pair(w)
    gpu.advance(1)
    ora.advance(1)
    check(gpu, ora, 0.03, 0.5, rel=2e-6, what="Euler step 1")
    gpu.advance(2)
    ora.advance(2)
    check(gpu, ora, 0.03, 0.5, rel=1e-5, what="step 3 (AB3 + 2 AM4)")
    gpu.advance(197)
    ora.advance(197)
    check(gpu, ora, 0.03, 0.5, rel=1e-4, what="step 200")
    ge, _, _ = gpu.state_numpy()
    b, _ = ora.bathy()
    assert np.all(ge >= b.astype(np.float32) - 1e-6)


def test_partially_reflective_sponge_parity():
    """Partially reflective sponges (target reflection 0.5 north, 0.2
    south, beside the oblique wave maker and the beach of the mixed case)
    match the oracle; R = 1 leaves the GPU state equal to a solid wall's, bit
    for bit."""
    ws = _ws()
    w = _mixed_case(150, 70)
    gpu, ora = build_pair(w)
    for d in (gpu, ora):
        d.set_boundary(wl.NORTH, wl.SPONGE, 12, sponge_reflect=0.5)
        d.set_boundary(wl.SOUTH, wl.SPONGE, 8, sponge_reflect=0.2)
    say("case: partially reflective sponges 150x70")
    gpu.advance(200)
    ora.advance(200)
    check(gpu, ora, 0.03, 0.5, rel=1e-4, what="step 200")
    w2 = _mixed_case(96, 40, seed=5)
    a, _ = build_pair(w2)
    b, _ = build_pair(w2)
    a.set_boundary(wl.SOUTH, wl.SPONGE, 8, sponge_reflect=1.0)
    b.set_boundary(wl.SOUTH, wl.SOLID)
    a.advance(60)
    b.advance(60)
    for x, y in zip(a.state_numpy(), b.state_numpy()):
        assert np.array_equal(x, y)
    with pytest.raises(ws.WaveStepError):
        a.set_boundary(wl.EAST, wl.SPONGE, 8, sponge_reflect=-0.1)


def test_corrector_tolerance_mode():
    """Corrector iteration until convergence on the GPU: a tolerance no
    change exceeds stops after one corrector and one no change meets runs the
    cap, equal bit for bit to the fixed-count runs (sponge and wave maker
    included); in between, the per-step counts vary, every step that stopped
    early reports changes within the tolerance, and the oracle stepped with
    the same counts matches the state.  Batches refuse the mode."""
    ws = _ws()
    w = _mixed_case(96, 40, seed=5)
    say("case: corrector tolerance mode 96x40")
    fixed1, _ = build_pair(w, n_corr=1)
    loose, _ = build_pair(w, n_corr=4)
    loose.set_corrector_tolerance(1e9, 1e9)
    fixed3, _ = build_pair(w, n_corr=3)
    tight, _ = build_pair(w, n_corr=3)
    tight.set_corrector_tolerance(1e-30, 1e-30)
    for d in (fixed1, loose, fixed3, tight):
        d.advance(40)
    for a, b in ((fixed1, loose), (fixed3, tight)):
        for x, y in zip(a.state_numpy(), b.state_numpy()):
            assert np.array_equal(x, y)
    assert loose.corrector_stats()[:2] == (1, 38) and tight.corrector_stats()[:2] == (3, 114)
    tol_w, tol_pq = 2e-5, 3e-4
    gpu, ora = build_pair(w, n_corr=4)
    gpu.set_corrector_tolerance(tol_w, tol_pq)
    counts = []
    for n in range(80):
        gpu.advance(1)
        last, _, dw, dpq = gpu.corrector_stats()
        counts.append(last)
        if 0 < last < 4:
            assert dw <= tol_w and dpq <= tol_pq, (n, last, dw, dpq)
        ora.set_n_corr(max(last, 0))
        ora.advance(1)
    say("  counts %s" % counts)
    assert counts[:2] == [0, 0] and len(set(counts[2:])) > 1, counts
    check(gpu, ora, 0.03, 0.5, rel=1e-4, what="tolerance mode, step 80")
    B = ws.Batch(2)
    with pytest.raises(ws.WaveStepError):
        B.attach(gpu)
    gpu.set_corrector_tolerance(0.0, 0.0)
    B.attach(gpu)
    with pytest.raises(ws.WaveStepError):
        gpu.set_corrector_tolerance(1e-5, 1e-5)
    B.close()


def test_parameter_changes_while_running_parity():
    """Runtime parameter changes on the GPU follow the oracle: quadratic
    friction and a new theta, then a smaller time step (restarting the
    multistep history), then the NLSW model, with the partially reflective
    sponge rescaled to the new step.  A dispersive model the bed cannot carry
    is refused with WS_ENOTDD and the domain runs on unchanged."""
    ws = _ws()
    w = _mixed_case(96, 40, seed=5)
    gpu, ora = build_pair(w)
    for d in (gpu, ora):
        d.set_boundary(wl.NORTH, wl.SPONGE, 10, sponge_reflect=0.4)
    say("case: runtime parameter changes 96x40")
    gpu.advance(30)
    ora.advance(30)
    gpu.update(friction=1, friction_coef=0.01, theta=1.5)
    ora.update(friction=1, fcoef=0.01, theta=1.5)
    gpu.advance(30)
    ora.advance(30)
    check(gpu, ora, 0.03, 0.5, rel=1e-4, what="friction, theta")
    gpu.update(dt=0.7 * w.dt)
    ora.update(dt=0.7 * w.dt)
    assert gpu.query()[0] == 0
    gpu.advance(40)
    ora.advance(40)
    check(gpu, ora, 0.03, 0.5, rel=1e-4, what="new dt")
    gpu.update(model=ws.NLSW)
    ora.update(model=o.NLSW)
    gpu.advance(30)
    ora.advance(30)
    check(gpu, ora, 0.03, 0.5, rel=1e-4, what="NLSW")
    with pytest.raises(ws.WaveStepError):
        gpu.update(nx=97)
    nx, ny, dx = 60, 8, 0.05
    zc = np.full(nx + 1, 0.2)
    zc[:40], zc[40], zc[41] = -1.1, -0.1, -0.01
    z = zc[None, :] * np.ones((ny + 1, 1))
    d = ws.Domain(nx, ny, dx, dx, 0.002, z, model=ws.NLSW)
    d.advance(3)
    before = d.state_numpy()
    with pytest.raises(ws.WaveStepError) as err:
        d.update(model=ws.BSNQ)
    assert err.value.status == ws.ENOTDD
    assert all(np.array_equal(x, y) for x, y in zip(before, d.state_numpy()))
    d.advance(3)
    assert d.query()[0] == 6


def _tiny_case(nx, ny):
    dx = 0.1
    X = np.arange(nx + 1)[None, :] * dx
    z = (-0.5 + 0.05 * np.sin(X)) * np.ones((ny + 1, 1))
    sides = wl.walls()
    sides[wl.WEST] = wl.Side(wl.WAVES, 2, [0.01], [1.0], [0.2], [0.0])
    sides[wl.EAST] = wl.Side(wl.SPONGE, max(1, nx // 2))
    return wl.Workload("tiny_%dx%d" % (nx, ny), nx, ny, dx, dx, wl.courant_dt(0.2, dx, 0.55), z, sides)


@pytest.mark.parametrize("nx,ny", [(2, 2), (3, 2), (2, 7), (17, 5)])
def test_tiny_grids(nx, ny):
    """The smallest grids (one partial strip, one partial tile, reduced
    systems of a few unknowns, a wave maker and a sponge wider than half the
    domain): parity with the oracle after a water edit and 40 steps."""
    say("case: tiny grid %dx%d" % (nx, ny))
    w = _tiny_case(nx, ny)
    gpu, ora = build_pair(w)
    for d in (gpu, ora):
        assert d.apply_edit(_ws().EDIT_WATER, 0.5 * nx * w.dx, 0.5 * ny * w.dy, 0.02, 0.1) == 0
    gpu.advance(40)
    ora.advance(40)
    check(gpu, ora, 0.02, 0.5, rel=1e-4, what="tiny %dx%d" % (nx, ny))


def test_degenerate_calls():
    """Zero steps change nothing; an empty batch advances and syncs; a grid
    whose reduced systems would exceed the library's limit, a bad side and a
    bad edit kind are refused with WS_EINVAL."""
    ws = _ws()
    w = _tiny_case(17, 5)
    gpu, _ = build_pair(w)
    gpu.advance(3)
    before = gpu.state_numpy()
    gpu.advance(0)
    assert gpu.query()[0] == 3 and all(np.array_equal(x, y) for x, y in zip(before, gpu.state_numpy()))
    B = ws.Batch(2)
    B.advance(5)
    B.sync()
    B.close()
    with pytest.raises(ws.WaveStepError) as e:
        ws.Domain(16400, 2, 0.1, 0.1, 0.01, -np.ones((3, 16401)))
    assert e.value.status == ws.EINVAL
    with pytest.raises(ws.WaveStepError) as e:
        gpu.set_boundary(5, ws.SPONGE, 4)
    assert e.value.status == ws.EINVAL
    with pytest.raises(ws.WaveStepError) as e:
        gpu.apply_edit(7, 0.5, 0.2, 0.01, 0.1)
    assert e.value.status == ws.EINVAL
    assert gpu.query()[0] == 3


@pytest.mark.parametrize("params", [dict(model=1), dict(friction=1, friction_coef=0.01),
                                    dict(friction=2, friction_coef=0.02),
                                    dict(n_corr=1), dict(n_corr=3, fstar_extrap=2),
                                    dict(fstar_extrap=0), dict(theta=1.0)])
def test_model_variants(params):
    say("case: variant %s" % params)
    w = _mixed_case(96, 40, seed=5)
    gpu, ora = build_pair(w, **params)
    gpu.advance(120)
    ora.advance(120)
    check(gpu, ora, 0.03, 0.5, rel=1e-4, what=str(params))


# ----------------------------------------------------------- exact properties
def test_lake_at_rest_is_bitwise_zero_on_gpu():
    """Pre-balanced fluxes: a lake at rest on a non-flat, fully wet bottom
    (bumps, a corner step) stays exactly at rest in FP32."""
    say("case: lake at rest 200x90")
    ws = _ws()
    nx, ny, dx = 200, 90, 0.1
    rng = np.random.default_rng(1)
    z = wl.gaussian_bumps(-1.0 * np.ones((ny + 1, nx + 1)), dx, dx, rng, n=12,
                          amp=(-0.4, 0.4), sigma=(0.2, 0.8))
    z[40:, 70:] += 0.5
    D = ws.Domain(nx, ny, dx, dx, wl.courant_dt(0.2, dx, 1.5), z)
    D.advance(300)
    e, P, Q = D.state_numpy()
    assert np.all(e == 0.0) and np.all(P == 0.0) and np.all(Q == 0.0)


def test_edits_and_state_round_trip():
    say("case: edits 100x60")
    ws = _ws()
    w = _mixed_case(100, 60, seed=8)
    gpu, ora = build_pair(w)
    gpu.advance(20)
    ora.advance(20)
    for (kind, x0, y0, a, s) in [(ws.EDIT_WATER, 1.5, 1.2, 0.05, 0.3),
                                 (ws.EDIT_TERRAIN, 3.9, 1.0, 0.3, 0.4),
                                 (ws.EDIT_TERRAIN, 2.0, 2.0, -0.2, 0.3)]:
        assert gpu.apply_edit(kind, x0, y0, a, s) == 0
        assert ora.apply_edit(kind, x0, y0, a, s) == 0
    gpu.advance(30)
    ora.advance(30)
    check(gpu, ora, 0.05, 0.5, rel=1e-4, what="after edits")
    # hot start from the oracle's state restarts both histories identically
    oe, oP, oQ = ora.state()
    gpu.set_state(oe.astype(np.float32), oP.astype(np.float32), oQ.astype(np.float32), t=ora.t)
    ora.set_state(oe.astype(np.float32).astype(np.float64), oP.astype(np.float32).astype(np.float64),
                  oQ.astype(np.float32).astype(np.float64), t=ora.t)
    gpu.advance(10)
    ora.advance(10)
    check(gpu, ora, 0.05, 0.5, rel=1e-4, what="after hot start")
    # depth read-back: h = w - cell bottom
    gh, _, _ = gpu.state_numpy(ws.READ_H)
    ge, _, _ = gpu.state_numpy(ws.READ_W)
    b, _ = ora.bathy()
    assert np.abs(gh - (ge - b)).max() < 1e-5


def test_terrain_edit_keeps_velocity_like_oracle():
    """Bed raised through a uniform current: surface and depth-averaged
    velocity kept where wet, no momentum where the bump emerges; element by
    element against the oracle right after the edit and 20 steps later."""
    say("case: terrain edit under a current 64x48")
    ws = _ws()
    nx, ny, dx, h0 = 64, 48, 0.1, 0.3
    z = -h0 * np.ones((ny + 1, nx + 1))
    gpu = ws.Domain(nx, ny, dx, dx, 0.004, z)
    ora = o.Domain(nx, ny, dx, dx, 0.004, z)
    w0 = np.zeros((ny, nx))
    P0, Q0 = h0 * 0.4 * np.ones((ny, nx)), h0 * -0.25 * np.ones((ny, nx))
    gpu.set_state(w0.astype(np.float32), P0.astype(np.float32), Q0.astype(np.float32))
    ora.set_state(w0, P0, Q0)
    assert gpu.apply_edit(ws.EDIT_TERRAIN, 3.2, 2.4, 0.5, 0.6) == 0
    assert ora.apply_edit(ws.EDIT_TERRAIN, 3.2, 2.4, 0.5, 0.6) == 0
    ge, gP, gQ = gpu.state_numpy()
    oe, oP, oQ = ora.state()
    assert np.abs(ge - oe).max() <= 1e-6 and np.abs(gP - oP).max() <= 1e-6 * 0.12
    assert np.abs(gQ - oQ).max() <= 1e-6 * 0.12
    gpu.advance(20)
    ora.advance(20)
    check(gpu, ora, 0.3, h0, rel=1e-4, what="20 steps after the edit")


def test_restore_after_time_step_change_restarts_history():
    """A snapshot restored after ws_update_grid changed dt brings back the
    state, bathymetry and time but restarts the multistep history (step 0,
    two Euler steps at the new dt): the run then matches the oracle
    hot-started from the same state at the new dt."""
    ws = _ws()
    w = wl.config2(nx=160, ny=72, seed=9)
    say("case: restore after a time-step change, %s" % w.name)
    gpu, ora = build_pair(w)
    gpu.advance(20)
    ora.advance(20)
    snap = gpu.snapshot()
    s20 = ora.state()
    t20 = ora.t
    gpu.advance(10)
    dt2 = 0.5 * w.dt
    gpu.update(dt=dt2)
    gpu.restore(snap)
    step, t, health = gpu.query()
    assert step == 0 and t == t20 and health == 0
    z = w.z.astype(np.float32).astype(np.float64)
    ora2 = o.Domain(w.nx, w.ny, w.dx, w.dy, dt2, z)
    for s, side in enumerate(w.sides):
        if side.kind != wl.SOLID:
            ora2.set_boundary(s, side.kind, side.width, side.amp, side.period, side.theta,
                              side.phase or None)
    ora2.set_state(*s20, t=t20)
    for n in (2, 28):
        gpu.advance(n)
        ora2.advance(n)
        check(gpu, ora2, 0.03, 0.5, rel=1e-4, what="after restore, step %d at dt/2" % ora2.step)
    # a snapshot restored at its own time step keeps the history
    gpu.update(dt=w.dt)
    gpu.restore(snap)
    assert gpu.query()[0] == 20


def test_steep_terrain_edit_rejected_unchanged():
    say("case: rejected terrain edit")
    ws = _ws()
    nx, ny, dx = 40, 30, 0.1
    D = ws.Domain(nx, ny, dx, dx, 0.01, 0.1 * np.ones((ny + 1, nx + 1)))
    before = D.state_numpy(ws.READ_H)
    assert D.apply_edit(ws.EDIT_TERRAIN, 2.0, 1.5, -6.0, 0.06) == ws.ENOTDD
    after = D.state_numpy(ws.READ_H)
    assert all(np.array_equal(a, b) for a, b in zip(before, after))


# -------------------------------------------------------------- full sizes
def test_config2_full_size_500_steps():
    """Config 2 at its full 1024 x 512 size for 500 steps (beach with a moving
    shoreline, seeded bumps, west sine maker a = 0.03 m, T = 2 s): eta within
    1e-4 a over the cells wet in both runs, P and Q within 1e-4 a sqrt(g d);
    the shoreline (cells wet in one run only) reported."""
    say("case: config2 1024x512, 500 steps")
    w = wl.config2(steps=500)
    gpu, ora = build_pair(w)
    a, d = 0.03, 0.5
    for n in (3, 497):
        gpu.advance(n)
        ora.advance(n)
    ge, gP, gQ = gpu.state_numpy()
    oe, oP, oQ = ora.state()
    b, _ = ora.bathy()
    wet = ((oe - b) > 1e-4) & ((ge - b) > 1e-4)
    shore = ((oe - b) > 1e-4) != ((ge - b) > 1e-4)
    de = np.abs(ge - oe)[wet].max()
    dP, dQ = np.abs(gP - oP).max(), np.abs(gQ - oQ).max()
    say("  step 500: wet cells %d, max|d eta| wet = %.3e (1e-4 a = %.1e), max|dP| = %.3e, "
        "max|dQ| = %.3e; cells wet in one run only: %d" % (wet.sum(), de, 1e-4 * a, dP, dQ, shore.sum()))
    assert de <= 1e-4 * a
    c = math.sqrt(G * d)
    assert dP <= 1e-4 * a * c and dQ <= 1e-4 * a * c
    assert np.all(ge >= b.astype(np.float32) - 1e-6)          # w >= B everywhere
    step, t, health = gpu.query()
    assert health == 0 and step == ora.step == 500


def _cached_tuning(nx, ny, n_corr=2, model=0):
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_1611_05984_amd", "tuning_cache.txt")
    for line in open(path):
        f = [int(v) for v in line.split()]
        if f[:4] == [nx, ny, n_corr, model]:
            return path, tuple(f[4:8])
    raise AssertionError("no cached tuning for %dx%d" % (nx, ny))


def test_config3_benchmark_shapes_100_steps():
    """Config 3 at 4096 x 4096 in the launch configuration the benchmark times:
    the tuning is read from the autotuner's cache exactly as bench.py does
    (8-row stencil strips, the factored reduced solve in workgroup form), then
    100 steps (two Euler steps, 98 AB3 + 2 AM4 steps) against the oracle,
    with the 64-component JONSWAP maker and the east sponge.  a0 = Hs/2."""
    say("case: config3 4096x4096, benchmark launch shapes, 100 steps")
    ws = _ws()
    w = wl.config3()
    gpu, ora = build_pair(w)
    path, want = _cached_tuning(w.nx, w.ny)
    got = gpu.tune(cache_path=path)
    say("  tuning from the cache: %s" % (got,))
    assert tuple(got) == want and want[2] == ws.SOLVE_LU
    a0, depth = 0.5, 30.0
    for n in (3, 97):
        gpu.advance(n)
        ora.advance(n)
        check(gpu, ora, a0, depth, rel=(2e-5 if ora.step == 3 else 1e-4), what="config3 step %d" % ora.step)


def test_maximum_grid_transposition_symmetry():
    """The largest square grid the library accepts (14640 x 14640, 2.1e8
    cells, ragged against the 64-column tiles: five padded fields just under
    4 GiB, the limit of the stencil's 32-bit field offsets) runs every kernel
    at its largest offsets.  Two
    water humps mirrored across the diagonal, one where offsets are small
    (top right) and one where they are largest (bottom left), over a
    transposition-symmetric bed: after 40 steps eta(i, j) = eta(j, i) and
    P(i, j) = Q(j, i) to FP32 rounding, far from both humps the lake is
    still exactly at rest, and the volume is conserved.  An access that went
    wrong with the offset would break the symmetry by O(1)."""
    ws = _ws()
    n, dx, depth, amp = 14640, 1.0, 2.0, 0.1
    assert ws.workspace_bytes(ws.grid(n, n, dx, dx, 0.01)) > 0
    assert ws.workspace_bytes(ws.grid(n + 1, n + 1, dx, dx, 0.01)) == 0   # the next square is refused
    dt = wl.courant_dt(0.2, dx, depth)
    c = (np.arange(n + 1) - n / 2) * dx
    r2 = c[:, None] ** 2 + c[None, :] ** 2
    z = (-depth + 0.5 * np.exp(-r2 / (2 * (200 * dx) ** 2))).astype(np.float32)  # symmetric mound
    say("case: maximum grid %dx%d (workspace %.1f GB)" % (n, n, ws.workspace_bytes(ws.grid(n, n, dx, dx, dt)) / 1e9))
    d = ws.Domain(n, n, dx, dx, dt, z)
    del z, c, r2
    d.set_tuning(8, 256, ws.SOLVE_LU)
    lo, hi = 0.1 * n * dx, 0.9 * n * dx
    assert d.apply_edit(ws.EDIT_WATER, hi, lo, amp, 20 * dx) == 0   # x large, y small: small offsets
    assert d.apply_edit(ws.EDIT_WATER, lo, hi, amp, 20 * dx) == 0   # x small, y large: largest offsets
    w0, _, _ = d.state_numpy()
    v0 = float(np.sum(w0, dtype=np.float64))
    del w0
    d.advance(40)
    step, _, health = d.query()
    say("  40 steps done: step %d health %d" % (step, health))
    assert step == 40 and health == 0
    w, P, Q = d.state_numpy()
    d.close()
    assert np.isfinite(w).all() and np.isfinite(P).all() and np.isfinite(Q).all()
    cpq = amp * math.sqrt(9.81 * depth)
    dw = float(np.max(np.abs(w - w.T)))
    dpq = float(np.max(np.abs(P - Q.T)))
    say("  max |eta - eta^T| = %.3e, max |P - Q^T| = %.3e, max eta = %.3e" % (dw, dpq, float(w.max())))
    assert float(w.max()) > 0.1 * amp                 # the humps are still there
    assert dw <= 1e-4 * amp and dpq <= 1e-4 * cpq
    # the waves travel about 8 m in 40 steps: the middle of the basin is at rest, exactly
    m = n // 2
    assert not np.any(w[m - 1000:m + 1000, m - 1000:m + 1000])
    assert not np.any(P[m - 1000:m + 1000, m - 1000:m + 1000]) and not np.any(Q[m - 1000:m + 1000, m - 1000:m + 1000])
    v1 = float(np.sum(w, dtype=np.float64))
    say("  volume change %.3e of %.3e" % (v1 - v0, v0))
    assert abs(v1 - v0) <= 1e-4 * abs(v0)
