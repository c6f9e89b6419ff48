"""The sec. 4.2 and 4.3 setups on the GPU path: element-by-element parity
with the oracle over a short run at full size, then self-consistency of long
runs (no measured data is available: the checks are the qualitative physics
those experiments show, with margins wide enough for any reasonable reading).
"""
import math
import sys

import numpy as np
import pytest

import oracle as o
from paper_1611_05984_amd import workloads as wl

pytestmark = pytest.mark.gpu
G = 9.81


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def pair(w, oracle_too=True):
    from paper_1611_05984_amd import wavestep as ws
    z = w.z.astype(np.float32).astype(np.float64)
    g = ws.Domain(w.nx, w.ny, w.dx, w.dy, w.dt, z)
    r = o.Domain(w.nx, w.ny, w.dx, w.dy, w.dt, z) if oracle_too else None
    for s, side in enumerate(w.sides):
        if side.kind == wl.SOLID:
            continue
        g.set_boundary(s, side.kind, side.width, side.amp, side.period, side.theta, side.phase or None)
        if r:
            r.set_boundary(s, side.kind, side.width, side.amp, side.period, side.theta, side.phase or None)
    for (H, th, x0, y0) in w.solitary:
        g.add_solitary(H, th, x0, y0)
        if r:
            r.add_solitary(H, th, x0, y0)
    return g, r


def test_whalin_short_parity():
    w = wl.whalin()
    say("case: %s, 400 steps vs oracle" % w.name)
    g, r = pair(w)
    g.advance(400)
    r.advance(400)
    ge, gP, gQ = g.state_numpy()
    oe, oP, oQ = r.state()
    a, c = 0.0075, math.sqrt(G * 0.4572)
    de, dP, dQ = np.abs(ge - oe).max(), np.abs(gP - oP).max(), np.abs(gQ - oQ).max()
    say("  max|d eta| %.3e  |dP| %.3e  |dQ| %.3e" % (de, dP, dQ))
    assert de <= 1e-4 * a and max(dP, dQ) <= 1e-4 * a * c


def harmonics(series, dt_sample, period, n_harm=3):
    """Amplitudes of the first n_harm harmonics of 1/period per column of
    series (time x space), from whole periods of samples."""
    n = series.shape[0]
    spec = np.fft.rfft(series - series.mean(axis=0), axis=0) * 2.0 / n
    freqs = np.fft.rfftfreq(n, dt_sample)
    out = []
    for h in range(1, n_harm + 1):
        k = int(np.argmin(np.abs(freqs - h / period)))
        out.append(np.abs(spec[k]))
    return out


def test_whalin_focusing_and_harmonics():
    """Regular waves over the shoal focus behind it and shed higher
    harmonics: along the centreline the first harmonic grows well above the
    incident amplitude and a second harmonic appears, while upstream of the
    shoal the first harmonic stays near the maker amplitude."""
    w = wl.whalin()
    g, _ = pair(w, oracle_too=False)
    a, T = 0.0075, 2.0
    spin_up, every, periods = 24000, 20, 4
    say("case: %s, %d + %d steps" % (w.name, spin_up, int(periods * T / w.dt)))
    g.advance(spin_up)
    jc = w.ny // 2
    rows = []
    for _ in range(int(periods * T / w.dt) // every):
        g.advance(every)
        e, _, _ = g.state_numpy()
        rows.append(e[jc].astype(np.float64))
    assert g.query()[2] == 0
    h1, h2, h3 = harmonics(np.array(rows), every * w.dt, T)
    x = (np.arange(w.nx) + 0.5) * w.dx
    up = (x > 2.0) & (x < 6.0)
    shoal = (x > 14.0) & (x < 28.0)
    say("  upstream h1/a %.2f..%.2f; shoal max h1/a %.2f at x=%.1f m, max h2/a %.2f, max h3/a %.2f"
        % (h1[up].min() / a, h1[up].max() / a, h1[shoal].max() / a, x[shoal][np.argmax(h1[shoal])],
           h2[shoal].max() / a, h3[shoal].max() / a))
    assert 0.7 < h1[up].mean() / a < 1.4
    assert h1[shoal].max() > 1.5 * a
    assert h2[shoal].max() > 0.2 * a


def test_conical_island_parity_and_wraparound():
    """Solitary wave on the conical island: short parity with the oracle at
    full size, then the wave runs up the front face and wraps around the
    island, wetting its lee side."""
    w = wl.conical_island(h_over_d=0.09)
    say("case: %s" % w.name)
    g, r = pair(w)
    g.advance(60)
    r.advance(60)
    ge, gP, gQ = g.state_numpy()
    oe, oP, oQ = r.state()
    H, c = 0.09 * 0.32, math.sqrt(G * 0.32)
    de, dP = np.abs(ge - oe).max(), max(np.abs(gP - oP).max(), np.abs(gQ - oQ).max())
    say("  60 steps: max|d eta| %.3e  |dP,dQ| %.3e" % (de, dP))
    assert de <= 1e-4 * H and dP <= 1e-4 * H * c
    b, dstill = r.bathy()
    X = (np.arange(w.nx) + 0.5) * w.dx - 15.0
    Y = (np.arange(w.ny) + 0.5) * w.dx - 15.0
    R = np.sqrt(X[None, :] ** 2 + Y[:, None] ** 2)
    ring = (dstill == 0) & (R > 1.1) & (R < 2.6)       # dry island face above the still water
    front = ring & (X[None, :] < -0.5)
    lee = ring & (X[None, :] > 0.5) & (np.abs(Y[:, None]) < 1.0)
    wet_front = np.zeros_like(front)
    wet_lee = np.zeros_like(lee)
    hmax = 0.0
    for _ in range(30):                               # 14.7 s simulated more
        g.advance(100)
        hh, _, _ = g.state_numpy(what=1)
        wet_front |= front & (hh > 1e-3)
        wet_lee |= lee & (hh > 1e-3)
        hmax = max(hmax, float(hh[front].max()))
    assert g.query()[2] == 0
    say("  run-up: wetted front-face cells %d of %d, lee cells %d of %d, max depth on the face %.3f m"
        % (wet_front.sum(), front.sum(), wet_lee.sum(), lee.sum(), hmax))
    assert wet_front.sum() > 10 and wet_lee.sum() > 5
