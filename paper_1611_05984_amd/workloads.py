"""Seeded synthetic inputs for the wave-solver workloads.

This module only draws inputs: corner bathymetry arrays, initial solitary
waves, wave-maker component tables, domain lists and arrival traces.  It holds
none of the solver's arithmetic; both the GPU library and the CPU oracle
receive the arrays it returns.  Every generator is deterministic in its seed
(``numpy.random.default_rng``); the draw order is fixed and documented per
function.

Bathymetry convention: ``z`` has shape (ny+1, nx+1) and samples the bottom
elevation at the cell corners (i*dx, j*dy); the still water level is 0, so
z < 0 is under water.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

G = 9.81
SOLID, SPONGE, WAVES = 0, 1, 2
WEST, EAST, SOUTH, NORTH = 0, 1, 2, 3


@dataclass
class Side:
    kind: int = SOLID
    width: int = 2
    amp: list = field(default_factory=list)
    period: list = field(default_factory=list)
    theta: list = field(default_factory=list)
    phase: list = field(default_factory=list)


@dataclass
class Workload:
    """One domain: grid, time step, bathymetry, boundaries, initial waves."""
    name: str
    nx: int
    ny: int
    dx: float
    dy: float
    dt: float
    z: np.ndarray
    sides: list
    solitary: list = field(default_factory=list)   # (H, theta, x0, y0)
    steps: int = 0

    @property
    def cells(self) -> int:
        return self.nx * self.ny


def courant_dt(courant: float, dx: float, depth_max: float) -> float:
    """Time step for a Courant number sqrt(g d_max) dt / dx."""
    return courant * dx / math.sqrt(G * depth_max)


def walls():
    return [Side(SOLID), Side(SOLID), Side(SOLID), Side(SOLID)]


# --------------------------------------------------------------- config 1
def config1(nx: int = 128, ny: int = 64) -> Workload:
    """128x64 cells at 0.1 m, flat bottom 1 m deep, solitary wave H = 0.1 m
    at x = 3 m travelling +x, walls, Courant 0.2, 500 steps.  No randomness."""
    dx = 0.1
    z = -np.ones((ny + 1, nx + 1))
    return Workload("solitary_basin_%dx%d" % (nx, ny), nx, ny, dx, dx,
                    courant_dt(0.2, dx, 1.0), z, walls(),
                    solitary=[(0.1, 0.0, 3.0, 0.5 * ny * dx)], steps=500)


def config1_long(nx: int = 1024, ny: int = 8) -> Workload:
    """Long-channel variant of config 1 (102.4 m) for the speed/shape check:
    same depth, height, grid spacing and Courant number, crest at x = 30 m."""
    w = config1(nx, ny)
    w.name = "solitary_channel_%dx%d" % (nx, ny)
    w.solitary = [(0.1, 0.0, 30.0, 0.5 * ny * w.dy)]
    return w


# --------------------------------------------------------------- config 2
def gaussian_bumps(z, dx, dy, rng, n=20, amp=(-0.05, 0.05), sigma=(0.2, 1.0)):
    """Add n Gaussian bumps to corner bathymetry.  Draw order per bump:
    centre x, centre y (uniform over the domain), amplitude, sigma."""
    ny1, nx1 = z.shape
    X = np.arange(nx1)[None, :] * dx
    Y = np.arange(ny1)[:, None] * dy
    Lx, Ly = (nx1 - 1) * dx, (ny1 - 1) * dy
    for _ in range(n):
        cx, cy = rng.uniform(0, Lx), rng.uniform(0, Ly)
        a, s = rng.uniform(*amp), rng.uniform(*sigma)
        z = z + a * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * s * s))
    return z


def config2(nx: int = 1024, ny: int = 512, seed: int = 2, steps: int = 10000) -> Workload:
    """Plane beach with a wet/dry shoreline and a west sine wave maker.

    dx = 0.05 m; z = max(-0.5, (x - x_s)/20) with the shoreline x_s at 0.805 of
    the domain length (41.2 m at 1024 cells), dry land up to the east wall;
    20 seeded Gaussian bumps (amplitude U(-0.05, 0.05) m, sigma U(0.2, 1.0) m).
    West: sine waves a = 0.03 m, T = 2 s, normal incidence; other sides walls.
    Courant 0.2 on the deepest water."""
    rng = np.random.default_rng(seed)
    dx = 0.05
    Lx = nx * dx
    X = np.arange(nx + 1)[None, :] * dx
    z = np.maximum(-0.5, (X - 0.805 * Lx) / 20.0) * np.ones((ny + 1, 1))
    z = gaussian_bumps(z, dx, dx, rng)
    dmax = float(max(1e-3, -z.min()))
    sides = walls()
    sides[WEST] = Side(WAVES, 2, [0.03], [2.0], [0.0], [0.0])
    return Workload("beach_%dx%d" % (nx, ny), nx, ny, dx, dx, courant_dt(0.2, dx, dmax), z,
                    sides, steps=steps)


# --------------------------------------------------------------- config 3
def fractal_noise(shape, dx, rng, rms=0.5, slope=-3.0):
    """Zero-mean Gaussian random field with power spectrum ~ |k|^slope by
    spectral synthesis, scaled to the given RMS.  Draws: one complex normal
    array of the FFT shape (real part, then imaginary part)."""
    ny, nx = shape
    kx = np.fft.rfftfreq(nx, dx)
    ky = np.fft.fftfreq(ny, dx)
    k = np.sqrt(kx[None, :] ** 2 + ky[:, None] ** 2)
    k[0, 0] = np.inf
    amp = k ** (slope / 2.0)
    re = rng.standard_normal(amp.shape)
    im = rng.standard_normal(amp.shape)
    f = np.fft.irfft2(amp * (re + 1j * im), s=(ny, nx))
    f -= f.mean()
    return f * (rms / f.std())


def jonswap_components(n=64, Hs=1.0, Tp=8.0, gamma=3.3, fmin=0.5, fmax=2.0, rng=None):
    """n wave components from a JONSWAP spectrum on equal frequency bins over
    [fmin, fmax]*fp; amplitudes sqrt(2 S df) rescaled so 4 sqrt(sum a^2/2) = Hs;
    phases U[0, 2 pi) drawn in component order.  Returns (amp, period, phase)."""
    fp = 1.0 / Tp
    df = (fmax - fmin) * fp / n
    f = fmin * fp + (np.arange(n) + 0.5) * df
    sigma = np.where(f <= fp, 0.07, 0.09)
    r = np.exp(-((f - fp) ** 2) / (2 * sigma ** 2 * fp ** 2))
    S = G ** 2 * (2 * np.pi) ** -4 * f ** -5 * np.exp(-1.25 * (fp / f) ** 4) * gamma ** r
    a = np.sqrt(2 * S * df)
    a *= Hs / (4.0 * np.sqrt(np.sum(a ** 2) / 2.0))
    phase = rng.uniform(0, 2 * np.pi, n) if rng is not None else np.zeros(n)
    return a, 1.0 / f, phase


def config3(n: int = 4096, seed: int = 3, dx: float = 1.0, steps: int = 1000) -> Workload:
    """Continental shelf 30 m -> 5 m, d(x) = 17.5 - 12.5 tanh((x - L/2)/(0.1 L)),
    plus fractal noise (|k|^-3, RMS 0.5 m) on the corners; 64 JONSWAP components
    (Hs 1 m, Tp 8 s, gamma 3.3) at the west side, 64-cell sponge east, walls
    north/south; Courant 0.2.  Draw order: noise field, then wave phases."""
    rng = np.random.default_rng(seed)
    L = n * dx
    X = np.arange(n + 1)[None, :] * dx
    d = 17.5 - 12.5 * np.tanh((X - 0.5 * L) / (0.1 * L))
    z = -d * np.ones((n + 1, 1)) + fractal_noise((n + 1, n + 1), dx, rng)
    a, T, ph = jonswap_components(rng=rng)
    sides = walls()
    sides[WEST] = Side(WAVES, 2, list(a), list(T), [0.0] * len(a), list(ph))
    sides[EAST] = Side(SPONGE, 64)
    dmax = float(-z.min())
    return Workload("shelf_%dx%d" % (n, n), n, n, dx, dx, courant_dt(0.2, dx, dmax),
                    z.astype(np.float64), sides, steps=steps)


# --------------------------------------------------------------- config 4
def beach_or_flat(nx, ny, dx, depth, slope, toe_frac=0.8):
    X = np.arange(nx + 1)[None, :] * dx
    if slope is None:
        return -depth * np.ones((ny + 1, nx + 1))
    Lx = nx * dx
    return np.maximum(-depth, slope * (X - toe_frac * Lx)) * np.ones((ny + 1, 1))


def config4(n_domains: int = 256, seed: int = 4, lo: int = 256, hi: int = 1024,
            steps: int = 2000) -> list:
    """Ensemble of independent domains: nx, ny ~ U{lo..hi}; dx = 0.1 m; depth
    1 m; half flat, half plane beach z = max(-1, s (x - 0.8 L)) with
    s ~ U[1/50, 1/10]; a solitary wave H = U(0.05, 0.4) * 1 m at x0 = 0.3 L,
    normal incidence; walls; Courant 0.2.  Draw order per domain: nx, ny,
    flat-or-beach, slope (beach only), H."""
    rng = np.random.default_rng(seed)
    out = []
    dx, depth = 0.1, 1.0
    for k in range(n_domains):
        nx = int(rng.integers(lo, hi + 1))
        ny = int(rng.integers(lo, hi + 1))
        beach = bool(rng.integers(0, 2))
        slope = float(rng.uniform(1 / 50, 1 / 10)) if beach else None
        H = float(rng.uniform(0.05, 0.4)) * depth
        z = beach_or_flat(nx, ny, dx, depth, slope)
        out.append(Workload("ens%03d_%dx%d" % (k, nx, ny), nx, ny, dx, dx,
                            courant_dt(0.2, dx, depth), z, walls(),
                            solitary=[(H, 0.0, 0.3 * nx * dx, 0.5 * ny * dx)], steps=steps))
    return out


# --------------------------------------------------------------- config 5
@dataclass
class Session:
    arrival: float
    nx: int
    depth: float
    slope: float
    steps: int
    edits: list   # (step, kind, x0, y0, amp, sigma)
    courant: float = 0.2
    eps: float = 5e-12    # desingularization threshold of the session's solver


def config5_trace(rate: float = 4.0, duration: float = 600.0, seed: int = 5,
                  sizes=(512, 1024, 2048), edit_every: int = 50, steps=(500, 2000),
                  sigma_cells=(10.0, 40.0), water_amp=(0.1, 0.5), terrain_amp=(0.2, 1.0),
                  eps: float = 5e-12) -> list:
    """Poisson arrivals (rate per second) over `duration` seconds.  Per
    session, in draw order: inter-arrival gap, grid size (uniform over
    `sizes`), offshore depth U[0.5, 2] m, beach slope U[1/50, 1/10], session
    length U{steps[0]..steps[1]} (default 500..2000) steps, then for each edit (every `edit_every` steps):
    kind (0 water hump A ~ U[0.1, 0.5] m, 1 terrain A ~ U[0.2, 1] m, p = 1/2),
    sigma ~ U[10, 40] cells, centre uniform, amplitude (ranges adjustable for
    small test traces)."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    dx = 0.1
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        depth = float(rng.uniform(0.5, 2.0))
        slope = float(rng.uniform(1 / 50, 1 / 10))
        n_steps = int(rng.integers(steps[0], steps[1] + 1))
        edits = []
        for s in range(edit_every, n_steps + 1, edit_every):
            kind = int(rng.integers(0, 2))
            sigma = float(rng.uniform(*sigma_cells)) * dx
            x0, y0 = float(rng.uniform(0, n * dx)), float(rng.uniform(0, n * dx))
            amp = float(rng.uniform(*water_amp)) if kind == 0 else float(rng.uniform(*terrain_amp))
            edits.append((s, kind, x0, y0, amp, sigma))
        out.append(Session(t, n, depth, slope, n_steps, edits, eps=eps))
    return out


def session_workload(s: Session) -> Workload:
    dx = 0.1
    z = beach_or_flat(s.nx, s.nx, dx, s.depth, s.slope)
    return Workload("session_%d" % s.nx, s.nx, s.nx, dx, dx, courant_dt(s.courant, dx, s.depth), z,
                    walls(), steps=s.steps)


# ------------------------------------------------- sec. 4.2 and 4.3 setups
def whalin(nx: int = 2000, ny: int = 65, amp: float = 0.0075, period: float = 2.0,
           dt: float = 0.001, steps: int = 20000) -> Workload:
    """Semicircular shoal (sec. 4.2): 35 m x 6.096 m on nx x ny cells, bottom of
    eq. 37 as heights above the tank floor with the still water 0.4572 m above
    it (depth 0.4572 m falling to 0.1524 m over the shoal), west sine maker
    (a, T), 5 m sponge east, walls north and south, fixed dt.  Eq. 37's middle
    branch is read as (x - 10.67 + G)/25: as printed it falls below the floor
    instead of rising to 0.3048 m at x = 18.29 - G.  No random draws."""
    Lx, Ly, h0 = 35.0, 6.096, 0.4572
    dx, dy = Lx / nx, Ly / ny
    X = np.arange(nx + 1)[None, :] * dx
    Y = np.arange(ny + 1)[:, None] * dy
    Gy = np.sqrt(np.clip(Y * (Ly - Y), 0.0, None))
    zf = np.where(X < 10.67 - Gy, 0.0, np.where(X < 18.29 - Gy, (X - 10.67 + Gy) / 25.0, 0.3048))
    z = zf - h0
    sides = walls()
    sides[WEST] = Side(WAVES, 2, [amp], [period], [0.0], [0.0])
    sides[EAST] = Side(SPONGE, int(round(5.0 / dx)))
    return Workload("whalin_%dx%d" % (nx, ny), nx, ny, dx, dy, dt, z, sides, steps=steps)


def conical_island(n: int = 601, h_over_d: float = 0.09, depth: float = 0.32, dt: float = 0.005,
                   x0: float = 5.0, sponge_m: float = 2.0, steps: int = 4000) -> Workload:
    """Solitary wave on a conical island (sec. 4.3): 30 m x 30 m on n x n cells,
    depth 0.32 m, island centred, base diameter 7.2 m, side slope 1/4 (height
    above the floor (3.6 - r)/4, flat top at 0.625 m above the floor, i.e.
    radius 1.1 m: the paper gives diameter and slope only), soliton H = h/d *
    depth with its crest along y at x0, sponges west and east (width sponge_m),
    walls north and south, fixed dt.  No random draws."""
    L = 30.0
    dx = L / n
    X = np.arange(n + 1)[None, :] * dx - 0.5 * L
    Y = np.arange(n + 1)[:, None] * dx - 0.5 * L
    r = np.sqrt(X * X + Y * Y)
    above = np.clip((3.6 - r) / 4.0, 0.0, 0.625)
    z = -depth + above
    sides = walls()
    w = int(round(sponge_m / dx))
    sides[WEST] = Side(SPONGE, w)
    sides[EAST] = Side(SPONGE, w)
    return Workload("conical_%dx%d_H%.2f" % (n, n, h_over_d), n, n, dx, dx, dt, z, sides,
                    solitary=[(h_over_d * depth, 0.0, x0, 0.5 * L)], steps=steps)
