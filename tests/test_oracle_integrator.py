"""Order of the oracle's multistep time integrator (sec. 2.3, eqs. 15-20).

The Euler start-up (two first-order steps, sec. 2.3) caps the global order of
any run that starts from a single state at 2, so a consistent but lower-order
Adams table (AB2 in place of AB3, AM3 in place of AM4) would pass a plain
self-convergence test.  These tests load an exact multistep history instead
(`set_clock`, `set_history`), so every step is a full AB3 predictor plus K
AM4 correctors, and measure the order against solutions known in closed form:

* local error of one step on a flow whose semi-discrete right-hand side is
  exact (E, F and G all non-zero): order 4 for AB3 alone (K = 0), order 5
  with AM4 correctors (K >= 1);
* global error of many steps on the friction decay of a uniform current:
  order 3 for K = 0, order 4 for K >= 1.
"""
import math

import numpy as np
import pytest

import oracle as o

D0 = 1.0  # still water depth of the flat basin (m)


# ------------------------------------------------------------ local error
def _divergent_flow(case, C, t, h0=1.0):
    """Depth h and the rates a, c of the flow P = a x, Q = c y on a flat bed.

    With h uniform and P, Q linear the reconstruction is exact, the
    central-upwind flux reduces to the physical flux of eq. 1, and the
    dispersive terms and F*, G* vanish (eta is uniform, Q_xy = P_xy = 0), so
    the semi-discrete system is exactly
        dh/dt = -(a + c),  da/dt = -a (2a + c)/h,  dc/dt = -c (a + 2c)/h
    (the x-momentum flux P^2/h gives 2 a P / h, the cross flux PQ/h gives
    c P / h).  Closed forms: c = 0 gives a = C h^2, h = h0 / (1 + C h0 t);
    a = c gives a = C h^(3/2), h = (h0^(-1/2) + C t)^(-2).  The walls at
    x = 0 and y = 0 mirror P and Q oddly, which these fields already are."""
    if case == "x":
        h = h0 / (1.0 + C * h0 * t)
        return h, C * h * h, 0.0
    if case == "y":
        h = h0 / (1.0 + C * h0 * t)
        return h, 0.0, C * h * h
    h = (h0 ** -0.5 + C * t) ** -2
    a = C * h ** 1.5
    return h, a, a


def _one_step_error(case, K, dt, n=48, dx=1.0, C=0.02, tn=0.0):
    """Largest error of w, P, Q after one step from the exact state and the
    exact history, over the cells no wall-inconsistent value reaches (the
    fields are not linear at the north and east walls)."""
    D = o.Domain(n, n, dx, dx, dt, -D0 * np.ones((n + 1, n + 1)), n_corr=K)
    x = (np.arange(n) + 0.5) * dx
    X, Y = np.meshgrid(x, x)

    def state(t):
        h, a, c = _divergent_flow(case, C, t)
        return (h - D0) * np.ones_like(X), a * X, c * Y

    def rhs(t):
        h, a, c = _divergent_flow(case, C, t)
        return (-(a + c) * np.ones_like(X), -a * (2 * a + c) * X / h, -c * (a + 2 * c) * Y / h)

    D.set_state(*state(tn), t=tn)
    D.set_clock(2, tn)
    D.set_history(1, *rhs(tn - dt))
    D.set_history(2, *rhs(tn - 2 * dt))
    D.advance(1)
    assert D.step == 3 and abs(D.t - (tn + dt)) < 1e-12
    got, want = D.state(), state(tn + dt)
    m = (slice(0, 16), slice(0, 16))
    return [float(np.abs(g[m] - e[m]).max()) for g, e in zip(got, want)]


@pytest.mark.parametrize("K", [0, 1, 2])
@pytest.mark.parametrize("case", ["x", "y", "xy"])
def test_adams_local_error_order(case, K):
    """One AB3 step has local error O(dt^4); AB3 followed by K >= 1 AM4
    correctors O(dt^5).  An AB2 table (order 2) would show 3, an AM3
    corrector (order 3) 4.  Checked separately for w, P and Q, so each of
    the three update formulas of eqs. 15-20 is pinned."""
    dts = (0.8, 0.4, 0.2, 0.1)
    errs = np.array([_one_step_error(case, K, dt) for dt in dts])   # (dt, field)
    want = 4.0 if K == 0 else 5.0
    active = {"x": (0, 1), "y": (0, 2), "xy": (0, 1, 2)}[case]
    for f in range(3):
        if f not in active:
            assert errs[:, f].max() < 1e-17, (case, K, f, errs[:, f])  # that discharge stays zero
            continue
        e = errs[:, f]
        assert e[-1] > 1e-14, (case, K, f, e)     # well above round-off
        orders = np.log2(e[:-1] / e[1:])
        assert orders.min() >= want - 0.2 and orders.max() <= want + 0.3, (case, K, f, e, orders)


# ----------------------------------------------------------- global error
def _friction_decay_error(direction, K, N, T=20.0, f=0.05, P0=1.0, n=1024, dx=60.0):
    """A uniform current on a flat bed under quadratic friction (eq. 31):
    uniform h and discharge make E = 0 and every flux difference zero, so
    dP/dt = -f P |P| / h^2 with h = d, and P(t) = P0 / (1 + k P0 t),
    k = f / d^2.  Run N steps to time T from the exact history; the walls
    stop the current, but in N steps of K + 1 passes nothing they change
    travels further than 2 (K + 1) N cells, and the reading is taken at the
    channel's middle, 512 cells from either wall."""
    dt = T / N
    nx, ny = (n, 2) if direction == "x" else (2, n)
    D = o.Domain(nx, ny, dx, dx, dt, -D0 * np.ones((ny + 1, nx + 1)), n_corr=K,
                 friction=o.FRIC_QUAD, fcoef=f)
    k = f / D0 ** 2
    exact = lambda t: P0 / (1.0 + k * P0 * t)
    one = np.ones((ny, nx))
    zero = 0.0 * one

    def discharge(v):
        return (v * one, zero) if direction == "x" else (zero, v * one)

    def rhs(t):
        F, G = discharge(-k * exact(t) ** 2)
        return zero, F, G

    D.set_state(zero, *discharge(exact(0.0)), t=0.0)
    D.set_clock(2, 0.0)
    D.set_history(1, *rhs(-dt))
    D.set_history(2, *rhs(-2 * dt))
    D.advance(N)
    w, P, Q = D.state()
    mid = P[0, n // 2] if direction == "x" else Q[n // 2, 0]
    return abs(mid - exact(T)), float(np.abs(w).max())


@pytest.mark.parametrize("K", [0, 1, 2])
@pytest.mark.parametrize("direction", ["x", "y"])
def test_adams_global_order_friction_decay(direction, K):
    """Global error at a fixed time over N = 8 .. 64 steps: order 3 for the
    AB3 predictor alone, 4 with AM4 correctors (an AB2 or AM3 table gives 2
    or 3).  The whole channel, walls included, stays bounded."""
    runs = [_friction_decay_error(direction, K, N) for N in (8, 16, 32, 64)]
    e = np.array([r[0] for r in runs])
    assert max(r[1] for r in runs) < 0.5, runs
    assert e[-1] > 1e-12, e
    orders = np.log2(e[:-1] / e[1:])
    want = 2.8 if K == 0 else 3.8
    assert orders.min() >= want, (direction, K, e, orders)
    # and the error constant is that of the method, not of a lower order one
    # whose constant happens to be small: the finest run is accurate
    assert e[-1] < (4e-6 if K == 0 else 3e-8), e


def test_exact_history_matches_self_started_run():
    """set_clock/set_history only replace the start-up: loading the history
    a run computed itself and its state reproduces that run bit for bit."""
    n, dx, dt = 24, 0.1, 0.01
    z = -np.ones((n + 1, n + 1))
    x = (np.arange(n) + 0.5) * dx
    X, Y = np.meshgrid(x, x)
    w0 = 0.01 * np.exp(-((X - 1.0) ** 2 + (Y - 1.3) ** 2) / 0.2)
    A = o.Domain(n, n, dx, dx, dt, z)
    A.set_state(w0, 0 * w0, 0 * w0)
    A.advance(1)
    r1 = A.eval_rhs(*A.state(), t=A.t)       # level 1: right-hand side after step 1
    A.advance(1)
    r2 = A.eval_rhs(*A.state(), t=A.t)       # level 2
    A.advance(1)
    s3 = A.state()
    A.advance(1)                             # step 4 uses levels 3, 2, 1
    # B starts at step 4 with the state after step 3, level 2 (lag 1), level 1 (lag 2)
    B = o.Domain(n, n, dx, dx, dt, z)
    B.set_state(*s3, t=3 * dt)
    B.set_clock(3, 3 * dt)
    B.set_history(1, r2["E"], r2["F"], r2["G"], r2["Fs"], r2["Gs"])
    B.set_history(2, r1["E"], r1["F"], r1["G"], r1["Fs"], r1["Gs"])
    B.advance(1)
    assert all(np.array_equal(a, b) for a, b in zip(A.state(), B.state()))
    assert math.isclose(A.t, B.t) and A.step == B.step == 4
