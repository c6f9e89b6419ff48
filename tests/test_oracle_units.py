"""Pins of the oracle's building blocks against closed forms, library solvers
and the governing equations (eqs. 1-3, 7, 12, 23, 29, 30 of the paper).

Every check here compares the oracle with something other than its own
formula: a library routine (scipy banded solver), an exact property
(polynomial exactness of a stencil, flux consistency, conservation of the cell
mean), or the continuous equations evaluated symbolically.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import sympy as sp

import oracle as o

G = 9.81
B = 1.0 / 15.0


# ------------------------------------------------------------ tridiagonal
def test_thomas_matches_banded_library_solver():
    rng = np.random.default_rng(11)
    for n in (2, 3, 17, 256, 1001):
        a = rng.uniform(-1, 1, n)
        c = rng.uniform(-1, 1, n)
        b = np.abs(a) + np.abs(c) + rng.uniform(0.05, 2.0, n)
        b *= rng.choice([-1, 1], n)
        a[0] = 0.0
        c[-1] = 0.0
        r = rng.standard_normal(n)
        ab = np.zeros((3, n))
        ab[0, 1:] = c[:-1]
        ab[1] = b
        ab[2, :-1] = a[1:]
        x_ref = scipy.linalg.solve_banded((1, 1), ab, r)
        x = o.thomas(a, b, c, r)
        np.testing.assert_allclose(x, x_ref, rtol=1e-12, atol=1e-13 * np.abs(x_ref).max())


def _flat(nx, ny, d=1.0):
    return -d * np.ones((ny + 1, nx + 1))


def test_solve_inverts_the_ustar_operator_walls_and_wavemaker():
    """The row/column solves (eqs. 21-22 with boundary folds) invert exactly the
    operator U* = A P_{i-1} + B P_i + C P_{i+1} that the step applies to P with
    its ghost values: solve(U*(P)) == P for walls and for a wave-maker side."""
    rng = np.random.default_rng(5)
    nx, ny, dx = 24, 20, 0.1
    X = np.arange(nx + 1)[None, :] * dx
    z = -(0.6 + 0.04 * X + 0.2 * np.sin(np.arange(ny + 1)[:, None] * 0.3)) * np.ones((1, nx + 1))
    for west in (o.SOLID, o.WAVES):
        D = o.Domain(nx, ny, dx, dx, 0.01, z)
        if west == o.WAVES:
            D.set_boundary(o.WEST, o.WAVES, 2, [0.02], [1.7], [0.3], [0.4])
            D.set_boundary(o.SOUTH, o.WAVES, 2, [0.01], [2.1], [1.2], [1.0])
        w = 0.01 * rng.standard_normal((ny, nx))
        P = rng.standard_normal((ny, nx))
        Q = rng.standard_normal((ny, nx))
        t = 0.37
        r = D.eval_rhs(w, P, Q, t)
        P2, Q2 = D.eval_solve(r["U"], r["V"], t)
        np.testing.assert_allclose(P2, P, rtol=0, atol=1e-12)
        np.testing.assert_allclose(Q2, Q, rtol=0, atol=1e-12)


def test_ustar_operator_matches_eq7_on_polynomials():
    """Eq. (23) discretizes eq. (7): U* = P - d d_x P_x / 3 - (B + 1/3) d^2 P_xx.
    Central differences are exact for quadratic P and linear d, so away from
    the walls the discrete U*, V* equal eqs. (7)-(8) evaluated exactly."""
    nx, ny, dx, dy = 30, 26, 0.2, 0.15
    cx = np.arange(nx + 1) * dx
    cy = np.arange(ny + 1) * dy
    z = -(1.0 + 0.08 * cx[None, :] + 0.05 * cy[:, None])  # d = 1 + 0.08x + 0.05y
    D = o.Domain(nx, ny, dx, dy, 0.01, z)
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    X, Y = np.meshgrid(x, y)
    P = 0.3 + 0.2 * X - 0.7 * X ** 2 + 0.1 * X * Y + 0.05 * Y ** 2
    Q = -0.1 + 0.4 * Y + 0.3 * Y ** 2 - 0.2 * X * Y + 0.1 * X ** 2
    d = 1.0 + 0.08 * X + 0.05 * Y
    Ux = P - d * 0.08 * (0.2 - 1.4 * X + 0.1 * Y) / 3.0 - (B + 1 / 3) * d ** 2 * (-1.4)
    Vy = Q - d * 0.05 * (0.4 + 0.6 * Y - 0.2 * X) / 3.0 - (B + 1 / 3) * d ** 2 * (0.6)
    r = D.eval_rhs(np.zeros_like(P), P, Q)
    s = (slice(2, -2), slice(2, -2))
    np.testing.assert_allclose(r["U"][s], Ux[s], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(r["V"][s], Vy[s], rtol=1e-12, atol=1e-12)


# ---------------------------------------------------- reconstruction, KP07
def test_minmod_cases():
    assert o.minmod3(1.0, 2.0, 3.0) == 1.0
    assert o.minmod3(3.0, 0.5, 2.0) == 0.5
    assert o.minmod3(-1.0, -2.0, -0.5) == -0.5
    assert o.minmod3(1.0, -1.0, 2.0) == 0.0
    assert o.minmod3(0.0, 1.0, 2.0) == 0.0


def test_reconstruction_exact_on_linear_data_and_zero_slope_on_constants():
    for th in (1.0, 1.3, 2.0):
        lo, hi = o.reconstruct([1.0, 1.5, 2.0], [-3.0, -1.0, 1.0], [0.2, 0.2, 0.2], -5, -5, th)
        np.testing.assert_allclose(lo, [1.25, -2.0, 0.2], rtol=0, atol=1e-15)
        np.testing.assert_allclose(hi, [1.75, 0.0, 0.2], rtol=0, atol=1e-15)


def test_positivity_correction_keeps_mean_and_nonnegative_depth():
    rng = np.random.default_rng(3)
    for _ in range(2000):
        blo, bhi = rng.uniform(-1, 1, 2)
        bc = 0.5 * (blo + bhi)
        w0 = bc + abs(rng.standard_normal()) * rng.choice([0.0, 1e-3, 0.3])
        w = [w0 + rng.standard_normal(), w0, w0 + rng.standard_normal()]
        lo, hi = o.reconstruct(w, [0, 0, 0], [0, 0, 0], blo, bhi, 1.3)
        assert abs(0.5 * (lo[0] + hi[0]) - w0) <= 1e-14 * (1 + abs(w0))
        assert lo[0] >= blo - 1e-14 and hi[0] >= bhi - 1e-14


def test_desingularization_eq14():
    eps = 5e-12
    for h in (1e-2, 0.1, 1.0, 30.0):
        for m in (-2.0, 0.3, 5.0):
            assert abs(o.desing(h, m, eps) - m / h) <= 4 * np.finfo(float).eps * abs(m / h)
    assert o.desing(0.0, 1.0, eps) == 0.0
    h0 = eps ** 0.25                      # continuous across h^4 = eps
    assert abs(o.desing(h0 * (1 - 1e-9), 1.0, eps) - o.desing(h0 * (1 + 1e-9), 1.0, eps)) < 1e-6 / h0
    # far below the threshold u -> sqrt(2) h m / sqrt(eps): bounded, vanishing with h
    for h in (1e-6, 1e-8, 1e-10):
        assert abs(o.desing(h, 1.0, eps) / (math.sqrt(2) * h / math.sqrt(eps)) - 1) < 1e-6


def test_central_upwind_flux_consistency_and_wall_zero_mass_flux():
    rng = np.random.default_rng(7)
    for _ in range(200):
        bf = rng.uniform(-2, 0)
        h = rng.uniform(0.05, 3)
        U = np.array([bf + h, rng.standard_normal(), rng.standard_normal()])
        H = o.cu_flux(G, 5e-12, bf, U, U)
        u, v = U[1] / h, U[2] / h
        expect = [U[1], U[1] * u + 0.5 * G * h * h, U[1] * v]   # F(U) of eq. (1)
        np.testing.assert_allclose(H, expect, rtol=1e-12, atol=1e-12)
        mirror = np.array([U[0], -U[1], U[2]])                  # wall ghost: normal flux odd
        Hw = o.cu_flux(G, 5e-12, bf, mirror, U)
        assert Hw[0] == 0.0
    # both sides dry: no flux
    assert np.all(o.cu_flux(G, 5e-12, 0.0, np.zeros(3), np.zeros(3)) == 0.0)


# ----------------------------------------------------- RHS vs eqs. (1)-(3)
def _mms_fields():
    x, y = sp.symbols("x y")
    z = -1.0 - 0.1 * x - 0.05 * y + 0.02 * sp.sin(x)
    eta = 0.03 * sp.sin(0.4 * x + 0.3 * y + 0.2)
    P = 0.2 + 0.1 * x + 0.05 * y ** 2
    Q = -0.1 + 0.08 * y + 0.03 * x ** 2
    return x, y, z, eta, P, Q


def _mms_exact(nx, ny, dx, dy):
    """E, F, G, F*, G* from the governing equations (1)-(3) written out
    symbolically: F, G are every non-time-derivative term of the momentum
    equations moved to the right side, F*, G* the coefficients of the mixed
    time-derivative terms of psi_1, psi_2 (eq. 3 with its first d d_x read as
    d d_y, as symmetry with eq. 2 requires)."""
    x, y, z, eta, P, Q = _mms_fields()
    g, Bs = G, sp.Rational(1, 15)
    d = -z                       # still water level 0, wet everywhere
    h = eta - z
    Fx = sp.Matrix([P, P ** 2 / h + g * h ** 2 / 2, P * Q / h])
    Gy = sp.Matrix([Q, P * Q / h, Q ** 2 / h + g * h ** 2 / 2])
    dd = lambda f, *v: sp.diff(f, *v)
    psi1_eta = (-Bs * g * d ** 3 * (dd(eta, x, 3) + dd(eta, x, y, y))
                - d * dd(d, x) * (2 * Bs * g * d * dd(eta, x, 2) + Bs * g * d * dd(eta, y, 2))
                - d * dd(d, y) * (Bs * g * d * dd(eta, x, y)))
    psi2_eta = (-Bs * g * d ** 3 * (dd(eta, y, 3) + dd(eta, x, x, y))
                - d * dd(d, y) * (2 * Bs * g * d * dd(eta, y, 2) + Bs * g * d * dd(eta, x, 2))
                - d * dd(d, x) * (Bs * g * d * dd(eta, x, y)))
    E = -(dd(Fx[0], x) + dd(Gy[0], y))
    F = -(dd(Fx[1], x) + dd(Gy[1], y)) - g * h * dd(z, x) - psi1_eta
    Gm = -(dd(Fx[2], x) + dd(Gy[2], y)) - g * h * dd(z, y) - psi2_eta
    # mixed time-derivative terms of psi_1 (eq. 2) carry Q_t; of psi_2 carry P_t
    Fs = (Bs + sp.Rational(1, 3)) * d ** 2 * dd(Q, x, y) + d * dd(d, x) * dd(Q, y) / 6 + d * dd(d, y) * dd(Q, x) / 6
    Gs = (Bs + sp.Rational(1, 3)) * d ** 2 * dd(P, x, y) + d * dd(d, y) * dd(P, x) / 6 + d * dd(d, x) * dd(P, y) / 6
    X, Y = np.meshgrid((np.arange(nx) + 0.5) * dx, (np.arange(ny) + 0.5) * dy)
    ev = lambda f: sp.lambdify((x, y), f, "numpy")(X, Y) * np.ones_like(X)
    cx, cy = np.meshgrid(np.arange(nx + 1) * dx, np.arange(ny + 1) * dy)
    zc = sp.lambdify((x, y), z, "numpy")(cx, cy) * np.ones_like(cx)
    return zc, ev(eta), ev(P), ev(Q), {"E": ev(E), "F": ev(F), "G": ev(Gm), "Fs": ev(Fs), "Gs": ev(Gs)}


@pytest.mark.parametrize("term", ["E", "F", "G", "Fs", "Gs"])
def test_rhs_converges_to_governing_equations(term):
    """Manufactured smooth, monotone state on smooth bathymetry: the oracle's
    discrete E, F, G, F*, G* converge at second order to the terms of
    eqs. (1)-(3).  A dropped term, a sign or a wrong index gives an O(1) error."""
    Lx, Ly = 2.4, 1.8
    errs = []
    for n in (24, 48, 96):
        nx, ny = n, int(n * Ly / Lx)
        dx, dy = Lx / nx, Ly / ny
        zc, eta, P, Q, ex = _mms_exact(nx, ny, dx, dy)
        D = o.Domain(nx, ny, dx, dy, 0.01, zc)
        r = D.eval_rhs(eta, P, Q)
        b = n // 6           # stay clear of the mirrored ghost cells at the walls
        s = (slice(b, -b), slice(b, -b))
        scale = np.abs(ex[term][s]).max()
        errs.append(np.abs(r[term][s] - ex[term][s]).max() / scale)
    order = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert errs[-1] < 5e-3, errs
    assert min(order) > 1.7, (errs, order)


# -------------------------------------------------------------- forcing
def test_eckart_limits_and_error_band():
    """Eq. (29) against the exact linear dispersion relation
    omega^2 = g k tanh(k d): exact in the shallow and deep limits, within
    Eckart's few-percent band in between."""
    def k_exact(om, d):
        k = om / math.sqrt(G * d)
        for _ in range(100):
            f = G * k * math.tanh(k * d) - om * om
            fp = G * math.tanh(k * d) + G * k * d / math.cosh(k * d) ** 2
            k -= f / fp
        return k
    d = 1.0
    for om in np.linspace(0.05, 12.0, 60):
        ke, kx = o.eckart_k(om, d), k_exact(om, d)
        assert abs(ke / kx - 1) < 0.055
    assert abs(o.eckart_k(0.01, d) / (0.01 / math.sqrt(G * d)) - 1) < 1e-4      # shallow
    assert abs(o.eckart_k(20.0, d) / (400.0 / G) - 1) < 1e-12                     # deep


def test_sponge_coefficient_eq30():
    Ls = 3.0
    assert o.sponge_gamma(0.0, Ls) == 0.0
    assert abs(o.sponge_gamma(Ls / 2, Ls) - 0.5) < 1e-15
    assert o.sponge_gamma(Ls, Ls) == 1.0 and o.sponge_gamma(2 * Ls, Ls) == 1.0
    g = [o.sponge_gamma(x, Ls) for x in np.linspace(0, Ls, 50)]
    assert np.all(np.diff(g) > 0)


def test_solitary_superposition_eqs33_36():
    """Crest height H at (x0, y0), discharge c_s * eta along theta with
    c_s = sqrt(g (H + d)), half-height where k_s r = acosh(sqrt 2) with
    k_s = sqrt(3 H / (4 d^3)) (the KdV soliton)."""
    nx, ny, dx = 400, 4, 0.05
    D = o.Domain(nx, ny, dx, dx, 0.01, _flat(nx, ny, 0.8))
    H, x0 = 0.12, 10.025
    D.add_solitary(H, 0.0, x0, 0.1)
    w, P, Q = D.state()
    x = (np.arange(nx) + 0.5) * dx
    k = np.argmin(abs(x - x0))
    assert abs(w[0, k] - H) < 1e-12
    cs = math.sqrt(G * (H + 0.8))
    np.testing.assert_allclose(P, cs * w, rtol=1e-13)
    assert np.all(Q == 0.0)
    ks = math.sqrt(3 * H / (4 * 0.8 ** 3))
    xh = x0 + math.acosh(math.sqrt(2.0)) / ks
    assert abs(np.interp(xh, x, w[0]) - H / 2) < 2e-3 * H
