"""FP64 CPU oracle for the extended-Boussinesq time step (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
import this package.  It wraps ``liboracle.so`` (built from
``wave_oracle.c`` by ``oracle/build.py``) with ctypes and numpy; it shares no
code with the GPU library.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

BSNQ, NLSW = 0, 1
FRIC_NONE, FRIC_QUAD, FRIC_MANNING = 0, 1, 2
WEST, EAST, SOUTH, NORTH = 0, 1, 2, 3
SOLID, SPONGE, WAVES = 0, 1, 2
EDIT_WATER, EDIT_TERRAIN = 0, 1


class Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("n_corr", C.c_int32),
                ("model", C.c_int32), ("friction", C.c_int32), ("fstar_extrap", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dt", C.c_double),
                ("g", C.c_double), ("ws", C.c_double), ("Bdisp", C.c_double),
                ("theta", C.c_double), ("eps", C.c_double), ("fcoef", C.c_double)]


_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def lib():
    """Load (building on first use if absent) the oracle shared library."""
    global _lib
    if _lib is None:
        path = _build.LIB
        if os.environ.get("WAVESTEP_ORACLE_SANITIZE") == "1":
            path = _build.SAN_LIB
            if not os.path.exists(path):
                _build.build(sanitize=True)
        elif not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        L.or_create.restype = C.c_void_p
        L.or_create.argtypes = [C.POINTER(Params), _dp]
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_set_boundary.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int,
                                      _dp, _dp, _dp, _dp, C.c_double]
        L.or_set_sponge_reflect.argtypes = [C.c_void_p, C.c_int, C.c_double]
        L.or_set_corrector_tolerance.argtypes = [C.c_void_p, C.c_double, C.c_double]
        L.or_set_n_corr.argtypes = [C.c_void_p, C.c_int]
        L.or_update_params.argtypes = [C.c_void_p, C.POINTER(Params)]
        L.or_corrector_stats.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int64),
                                         _dp, _dp]
        L.or_set_state.argtypes = [C.c_void_p, _dp, _dp, _dp, C.c_double]
        L.or_get_state.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.or_get_bathy.argtypes = [C.c_void_p, _dp, _dp]
        L.or_add_solitary.argtypes = [C.c_void_p] + [C.c_double] * 4
        L.or_apply_edit.argtypes = [C.c_void_p, C.c_int] + [C.c_double] * 4
        L.or_advance.argtypes = [C.c_void_p, C.c_int64]
        L.or_get_step.restype = C.c_int64
        L.or_get_step.argtypes = [C.c_void_p]
        L.or_get_time.restype = C.c_double
        L.or_get_time.argtypes = [C.c_void_p]
        L.or_diag_dominant.argtypes = [C.c_void_p]
        L.or_eval_rhs.argtypes = [C.c_void_p, _dp, _dp, _dp, C.c_double] + [_dp] * 7
        L.or_set_threads.restype = C.c_int
        L.or_set_threads.argtypes = [C.c_int]
        L.or_set_clock.argtypes = [C.c_void_p, C.c_int64, C.c_double]
        L.or_set_history.argtypes = [C.c_void_p, C.c_int] + [_dp] * 5
        L.or_eval_solve.argtypes = [C.c_void_p, _dp, _dp, C.c_double, _dp, _dp]
        L.or_thomas.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _dp]
        L.or_eckart_k.restype = C.c_double
        L.or_eckart_k.argtypes = [C.c_double] * 3
        L.or_minmod3.restype = C.c_double
        L.or_minmod3.argtypes = [C.c_double] * 3
        L.or_desing.restype = C.c_double
        L.or_desing.argtypes = [C.c_double] * 3
        L.or_sponge_gamma.restype = C.c_double
        L.or_sponge_gamma.argtypes = [C.c_double] * 2
        L.or_cu_flux.argtypes = [C.c_double, C.c_double, C.c_double, _dp, _dp, _dp]
        L.or_reconstruct.argtypes = [_dp, _dp, _dp, C.c_double, C.c_double, C.c_double, _dp]
        _lib = L
    return _lib


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None:
        assert a.size == n, (a.shape, n)
    return a


class Domain:
    """One rectangular domain advanced by the FP64 oracle.

    ``z`` holds the bathymetry at cell corners, shape (ny+1, nx+1), elevation
    above the datum (negative under still water when w_s = 0).  Fields are
    returned as (ny, nx) arrays, x fastest.
    """

    def __init__(self, nx, ny, dx, dy, dt, z, *, g=9.81, ws=0.0, B=1.0 / 15.0,
                 theta=1.3, eps=5e-12, n_corr=2, model=BSNQ, friction=FRIC_NONE,
                 fcoef=0.0, fstar_extrap=1):
        self.nx, self.ny = int(nx), int(ny)
        self.p = Params(nx=nx, ny=ny, n_corr=n_corr, model=model, friction=friction,
                        fstar_extrap=fstar_extrap,
                        dx=dx, dy=dy, dt=dt, g=g, ws=ws, Bdisp=B, theta=theta, eps=eps,
                        fcoef=fcoef)
        z = _f64(z, (ny + 1) * (nx + 1))
        h = lib().or_create(C.byref(self.p), z)
        if not h:
            raise ValueError("oracle: invalid grid parameters")
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_destroy(self._h)
            self._h = None

    def set_boundary(self, side, btype, width=2, amp=(), period=(), theta=(), phase=None,
                     ref_depth=0.0, sponge_reflect=0.0):
        n = len(amp)
        ph = np.zeros(n) if phase is None else phase
        z = np.zeros(1)
        rc = lib().or_set_boundary(self._h, side, btype, int(width), n,
                                   _f64(amp) if n else z, _f64(period) if n else z,
                                   _f64(theta) if n else z, _f64(ph) if n else z,
                                   float(ref_depth))
        if rc == 0 and btype == SPONGE:
            rc = lib().or_set_sponge_reflect(self._h, side, float(sponge_reflect))
        if rc:
            raise ValueError("oracle: bad boundary")

    def set_corrector_tolerance(self, tol_w, tol_pq):
        """Iterate the corrector until the largest change of w is within
        tol_w and that of P, Q within tol_pq (at most n_corr times); tol_w
        <= 0: the fixed count."""
        if lib().or_set_corrector_tolerance(self._h, float(tol_w), float(tol_pq)):
            raise ValueError("oracle: bad tolerance")

    def update(self, **kw):
        """Change parameters of the running domain (fields of Params: model,
        friction, fcoef, Bdisp, theta, eps, g, fstar_extrap, dt); a new dt
        restarts the multistep history.  ValueError if refused."""
        p = Params.from_buffer_copy(self.p)
        for k, v in kw.items():
            if not hasattr(p, k):
                raise ValueError("unknown parameter %s" % k)
            setattr(p, k, v)
        rc = lib().or_update_params(self._h, C.byref(p))
        if rc:
            raise ValueError("oracle: parameter update refused (%d)" % rc)
        self.p = p

    def set_n_corr(self, n_corr):
        """Corrector count of the following steps (the cap in tolerance mode)."""
        if lib().or_set_n_corr(self._h, int(n_corr)):
            raise ValueError("oracle: bad corrector count")

    def corrector_stats(self):
        """(correctors of the last step, total since the tolerance was set,
        change of w and of P, Q after the last corrector)."""
        last, total = C.c_int(0), C.c_int64(0)
        dw, dpq = np.zeros(1), np.zeros(1)
        lib().or_corrector_stats(self._h, C.byref(last), C.byref(total), _f64(dw), _f64(dpq))
        return last.value, total.value, float(dw[0]), float(dpq[0])

    def set_state(self, w, P, Q, t=0.0):
        n = self.nx * self.ny
        lib().or_set_state(self._h, _f64(w, n), _f64(P, n), _f64(Q, n), float(t))

    def state(self):
        shp = (self.ny, self.nx)
        w, P, Q = np.empty(shp), np.empty(shp), np.empty(shp)
        lib().or_get_state(self._h, w, P, Q)
        return w, P, Q

    def bathy(self):
        b, d = np.empty((self.ny, self.nx)), np.empty((self.ny, self.nx))
        lib().or_get_bathy(self._h, b, d)
        return b, d

    def add_solitary(self, H, theta, x0, y0):
        if lib().or_add_solitary(self._h, H, theta, x0, y0):
            raise ValueError("oracle: solitary wave needs positive depth at its crest")

    def apply_edit(self, kind, x0, y0, amp, sigma):
        return lib().or_apply_edit(self._h, kind, x0, y0, amp, sigma)

    def advance(self, n):
        return lib().or_advance(self._h, int(n))

    @property
    def step(self):
        return lib().or_get_step(self._h)

    @property
    def t(self):
        return lib().or_get_time(self._h)

    def diag_dominant(self):
        return bool(lib().or_diag_dominant(self._h))

    def set_clock(self, step, t):
        """Set the count of completed steps and the time (test access)."""
        if lib().or_set_clock(self._h, int(step), float(t)):
            raise ValueError("oracle: bad step count")

    def set_history(self, lag, E, F, G, Fs=None, Gs=None):
        """Load the right-hand side of level n-lag (lag 1 or 2, relative to
        the next step) into the multistep history (test access); arrays of
        shape (ny, nx), None for zeros."""
        n = self.nx * self.ny
        z = np.zeros(n)
        arrs = [z if a is None else _f64(a, n) for a in (E, F, G, Fs, Gs)]
        if lib().or_set_history(self._h, int(lag), *arrs):
            raise ValueError("oracle: bad history lag")

    def eval_rhs(self, w, P, Q, t=0.0):
        """(E, F, G, F*, G*, U*, V*) of an interior state, ghosts at time t."""
        n = self.nx * self.ny
        outs = [np.empty((self.ny, self.nx)) for _ in range(7)]
        lib().or_eval_rhs(self._h, _f64(w, n), _f64(P, n), _f64(Q, n), float(t), *outs)
        return dict(zip(("E", "F", "G", "Fs", "Gs", "U", "V"), outs))

    def eval_solve(self, U, V, t=0.0):
        n = self.nx * self.ny
        P, Q = np.empty((self.ny, self.nx)), np.empty((self.ny, self.nx))
        lib().or_eval_solve(self._h, _f64(U, n), _f64(V, n), float(t), P, Q)
        return P, Q


def set_threads(n=0):
    """OpenMP threads of the oracle's loops (n <= 0: unchanged); returns the
    number in use."""
    return int(lib().or_set_threads(int(n)))


def thomas(a, b, c, r):
    n = len(b)
    x = np.empty(n)
    lib().or_thomas(n, _f64(a, n), _f64(b, n), _f64(c, n), _f64(r, n), x)
    return x


def eckart_k(omega, d, g=9.81):
    return lib().or_eckart_k(omega, d, g)


def minmod3(a, b, c):
    return lib().or_minmod3(a, b, c)


def desing(h, m, eps=5e-12):
    return lib().or_desing(h, m, eps)


def sponge_gamma(dist, Ls):
    return lib().or_sponge_gamma(dist, Ls)


def cu_flux(g, eps, bf, L, R):
    H = np.empty(3)
    lib().or_cu_flux(g, eps, bf, _f64(L, 3), _f64(R, 3), H)
    return H


def reconstruct(w, n, t, b_lo, b_hi, theta=1.3):
    """Face values ((w, n, t) at the low face, (w, n, t) at the high face)."""
    out = np.empty(6)
    lib().or_reconstruct(_f64(w, 3), _f64(n, 3), _f64(t, 3), b_lo, b_hi, theta, out)
    return out[:3], out[3:]
