"""ctypes binding of libwavestep.so (C ABI in include/wavestep.h).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  PyTorch provides the device memory (the workspace is a uint8 tensor
owned by the Domain object) and the stream (torch's current stream by
default).  The library must be built (``python -m paper_1611_05984_amd.build``
or ``__graft_entry__.build()``); loading fails with an error otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwavestep.so")

OK, EINVAL, ENOMEM, EHIP, ENOTDD, ENONFINITE, EBUSY = 0, -1, -2, -3, -4, -5, -6
BSNQ, NLSW = 0, 1
FRIC_NONE, FRIC_QUAD, FRIC_MANNING = 0, 1, 2
WEST, EAST, SOUTH, NORTH = 0, 1, 2, 3
SOLID, SPONGE, WAVES = 0, 1, 2
EDIT_WATER, EDIT_TERRAIN = 0, 1
READ_W, READ_H = 0, 1
STATIC_WORKSPACE_BYTES = 80 << 20      # WS_STATIC_WORKSPACE_BYTES of the C header
SOLVE_PCR, SOLVE_THOMAS, SOLVE_LU, SOLVE_LU2, SOLVE_PCR_WAVE = 0, 1, 2, 3, 4
K_PREDICTOR, K_CORRECTOR, K_REDUCE, K_SOLVE, K_EXPAND, K_COUNT = 0, 1, 2, 3, 4, 5
KERNEL_NAMES = ("k_stencil[predictor]", "k_stencil[corrector]", "k_reduce", "reduced_solve", "k_expand")


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("n_corr", C.c_int32),
                ("model", C.c_int32), ("friction", C.c_int32), ("fstar_extrap", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dt", C.c_double), ("g", C.c_double),
                ("still_water", C.c_double), ("Bcoef", C.c_double), ("theta", C.c_double),
                ("eps", C.c_double), ("friction_coef", C.c_double)]


class Boundary(C.Structure):
    _fields_ = [("type", C.c_int32), ("width_cells", C.c_int32), ("n_comp", C.c_int32),
                ("reserved", C.c_int32), ("amp", C.POINTER(C.c_double)),
                ("period", C.POINTER(C.c_double)), ("theta_rad", C.POINTER(C.c_double)),
                ("phase", C.POINTER(C.c_double)), ("ref_depth", C.c_double),
                ("sponge_reflect", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("stencil_rows", C.c_int32), ("pcr_threads", C.c_int32), ("solver", C.c_int32),
                ("corrector_rows", C.c_int32), ("reserved", C.c_int32 * 4)]


class WaveStepError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("wavestep status %d: %s" % (status, msg))
        self.status = status


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libwavestep.so is not built (%s); run paper_1611_05984_amd/build.py"
                               % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, f64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
        sigs = {
            "ws_grid_defaults": (None, [C.POINTER(Grid), i32, i32]),
            "ws_workspace_bytes": (sz, [C.POINTER(Grid)]),
            "ws_domain_init": (C.c_int, [C.POINTER(Grid), vp, vp, sz, vp, C.POINTER(vp)]),
            "ws_domain_init_static": (C.c_int, [C.POINTER(Grid), vp, vp, C.POINTER(vp)]),
            "ws_domain_destroy": (C.c_int, [vp]),
            "ws_set_boundary": (C.c_int, [vp, i32, C.POINTER(Boundary)]),
            "ws_set_state": (C.c_int, [vp, vp, vp, vp, i32, f64, vp]),
            "ws_add_solitary": (C.c_int, [vp, f64, f64, f64, f64, vp]),
            "ws_advance": (C.c_int, [vp, i64, vp]),
            "ws_read": (C.c_int, [vp, i32, vp, vp, vp, i32, vp]),
            "ws_read_gauges": (C.c_int, [vp, i32, vp, vp, vp]),
            "ws_apply_edit": (C.c_int, [vp, i32, f64, f64, f64, f64, vp]),
            "ws_query": (C.c_int, [vp, vp, C.POINTER(i64), C.POINTER(f64), C.POINTER(i32)]),
            "ws_last_error": (C.c_char_p, []),
            "ws_profile_enable": (C.c_int, [vp, i32]),
            "ws_profile_collect": (C.c_int, [vp, vp, C.POINTER(f64), C.POINTER(i64), i32]),
            "ws_snapshot_bytes": (sz, [vp]),
            "ws_snapshot_bytes_grid": (sz, [C.POINTER(Grid)]),
            "ws_snapshot": (C.c_int, [vp, vp, sz, vp]),
            "ws_restore": (C.c_int, [vp, vp, sz, vp]),
            "ws_get_tuning": (C.c_int, [vp, C.POINTER(Tuning)]),
            "ws_set_tuning": (C.c_int, [vp, C.POINTER(Tuning)]),
            "ws_batch_set_tuning": (C.c_int, [vp, C.POINTER(Tuning)]),
            "ws_tune": (C.c_int, [vp, C.c_char_p, vp, C.POINTER(Tuning)]),
            "ws_batch_tune": (C.c_int, [vp, vp, C.POINTER(Tuning)]),
            "ws_batch_workspace_bytes": (sz, [i32]),
            "ws_batch_create": (C.c_int, [i32, vp, sz, C.POINTER(vp)]),
            "ws_batch_destroy": (C.c_int, [vp]),
            "ws_batch_attach": (C.c_int, [vp, vp, C.POINTER(i32)]),
            "ws_batch_detach": (C.c_int, [vp, i32]),
            "ws_batch_advance": (C.c_int, [vp, i64, vp]),
            "ws_batch_set_stop": (C.c_int, [vp, i32, i64]),
            "ws_batch_status": (C.c_int, [vp, i32, C.POINTER(i64), C.POINTER(f64), C.POINTER(i32)]),
            "ws_batch_sync": (C.c_int, [vp, vp]),
            "ws_set_corrector_tolerance": (C.c_int, [vp, f64, f64]),
            "ws_update_grid": (C.c_int, [vp, C.POINTER(Grid), vp]),
            "ws_corrector_stats": (C.c_int, [vp, C.POINTER(i32), C.POINTER(i64), C.POINTER(f64),
                                             C.POINTER(f64)]),
        }
        for name, (res, args) in sigs.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status, what=""):
    if status != OK:
        raise WaveStepError(status, (what + ": " if what else "") +
                            lib().ws_last_error().decode(errors="replace"))


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


def grid(nx, ny, dx, dy, dt, **kw) -> Grid:
    g = Grid()
    lib().ws_grid_defaults(C.byref(g), int(nx), int(ny))
    g.dx, g.dy, g.dt = float(dx), float(dy), float(dt)
    for k, v in kw.items():
        setattr(g, k, v)
    return g


def workspace_bytes(g: Grid) -> int:
    return int(lib().ws_workspace_bytes(C.byref(g)))


def snapshot_bytes(g: Grid) -> int:
    return int(lib().ws_snapshot_bytes_grid(C.byref(g)))


class Domain:
    """One domain resident on the GPU.

    z: bottom elevation at the (ny+1) x (nx+1) cell corners (numpy or torch).
    Fields are exchanged as float32 CUDA tensors of shape (ny, nx).
    """

    def __init__(self, nx, ny, dx, dy, dt, z, device="cuda", stream=None, static_workspace=False,
                 **params):
        """static_workspace: use the library's static device array as the
        workspace (ws_domain_init_static: one such domain per device, grids up
        to STATIC_WORKSPACE_BYTES) instead of a tensor allocated here."""
        import torch
        self.device = torch.device(device)
        self.g = grid(nx, ny, dx, dy, dt, **params)
        self.nx, self.ny = int(nx), int(ny)
        nbytes = workspace_bytes(self.g)
        if nbytes == 0:
            raise WaveStepError(EINVAL, "invalid grid parameters")
        zt = torch.as_tensor(np.asarray(z) if not torch.is_tensor(z) else z,
                             dtype=torch.float32).to(self.device).contiguous()
        if zt.numel() != (ny + 1) * (nx + 1):
            raise ValueError("z must hold (ny+1)*(nx+1) corner values")
        h = C.c_void_p()
        if static_workspace:
            self.workspace = None
            with torch.cuda.device(self.device):
                _check(lib().ws_domain_init_static(C.byref(self.g), _dptr(zt), _stream(stream),
                                                   C.byref(h)), "ws_domain_init_static")
        else:
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            _check(lib().ws_domain_init(C.byref(self.g), _dptr(zt), _dptr(self.workspace), nbytes,
                                        _stream(stream), C.byref(h)), "ws_domain_init")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().ws_domain_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_boundary(self, side, kind, width=2, amp=(), period=(), theta=(), phase=None,
                     ref_depth=0.0, sponge_reflect=0.0):
        n = len(amp)
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in
                (amp, period, theta, phase if phase is not None else np.zeros(n))]
        ptrs = [a.ctypes.data_as(C.POINTER(C.c_double)) for a in arrs]
        b = Boundary(int(kind), int(width), n, 0, *ptrs, float(ref_depth), float(sponge_reflect))
        _check(lib().ws_set_boundary(self._h, int(side), C.byref(b)), "ws_set_boundary")

    def set_state(self, w, P, Q, t=0.0, stream=None):
        import torch
        ts = [torch.as_tensor(a, dtype=torch.float32).to(self.device).contiguous() for a in (w, P, Q)]
        for a in ts:
            assert a.shape == (self.ny, self.nx), a.shape
        _check(lib().ws_set_state(self._h, *[_dptr(a) for a in ts], self.nx, float(t),
                                  _stream(stream)), "ws_set_state")
        self._keep = ts   # keep the inputs alive until the copy kernel has run

    def add_solitary(self, H, theta, x0, y0, stream=None):
        _check(lib().ws_add_solitary(self._h, H, theta, x0, y0, _stream(stream)), "ws_add_solitary")

    def advance(self, n, stream=None):
        _check(lib().ws_advance(self._h, int(n), _stream(stream)), "ws_advance")

    def read(self, what=READ_W, stream=None):
        import torch
        out = [torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device)
               for _ in range(3)]
        _check(lib().ws_read(self._h, int(what), *[_dptr(a) for a in out], self.nx,
                             _stream(stream)), "ws_read")
        return tuple(out)

    def state_numpy(self, what=READ_W):
        import torch
        out = self.read(what)
        torch.cuda.current_stream().synchronize()
        return tuple(a.cpu().numpy() for a in out)

    def gauges(self, ij, out=None, stream=None):
        """State at gauge cells: ij is an int32 CUDA tensor of shape (n, 2)
        holding (i, j) pairs; writes (w, h, P, Q) per gauge into `out` (a
        float32 CUDA tensor of n * 4 elements, e.g. a row of a time-series
        buffer; allocated when None) without synchronizing, and returns it."""
        import torch
        assert ij.dtype == torch.int32 and ij.is_cuda and ij.is_contiguous() and ij.shape[-1] == 2
        n = ij.numel() // 2
        if out is None:
            out = torch.empty((n, 4), dtype=torch.float32, device=self.device)
        assert out.dtype == torch.float32 and out.is_contiguous() and out.numel() == 4 * n
        _check(lib().ws_read_gauges(self._h, n, _dptr(ij), _dptr(out), _stream(stream)), "ws_read_gauges")
        return out

    def apply_edit(self, kind, x0, y0, amp, sigma, stream=None):
        """Returns the status (0, or ENOTDD for a rejected terrain edit)."""
        st = lib().ws_apply_edit(self._h, int(kind), x0, y0, amp, sigma, _stream(stream))
        if st not in (OK, ENOTDD):
            _check(st, "ws_apply_edit")
        return st

    def update(self, stream=None, **params):
        """Change parameters of the running domain (model, friction,
        friction_coef, Bcoef, theta, eps, g, fstar_extrap, dt); the grid
        shape, n_corr and still_water are fixed.  A new dt restarts the
        multistep history."""
        g = Grid.from_buffer_copy(self.g)
        for k, v in params.items():
            if not hasattr(g, k):
                raise ValueError("unknown parameter %s" % k)
            setattr(g, k, v)
        _check(lib().ws_update_grid(self._h, C.byref(g), _stream(stream)), "ws_update_grid")
        self.g = g

    def set_corrector_tolerance(self, tol_w, tol_pq):
        """Iterate the corrector until the largest change of w is within
        tol_w (m) and that of P, Q within tol_pq (m^2/s), at most n_corr
        times; tol_w <= 0 restores the fixed count."""
        _check(lib().ws_set_corrector_tolerance(self._h, float(tol_w), float(tol_pq)),
               "ws_set_corrector_tolerance")

    def corrector_stats(self):
        """(correctors of the last step, total since the tolerance was set,
        change of w and of P, Q after the last corrector)."""
        last, total, dw, dpq = C.c_int32(0), C.c_int64(0), C.c_double(0), C.c_double(0)
        _check(lib().ws_corrector_stats(self._h, C.byref(last), C.byref(total), C.byref(dw),
                                        C.byref(dpq)), "ws_corrector_stats")
        return last.value, total.value, dw.value, dpq.value

    def query(self, stream=None):
        step, t, health = C.c_int64(), C.c_double(), C.c_int32()
        st = lib().ws_query(self._h, _stream(stream), C.byref(step), C.byref(t), C.byref(health))
        if st not in (OK, ENONFINITE):
            _check(st, "ws_query")
        return step.value, t.value, health.value

    def snapshot(self, stream=None, out=None):
        """Device snapshot (uint8 tensor) of state, history, bathymetry, step
        and time; into `out` when it is given and large enough."""
        import torch
        n = int(lib().ws_snapshot_bytes(self._h))
        buf = out if out is not None and out.numel() >= n else torch.empty(n, dtype=torch.uint8,
                                                                            device=self.device)
        _check(lib().ws_snapshot(self._h, _dptr(buf), n, _stream(stream)), "ws_snapshot")
        return buf

    def restore(self, buf, stream=None):
        _check(lib().ws_restore(self._h, _dptr(buf), buf.numel(), _stream(stream)), "ws_restore")

    def tuning(self):
        """(stencil rows, PCR threads, reduced solver, corrector-pass stencil
        rows or 0 for the same as the first) of this domain."""
        t = Tuning()
        _check(lib().ws_get_tuning(self._h, C.byref(t)), "ws_get_tuning")
        return t.stencil_rows, t.pcr_threads, t.solver, t.corrector_rows

    def set_tuning(self, stencil_rows, pcr_threads, solver=SOLVE_PCR, corrector_rows=0):
        t = Tuning(int(stencil_rows), int(pcr_threads), int(solver), int(corrector_rows))
        _check(lib().ws_set_tuning(self._h, C.byref(t)), "ws_set_tuning")

    def tune(self, cache_path=None, stream=None):
        """Run the autotuner on this grid (or read its cache); returns the choice."""
        t = Tuning()
        path = cache_path.encode() if cache_path else None
        _check(lib().ws_tune(self._h, path, _stream(stream), C.byref(t)), "ws_tune")
        return t.stencil_rows, t.pcr_threads, t.solver, t.corrector_rows

    def profile(self, on=True):
        _check(lib().ws_profile_enable(self._h, 1 if on else 0), "ws_profile_enable")

    def profile_collect(self, stream=None):
        """{kernel class: (summed ms, launches)} since the last collection."""
        ms = (C.c_double * K_COUNT)()
        n = (C.c_int64 * K_COUNT)()
        _check(lib().ws_profile_collect(self._h, _stream(stream), ms, n, K_COUNT), "ws_profile_collect")
        return {KERNEL_NAMES[k]: (ms[k], n[k]) for k in range(K_COUNT)}


class Batch:
    """Many domains advanced together: one launch per phase for all of them,
    one step captured as a HIP graph on the batch's own stream and replayed.

    Attached domains are advanced only through the batch; after ``advance``
    call ``sync`` before using them individually (read, query, edits, ...).
    Work the caller queued on its current stream before ``advance`` (states,
    edits) is ordered before the batch's steps.
    """

    def __init__(self, max_domains, device="cuda"):
        import torch
        self.device = torch.device(device)
        self.max = int(max_domains)
        nbytes = int(lib().ws_batch_workspace_bytes(self.max))
        if nbytes == 0:
            raise WaveStepError(EINVAL, "invalid batch size")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.Stream(device=self.device)   # default priority
        h = C.c_void_p()
        _check(lib().ws_batch_create(self.max, _dptr(self.workspace), nbytes, C.byref(h)),
               "ws_batch_create")
        self._h = h
        self.domains = {}

    def attach(self, dom: Domain) -> int:
        slot = C.c_int32()
        _check(lib().ws_batch_attach(self._h, dom._h, C.byref(slot)), "ws_batch_attach")
        self.domains[slot.value] = dom
        return slot.value

    def detach(self, slot: int):
        _check(lib().ws_batch_detach(self._h, int(slot)), "ws_batch_detach")
        return self.domains.pop(int(slot))

    def set_tuning(self, stencil_rows, pcr_threads, solver=SOLVE_PCR, corrector_rows=0):
        t = Tuning(int(stencil_rows), int(pcr_threads), int(solver), int(corrector_rows))
        _check(lib().ws_batch_set_tuning(self._h, C.byref(t)), "ws_batch_set_tuning")

    def tune(self):
        """Run the batch autotuner on the attached domains; returns the choice."""
        t = Tuning()
        _check(lib().ws_batch_tune(self._h, C.c_void_p(self.stream.cuda_stream), C.byref(t)), "ws_batch_tune")
        return t.stencil_rows, t.pcr_threads, t.solver, t.corrector_rows

    def set_stop(self, slot, stop_step):
        """Do not advance the domain in `slot` past step `stop_step` (-1: no limit)."""
        _check(lib().ws_batch_set_stop(self._h, int(slot), int(stop_step)), "ws_batch_set_stop")

    def advance(self, n):
        import torch
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        _check(lib().ws_batch_advance(self._h, int(n), C.c_void_p(self.stream.cuda_stream)),
               "ws_batch_advance")

    def sync(self):
        _check(lib().ws_batch_sync(self._h, C.c_void_p(self.stream.cuda_stream)), "ws_batch_sync")

    def status(self, slot):
        """(step, t, health) of the domain in `slot` as of the last sync."""
        step, t, health = C.c_int64(), C.c_double(), C.c_int32()
        _check(lib().ws_batch_status(self._h, int(slot), C.byref(step), C.byref(t), C.byref(health)),
               "ws_batch_status")
        return step.value, t.value, health.value

    def close(self):
        if getattr(self, "_h", None):
            lib().ws_batch_destroy(self._h)
            self._h = None
            self.domains = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
