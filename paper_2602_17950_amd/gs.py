"""ctypes binding of ``libgs.so`` (the C ABI declared in include/gs.h).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels. PyTorch provides device memory and streams for the device-pointer
entry points. Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgs.so")

GS_OK, GS_EINVAL, GS_ENOMEM, GS_EDEVICE, GS_ENONFINITE, GS_ECANCELED = 0, -1, -2, -3, -4, -5
GS_WMAXITER, GS_WSTAGNATED, GS_WEXISTENCE = 1, 2, 3
GS_PENDING = 16
GS_STOP_ENERGY, GS_STOP_RESIDUAL, GS_STOP_EITHER, GS_STOP_WAVEFN = 0, 1, 2, 3
GS_PC_COMBINED, GS_PC_KINETIC, GS_PC_POTENTIAL = 0, 1, 2
GS_LS_ALG2, GS_LS_EXACT = 0, 1
GS_FP64, GS_FP32, GS_MIXED = 0, 1, 2
GS_NYQ_KEEP, GS_NYQ_ZERO = 0, 1

EXPORTS = ("gs_create", "gs_destroy", "gs_default_options", "gs_footprint_bytes", "gs_solve",
           "gs_solve_device", "gs_fft", "gs_hamiltonian", "gs_precondition", "gs_kernel_timer_start",
           "gs_kernel_timer_read", "gs_last_error", "gs_set_hbm_budget", "gs_memory_stats",
           "gs_batch_solve", "gs_submit", "gs_progress", "gs_poll", "gs_wait", "gs_cancel",
           "gs_interpolate", "gs_existence_check", "gs_fft_noalloc", "gs_set_autotune",
           "gs_autotune_report")

KERNEL_KINDS = {"hl_fwd": 0, "hl_mid": 1, "hl_inv": 2, "pre_fwd": 3, "pre_mid": 4, "pre_inv": 5,
                "eval": 6, "resid": 7, "lsred": 9, "hl_fwd2": 10, "hl_inv2": 11, "ctrl": 12}


class GsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gs error {code}: {msg}")
        self.code = code


class gs_grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("L", C.c_double * 3)]


class gs_trap(C.Structure):
    _fields_ = [("g", C.c_double * 3), ("q2", C.c_double), ("q4", C.c_double),
                ("V", C.POINTER(C.c_double))]


class gs_params(C.Structure):
    _fields_ = [("omega", C.c_double), ("gamma", C.c_double), ("c0", C.c_double), ("c1", C.c_double)]


class gs_options(C.Structure):
    _fields_ = [("stop_kind", C.c_int), ("tol", C.c_double), ("max_iter", C.c_int),
                ("precision", C.c_int), ("switch_resid", C.c_double), ("fp32_max_iter", C.c_int),
                ("stall_window", C.c_int), ("theta_trial", C.c_double), ("sigma", C.c_double),
                ("max_backtrack", C.c_int), ("check_every", C.c_int), ("cm_levels", C.c_int),
                ("dir_precision", C.c_int), ("precond", C.c_int), ("line_search", C.c_int),
                ("nyquist_odd", C.c_int)]


class gs_result(C.Structure):
    _fields_ = [("E", C.c_double), ("mu", C.c_double), ("mu_comp", C.c_double * 3),
                ("norm_comp", C.c_double * 3), ("e_kin", C.c_double), ("e_pot", C.c_double),
                ("e_rot", C.c_double), ("e_spin", C.c_double), ("e_soc", C.c_double),
                ("virial", C.c_double), ("resid_inf", C.c_double), ("dE_last", C.c_double),
                ("iters", C.c_int), ("iters_fp32", C.c_int), ("backtracks", C.c_int),
                ("resets", C.c_int), ("status", C.c_int), ("wall_s", C.c_double),
                ("iters_coarse", C.c_int), ("dphi_inf", C.c_double)]

    def to_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if isinstance(v, C.Array) else v
        return d


class gs_request(C.Structure):
    _fields_ = [("grid", gs_grid), ("trap", gs_trap), ("params", gs_params), ("options", gs_options),
                ("d_psi0", C.c_void_p), ("d_psi_out", C.c_void_p)]


_lib = None


def load():
    """Load libgs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(or python -m paper_2602_17950_amd.build)")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    lib.gs_create.argtypes = [C.POINTER(vp), C.c_int]
    lib.gs_destroy.argtypes = [vp]
    lib.gs_destroy.restype = None
    lib.gs_default_options.argtypes = [C.POINTER(gs_options)]
    lib.gs_default_options.restype = None
    lib.gs_footprint_bytes.argtypes = [C.POINTER(gs_grid), C.POINTER(gs_options)]
    lib.gs_footprint_bytes.restype = C.c_size_t
    lib.gs_solve.argtypes = [vp, C.POINTER(gs_grid), C.POINTER(gs_trap), C.POINTER(gs_params),
                             C.POINTER(gs_options), vp, vp, C.POINTER(gs_result)]
    lib.gs_solve_device.argtypes = [vp, C.POINTER(gs_grid), C.POINTER(gs_trap), C.POINTER(gs_params),
                                    C.POINTER(gs_options), vp, vp, C.POINTER(gs_result), vp]
    lib.gs_fft.argtypes = [vp, C.POINTER(gs_grid), C.c_int, C.c_int, vp, vp, vp]
    lib.gs_fft_noalloc.argtypes = [vp, C.POINTER(gs_grid), C.c_int, C.c_int, vp, vp, vp]
    lib.gs_hamiltonian.argtypes = [vp, C.POINTER(gs_grid), C.POINTER(gs_trap), C.POINTER(gs_params),
                                   C.c_int, vp, vp, C.POINTER(gs_result), vp]
    lib.gs_precondition.argtypes = [vp, C.POINTER(gs_grid), C.POINTER(gs_trap), C.POINTER(gs_params),
                                    C.c_int, vp, vp, vp, vp]
    lib.gs_kernel_timer_start.argtypes = [vp, C.c_int]
    lib.gs_kernel_timer_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                         C.POINTER(C.c_longlong)]
    lib.gs_last_error.restype = C.c_char_p
    lib.gs_set_hbm_budget.argtypes = [vp, C.c_size_t]
    lib.gs_memory_stats.argtypes = [vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
    lib.gs_batch_solve.argtypes = [vp, C.c_int, C.POINTER(gs_request), C.POINTER(gs_result)]
    lib.gs_submit.argtypes = [vp, C.POINTER(gs_request), C.POINTER(C.c_uint64)]
    lib.gs_progress.argtypes = [vp, C.c_int]
    lib.gs_poll.argtypes = [vp, C.c_uint64, C.POINTER(gs_result)]
    lib.gs_wait.argtypes = [vp, C.c_uint64, C.POINTER(gs_result)]
    lib.gs_cancel.argtypes = [vp, C.c_uint64]
    lib.gs_interpolate.argtypes = [vp, C.POINTER(gs_grid), vp, C.POINTER(gs_grid), vp, vp]
    lib.gs_existence_check.argtypes = [C.POINTER(gs_grid), C.POINTER(gs_trap), C.POINTER(gs_params)]
    lib.gs_set_autotune.argtypes = [vp, C.c_int]
    lib.gs_autotune_report.argtypes = [vp]
    lib.gs_autotune_report.restype = C.c_char_p
    _lib = lib
    return lib


def last_error() -> str:
    return load().gs_last_error().decode()


def _check(rc):
    if rc < 0:
        raise GsError(rc, last_error())
    return rc


def make_grid(dim, n, L) -> gs_grid:
    g = gs_grid()
    g.dim = dim
    for a in range(3):
        g.n[a] = int(n[a]) if a < dim else 1
        g.L[a] = float(L[a]) if a < dim else 1.0
    return g


def grid_of(pb) -> gs_grid:
    return make_grid(pb.dim, pb.n, pb.L)


def trap_of(pb, V=None):
    t = gs_trap()
    for a in range(3):
        t.g[a] = float(pb.g[a]) if a < len(pb.g) else 1.0
    t.q2, t.q4 = float(pb.q2), float(pb.q4)
    keep = None
    if V is not None:
        keep = np.ascontiguousarray(V, dtype=np.float64)
        t.V = keep.ctypes.data_as(C.POINTER(C.c_double))
    return t, keep


def params_of(pb) -> gs_params:
    return gs_params(pb.omega, pb.gamma, pb.c0, pb.c1)


def default_options(**kw) -> gs_options:
    o = gs_options()
    load().gs_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(f"gs_options has no field {k}")
        setattr(o, k, v)
    return o


def existence_check(pb) -> int:
    """GS_OK or GS_WEXISTENCE: whether pb satisfies the hypotheses of the
    existence theorem of Sec. 2.1 (host-side check, no device needed)."""
    g, (t, keep), p = grid_of(pb), trap_of(pb), params_of(pb)
    return _check(load().gs_existence_check(C.byref(g), C.byref(t), C.byref(p)))


def footprint_bytes(pb, precision=GS_FP64, **kw) -> int:
    """Device bytes of a solve of pb (0 for an invalid grid or options); kw: other option fields."""
    g = grid_of(pb)
    o = default_options(precision=precision, **kw)
    return int(load().gs_footprint_bytes(C.byref(g), C.byref(o)))


def make_request(pb, psi0, out, options: gs_options | None = None, V=None):
    """gs_request for problem pb with device tensors psi0 (or None) and out
    (complex128, shape (3,)+grid). Returns (request, keep-alive object)."""
    q = gs_request()
    q.grid = grid_of(pb)
    t, keep = trap_of(pb, V)
    q.trap = t
    q.params = params_of(pb)
    q.options = options or default_options()
    q.d_psi0 = None if psi0 is None else psi0.data_ptr()
    q.d_psi_out = out.data_ptr()
    return q, keep


def _result(rc, res):
    """Result dict of a completed request; raises for a failed call (as opposed
    to a request that completed with a negative status)."""
    if rc < 0 and res.status != rc:
        raise GsError(rc, last_error())
    d = res.to_dict()
    d["rc"] = rc
    if rc < 0:
        d["error"] = last_error()
    return d


def _stream_ptr(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(int(stream))


class Context:
    """One library context on one HIP device."""

    def __init__(self, device: int = 0):
        lib = load()
        self._h = C.c_void_p()
        _check(lib.gs_create(C.byref(self._h), int(device)))
        self.device = device
        # ticket -> the request's guess, output and sampled V: the library reads
        # the guess at admission and writes the output at completion, so they
        # are held until the ticket's result has been taken
        self._held = {}

    def close(self):
        if self._h:
            load().gs_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- solves ---------------------------------------------------------------
    def solve(self, pb, psi0=None, options: gs_options | None = None, V=None):
        """Ground state from a host initial guess (numpy complex128, shape
        (3,)+grid). Returns (psi, result dict)."""
        g, (t, keep), p = grid_of(pb), trap_of(pb, V), params_of(pb)
        o = options or default_options()
        shape = (3,) + tuple(pb.shape)
        src = None
        if psi0 is not None:
            src = np.ascontiguousarray(psi0, dtype=np.complex128)
            if src.shape != shape:
                raise ValueError(f"psi0 shape {src.shape} != {shape}")
        out = np.empty(shape, dtype=np.complex128)
        res = gs_result()
        rc = load().gs_solve(self._h, C.byref(g), C.byref(t), C.byref(p), C.byref(o),
                             None if src is None else src.ctypes.data_as(C.c_void_p),
                             out.ctypes.data_as(C.c_void_p), C.byref(res))
        _check(rc)
        d = res.to_dict()
        d["rc"] = rc
        return out, d

    def solve_device(self, pb, psi0, out, options: gs_options | None = None, stream=None, V=None):
        """Device variant: psi0 (or None) and out are complex128 torch tensors on
        this context's device, shape (3,)+grid. Returns the result dict."""
        g, (t, keep), p = grid_of(pb), trap_of(pb, V), params_of(pb)
        o = options or default_options()
        res = gs_result()
        rc = load().gs_solve_device(self._h, C.byref(g), C.byref(t), C.byref(p), C.byref(o),
                                    None if psi0 is None else C.c_void_p(psi0.data_ptr()),
                                    C.c_void_p(out.data_ptr()), C.byref(res), _stream_ptr(stream))
        _check(rc)
        d = res.to_dict()
        d["rc"] = rc
        return d

    # -- batching and serving -------------------------------------------------
    def batch_solve(self, requests):
        """requests: list of (pb, psi0 tensor or None, out tensor, options or
        None, V or None). Runs them all with continuous batching; returns the
        result dicts in order."""
        n = len(requests)
        arr = (gs_request * max(n, 1))()
        keep = []
        for i, (pb, psi0, out, opt, V) in enumerate(requests):
            q, k = make_request(pb, psi0, out, opt, V)
            arr[i] = q
            keep.append(k)
        res = (gs_result * max(n, 1))()
        _check(load().gs_batch_solve(self._h, n, arr, res))
        out = []
        for i in range(n):
            d = res[i].to_dict()
            d["rc"] = res[i].status
            out.append(d)
        return out

    def submit(self, pb, psi0, out, options: gs_options | None = None, V=None) -> int:
        """Queue a request (psi0 may be None); psi0 and out are kept alive by the
        context until poll() or wait() has returned the ticket's result."""
        q, keep = make_request(pb, psi0, out, options, V)
        t = C.c_uint64()
        _check(load().gs_submit(self._h, C.byref(q), C.byref(t)))
        self._held[t.value] = (psi0, out, keep)
        return t.value

    def progress(self, block: bool = False) -> int:
        return _check(load().gs_progress(self._h, int(bool(block))))

    def poll(self, ticket: int):
        """None while the request runs, else its result dict (ticket released)."""
        res = gs_result()
        rc = load().gs_poll(self._h, C.c_uint64(ticket), C.byref(res))
        if rc == GS_PENDING:
            return None
        self._held.pop(ticket, None)
        return _result(rc, res)

    def wait(self, ticket: int):
        res = gs_result()
        rc = load().gs_wait(self._h, C.c_uint64(ticket), C.byref(res))
        self._held.pop(ticket, None)
        return _result(rc, res)

    def cancel(self, ticket: int):
        _check(load().gs_cancel(self._h, C.c_uint64(ticket)))

    def set_hbm_budget(self, nbytes: int):
        _check(load().gs_set_hbm_budget(self._h, C.c_size_t(int(nbytes))))

    def memory_stats(self):
        b, r, a = C.c_size_t(), C.c_size_t(), C.c_size_t()
        _check(load().gs_memory_stats(self._h, C.byref(b), C.byref(r), C.byref(a)))
        return {"budget": b.value, "reserved": r.value, "allocated": a.value}

    # -- schedules of the FFT passes ------------------------------------------------
    def set_autotune(self, on: bool):
        _check(load().gs_set_autotune(self._h, int(bool(on))))

    def autotune_report(self):
        """Per class and bucket of running solves: the chosen schedule of every
        FFT pass and the mean launch time of each candidate (list of dicts)."""
        import json
        r = load().gs_autotune_report(self._h)
        if r is None:
            raise GsError(GS_EINVAL, last_error())
        return json.loads(r.decode())

    # -- measurement ---------------------------------------------------------------
    def kernel_timer_start(self, kind):
        """Time every launch of one kernel kind (name in KERNEL_KINDS or int; None = off)."""
        k = -1 if kind is None else (KERNEL_KINDS[kind] if isinstance(kind, str) else int(kind))
        _check(load().gs_kernel_timer_start(self._h, k))

    def kernel_timer_read(self):
        ms, by, n = C.c_double(), C.c_double(), C.c_longlong()
        _check(load().gs_kernel_timer_read(self._h, C.byref(ms), C.byref(by), C.byref(n)))
        return {"ms": ms.value, "bytes": by.value, "launches": n.value}

    # -- operator-level calls ----------------------------------------------------
    def fft(self, grid: gs_grid, x, out, sign: int, precision=GS_FP64, stream=None):
        _check(load().gs_fft(self._h, C.byref(grid), int(precision), int(sign),
                             C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def fft_noalloc(self, grid: gs_grid, x, out, sign: int, precision=GS_FP64, stream=None):
        """gs_fft without device allocation (at most 2^18 points per component)."""
        _check(load().gs_fft_noalloc(self._h, C.byref(grid), int(precision), int(sign),
                                     C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def interpolate(self, grid_c: gs_grid, x, grid_f: gs_grid, out, stream=None):
        """Fourier interpolation of complex128 device field x on grid_c to grid_f."""
        _check(load().gs_interpolate(self._h, C.byref(grid_c), C.c_void_p(x.data_ptr()), C.byref(grid_f),
                                     C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def hamiltonian(self, pb, psi, out, precision=GS_FP64, stream=None, V=None):
        g, (t, keep), p = grid_of(pb), trap_of(pb, V), params_of(pb)
        res = gs_result()
        _check(load().gs_hamiltonian(self._h, C.byref(g), C.byref(t), C.byref(p), int(precision),
                                     C.c_void_p(psi.data_ptr()), C.c_void_p(out.data_ptr()),
                                     C.byref(res), _stream_ptr(stream)))
        return res.to_dict()

    def precondition(self, pb, psi, r, out, precision=GS_FP64, stream=None, V=None):
        g, (t, keep), p = grid_of(pb), trap_of(pb, V), params_of(pb)
        _check(load().gs_precondition(self._h, C.byref(g), C.byref(t), C.byref(p), int(precision),
                                      C.c_void_p(psi.data_ptr()), C.c_void_p(r.data_ptr()),
                                      C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out
