"""Thin Python binding of libmatex.so (the C ABI in include/matex.h).

Argument marshalling only: every numeric step runs in the library's HIP
kernels. PyTorch supplies device memory (tensors on a gfx950 device) and the
current stream. The library must have been built (`build.py`); there is no
fallback, so a missing or unloadable library raises at import of the first
call.

Layouts (torch shapes): a batch of right-hand sides is (nrhs, n) (column-major
n x nrhs in the C ABI); krylov outputs are (n_tau, nrhs, n); probe outputs are
(n_probe, n_out).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmatex.so")

MATEX_OK, MATEX_E_INVALID, MATEX_E_NOT_SPD, MATEX_E_OOM, MATEX_E_HIP, MATEX_E_NOCONV, \
    MATEX_E_UNSUPPORTED, MATEX_E_NONFINITE = range(8)
MATEX_PLAIN, MATEX_BATCHED = 0, 1
MATEX_RATIONAL, MATEX_INVERTED = 0, 1

_i32, _i64, _f64, _vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
_pi32, _pi64, _pf64 = (ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                       ctypes.POINTER(ctypes.c_double))


class Netlist(ctypes.Structure):
    _fields_ = [("n", _i64), ("n_branch", _i64), ("br_a", _pi32), ("br_b", _pi32),
                ("br_g", _pf64), ("c_node", _pf64), ("n_pad", _i32), ("pad_node", _pi32),
                ("pad_g", _pf64), ("vdd", _f64), ("coord", _pi32)]


class FactorOpts(ctypes.Structure):
    _fields_ = [("n_shifts", _i32), ("leaf_max", _i32), ("subtree_levels", _i32),
                ("batched_schedule", _i32)]


class FactorInfo(ctypes.Structure):
    _fields_ = [("n", _i64), ("nnz_l", _i64), ("panel_doubles", _i64), ("n_supernodes", _i32),
                ("n_levels", _i32), ("n_shifts", _i32), ("max_nr", _i32), ("gamma", _f64),
                ("seconds_analyse", _f64), ("seconds_numeric", _f64), ("device_bytes", _i64),
                ("subtree_levels", _i32), ("subtree_blocks", _i32), ("nnz_l_exact", _i64),
                ("n_upd", _i64), ("seconds_tune", _f64)]


class Problem(ctypes.Structure):
    _fields_ = [("n_src", _i32), ("node", _pi32), ("amp", _pf64), ("delay", _pi64),
                ("rise", _pi64), ("width", _pi64), ("fall", _pi64), ("group", _pi32),
                ("t_end", _i64), ("n_out", _i32), ("t_out", _pi64), ("n_probe", _i32),
                ("probe", _pi32)]


class RunOpts(ctypes.Structure):
    _fields_ = [("tol", _f64), ("m_max", _i32), ("mode", _i32), ("h_min", _i64),
                ("shift_ratio", _f64), ("output_droop", _i32), ("batched_independent", _i32),
                ("krylov", _i32), ("reserved_", _i32)]


class Stats(ctypes.Structure):
    _fields_ = [("subtasks", _i64), ("segments", _i64), ("bases", _i64),
                ("solve_pairs_m", _i64), ("solve_pairs_g", _i64), ("krylov_dims", _i64),
                ("m_peak", _i32), ("halvings", _i32), ("shift_downs", _i32), ("pad_", _i32),
                ("seconds", _f64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


EXPORTS = ["matex_factor", "matex_factor_free", "matex_factor_get_info", "matex_factor_describe",
           "matex_solve",
           "matex_solve_noalloc",
           "matex_krylov_step", "matex_transient", "matex_trapezoidal", "matex_transient_many",
           "matex_adjoint",
           "matex_time_solves", "matex_sync", "matex_last_error", "matex_version"]

_lib = None


def lib():
    """Load libmatex.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1511_04519_amd/build.py")
        # torch's HIP runtime must be the process's first: the library then
        # shares its device context and streams
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        L.matex_factor.argtypes = [ctypes.POINTER(Netlist), _f64, ctypes.POINTER(FactorOpts), _vp,
                                   ctypes.POINTER(_vp)]
        L.matex_factor_free.argtypes = [_vp]
        L.matex_factor_get_info.argtypes = [_vp, ctypes.POINTER(FactorInfo)]
        L.matex_factor_describe.argtypes = [_vp, ctypes.c_char_p, ctypes.c_size_t]
        L.matex_factor_describe.restype = ctypes.c_size_t
        L.matex_solve.argtypes = [_vp, _i32, _i32, _vp, _vp, _vp, _vp]
        L.matex_solve_noalloc.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp]
        L.matex_krylov_step.argtypes = [_vp, _i32, _i32, _vp, _i32, _pf64, _i32, _f64, _vp, _pi32,
                                        _pf64, _vp]
        L.matex_transient.argtypes = [_vp, ctypes.POINTER(Problem), ctypes.POINTER(RunOpts), _vp,
                                      _vp, ctypes.POINTER(Stats), _vp]
        L.matex_trapezoidal.argtypes = [_vp, ctypes.POINTER(Problem), _i64, ctypes.POINTER(RunOpts), _vp, _vp,
                                        ctypes.POINTER(Stats), _vp]
        L.matex_transient_many.argtypes = [_i32, ctypes.POINTER(_vp), ctypes.POINTER(Problem),
                                           ctypes.POINTER(RunOpts), ctypes.POINTER(_vp),
                                           ctypes.POINTER(_vp), ctypes.POINTER(Stats), _i32, _vp]
        L.matex_adjoint.argtypes = [_vp, ctypes.POINTER(Problem), ctypes.POINTER(RunOpts), _vp,
                                    _vp, _vp, _vp]
        L.matex_time_solves.argtypes = [_vp, _i32, _i32, _i32, _pf64, _pf64, _vp]
        L.matex_sync.argtypes = [_vp]
        L.matex_last_error.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
        L.matex_last_error.restype = ctypes.c_size_t
        L.matex_version.restype = ctypes.c_char_p
        for name in ("matex_factor", "matex_factor_free", "matex_factor_get_info", "matex_solve",
                     "matex_solve_noalloc",
                     "matex_krylov_step", "matex_transient", "matex_trapezoidal", "matex_transient_many",
                     "matex_adjoint", "matex_time_solves", "matex_sync"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


class MatexError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"matex status {status}: {msg}")
        self.status = status


def last_error() -> str:
    buf = ctypes.create_string_buffer(1024)
    lib().matex_last_error(buf, 1024)
    return buf.value.decode()


def _check(st, allow=()):
    if st != MATEX_OK and st not in allow:
        raise MatexError(st, last_error())
    return st


def _p(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype)) if a is not None else None


def _stream():
    """torch's current HIP stream (NULL = default stream when no device is
    visible, which only the argument checks before any device work see)."""
    import torch
    if not torch.cuda.is_available():
        return None
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class FactorHandle:
    """Owns a matex_factor_t; keeps the host arrays alive only during the call."""

    def __init__(self, handle, info):
        self.handle = handle
        self.info = info
        self._free = lib().matex_factor_free   # still reachable at interpreter exit

    def __del__(self):
        h = getattr(self, "handle", None)
        free = getattr(self, "_free", None)
        if h and free is not None:
            free(h)
            self.handle = None


def matex_factor(netlist, gamma: float, n_shifts: int = 6, leaf_max: int = 16,
                 use_coords: bool = True, subtree_levels: int = 0,
                 batched_schedule: int = 0) -> FactorHandle:
    """Factor C + gamma_k G for the shift ladder and G (see matex.h)."""
    a = np.ascontiguousarray(netlist.br_a, np.int32)
    b = np.ascontiguousarray(netlist.br_b, np.int32)
    g = np.ascontiguousarray(netlist.br_g, np.float64)
    c = np.ascontiguousarray(netlist.c_node, np.float64)
    pn = np.ascontiguousarray(netlist.pad_node, np.int32)
    pg = np.ascontiguousarray(netlist.pad_g, np.float64)
    crd = np.ascontiguousarray(netlist.coord, np.int32) if use_coords else None
    nl = Netlist(netlist.n, a.size, _p(a, ctypes.c_int32), _p(b, ctypes.c_int32),
                 _p(g, ctypes.c_double), _p(c, ctypes.c_double), pn.size, _p(pn, ctypes.c_int32),
                 _p(pg, ctypes.c_double), float(netlist.vdd),
                 _p(crd, ctypes.c_int32) if crd is not None else None)
    opts = FactorOpts(n_shifts, leaf_max, subtree_levels, batched_schedule)
    h = ctypes.c_void_p()
    _check(lib().matex_factor(ctypes.byref(nl), float(gamma), ctypes.byref(opts), _stream(),
                              ctypes.byref(h)))
    info = FactorInfo()
    _check(lib().matex_factor_get_info(h, ctypes.byref(info)))
    return FactorHandle(h, {k: getattr(info, k) for k, _ in FactorInfo._fields_})


def matex_factor_describe(f: FactorHandle) -> str:
    """The factor's sweep schedules, one line per level."""
    n = lib().matex_factor_describe(f.handle, None, 0)
    buf = ctypes.create_string_buffer(n + 1)
    lib().matex_factor_describe(f.handle, buf, n + 1)
    return buf.value.decode()


def matex_solve(f: FactorHandle, which: int, b, scale=None):
    """x = A_which^-1 (scale * b); b is a (n,) or (nrhs, n) float64 device tensor."""
    import torch
    b2 = b.reshape(-1, f.info["n"]).contiguous()
    x = torch.empty_like(b2)
    sc = scale.contiguous() if scale is not None else None
    _check(lib().matex_solve(f.handle, which, b2.shape[0], _ptr(b2), _ptr(sc), _ptr(x), _stream()))
    return x.reshape(b.shape)


def matex_solve_noalloc(f: FactorHandle, which: int, b, x, scale=None):
    """x = A_which^-1 (scale * b) for one (n,) float64 device vector into the
    caller's x, through the library's allocation-free entry point (nothing
    allocated by the library; asynchronous on torch's current stream)."""
    _check(lib().matex_solve_noalloc(f.handle, which, _ptr(b), _ptr(scale), _ptr(x), _stream()))
    return x


def matex_krylov_step(f: FactorHandle, v, taus, shift: int = 0, m_max: int = 20,
                      tol: float = 1e-12):
    """e^{tau A} v for every tau (seconds). v: (n,) or (nrhs, n) device tensor.
    shift: index of the ladder's shift (rational space), or -1 for the
    inverted space (X1 = G). Returns (out (n_tau, nrhs, n), m_used[nrhs],
    est[nrhs], converged)."""
    import torch
    n = f.info["n"]
    v2 = v.reshape(-1, n).contiguous()
    nrhs = v2.shape[0]
    t = np.ascontiguousarray(taus, np.float64)
    out = torch.empty((t.size, nrhs, n), dtype=torch.float64, device=v.device)
    m_used = np.zeros(nrhs, np.int32)
    est = np.zeros(nrhs)
    st = _check(lib().matex_krylov_step(f.handle, shift, nrhs, _ptr(v2), t.size,
                                        _p(t, ctypes.c_double), m_max, float(tol), _ptr(out),
                                        _p(m_used, ctypes.c_int32), _p(est, ctypes.c_double),
                                        _stream()), allow=(MATEX_E_NOCONV,))
    return out, m_used, est, st == MATEX_OK


def _problem_struct(prob, keep):
    s = prob.sources
    arrs = dict(node=np.ascontiguousarray(s.node, np.int32), amp=np.ascontiguousarray(s.amp, np.float64),
                delay=np.ascontiguousarray(s.delay, np.int64), rise=np.ascontiguousarray(s.rise, np.int64),
                width=np.ascontiguousarray(s.width, np.int64), fall=np.ascontiguousarray(s.fall, np.int64),
                group=np.ascontiguousarray(s.group, np.int32),
                t_out=np.ascontiguousarray(prob.t_out, np.int64),
                probe=np.ascontiguousarray(prob.probe, np.int32))
    keep.append(arrs)
    return Problem(arrs["node"].size, _p(arrs["node"], ctypes.c_int32), _p(arrs["amp"], ctypes.c_double),
                   _p(arrs["delay"], ctypes.c_int64), _p(arrs["rise"], ctypes.c_int64),
                   _p(arrs["width"], ctypes.c_int64), _p(arrs["fall"], ctypes.c_int64),
                   _p(arrs["group"], ctypes.c_int32), int(prob.t_end), arrs["t_out"].size,
                   _p(arrs["t_out"], ctypes.c_int64), arrs["probe"].size, _p(arrs["probe"], ctypes.c_int32))


def matex_transient(f: FactorHandle, prob, tol: float = 1e-11, m_max: int = 20,
                    mode: int = MATEX_PLAIN, h_min: int = 1, device="cuda", final: bool = True,
                    shift_ratio: float = 1.0, droop: bool = False, independent: bool = False,
                    krylov: int = MATEX_RATIONAL):
    """Alg. 2 over every subtask, summed. Returns (x at probes (n_probe, n_out),
    x(t_end) (n,) or None, stats dict); with droop=True the droop y = Vdd - x
    instead of x."""
    import torch
    keep = []
    pr = _problem_struct(prob, keep)
    out = torch.empty((prob.probe.size, prob.t_out.size), dtype=torch.float64, device=device)
    fin = torch.empty(f.info["n"], dtype=torch.float64, device=device) if final else None
    st = Stats()
    opts = RunOpts(float(tol), int(m_max), int(mode), int(h_min), float(shift_ratio), int(droop),
                   int(bool(independent)), int(krylov))
    _check(lib().matex_transient(f.handle, ctypes.byref(pr), ctypes.byref(opts), _ptr(out), _ptr(fin),
                                 ctypes.byref(st), _stream()))
    return out, fin, st.as_dict()


def matex_trapezoidal(f: FactorHandle, prob, h_fs: int, device="cuda", final: bool = True,
                      droop: bool = False):
    """The trapezoidal rule at the fixed step h_fs (fs); f must be factored
    with gamma = h / 2. Returns (x at probes (n_probe, n_out), x(t_end) or
    None, stats dict), or the droop with droop=True."""
    import torch
    keep = []
    pr = _problem_struct(prob, keep)
    out = torch.empty((prob.probe.size, prob.t_out.size), dtype=torch.float64, device=device)
    fin = torch.empty(f.info["n"], dtype=torch.float64, device=device) if final else None
    st = Stats()
    opts = RunOpts(1.0, 1, MATEX_PLAIN, 1, 1.0, int(droop), 0)
    _check(lib().matex_trapezoidal(f.handle, ctypes.byref(pr), int(h_fs), ctypes.byref(opts), _ptr(out),
                                   _ptr(fin), ctypes.byref(st), _stream()))
    return out, fin, st.as_dict()


def matex_transient_many(factors, probs, tol: float = 1e-11, m_max: int = 20,
                         mode: int = MATEX_PLAIN, h_min: int = 1, n_streams: int = 4,
                         device="cuda", final: bool = True, shift_ratio: float = 1.0,
                         krylov: int = MATEX_RATIONAL, droop: bool = False):
    """Independent instances (own factor each) advanced concurrently on
    n_streams library streams. Returns a list of (x, x_final or None, stats)."""
    import torch
    k = len(factors)
    assert len(probs) == k
    keep = []
    prs = (Problem * max(1, k))(*[_problem_struct(q, keep) for q in probs])
    outs = [torch.empty((q.probe.size, q.t_out.size), dtype=torch.float64, device=device) for q in probs]
    fins = [torch.empty(F.info["n"], dtype=torch.float64, device=device) for F in factors] if final else None
    fh = (_vp * max(1, k))(*[F.handle.value for F in factors])
    po = (_vp * max(1, k))(*[_ptr(t) for t in outs])
    pf = (_vp * max(1, k))(*[_ptr(t) for t in fins]) if final else None
    opts = (RunOpts * max(1, k))(*[RunOpts(float(tol), int(m_max), int(mode), int(h_min),
                                           float(shift_ratio), int(droop), 0, int(krylov))
                                   for _ in range(k)])
    sts = (Stats * max(1, k))()
    _check(lib().matex_transient_many(k, fh, prs, opts, po, pf, sts, int(n_streams), _stream()))
    return [(outs[i], fins[i] if final else None, sts[i].as_dict()) for i in range(k)]


def matex_time_solves(f: FactorHandle, which: int = 0, reps: int = 50, nrhs: int = 1):
    """Mean seconds of one substitution pair on nrhs right-hand sides
    (event-timed on the current stream) and its algorithmic bytes."""
    sec = ctypes.c_double()
    byt = ctypes.c_double()
    _check(lib().matex_time_solves(f.handle, which, nrhs, reps, ctypes.byref(sec),
                                   ctypes.byref(byt), _stream()))
    return sec.value, byt.value


def matex_sync():
    """Waits for the library's work on torch's current stream; raises
    MatexError (MATEX_E_HIP) if HIP reports a pending error."""
    _check(lib().matex_sync(_stream()))


def matex_adjoint(f: FactorHandle, prob, dJdx, tol: float = 1e-10, m_max: int = 30,
                  h_min: int = 1, grad_c: bool = False, shift_ratio: float = 1.0):
    """Gradients of an objective J of the probe voltages. dJdx: device tensor
    (n_probe, n_out) = dJ/dx at the probes and output times. Returns
    (dJ/d amplitude (n_src,), dJ/d c (n,) or None)."""
    import torch
    keep = []
    pr = _problem_struct(prob, keep)
    d = dJdx.contiguous()
    ga = torch.empty(prob.sources.n_src, dtype=torch.float64, device=d.device)
    gc = torch.empty(f.info["n"], dtype=torch.float64, device=d.device) if grad_c else None
    opts = RunOpts(float(tol), int(m_max), MATEX_PLAIN, int(h_min), float(shift_ratio))
    _check(lib().matex_adjoint(f.handle, ctypes.byref(pr), ctypes.byref(opts), _ptr(d), _ptr(ga),
                               _ptr(gc), _stream()))
    return ga, gc
