"""Circuit model of the oracle: MNA matrices, pulse inputs, transition spots.

Test infrastructure (see the package docstring).

Sec. 2.1, Eq. 1: C x' = -G x + B u(t). For an RC grid, C is the diagonal of
node-to-ground capacitances, G is the branch-conductance Laplacian plus the
Norton pad conductances on the diagonal, and B u injects Vdd * g_pad at each
pad and draws the sink currents out of their nodes.

Droop form used throughout the oracle. G * 1 = g_pad (the Laplacian kills the
constant vector), so with no sinks x = Vdd * 1 is the DC solution. With
y = Vdd * 1 - x,  C y' = -G y + i(t),  y(0) = 0,  where i(t) collects the sink
currents. In the paper's ODE form (Eq. 3) A = -C^-1 G and b(t) = C^-1 i(t).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib

FS = 1e-15  # seconds per femtosecond


def assemble_G(nl):
    """Full symmetric CSR (rowptr int64, col int32, val f64) of G (Eq. 1)."""
    n = nl.n
    a = np.asarray(nl.br_a, dtype=np.int64)
    b = np.asarray(nl.br_b, dtype=np.int64)
    g = np.asarray(nl.br_g, dtype=np.float64)
    p = np.asarray(nl.pad_node, dtype=np.int64)
    rows = np.concatenate([a, b, a, b, p])
    cols = np.concatenate([b, a, a, b, p])
    vals = np.concatenate([-g, -g, g, g, np.asarray(nl.pad_g, dtype=np.float64)])
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    key, vals = key[order], vals[order]
    uniq, start = np.unique(key, return_index=True)
    summed = np.add.reduceat(vals, start)
    r = (uniq // n).astype(np.int64)
    c = (uniq % n).astype(np.int32)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr, c, summed


def csr_add_diag(rowptr, col, val, d, alpha=1.0):
    """CSR of alpha*A + diag(d) for A whose pattern contains the diagonal."""
    out = alpha * val.copy()
    n = rowptr.size - 1
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    diag = rows == col
    out[diag] += d[rows[diag]]
    return out


def csr_matvec(rowptr, col, val, x):
    n = rowptr.size - 1
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    y = np.zeros(n)
    np.add.at(y, rows, val * x[col])
    return y


def csr_dense(rowptr, col, val):
    n = rowptr.size - 1
    D = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    D[rows, col] = val
    return D


class Cholesky:
    """Sparse Cholesky A = P^T L L^T P of a symmetric positive-definite CSR
    matrix (both triangles given); .solve applies A^{-1}, i.e. the
    forward/backward substitution pair of Alg. 1."""

    def __init__(self, rowptr, col, val, nested_dissection=True):
        L = _lib.lib()
        self.n = rowptr.size - 1
        self._rp = np.ascontiguousarray(rowptr, dtype=np.int64)
        self._ci = np.ascontiguousarray(col, dtype=np.int32)
        self._v = np.ascontiguousarray(val, dtype=np.float64)
        h = ctypes.c_void_p()
        st = L.orc_chol_factor(self.n,
                               self._rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                               self._ci.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               self._v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               1 if nested_dissection else 0, ctypes.byref(h))
        self._h = h
        if st != 0:
            L.orc_chol_free(h)
            self._h = None
            raise np.linalg.LinAlgError(f"not positive definite (status {st})")
        self.nnz = int(L.orc_chol_nnz(h))

    def solve(self, b):
        b = np.array(b, dtype=np.float64, order="F", copy=True)
        nrhs = 1 if b.ndim == 1 else b.shape[1]
        _lib.lib().orc_chol_solve(self._h, b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  nrhs)
        return b

    def export(self):
        """(colptr, rowidx, val, perm) of L with L[perm, :][:, perm]... i.e. the
        factor of the permuted matrix A[perm][:, perm]."""
        n, nnz = self.n, self.nnz
        cp = np.empty(n + 1, dtype=np.int64)
        ri = np.empty(nnz, dtype=np.int32)
        v = np.empty(nnz)
        pm = np.empty(n, dtype=np.int32)
        _lib.lib().orc_chol_export(self._h, cp.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   ri.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   pm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        return cp, ri, v, pm

    def __del__(self):
        if getattr(self, "_h", None):
            _lib.lib().orc_chol_free(self._h)
            self._h = None


# ---------------------------------------------------------------- inputs

def pulse(t_fs, delay, rise, width, fall):
    """Unit trapezoidal pulse (Fig. 3 timing; SPICE PULSE shape, one period):
    0 before delay, linear rise over `rise`, flat for `width`, linear fall over
    `fall`, 0 afterwards. All times in fs; t may be a scalar."""
    t = np.asarray(t_fs, dtype=np.float64)
    d = delay.astype(np.float64)
    r = rise.astype(np.float64)
    w = width.astype(np.float64)
    f = fall.astype(np.float64)
    out = np.zeros(np.broadcast(t, d).shape)
    up = (t > d) & (t <= d + r)
    out = np.where(up, (t - d) / r, out)
    top = (t > d + r) & (t <= d + r + w)
    out = np.where(top, 1.0, out)
    down = (t > d + r + w) & (t < d + r + w + f)
    out = np.where(down, 1.0 - (t - d - r - w) / f, out)
    return out


def pulse_slope(t_a, delay, rise, width, fall):
    """Slope (per fs) of the unit pulse on the piece that starts at t_a, i.e.
    on [t_a, next transition spot)."""
    t = float(t_a)
    d, r, w, f = (x.astype(np.float64) for x in (delay, rise, width, fall))
    s = np.zeros(d.shape)
    s = np.where((t >= d) & (t < d + r), 1.0 / r, s)
    s = np.where((t >= d + r + w) & (t < d + r + w + f), -1.0 / f, s)
    return s


def source_spots(src, idx):
    """Local transition spots (Sec. 3.1 definition): the corners of each
    selected source's pulse, as integer fs."""
    d = src.delay[idx]
    return np.concatenate([d, d + src.rise[idx], d + src.rise[idx] + src.width[idx],
                           d + src.rise[idx] + src.width[idx] + src.fall[idx]])


def transition_spots(src, idx, t_end):
    """Sorted transition spots of the sources `idx` inside (0, t_end), plus 0 and
    t_end (Sec. 2.2, the maximum step ends at the next spot)."""
    ts = source_spots(src, idx)
    ts = ts[(ts > 0) & (ts < t_end)]
    return np.unique(np.concatenate([[0], ts, [t_end]])).astype(np.int64)


def current(src, idx, n, t_fs):
    """Sink current vector i(t) (A) of the sources `idx` at time t."""
    i = np.zeros(n)
    u = pulse(t_fs, src.delay[idx], src.rise[idx], src.width[idx], src.fall[idx])
    np.add.at(i, src.node[idx], src.amp[idx] * u)
    return i


def current_slope(src, idx, n, t_a):
    """Slope of i(t) in A/s on the piece starting at t_a."""
    s = np.zeros(n)
    sl = pulse_slope(t_a, src.delay[idx], src.rise[idx], src.width[idx], src.fall[idx])
    np.add.at(s, src.node[idx], src.amp[idx] * sl / FS)
    return s


def subtasks(src):
    """Source decomposition (Sec. 3.1, grouping by pulse shape): the groups'
    source index lists, in increasing group id."""
    return [np.nonzero(src.group == g)[0] for g in np.unique(src.group)]
