"""Exact and classical references for the droop transient (oracle).

Test infrastructure (see the package docstring).

  * modal():  the exact solution of Eq. 4 for piecewise-linear inputs, mode by
    mode. S = C^-1/2 G C^-1/2 = Q diag(lam) Q^T (symmetric eigendecomposition,
    a library step). In q = Q^T C^1/2 y every mode obeys the scalar ODE
    q' = -lam q + f(t) with f linear between transition spots, whose exact
    solution over a step tau is
      q(t+tau) = e^{-lam tau} q(t) + f(t) tau phi1(lam tau) + f' tau^2 phi2(lam tau),
      phi1(z) = (1 - e^{-z})/z,  phi2(z) = (z - 1 + e^{-z})/z^2.
    No Krylov projection and no matrix exponential: exact up to rounding.
  * dense_eq5(): Eq. 5 literally, with dense A = -C^-1 G, A^-1 = -G^-1 C and the
    oracle's Pade expm; for grids of a few hundred nodes.
  * trapezoidal(): Eq. 2 with a fixed step on a grid that contains every
    transition spot and output time when `align` is set.
All three work in the droop form y = Vdd - x (see circuit.py).
"""
from __future__ import annotations

import numpy as np

from .circuit import (FS, Cholesky, assemble_G, csr_add_diag, csr_dense, current,
                      current_slope, subtasks, transition_spots)
from .expm import expm


def phi1(z):
    z = np.asarray(z, dtype=np.float64)
    out = np.ones_like(z)
    nz = z != 0
    out[nz] = -np.expm1(-z[nz]) / z[nz]
    return out


def phi2(z):
    """(z - 1 + e^-z)/z^2, by its Taylor series sum_k (-z)^k/(k+2)! for small z."""
    z = np.asarray(z, dtype=np.float64)
    out = np.empty_like(z)
    small = np.abs(z) < 0.1
    zs = z[small]
    acc = np.zeros_like(zs)
    term = np.full_like(zs, 0.5)
    for k in range(20):
        acc += term
        term = term * (-zs) / (k + 3)
    out[small] = acc
    zl = z[~small]
    out[~small] = (zl - 1.0 + np.exp(-zl)) / (zl * zl)
    return out


def _breakpoints(src, idx, t_end, t_out):
    ts = transition_spots(src, idx, t_end)
    return np.unique(np.concatenate([ts, t_out[(t_out >= 0) & (t_out <= t_end)]]))


def modal(prob, decompose: bool = False):
    """Exact droop y at (probe x t_out) and at t_end, by modal decomposition."""
    nl, src = prob.netlist, prob.sources
    n = nl.n
    rp, ci, gv = assemble_G(nl)
    G = csr_dense(rp, ci, gv)
    cs = np.sqrt(nl.c_node)
    S = G / cs[:, None] / cs[None, :]
    lam, Q = np.linalg.eigh(S)
    groups = subtasks(src) if decompose else [np.arange(src.n_src)]
    y_out = np.zeros((prob.probe.size, prob.t_out.size))
    y_end = np.zeros(n)
    for idx in groups:
        bp = _breakpoints(src, idx, prob.t_end, prob.t_out)
        q = np.zeros(n)
        # y(0) = G^-1 i(0): in modal form q = diag(1/lam) Q^T C^-1/2 i(0)
        q = (Q.T @ (current(src, idx, n, 0) / cs)) / lam
        k_out = 0
        for k in range(bp.size):
            t = bp[k]
            if k > 0:
                ta = bp[k - 1]
                tau = (t - ta) * FS
                fa = Q.T @ (current(src, idx, n, ta) / cs)
                fs = Q.T @ (current_slope(src, idx, n, ta) / cs)
                z = lam * tau
                q = np.exp(-z) * q + fa * tau * phi1(z) + fs * tau * tau * phi2(z)
            while k_out < prob.t_out.size and prob.t_out[k_out] == t:
                y_out[:, k_out] += ((Q @ q) / cs)[prob.probe]
                k_out += 1
        y_end += (Q @ q) / cs
    return y_out, y_end


def dense_eq5(prob):
    """Eq. 5 stepped between consecutive breakpoints (transition spots and
    output times), all sources together."""
    nl, src = prob.netlist, prob.sources
    n = nl.n
    idx = np.arange(src.n_src)
    rp, ci, gv = assemble_G(nl)
    G = csr_dense(rp, ci, gv)
    C = np.diag(nl.c_node)
    A = -np.linalg.solve(C, G)
    Ainv = -np.linalg.solve(G, C)
    bp = _breakpoints(src, idx, prob.t_end, prob.t_out)
    b = lambda t: current(src, idx, n, t) / nl.c_node
    x = np.linalg.solve(G, current(src, idx, n, 0))
    y_out = np.zeros((prob.probe.size, prob.t_out.size))
    k_out = 0
    for k in range(bp.size):
        t = bp[k]
        if k > 0:
            ta = bp[k - 1]
            h = (t - ta) * FS
            bt, bth = b(ta), b(t)
            db = (bth - bt) / h
            F = Ainv @ bt + Ainv @ (Ainv @ db)
            P = Ainv @ bth + Ainv @ (Ainv @ db)
            x = expm(h * A) @ (x + F) - P
        while k_out < prob.t_out.size and prob.t_out[k_out] == t:
            y_out[:, k_out] = x[prob.probe]
            k_out += 1
    return y_out, x


def trapezoidal(prob, h_fs: int, align: bool = True, factors=None):
    """Eq. 2 with fixed step h (fs): (C/h + G/2) y+ = (C/h - G/2) y + (i + i+)/2.
    With align, steps are cut at every transition spot and output time so the
    piecewise-linear input is sampled exactly; returns (y at probe x t_out,
    y(t_end), number of substitution pairs). `factors` may hold factors made
    beforehand: "G" (for the initial state) and, per step h in fs, the
    Cholesky of C/h + G/2; the missing ones are made here."""
    nl, src = prob.netlist, prob.sources
    n = nl.n
    idx = np.arange(src.n_src)
    rp, ci, gv = assemble_G(nl)
    c = nl.c_node
    if align:
        bp = _breakpoints(src, idx, prob.t_end, prob.t_out)
        grid = [0]
        for k in range(1, bp.size):
            ta, tb = bp[k - 1], bp[k]
            steps = max(1, int(np.ceil((tb - ta) / h_fs)))
            grid.extend(ta + (tb - ta) * np.arange(1, steps + 1) // steps)
        grid = np.array(grid, dtype=np.int64)
    else:
        grid = np.arange(0, prob.t_end + 1, h_fs, dtype=np.int64)
    facs = dict(factors or {})
    Gf = facs.pop("G", None) or Cholesky(rp, ci, gv)
    y = Gf.solve(current(src, idx, n, 0))
    y_out = np.zeros((prob.probe.size, prob.t_out.size))
    k_out = 0
    pairs = 0
    while k_out < prob.t_out.size and prob.t_out[k_out] == 0:
        y_out[:, k_out] = y[prob.probe]
        k_out += 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    for k in range(1, grid.size):
        h = int(grid[k] - grid[k - 1])
        hs = h * FS
        if h not in facs:
            facs[h] = Cholesky(rp, ci, csr_add_diag(rp, ci, gv, c / hs, alpha=0.5))
        Gy = np.zeros(n)
        np.add.at(Gy, rows, gv * y[ci])
        rhs = c / hs * y - 0.5 * Gy + 0.5 * (current(src, idx, n, grid[k - 1])
                                             + current(src, idx, n, grid[k]))
        y = facs[h].solve(rhs)
        pairs += 1
        while k_out < prob.t_out.size and prob.t_out[k_out] == grid[k]:
            y_out[:, k_out] = y[prob.probe]
            k_out += 1
    return y_out, y, pairs
