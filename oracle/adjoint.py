"""Gradients of an objective of the probe voltages, written from their
definitions (test infrastructure; see the package header).

The objective J depends on the node voltages x = Vdd - y at the probe rows
and output times; the caller gives dJ/dx there, shaped [n_probe, n_out].
Both routes run on the exact modal solution (reference.modal), so they carry
no Krylov truncation:

* amplitudes: the droop is linear in the source amplitudes (the responses of
  sources superpose, Sec. 3.1), so dx/da_k is minus the response to source k
  alone at unit amplitude and dJ/da_k = sum over probes and times of
  dJ/dx * dx/da_k. Exact up to rounding.
* node capacitances: the chain rule dJ/dc_i = sum dJ/dx * dx/dc_i with
  dx/dc_i = -dy/dc_i, by complex-step differentiation (Squire and Trapp,
  SIAM Rev. 40(1), 1998: dy/dc = Im y(c + i h) / h, no cancellation, exact to
  rounding) of the dense Eq. 5 solution, which is analytic in c; or, as a
  cross-check, by central differences of the droop (the modal solution's
  rounding limits those to about 1e-4 relative).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import reference as R
from .circuit import FS, assemble_G, csr_dense, current
from .expm import expm


def amp_gradient(prob, dJdx):
    """dJ/da_k for every source k (linearity in the amplitudes)."""
    src = prob.sources
    dJdx = np.asarray(dJdx, dtype=np.float64)
    grad = np.zeros(src.n_src)
    for k in range(src.n_src):
        one = dataclasses.replace(
            src, node=src.node[k:k + 1], amp=np.ones(1), delay=src.delay[k:k + 1],
            rise=src.rise[k:k + 1], width=src.width[k:k + 1], fall=src.fall[k:k + 1],
            group=np.zeros(1, np.int32))
        y_k, _ = R.modal(dataclasses.replace(prob, sources=one))
        grad[k] = -np.sum(dJdx * y_k)
    return grad


def droop_probes(prob, c_node=None):
    """Exact droop y at the probes, optionally with other capacitances."""
    if c_node is not None:
        prob = dataclasses.replace(prob, netlist=dataclasses.replace(prob.netlist, c_node=c_node))
    y, _ = R.modal(prob)
    return y


def x_probes(prob, c_node=None):
    """Exact x = Vdd - y at the probes."""
    return prob.netlist.vdd - droop_probes(prob, c_node)


def c_gradient_fd(prob, dJdx, nodes=None, rel: float = 1e-4):
    """dJ/dc_i (chain rule with the given dJ/dx; dy/dc_i by central
    differences of the exact droop). nodes: which i (default all)."""
    c = np.asarray(prob.netlist.c_node, dtype=np.float64)
    dJdx = np.asarray(dJdx, dtype=np.float64)
    nodes = np.arange(c.size) if nodes is None else np.asarray(nodes)
    grad = np.zeros(nodes.size)
    for q, i in enumerate(nodes):
        h = rel * c[i]
        cp = c.copy()
        cp[i] = c[i] + h
        cm = c.copy()
        cm[i] = c[i] - h
        dy = (droop_probes(prob, cp) - droop_probes(prob, cm)) / (2.0 * h)
        grad[q] = -np.sum(dJdx * dy)
    return grad


def _dense_eq5_droop(prob, c):
    """The droop at the probes by Eq. 5 stepped between consecutive
    breakpoints, for node capacitances c (real or complex): the same route as
    reference.dense_eq5, written for a complex c."""
    nl, src = prob.netlist, prob.sources
    n = nl.n
    idx = np.arange(src.n_src)
    rp, ci, gv = assemble_G(nl)
    G = csr_dense(rp, ci, gv).astype(c.dtype)
    A = -G / c[:, None]                      # -C^-1 G
    Ainv = -np.linalg.solve(G, np.diag(c))   # A^-1 = -G^-1 C
    bp = R._breakpoints(src, idx, prob.t_end, prob.t_out)
    y = np.linalg.solve(G, current(src, idx, n, 0).astype(c.dtype))
    out = np.zeros((prob.probe.size, prob.t_out.size), dtype=c.dtype)
    k_out = 0
    for k in range(bp.size):
        t = bp[k]
        if k > 0:
            ta = bp[k - 1]
            h = (t - ta) * FS
            bt, bth = current(src, idx, n, ta) / c, current(src, idx, n, t) / c
            db = (bth - bt) / h
            F = Ainv @ bt + Ainv @ (Ainv @ db)
            P = Ainv @ bth + Ainv @ (Ainv @ db)
            y = expm(h * A) @ (y + F) - P
        while k_out < prob.t_out.size and prob.t_out[k_out] == t:
            out[:, k_out] = y[prob.probe]
            k_out += 1
    return out


def c_gradient_cs(prob, dJdx, nodes=None, rel: float = 1e-20):
    """dJ/dc_i by complex-step differentiation of the dense Eq. 5 droop
    (small grids). nodes: which i (default all)."""
    c = np.asarray(prob.netlist.c_node, dtype=np.float64)
    dJdx = np.asarray(dJdx, dtype=np.float64)
    nodes = np.arange(c.size) if nodes is None else np.asarray(nodes)
    grad = np.zeros(nodes.size)
    for q, i in enumerate(nodes):
        cc = c.astype(np.complex128)
        h = rel * c[i]
        cc[i] += 1j * h
        dy = _dense_eq5_droop(prob, cc).imag / h
        grad[q] = -np.sum(dJdx * dy)
    return grad
