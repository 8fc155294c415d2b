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
* node capacitances: central differences of J in c_i with relative step rel;
  truncation O(rel^2), rounding O(eps / rel).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import reference as R


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


def x_probes(prob, c_node=None):
    """Exact x = Vdd - y at the probes, optionally with other capacitances."""
    if c_node is not None:
        prob = dataclasses.replace(prob, netlist=dataclasses.replace(prob.netlist, c_node=c_node))
    y, _ = R.modal(prob)
    return prob.netlist.vdd - y


def c_gradient_fd(prob, J, nodes=None, rel: float = 1e-5):
    """dJ/dc_i by central differences of the exact solution; J maps the probe
    voltages [n_probe, n_out] to a number. nodes: which i (default all)."""
    c = np.asarray(prob.netlist.c_node, dtype=np.float64)
    nodes = np.arange(c.size) if nodes is None else np.asarray(nodes)
    grad = np.zeros(nodes.size)
    for q, i in enumerate(nodes):
        h = rel * c[i]
        cp = c.copy()
        cp[i] = c[i] + h
        cm = c.copy()
        cm[i] = c[i] - h
        grad[q] = (J(x_probes(prob, cp)) - J(x_probes(prob, cm))) / (2.0 * h)
    return grad
