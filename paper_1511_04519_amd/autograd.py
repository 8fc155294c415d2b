"""torch.autograd over the library's transient and adjoint.

`transient(amp, c_node, prob)` returns the probe voltages x of the problem's
transient (matex_transient) for source amplitudes `amp` and node
capacitances `c_node`; its backward pass calls matex_adjoint, the continuous
adjoint of the exact solution propagated with the same rational Krylov
steps, for dJ/d amp and dJ/d c_node. Argument marshalling only: the forward
run and the gradients are computed by the library's kernels (a missing
library raises). The factor of C + gamma_k G and G is built for the
capacitances given and reused while they do not change (Alg. 2 factors once
before its time loop; a new C needs a new factor).
"""
from __future__ import annotations

import numpy as np
import torch

from . import instances as I
from . import matex as M


class FactorCache:
    """The last factor built and the capacitances it was built for."""

    def __init__(self, gamma: float, **factor_kw):
        self.gamma = gamma
        self.kw = factor_kw
        self.c = None
        self.F = None
        self.builds = 0

    def factor_for(self, netlist, c_node: np.ndarray):
        if self.F is None or self.c is None or not np.array_equal(self.c, c_node):
            nl = I.Netlist(netlist.n, netlist.br_a, netlist.br_b, netlist.br_g, c_node, netlist.pad_node,
                           netlist.pad_g, netlist.vdd, netlist.coord)
            self.F = M.matex_factor(nl, self.gamma, **self.kw)
            self.c = c_node.copy()
            self.builds += 1
        return self.F


def _with(prob, amp: np.ndarray, c_node: np.ndarray):
    nl = prob.netlist
    nl2 = I.Netlist(nl.n, nl.br_a, nl.br_b, nl.br_g, c_node, nl.pad_node, nl.pad_g, nl.vdd, nl.coord)
    s = prob.sources
    src = I.Sources(s.node, amp, s.delay, s.rise, s.width, s.fall, s.group)
    return I.Problem(prob.name, nl2, src, prob.t_end, prob.t_out, prob.probe, prob.gamma, prob.m_max)


class TransientFunction(torch.autograd.Function):
    """x = transient(amp, c_node); backward: (dJ/d amp, dJ/d c_node) from
    matex_adjoint with the incoming dJ/dx."""

    @staticmethod
    def forward(ctx, amp, c_node, prob, cache, tol, m_max, adj_tol, device):
        a = amp.detach().to("cpu", torch.float64).numpy().copy()
        c = c_node.detach().to("cpu", torch.float64).numpy().copy()
        F = cache.factor_for(prob.netlist, c)
        q = _with(prob, a, c)
        x, _, _ = M.matex_transient(F, q, tol=tol, m_max=m_max, device=device, final=False)
        ctx.F, ctx.q, ctx.adj_tol = F, q, adj_tol
        ctx.amp_dev, ctx.c_dev = amp.device, c_node.device
        return x

    @staticmethod
    def backward(ctx, gx):
        want_c = ctx.needs_input_grad[1]
        if not (ctx.needs_input_grad[0] or want_c):
            return (None,) * 8
        ga, gc = M.matex_adjoint(ctx.F, ctx.q, gx.detach().to(torch.float64).contiguous(), tol=ctx.adj_tol,
                                 m_max=30, grad_c=want_c)
        ga = ga.to(ctx.amp_dev) if ctx.needs_input_grad[0] else None
        gc = gc.to(ctx.c_dev) if want_c else None
        return ga, gc, None, None, None, None, None, None


def transient(amp: torch.Tensor, c_node: torch.Tensor, prob, cache: FactorCache | None = None,
              tol: float = 1e-11, m_max: int = 20, adj_tol: float = 1e-11, device="cuda"):
    """Probe voltages x (n_probe, n_out) of `prob` with amplitudes `amp`
    (n_src,) and capacitances `c_node` (n,), differentiable in both."""
    cache = cache or FactorCache(prob.gamma)
    return TransientFunction.apply(amp, c_node, prob, cache, tol, m_max, adj_tol, device)
