"""torch.autograd over the transient (forward: matex_transient, backward:
matex_adjoint) against the oracle's gradients: amplitudes by linearity of the
exact modal solution, capacitances by complex-step differentiation of the
dense Eq. 5 solution."""
import numpy as np
import pytest

from oracle import adjoint as A
from paper_1511_04519_amd import instances as I
from paper_1511_04519_amd import matex as M

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _note(msg):
    print(f"\n[case] {msg}", flush=True)


def test_autograd_linear_objective_matches_oracle():
    from paper_1511_04519_amd import autograd as AG
    _note("autograd: linear objective, amplitudes and capacitances")
    p = I.small(611, layers=1, nx=6, ny=5, n_src=4, t_end=1 * I.NS)
    w = np.random.default_rng(611).standard_normal((p.probe.size, p.t_out.size))
    w[:, ::2] = 0.0
    amp = torch.tensor(p.sources.amp, dtype=torch.float64, requires_grad=True)
    c = torch.tensor(p.netlist.c_node, dtype=torch.float64, requires_grad=True)
    cache = AG.FactorCache(p.gamma)
    x = AG.transient(amp, c, p, cache, tol=1e-12, adj_tol=1e-11)
    # the forward pass is the library's transient, bit for bit
    F = M.matex_factor(p.netlist, p.gamma)
    x_ref, _, _ = M.matex_transient(F, p, tol=1e-12, final=False)
    assert torch.equal(x, x_ref)
    J = (torch.as_tensor(w, device=x.device) * x).sum()
    J.backward()
    ra = A.amp_gradient(p, w)
    rc = A.c_gradient_cs(p, w)
    ea = np.abs(amp.grad.numpy() - ra).max() / np.abs(ra).max()
    ec = np.abs(c.grad.numpy() - rc).max() / np.abs(rc).max()
    print(f"amplitude rel err {ea:.3e}, capacitance rel err {ec:.3e}", flush=True)
    assert ea <= 1e-8
    assert ec <= 2e-6
    # unchanged capacitances reuse the factor; changed ones rebuild it
    AG.transient(amp.detach(), c.detach(), p, cache, tol=1e-12)
    assert cache.builds == 1
    c2 = c.detach().clone()
    c2[3] *= 1.5
    x2 = AG.transient(amp.detach(), c2, p, cache, tol=1e-12)
    assert cache.builds == 2
    nl = I.Netlist(p.netlist.n, p.netlist.br_a, p.netlist.br_b, p.netlist.br_g, c2.numpy(),
                   p.netlist.pad_node, p.netlist.pad_g, p.netlist.vdd, p.netlist.coord)
    q = I.Problem(p.name, nl, p.sources, p.t_end, p.t_out, p.probe)
    x2_ref, _, _ = M.matex_transient(M.matex_factor(nl, p.gamma), q, tol=1e-12, final=False)
    assert torch.equal(x2, x2_ref)


def test_autograd_droop_penalty_matches_oracle():
    """J = sum max(0, y - theta)^2 over the probes and output times (y the
    droop Vdd - x), theta the 90th percentile of the droops: dJ/dx comes from
    torch, the gradient from the adjoint."""
    from paper_1511_04519_amd import autograd as AG
    _note("autograd: thresholded droop objective")
    p = I.small(604, layers=2, nx=10, ny=8, n_src=7, t_end=2 * I.NS)
    y_ex = p.netlist.vdd - A.x_probes(p)
    theta = float(np.quantile(y_ex, 0.9))
    amp = torch.tensor(p.sources.amp, dtype=torch.float64, requires_grad=True)
    c = torch.tensor(p.netlist.c_node, dtype=torch.float64)
    x = AG.transient(amp, c, p, tol=1e-12, adj_tol=1e-10)
    J = ((p.netlist.vdd - x - theta).clamp(min=0.0) ** 2).sum()
    J.backward()
    dJdx = -2.0 * np.maximum(0.0, y_ex - theta)
    ra = A.amp_gradient(p, dJdx)
    err = np.abs(amp.grad.numpy() - ra).max() / np.abs(ra).max()
    print(f"amplitude rel err {err:.3e}", flush=True)
    assert err <= 1e-7
