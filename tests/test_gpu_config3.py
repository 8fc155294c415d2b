"""The uneven batch (independent 2-layer meshes of 10k to 300k nodes, each
with its own factor, advanced concurrently) on the seeded 8-instance subset
of the 128 meshes against the oracle's stored first 100 ps, and against the
same instances run one at a time (identical results)."""
import os

import numpy as np
import pytest

from paper_1511_04519_amd import instances as I
from paper_1511_04519_amd import matex as M

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "config3_head.npz")


def test_config3_subset_concurrent_matches_oracle():
    g = np.load(GOLD)
    sub = [int(k) for k in g["instances"]]
    t_end = int(g["t_end"])
    probs, factors = [], []
    for k in sub:
        p = I.config3(k)
        assert str(g[f"digest_{k}"]) == p.digest()
        probs.append(I.Problem(p.name, p.netlist, p.sources, t_end, p.t_out[p.t_out <= t_end], p.probe))
        factors.append(M.matex_factor(p.netlist, p.gamma))
    print(f"[gpu-test] config3 subset {sub}: n {[q.netlist.n for q in probs]}", flush=True)
    res = M.matex_transient_many(factors, probs, tol=1e-10, m_max=20, n_streams=8, final=False)
    for k, q, F, (x, _, st) in zip(sub, probs, factors, res):
        err = np.abs(x.cpu().numpy() - g[f"x_{k}"]).max()
        print(f"config3[{k}] n {q.netlist.n}: max |x_gpu - x_oracle| = {err:.3e} V, bases {st['bases']}",
              flush=True)
        assert err <= 1e-9
        x1, _, _ = M.matex_transient(F, q, tol=1e-10, m_max=20, final=False)
        assert np.array_equal(x.cpu().numpy(), x1.cpu().numpy())
