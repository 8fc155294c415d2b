"""The allocation-free solve (matex_solve_noalloc) against matex_solve with
one right-hand side: the same kernels in the same order, so the same bits,
on two calls in a row (the second on a smaller grid, so the shared scratch
holds the first call's larger contents), with and without a scale; and the
size limit of its scratch refused before any device work."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1511_04519_amd import instances as I
from paper_1511_04519_amd import matex as M

pytestmark = pytest.mark.gpu


def _solve_pair(F, which, b, scale):
    ref = M.matex_solve(F, which, b, scale)
    x = torch.full_like(b, float("nan"))
    M.matex_solve_noalloc(F, which, b, x, scale)
    torch.cuda.synchronize()
    return ref, x


def test_noalloc_solve_matches_matex_solve_twice_second_smaller():
    big = I.small(31, layers=2, nx=40, ny=37, n_src=4)
    small = I.small(32, layers=1, nx=9, ny=7, n_src=2)
    for prob, seed in ((big, 1), (small, 2)):
        F = M.matex_factor(prob.netlist, 1e-11)
        n = prob.netlist.n
        g = torch.Generator().manual_seed(seed)
        b = torch.randn(n, generator=g, dtype=torch.float64).cuda()
        c = torch.as_tensor(prob.netlist.c_node, dtype=torch.float64).cuda()
        for which, scale in ((0, c), (-1, None), (3, c)):
            ref, x = _solve_pair(F, which, b, scale)
            assert torch.equal(ref, x), (n, which, float((ref - x).abs().max()))
        # and the result solves the system: (C + gamma G) x = C b for shift 0
        ref, x = _solve_pair(F, 0, b, c)
        assert torch.isfinite(x).all()


def test_noalloc_solve_refuses_a_factor_beyond_its_scratch():
    """The 1M-node grid with one-node leaves needs 3 n + n_upd = 8.52 Mi
    doubles, beyond the 8 Mi of the scratch: refused before device work."""
    p = I.small(33, layers=1, nx=8, ny=8, n_src=1)
    F = M.matex_factor(p.netlist, 1e-11)
    assert 3 * F.info["n"] + F.info["n_upd"] <= (8 << 20)
    q = I.config2()
    F2 = M.matex_factor(q.netlist, q.gamma, leaf_max=1, n_shifts=1)
    need = 3 * F2.info["n"] + F2.info["n_upd"]
    assert need > (8 << 20), need
    b = torch.zeros(q.netlist.n, dtype=torch.float64, device="cuda")
    x = torch.full_like(b, 7.0)
    with pytest.raises(M.MatexError) as e:
        M.matex_solve_noalloc(F2, 0, b, x)
    assert e.value.status == M.MATEX_E_INVALID
    assert "64 MiB" in str(e.value)
    torch.cuda.synchronize()
    assert bool((x == 7.0).all())   # nothing written
