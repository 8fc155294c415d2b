"""Pins of the oracle's I-MATEX (the inverted Krylov subspace of Sec. 3.3.1,
X1 = G, X2 = C, H_m = H'^-1 with H' the Arnoldi matrix of A^-1) against facts
outside it: the single-RC closed form, the lemma of Sec. 3.3.3, scipy's
dense expm, the Arnoldi relation of the inverted operator, the Ritz values of
the slowest modes, and the exact modal solution of a transient."""
import numpy as np
import pytest
import scipy.linalg

from oracle import circuit as C
from oracle import reference as R
from oracle import rmatex as RM
from paper_1511_04519_amd import instances as I
from tests.helpers import single_rc, uniform_mesh

NS = I.NS


def _dense_A(nl):
    rp, ci, gv = C.assemble_G(nl)
    return -C.csr_dense(rp, ci, gv) / nl.c_node[:, None]


def test_imatex_single_rc_exact_at_m1():
    """C y' = -g y: the inverted space of one node is exact at m = 1 and
    gives V exp(-t g / c)."""
    c, g = 3e-14, 0.7
    s = RM.IMatex(single_rc(c, g))
    taus = np.array([1e-15, 1e-13, 1e-12, 5e-12, 3e-11])
    out, m, est, ok = s.expv(np.array([0.8]), taus, 1e-14, 20)
    assert ok and m == 1 and est == 0.0
    ref = 0.8 * np.exp(-taus * g / c)
    # the exponent -tau / (c/g) carries the rounding of the solve g^-1 c and
    # of its inverse: a few units of eps, times the exponent's size
    assert (np.abs(out[0] - ref) <= 1e-15 * (1 + taus * g / c) * ref).all()


def test_imatex_lemma_generalized_eigenvector():
    """Lemma of Sec. 3.3.3 for the inverted space: an eigenvector u of the
    pencil (-G, C) spans an invariant space, so m = 1 gives e^{lam t} u."""
    k, Rb, c, g0 = 7, 0.8, 2e-14, 0.03
    s = RM.IMatex(uniform_mesh(k, Rb, c, g0))
    ii, jj = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
    for pm, qm in [(0, 0), (1, 2), (3, 5), (6, 6)]:
        u = (np.cos(np.pi * pm * (ii + 0.5) / k) * np.cos(np.pi * qm * (jj + 0.5) / k)).ravel()
        lam = -(g0 + (2 / Rb) * (2 - np.cos(np.pi * pm / k) - np.cos(np.pi * qm / k))) / c
        taus = np.array([1e-14, 1e-12, 2e-11])
        out, m, est, ok = s.expv(u, taus, 1e-14, 20)
        assert ok and m == 1
        for q, tau in enumerate(taus):
            assert np.abs(out[:, q] - np.exp(lam * tau) * u).max() <= 1e-12 * np.abs(u).max()


@pytest.mark.parametrize("seed,tau", [(91, 2e-12), (92, 5e-11), (93, 1e-9)])
def test_imatex_expv_matches_scipy_dense(seed, tau):
    """e^{tau A} v from the inverted space against scipy's dense expm of
    A = -C^-1 G (a stiff RC mesh, n <= 200), at the tolerance asked."""
    p = I.small(seed, layers=2, nx=9, ny=8, n_src=3)
    A = _dense_A(p.netlist)
    v = np.random.default_rng(seed).random(p.netlist.n) * 1e-3
    s = RM.IMatex(p.netlist)
    out, m, est, ok = s.expv(v, [tau], 1e-13, 40)
    ref = scipy.linalg.expm(tau * A) @ v
    assert ok
    assert np.abs(out[:, 0] - ref).max() <= 1e-11 * np.abs(v).max()


def test_imatex_arnoldi_relation_and_ritz_values():
    """G^-1 C V_m = V_m H' + h v_{m+1} e_m^T with H' = -H_m^-1, an orthonormal
    V_m; and the eigenvalues of H_m closest to zero approach the slowest
    modes of A first (the reason for inverting, Sec. 3.3.1)."""
    p = I.small(94, nx=7, ny=6)
    nl = p.netlist
    A = _dense_A(nl)
    K = -np.linalg.inv(A)                       # G^-1 C
    s = RM.IMatex(nl)
    v = np.random.default_rng(5).random(nl.n)
    m = 10
    b, _ = s.arnoldi(v, [1e-12], 0.0, m)        # tol 0: runs to m
    V = b.V
    assert np.abs(V.T @ V - np.eye(m)).max() <= 1e-12
    Hp = -np.linalg.inv(b.Hm)
    resid = K @ V - V @ Hp
    assert np.abs(V.T @ resid).max() <= 1e-10 * np.abs(Hp).max()
    assert np.isclose(np.linalg.norm(resid), b.h_next, rtol=1e-8)
    lam = np.sort(np.linalg.eigvals(A).real)[::-1]           # slowest first
    ritz = np.sort(np.linalg.eigvals(b.Hm).real)[::-1]
    assert np.all(ritz < 0)
    assert abs(ritz[0] - lam[0]) <= 1e-8 * abs(lam[0])


@pytest.mark.parametrize("tol,bound", [(1e-10, 1e-9), (1e-12, 1e-11)])
def test_imatex_transient_matches_modal(tol, bound):
    """The whole Alg. 2 run with the inverted space (one factor, halving
    only) against the exact modal solution of the pulse-driven mesh."""
    p = I.small(95, layers=2, nx=8, ny=7, n_src=6, t_end=2 * NS)
    ym, _ = R.modal(p)
    x, _ = RM.IMatex(p.netlist).transient(p, tol=tol)
    err = np.abs((p.netlist.vdd - x) - ym).max() / np.abs(x).max()
    assert err <= bound
