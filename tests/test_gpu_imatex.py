"""Parity of the inverted Krylov subspace (I-MATEX, Sec. 3.3.1: X1 = G,
X2 = C, H_m = H'^-1) on the HIP path with the oracle's I-MATEX, scipy's dense
expm, the lemma of Sec. 3.3.3 and the exact modal solution."""
import numpy as np
import pytest
import scipy.linalg

from oracle import circuit as C
from oracle import reference as R
from oracle import rmatex as RM
from paper_1511_04519_amd import instances as I
from paper_1511_04519_amd import matex as M

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GAMMA = 1e-11
INV = M.MATEX_INVERTED


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def _note(msg):
    print(f"\n[case] {msg}", flush=True)


def test_inverted_krylov_step_matches_oracle_and_dense_expm():
    _note("inverted krylov_step 2x9x8")
    p = I.small(91, layers=2, nx=9, ny=8, n_src=3)
    nl = p.netlist
    F = M.matex_factor(nl, GAMMA)
    v = np.random.default_rng(5).random((2, nl.n)) * 1e-3
    taus = np.array([2e-12, 7.5e-12, 3e-11, 2e-10])
    tol = 1e-12
    out, m_used, est, ok = M.matex_krylov_step(F, _dev(v), taus, shift=-1, m_max=32, tol=tol)
    out = out.cpu().numpy()
    rp, ci, gv = C.assemble_G(nl)
    A = -C.csr_dense(rp, ci, gv) / nl.c_node[:, None]
    orc = RM.IMatex(nl)
    assert ok
    for r in range(2):
        ref, m_ref, est_ref, ok_ref = orc.expv(v[r], taus, tol, 32)
        assert ok_ref
        assert abs(int(m_used[r]) - m_ref) <= 1
        assert est[r] < tol
        for k, t in enumerate(taus):
            exact = scipy.linalg.expm(t * A) @ v[r]
            assert np.linalg.norm(out[k, r] - exact) <= 2 * tol
            assert np.linalg.norm(out[k, r] - ref[:, k]) <= (1e-13 if m_used[r] == m_ref else 3 * tol)


def test_inverted_krylov_step_eigenvector_exact_at_m1():
    """Lemma of Sec. 3.3.3 in the inverted space: m = 1 gives e^{lam t} u."""
    _note("inverted krylov_step eigenvector")
    from tests.helpers import uniform_mesh
    k, Rb, c, g0 = 9, 0.7, 3e-14, 0.02
    nl = uniform_mesh(k, Rb, c, g0)
    F = M.matex_factor(nl, GAMMA)
    ii, jj = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
    u = (np.cos(np.pi * 2 * (ii + 0.5) / k) * np.cos(np.pi * 5 * (jj + 0.5) / k)).ravel()
    lam = -(g0 + (2 / Rb) * (2 - np.cos(np.pi * 2 / k) - np.cos(np.pi * 5 / k))) / c
    taus = np.array([1e-13, 3e-12, 4e-11])
    out, m_used, est, ok = M.matex_krylov_step(F, _dev(u), taus, shift=-1, tol=1e-14)
    assert ok and m_used[0] == 1
    for q, t in enumerate(taus):
        assert np.abs(out[q, 0].cpu().numpy() - np.exp(lam * t) * u).max() <= 1e-12


@pytest.mark.parametrize("seed,layers,nx,ny,nsrc", [(101, 1, 8, 8, 5), (102, 2, 13, 11, 9),
                                                     (104, 3, 9, 12, 7)])
def test_inverted_transient_matches_oracle_and_modal(seed, layers, nx, ny, nsrc):
    _note(f"inverted transient seed={seed} {layers}x{nx}x{ny}")
    p = I.small(seed, layers=layers, nx=nx, ny=ny, n_src=nsrc, t_end=3 * I.NS)
    F = M.matex_factor(p.netlist, GAMMA)
    x, xf, st = M.matex_transient(F, p, tol=1e-12, m_max=30, krylov=INV)
    x = x.cpu().numpy()
    orc = RM.IMatex(p.netlist)
    xo, _ = orc.transient(p, tol=1e-12, m_max=30)
    ym, ym_end = R.modal(p)
    print(f"gpu bases {st['bases']} dims {st['krylov_dims']} halvings {st['halvings']}; "
          f"oracle bases {orc.stats.bases} dims {sum(orc.stats.m_hist)}", flush=True)
    assert st["shift_downs"] == 0
    assert np.abs(x - (p.netlist.vdd - ym)).max() <= 1e-10
    assert np.abs(x - xo).max() <= 1e-10
    assert np.abs(xf.cpu().numpy() - (p.netlist.vdd - ym_end)).max() <= 1e-10


def test_inverted_config0_matches_modal_truth():
    """32x32 workload with the inverted space: relative error <= 1e-9; the
    Krylov dimensions of both spaces are printed (Tab. 1's m_a and m_p)."""
    _note("inverted transient config0")
    p = I.config0()
    F = M.matex_factor(p.netlist, p.gamma)
    ym, _ = R.modal(p)
    for name, kr in (("R-MATEX", M.MATEX_RATIONAL), ("I-MATEX", INV)):
        x, _, st = M.matex_transient(F, p, tol=1e-11, m_max=30, krylov=kr)
        x = x.cpu().numpy()
        err = np.abs(x - (p.netlist.vdd - ym)).max() / np.abs(x).max()
        print(f"{name}: rel err {err:.2e}, bases {st['bases']}, m_a {st['krylov_dims'] / st['bases']:.2f}, "
              f"m_p {st['m_peak']}, pairs {st['solve_pairs_m']}", flush=True)
        assert err <= 1e-9


def test_inverted_batched_equals_plain():
    """The batched mode in the inverted space takes the plain mode's steps."""
    _note("inverted batched vs plain")
    p = I.small(121, layers=2, nx=12, ny=10, n_src=14, t_end=2 * I.NS, n_groups=5)
    F = M.matex_factor(p.netlist, GAMMA)
    xp, fp, sp = M.matex_transient(F, p, tol=1e-12, m_max=30, krylov=INV)
    xb, fb, sb = M.matex_transient(F, p, tol=1e-12, m_max=30, mode=M.MATEX_BATCHED, krylov=INV)
    ym, _ = R.modal(p)
    assert sb["bases"] == sp["bases"] and sb["krylov_dims"] == sp["krylov_dims"]
    assert np.abs(xb.cpu().numpy() - xp.cpu().numpy()).max() <= 1e-12
    assert np.abs(fb.cpu().numpy() - fp.cpu().numpy()).max() <= 1e-12
    assert np.abs(xp.cpu().numpy() - (p.netlist.vdd - ym)).max() <= 1e-10


def test_inverted_space_refusals():
    """The adjoint runs the rational space only; an unknown subspace is refused."""
    _note("inverted refusals")
    p = I.small(122, nx=6, ny=5, n_src=2, t_end=1 * I.NS)
    F = M.matex_factor(p.netlist, GAMMA)
    w = _dev(np.ones((p.probe.size, p.t_out.size)))
    opts = M.RunOpts(1e-10, 20, M.MATEX_PLAIN, 1, 1.0, 0, 0, INV)
    keep = []
    pr = M._problem_struct(p, keep)
    ga = torch.empty(p.sources.n_src, dtype=torch.float64, device="cuda:0")
    st = M.lib().matex_adjoint(F.handle, M.ctypes.byref(pr), M.ctypes.byref(opts), M._ptr(w), M._ptr(ga),
                               None, M._stream())
    assert st == M.MATEX_E_INVALID
    with pytest.raises(M.MatexError) as e:
        M.matex_transient(F, p, tol=1e-10, krylov=2)
    assert e.value.status == M.MATEX_E_INVALID


def test_inverted_uneven_instances():
    """Independent grids of uneven size in the inverted space, advanced
    concurrently: equal to one-at-a-time runs and to the modal solution."""
    _note("inverted uneven instances")
    probs = [I.small(131 + i, layers=1 + i % 2, nx=6 + 3 * i, ny=5 + 2 * i, n_src=3 + i, t_end=2 * I.NS)
             for i in range(4)]
    factors = [M.matex_factor(q.netlist, GAMMA) for q in probs]
    res = M.matex_transient_many(factors, probs, tol=1e-12, m_max=30, n_streams=3, krylov=INV)
    for q, F, (x, _, st) in zip(probs, factors, res):
        x1, _, st1 = M.matex_transient(F, q, tol=1e-12, m_max=30, krylov=INV, final=False)
        assert np.array_equal(x.cpu().numpy(), x1.cpu().numpy())
        assert st["bases"] == st1["bases"] and st["shift_downs"] == 0
        ym, _ = R.modal(q)
        assert np.abs(x.cpu().numpy() - (q.netlist.vdd - ym)).max() <= 1e-10
