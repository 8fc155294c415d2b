"""GPU parity of the batched mode (Sec. 3.1 subtasks advanced together).

Every case runs the same problem through the one-subtask-at-a-time path and
the batched path and compares both with the oracle and with the exact modal
solution. The batched path takes the same per-subtask decisions (offsets,
shift of the ladder, step-down, halving), so the two differ only by the
rounding of their reductions.
"""
import numpy as np
import pytest

from paper_1511_04519_amd import instances as I
from paper_1511_04519_amd import matex as M
from oracle import reference as R
from oracle import rmatex as RM

pytestmark = pytest.mark.gpu

GAMMA = 1e-11


def _note(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _run_both(F, p, tol):
    xp, fp, sp = M.matex_transient(F, p, tol=tol, m_max=20, mode=M.MATEX_PLAIN)
    xb, fb, sb = M.matex_transient(F, p, tol=tol, m_max=20, mode=M.MATEX_BATCHED)
    return (xp.cpu().numpy(), fp.cpu().numpy(), sp), (xb.cpu().numpy(), fb.cpu().numpy(), sb)


@pytest.mark.parametrize("seed,layers,nx,ny,nsrc,groups", [
    (401, 2, 12, 10, 16, 5),      # 5 subtasks, one batch
    (402, 1, 17, 13, 24, 24),     # one subtask per source
    (403, 3, 9, 8, 9, 1),         # a single subtask
])
def test_batched_matches_plain_oracle_modal(seed, layers, nx, ny, nsrc, groups):
    _note(f"batched seed={seed} {layers}x{nx}x{ny} sources={nsrc} groups={groups}")
    p = I.small(seed, layers=layers, nx=nx, ny=ny, n_src=nsrc, t_end=3 * I.NS, n_groups=groups)
    if groups == nsrc:
        p.sources.group[:] = np.arange(nsrc, dtype=np.int32)
    F = M.matex_factor(p.netlist, GAMMA)
    (xp, fp, sp), (xb, fb, sb) = _run_both(F, p, 1e-12)
    ym, ym_end = R.modal(p)
    xo, _ = RM.RMatex(p.netlist, GAMMA).transient(p, tol=1e-12, m_max=20)
    vdd = p.netlist.vdd
    print("plain", sp, "\nbatched", sb, flush=True)
    assert sb["subtasks"] == sp["subtasks"] == len(np.unique(p.sources.group))
    assert np.abs(xb - (vdd - ym)).max() <= 1e-10
    assert np.abs(xb - xo).max() <= 1e-10
    assert np.abs(xb - xp).max() <= 1e-10
    assert np.abs(fb - (vdd - ym_end)).max() <= 1e-10
    assert np.abs(fb - fp).max() <= 1e-10
    # same per-subtask steps; one multi-right-hand-side pair per lockstep
    # iteration instead of one pair per subtask and iteration
    assert sb["segments"] == sp["segments"]
    assert abs(sb["bases"] - sp["bases"]) <= 2
    assert sb["solve_pairs_m"] < sp["solve_pairs_m"] or sp["subtasks"] == 1


def test_batched_two_batches():
    """More subtasks than one batch holds (64): two batches summed."""
    _note("batched 70 subtasks")
    p = I.small(404, layers=1, nx=10, ny=9, n_src=70, t_end=2 * I.NS)
    p.sources.group[:] = np.arange(70, dtype=np.int32)
    F = M.matex_factor(p.netlist, GAMMA)
    (xp, fp, sp), (xb, fb, sb) = _run_both(F, p, 1e-12)
    ym, ym_end = R.modal(p)
    print("plain", sp, "\nbatched", sb, flush=True)
    assert sb["subtasks"] == 70
    assert np.abs(xb - (p.netlist.vdd - ym)).max() <= 1e-10
    assert np.abs(xb - xp).max() <= 1e-10
    assert np.abs(fb - (p.netlist.vdd - ym_end)).max() <= 1e-10


def test_batched_edge_cases():
    _note("batched edge cases")
    p = I.small(405, nx=7, ny=5, n_src=6, t_end=1 * I.NS, n_groups=3)
    F = M.matex_factor(p.netlist, GAMMA)
    # no sources: the grid stays at Vdd
    q = I.Problem("empty", p.netlist, I.Sources(*(np.zeros(0, dt) for dt in
                  (np.int32, float, np.int64, np.int64, np.int64, np.int64, np.int32))),
                  p.t_end, p.t_out, p.probe)
    x, xf, st = M.matex_transient(F, q, mode=M.MATEX_BATCHED)
    assert np.array_equal(x.cpu().numpy(), np.full(x.shape, p.netlist.vdd))
    assert np.array_equal(xf.cpu().numpy(), np.full(xf.shape, p.netlist.vdd))
    # one output time, repeated probes and a pad node; group ids with gaps
    p.sources.group[:] = np.where(p.sources.group == 1, 7, p.sources.group)
    q = I.Problem("one-out", p.netlist, p.sources, p.t_end, np.array([p.t_end // 3]),
                  np.array([0, 0, p.netlist.pad_node[0], 5], np.int32))
    x, _, st = M.matex_transient(F, q, tol=1e-12, mode=M.MATEX_BATCHED)
    ym, _ = R.modal(q)
    assert np.abs(x.cpu().numpy() - (1.0 - ym)).max() <= 1e-10
    # an output time on a transition spot, and at t = 0
    t_spot = int(p.sources.delay[0])
    q = I.Problem("spot", p.netlist, p.sources, p.t_end,
                  np.unique(np.array([0, t_spot, t_spot + 1, p.t_end])), p.probe)
    x, _, _ = M.matex_transient(F, q, tol=1e-12, mode=M.MATEX_BATCHED)
    ym, _ = R.modal(q)
    assert np.abs(x.cpu().numpy() - (1.0 - ym)).max() <= 1e-10
    # droop outputs: Vdd - x, plain and batched
    for md in (M.MATEX_PLAIN, M.MATEX_BATCHED):
        x, xf, _ = M.matex_transient(F, q, tol=1e-12, mode=md)
        y, yf, _ = M.matex_transient(F, q, tol=1e-12, mode=md, droop=True)
        assert np.abs((p.netlist.vdd - x.cpu().numpy()) - y.cpu().numpy()).max() <= 1e-15
        assert np.abs((p.netlist.vdd - xf.cpu().numpy()) - yf.cpu().numpy()).max() <= 1e-15
        assert np.abs(y.cpu().numpy() - ym).max() <= 1e-10
    # invalid mode
    with pytest.raises(M.MatexError) as e:
        M.matex_transient(F, q, mode=7)
    assert e.value.status == M.MATEX_E_INVALID


def test_uneven_instances_concurrent():
    """Independent grids of different sizes (own factor each) on concurrent
    streams: each instance gives exactly what a call on its own gives, and
    matches the oracle and the exact modal solution."""
    _note("uneven instances")
    shapes = [(1, 9, 7, 5), (2, 14, 11, 9), (1, 23, 6, 4), (3, 8, 8, 6), (2, 5, 17, 3), (1, 12, 12, 7)]
    probs = [I.small(500 + k, layers=L, nx=nx, ny=ny, n_src=ns, t_end=2 * I.NS)
             for k, (L, nx, ny, ns) in enumerate(shapes)]
    facs = [M.matex_factor(q.netlist, GAMMA) for q in probs]
    many = M.matex_transient_many(facs, probs, tol=1e-12, n_streams=3)
    for q, F, (x, xf, st) in zip(probs, facs, many):
        x1, xf1, st1 = M.matex_transient(F, q, tol=1e-12)
        assert np.array_equal(x.cpu().numpy(), x1.cpu().numpy())
        assert np.array_equal(xf.cpu().numpy(), xf1.cpu().numpy())
        assert st["segments"] == st1["segments"] and st["krylov_dims"] == st1["krylov_dims"]
        ym, _ = R.modal(q)
        assert np.abs(x.cpu().numpy() - (q.netlist.vdd - ym)).max() <= 1e-10
    # one failing instance: the call reports it by index
    bad = I.Problem("bad", probs[1].netlist, probs[1].sources, probs[1].t_end,
                    np.array([10, 5]), probs[1].probe)
    with pytest.raises(M.MatexError) as e:
        M.matex_transient_many(facs[:2], [probs[0], bad], n_streams=2)
    assert e.value.status == M.MATEX_E_INVALID and "instance 1" in str(e.value)


@pytest.mark.parametrize("seed,layers,nx,ny,nsrc,groups", [
    (421, 2, 14, 11, 20, 7), (422, 1, 19, 15, 30, 30), (423, 3, 10, 9, 12, 3)])
def test_batched_independent_equals_lockstep(seed, layers, nx, ny, nsrc, groups):
    """Subtasks advancing on their own (slope changes from solved timing
    columns) and in lockstep generations (whole-batch G solves) take the
    same steps and agree to rounding; both equal the oracle's modal truth."""
    _note(f"independent vs lockstep seed={seed}")
    p = I.small(seed, layers=layers, nx=nx, ny=ny, n_src=nsrc, t_end=3 * I.NS, n_groups=groups)
    F = M.matex_factor(p.netlist, GAMMA)
    xa, fa, sa = M.matex_transient(F, p, tol=1e-12, m_max=20, mode=M.MATEX_BATCHED, independent=True)
    xl, fl, sl = M.matex_transient(F, p, tol=1e-12, m_max=20, mode=M.MATEX_BATCHED)
    assert (sa["segments"], sa["bases"], sa["krylov_dims"]) == (sl["segments"], sl["bases"], sl["krylov_dims"])
    d = float((xa - xl).abs().max())
    print(f"max |independent - lockstep| = {d:.3e}, pairs {sa['solve_pairs_m']} vs {sl['solve_pairs_m']}", flush=True)
    assert d <= 1e-13
    assert float((fa - fl).abs().max()) <= 1e-13
    ym, _ = R.modal(p)
    assert np.abs(xa.cpu().numpy() - (p.netlist.vdd - ym)).max() <= 1e-10
