"""The one-vector iteration pipeline: checks on their own stream that wait for
their iteration's ticket, iterations launched ahead of the pending decision
(and cut short when it stops the process), and the device-clock diagnostics.
Expected values come from the CPU oracle (R-MATEX written from the paper)."""
import os

import numpy as np
import pytest

from oracle import rmatex as RM
from paper_1511_04519_amd import instances as I
from paper_1511_04519_amd import matex as M

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
GAMMA = 1e-11


def test_pipeline_counts_and_diagnostics(capfd):
    """Alg. 1 / Alg. 2 through the pipelined loop: the result matches the
    oracle; every kept Krylov dimension was computed once, and iterations
    computed past a stopping decision (counted in solve_pairs_m) are at most
    one per decision; the device-clock stamps (MATEX_HOST_TIMES=1) change no
    bit of the result."""
    print("\n[case] pipeline small seed=102 2x13x11", flush=True)
    p = I.small(102, layers=2, nx=13, ny=11, n_src=9, t_end=3 * I.NS)
    F = M.matex_factor(p.netlist, GAMMA)
    x, xf, st = M.matex_transient(F, p, tol=1e-12, m_max=20)
    torch.cuda.synchronize()
    x = x.cpu().numpy()
    xo, _ = RM.RMatex(p.netlist, GAMMA).transient(p, tol=1e-12, m_max=20)
    assert np.abs(x - xo).max() <= 1e-10
    discarded = st["solve_pairs_m"] - st["krylov_dims"]
    assert 0 <= discarded <= 2 * st["bases"], st
    old = os.environ.get("MATEX_HOST_TIMES")
    os.environ["MATEX_HOST_TIMES"] = "1"
    try:
        x2, xf2, st2 = M.matex_transient(F, p, tol=1e-12, m_max=20)
        torch.cuda.synchronize()
    finally:
        if old is None:
            del os.environ["MATEX_HOST_TIMES"]
        else:
            os.environ["MATEX_HOST_TIMES"] = old
    err = capfd.readouterr().err
    assert "[matex] stamps iter -> iter" in err
    assert np.array_equal(x2.cpu().numpy(), x)
    assert np.array_equal(xf2.cpu().numpy(), xf.cpu().numpy())
    assert st2["krylov_dims"] == st["krylov_dims"] and st2["segments"] == st["segments"]


def test_graph_replayed_iterations_match_eager(monkeypatch):
    """Krylov iterations replayed from captured graphs (MATEX_GRAPHS=1): each
    (shift, dimension) graph is replayed many times in one transient, between
    the checks' eager launches and the host's synchronisations; the outputs
    equal the eager launches' bit for bit, on two transients in a row."""
    import numpy as np
    from paper_1511_04519_amd import instances as I
    from paper_1511_04519_amd import matex as M
    p = I.small(91, layers=2, nx=14, ny=12, n_src=12, t_end=2 * I.NS)
    F = M.matex_factor(p.netlist, p.gamma)
    monkeypatch.setenv("MATEX_GRAPHS", "0")
    xe, fe, se = M.matex_transient(F, p, tol=1e-12)
    monkeypatch.setenv("MATEX_GRAPHS", "1")
    for _ in range(2):
        xg, fg, sg = M.matex_transient(F, p, tol=1e-12)
        assert np.array_equal(xg.cpu().numpy(), xe.cpu().numpy())
        assert np.array_equal(fg.cpu().numpy(), fe.cpu().numpy())
        assert (sg["bases"], sg["krylov_dims"]) == (se["bases"], se["krylov_dims"])


def test_tuner_cache_replays_the_schedule(monkeypatch, tmp_path):
    """With MATEX_TUNE_CACHE set, the first factor of a structure times the
    batched schedule's candidates and records the choice; a second factor of
    the same structure takes the recorded choice without timing, and
    another structure gets its own line."""
    from paper_1511_04519_amd import instances as I
    from paper_1511_04519_amd import matex as M
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("MATEX_TUNE_CACHE", str(path))
    p = I.small(93, layers=2, nx=30, ny=24, n_src=4)
    F1 = M.matex_factor(p.netlist, p.gamma)
    assert F1.info["seconds_tune"] > 0.0 and len(path.read_text().splitlines()) == 1
    F2 = M.matex_factor(p.netlist, p.gamma)
    assert F2.info["seconds_tune"] == 0.0
    assert M.matex_factor_describe(F2) == M.matex_factor_describe(F1)
    q = I.small(94, layers=1, nx=40, ny=20, n_src=4)
    M.matex_factor(q.netlist, q.gamma)
    assert len(path.read_text().splitlines()) == 2
    b = torch.as_tensor(np.random.default_rng(1).random((64, p.netlist.n)), device="cuda:0")
    x1 = M.matex_solve(F1, 0, b)
    x2 = M.matex_solve(F2, 0, b)
    assert torch.equal(x1, x2)
