"""GPU trapezoidal rule (Eq. 2 at a fixed step, the comparator of the
paper's runtime tables) against the oracle's trapezoidal stepping with the
same fixed grid (input sampled at the step ends)."""
import numpy as np
import pytest

from oracle import reference as R
from paper_1511_04519_amd import instances as I
from paper_1511_04519_amd import matex as M

pytestmark = pytest.mark.gpu
H = 10 * I.PS


def _note(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _factor_tr(p, h_fs=H):
    # C + (h/2) G = h (C/h + G/2): the step matrix, as the ladder's first shift
    return M.matex_factor(p.netlist, 0.5 * h_fs * 1e-15, n_shifts=1)


@pytest.mark.parametrize("which", ["config0", "small"])
def test_tr_matches_oracle(which):
    p = I.config0() if which == "config0" else I.small(77, layers=2, nx=13, ny=11, n_src=9, t_end=3 * I.NS)
    _note(f"trapezoidal {which}: n={p.netlist.n}, {p.t_end // H} steps")
    F = _factor_tr(p)
    y, yf, st = M.matex_trapezoidal(F, p, H, droop=True)
    y_ref, yend_ref, pairs = R.trapezoidal(p, H, align=False)
    err = np.abs(y.cpu().numpy() - y_ref).max()
    print(f"max |y_gpu - y_oracle| = {err:.3e} V (max droop {np.abs(y_ref).max():.3e}), steps {st['segments']}",
          flush=True)
    assert st["segments"] == pairs == p.t_end // H
    assert err <= 1e-12 * max(1.0, np.abs(y_ref).max())
    assert np.abs(yf.cpu().numpy() - yend_ref).max() <= 1e-12
    # x = Vdd - y
    x, _, _ = M.matex_trapezoidal(F, p, H, final=False)
    assert np.abs(x.cpu().numpy() - (p.netlist.vdd - y_ref)).max() <= 1e-12


def test_tr_config1_window_matches_oracle():
    p = I.config1()
    T = 200 * I.PS
    q = I.Problem(p.name, p.netlist, p.sources, T, p.t_out[p.t_out <= T], p.probe)
    _note("trapezoidal 180k-node grid, 20 steps")
    F = _factor_tr(q)
    y, _, st = M.matex_trapezoidal(F, q, H, droop=True, final=False)
    y_ref, _, _ = R.trapezoidal(q, H, align=False)
    err = np.abs(y.cpu().numpy() - y_ref).max()
    print(f"config1 window: max |y_gpu - y_oracle| = {err:.3e} V", flush=True)
    assert err <= 1e-12


def test_tr_argument_checks():
    p = I.small(78, nx=6, ny=6, n_src=2, t_end=1 * I.NS)
    F = _factor_tr(p)
    for h in (0, 7 * I.PS):   # zero; does not divide t_end
        with pytest.raises(M.MatexError) as e:
            M.matex_trapezoidal(F, p, h)
        assert e.value.status == M.MATEX_E_INVALID
    G2 = M.matex_factor(p.netlist, 1e-11, n_shifts=1)   # gamma 10 ps is not h / 2 = 5 ps
    with pytest.raises(M.MatexError) as e:
        M.matex_trapezoidal(G2, p, H)
    assert e.value.status == M.MATEX_E_INVALID
