"""R-MATEX: rational-Krylov exponential integrator for C y' = -G y + i(t)
(oracle, step by step in the paper's order).

Test infrastructure (see the package docstring).

Paper map:
  * Eq. 5 / Eq. 6: for an input that is linear on [t, t+h],
      x(t+h) = e^{hA} (x(t) + F(t,h)) - P(t,h),
      F = A^-1 b(t) + A^-2 (b(t+h) - b(t))/h,
      P = A^-1 b(t+h) + A^-2 (b(t+h) - b(t))/h.
    With A = -C^-1 G and b = C^-1 i (droop form, see circuit.py):
      A^-1 b(t) = -G^-1 i(t),  A^-2 (db/h) = G^-1 C G^-1 s  (s = di/dt),
    so with y0 = G^-1 i(t_a), z1 = G^-1 s, z2 = G^-1 C z1:
      F = -y0 + z2,   P(tau) = -y0 - tau z1 + z2,
      y(t_a + tau) = e^{tau A} v + y0 + tau z1 - z2,   v = y(t_a) - y0 + z2.
  * Alg. 1 with the R-MATEX inputs of Sec. 3.3.2: X1 = C + gamma G (factored
    once), X2 = C; each Arnoldi step is w = X1^-1 (X2 v_j), then modified
    Gram-Schmidt, h_{j+1,j} = ||w||, v_{j+1} = w / h_{j+1,j}.
  * Eq. 9: e^{hA} v ~= ||v|| V_m e^{h H_m} e_1 with H_m = (I - Ht_m^-1)/gamma.
  * Convergence (Sec. 3.3.3, the empirical estimate that replaces Eq. 8/10):
      r_m(h) = ||v|| * |h_{m+1,m} e_m^T e^{h H_m} e_1|,  stop when r < eps.
  * Alg. 2: the time loop. Krylov bases are generated at the transition spots
    of the subtask (its LTS) and reused for every later output time
    (snapshot) before the next spot by rescaling H_m with the step (Sec. 2.4).
  * Sec. 3.1: subtasks are groups of sources; by superposition the grid
    response is the sum of the subtask responses.

Readings where the paper is silent:
  * The check set of the stopping test is every snapshot offset in the
    segment plus the segment length.
  * The estimate is the larger of the paper's empirical form and the change
    of the approximation from dimension j-1 to j, ||v|| ||u_j - [u_{j-1}; 0]||
    with u_j = e^{tau H_j} e_1 and u_0 = 1. The paper's form alone is a single
    entry of u_j that can be accidentally tiny when tau is well below gamma
    (seen on the 32x32 mesh: 3e-13 estimated, 1.6e-9 true); the difference
    term bounds the previous iterate's error and keeps the test honest there.
    A safety factor S multiplies the estimate (S = 1 by default).
  * Happy breakdown: h_{j+1,j} <= 1e-14 max|h_ij| ends the process with the
    exact result.
  * Shift ladder. One shift gamma resolves e^{tau A} well only for tau from
    about gamma/10 upwards (Sec. 3.3.2 asks for gamma near the step sizes);
    two transition spots a few fs apart, or an output time just after a spot,
    ask for far shorter steps. So C + gamma_k G is factored once for each
    gamma_k = gamma * 10^-k, k < K (no refactorisation in the time loop). A
    segment uses the largest gamma_k with tau_1 >= rho * gamma_k, tau_1 being
    its first check offset (rho = 1 by default: gamma near the step, as
    Sec. 3.3.2 advises); with k > 0 the segment is cut after the last check
    offset <= 10 gamma_k and the rest starts a new segment (same input slope).
  * If m_max is reached without convergence, the segment is tried again with
    the next smaller shift (cut as above). With the smallest shift, the
    segment end is halved (in whole fs) until the checks that remain pass with
    the same basis; the next segment restarts there with the same input
    slope. Below h_min: failure.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .circuit import (FS, Cholesky, assemble_G, csr_add_diag, current,
                      current_slope, subtasks, transition_spots)
from .expm import expm


class NoConvergence(RuntimeError):
    pass


LADDER_LO = 1.0    # a shift serves check offsets tau >= LADDER_LO * gamma_k
LADDER_HI = 10.0   # ... and, below the top shift, tau <= LADDER_HI * gamma_k


def pick_shift(gammas, offsets_fs, lo=LADDER_LO):
    """Index of the shift for a segment whose sorted check offsets (fs) are
    given, and how many leading offsets it may cover."""
    tau1 = offsets_fs[0] * FS
    k = len(gammas) - 1
    for i, g in enumerate(gammas):
        if tau1 >= lo * g:
            k = i
            break
    if k == 0:
        return 0, len(offsets_fs)
    limit = LADDER_HI * gammas[k]
    cnt = int(np.searchsorted(np.asarray(offsets_fs) * FS, limit, side="right"))
    return k, max(1, cnt)


@dataclass
class KrylovBasis:
    """State kept by Alg. 2 between a Krylov generation and its snapshots."""
    V: np.ndarray        # n x m
    Hm: np.ndarray       # m x m, (I - Ht^-1)/gamma
    beta: float          # ||v||
    h_next: float        # h_{m+1,m}
    m: int
    exact: bool          # happy breakdown
    Hprev: np.ndarray | None = None   # H_{m-1}, for the difference term

    def expv(self, tau: float) -> np.ndarray:
        """||v|| V_m e^{tau H_m} e_1 (Eq. 9)."""
        if self.m == 0:
            return np.zeros(self.V.shape[0])
        e = expm(tau * self.Hm)[:, 0]
        return self.beta * (self.V @ e)

    def estimate(self, tau: float) -> float:
        """Larger of the empirical posterior estimate of Sec. 3.3.3,
        ||v|| h_{m+1,m} |e_m^T e^{tau H_m} e_1|, and the change from the
        dimension m-1 approximation (see the module docstring)."""
        if self.exact or self.m == 0:
            return 0.0
        u = expm(tau * self.Hm)[:, 0]
        paper = self.beta * self.h_next * abs(u[self.m - 1])
        if self.m == 1:
            diff = self.beta * abs(u[0] - 1.0)          # against u_0 = 1 (v itself)
        else:
            prev = expm(tau * self.Hprev)[:, 0]
            diff = self.beta * np.linalg.norm(u - np.concatenate([prev, [0.0]]))
        return max(paper, diff)


@dataclass
class Stats:
    solve_pairs_M: int = 0
    solve_pairs_G: int = 0
    bases: int = 0
    m_hist: list = field(default_factory=list)
    segments: int = 0
    halvings: int = 0
    shift_downs: int = 0


class RMatex:
    """Factors C + gamma G and G once (Alg. 2, LU_Decompose before the loop)."""

    def __init__(self, netlist, gamma: float, n_shifts: int = 5):
        self.nl = netlist
        self.n = netlist.n
        self.gammas = [gamma * 10.0 ** (-k) for k in range(n_shifts)]
        self.c = np.asarray(netlist.c_node, dtype=np.float64)
        rp, ci, gv = assemble_G(netlist)
        self.G = (rp, ci, gv)
        self.Gf = Cholesky(rp, ci, gv)
        self.Mfs = [Cholesky(rp, ci, csr_add_diag(rp, ci, gv, self.c, alpha=g))
                    for g in self.gammas]
        self.stats = Stats()
        self.trace = False

    # ---------------------------------------------------------- Alg. 1
    def arnoldi(self, v: np.ndarray, check_taus, tol: float, m_max: int,
                safety: float = 1.0, breakdown: float = 1e-14, shift: int = 0):
        """Rational Arnoldi on K_m((C + gamma G)^-1 C, v).

        `shift` selects gamma_k of the ladder. Returns (basis, converged). The stopping rule is checked at every j for
        the first and the last check offset; when both pass, every offset is
        checked (the first j at which all pass is the same either way)."""
        n = v.size
        gamma, Mf = self.gammas[shift], self.Mfs[shift]
        taus = np.sort(np.asarray(check_taus, dtype=np.float64))
        beta = float(np.linalg.norm(v))
        if beta == 0.0:
            return KrylovBasis(np.zeros((n, 0)), np.zeros((0, 0)), 0.0, 0.0, 0, True), True
        V = np.zeros((n, m_max + 1))
        Ht = np.zeros((m_max + 1, m_max))
        V[:, 0] = v / beta
        basis = None
        for j in range(m_max):
            w = Mf.solve(self.c * V[:, j])               # X1^-1 (X2 v_j)
            self.stats.solve_pairs_M += 1
            for i in range(j + 1):                         # modified Gram-Schmidt
                Ht[i, j] = w @ V[:, i]
                w = w - Ht[i, j] * V[:, i]
            Ht[j + 1, j] = np.linalg.norm(w)
            m = j + 1
            Hprev = basis.Hm if basis is not None else None
            Hm = (np.eye(m) - np.linalg.inv(Ht[:m, :m])) / gamma
            exact = Ht[j + 1, j] <= breakdown * np.abs(Ht[:m + 1, :m]).max()
            basis = KrylovBasis(V[:, :m].copy(), Hm, beta, float(Ht[j + 1, j]), m,
                                bool(exact), Hprev)
            if exact:
                self.stats.m_hist.append(m)
                return basis, True
            V[:, j + 1] = w / Ht[j + 1, j]
            ends = (taus[0], taus[-1])
            if all(safety * basis.estimate(t) < tol for t in ends):
                if all(safety * basis.estimate(t) < tol for t in taus):
                    self.stats.m_hist.append(m)
                    return basis, True
        self.stats.m_hist.append(basis.m)
        return basis, False

    def expv(self, v, taus, tol, m_max, safety=1.0, shift=0):
        """e^{tau A} v for every tau (s) with one basis (matex_krylov_step)."""
        basis, ok = self.arnoldi(v, taus, tol, m_max, safety, shift=shift)
        out = np.stack([basis.expv(t) for t in taus], axis=1)
        est = max((basis.estimate(t) for t in taus), default=0.0)
        return out, basis.m, est, ok

    # ---------------------------------------------------------- Alg. 2
    def subtask(self, src, idx, t_end: int, t_out: np.ndarray, probe, tol: float,
                m_max: int, safety: float = 1.0, h_min: int = 1, shift_ratio: float = LADDER_LO,
                t_start: int = 0):
        """Transient of one subtask (sources `idx`). Returns (y at probe rows for
        every t_out [n_probe x n_out], y(t_end) [n]). The run starts at t_start
        from the quasi-static state G^-1 i(t_start), which is exact at 0 (no
        source draws current before its delay) and otherwise forgets its error
        at the rate of the slowest mode; outputs before t_start stay 0."""
        n = self.n
        ts = transition_spots(src, idx, t_end)
        ts = np.unique(np.concatenate([[t_start], ts[ts > t_start]]))
        y = self.Gf.solve(current(src, idx, n, t_start))  # Local_Initial_Solution
        self.stats.solve_pairs_G += 1
        out = np.zeros((len(probe), t_out.size))
        k_out = int(np.searchsorted(t_out, t_start, side="left"))
        while k_out < t_out.size and t_out[k_out] <= t_start:
            out[:, k_out] = y[probe]
            k_out += 1
        t_a = t_start
        while t_a < t_end:
            t_b = int(ts[np.searchsorted(ts, t_a, side="right")])
            i_a = current(src, idx, n, t_a)
            s = current_slope(src, idx, n, t_a)            # A/s on [t_a, t_b)
            y0 = self.Gf.solve(i_a)
            z1 = self.Gf.solve(s)
            z2 = self.Gf.solve(self.c * z1)
            self.stats.solve_pairs_G += 3
            v = y - y0 + z2                                # x(t) + F(t, h)
            snaps = t_out[(t_out > t_a) & (t_out <= t_b)]
            offs = np.unique(np.concatenate([snaps, [t_b]]) - t_a)
            k, cnt = pick_shift(self.gammas, offs, shift_ratio)
            while True:
                if cnt < offs.size:                        # ladder cut
                    t_b = int(t_a + offs[cnt - 1])
                    snaps = snaps[snaps <= t_b]
                    offs = offs[:cnt]
                basis, ok = self.arnoldi(v, offs * FS, tol, m_max, safety, shift=k)
                self.stats.bases += 1
                if ok or k + 1 == len(self.gammas):
                    break
                # not converged: step down the ladder before halving
                k += 1
                cnt = max(1, int(np.searchsorted(offs * FS, LADDER_HI * self.gammas[k],
                                                 side="right")))
                self.stats.shift_downs += 1
            if not ok:
                # adaptive step: shrink the segment until the checks pass
                h = t_b - t_a
                while True:
                    h //= 2
                    self.stats.halvings += 1
                    if h < h_min:
                        raise NoConvergence(f"no convergence at t={t_a} fs")
                    cs = np.concatenate([snaps[snaps <= t_a + h] - t_a, [h]]) * FS
                    if all(safety * basis.estimate(t) < tol for t in cs):
                        break
                t_b = t_a + h
                snaps = snaps[snaps <= t_b]
            self.stats.segments += 1
            if self.trace:
                print(f"[oracle] seg t_a={t_a} t_b={t_b} shift={k} m={basis.m} conv={int(ok)} "
                      f"est={max(basis.estimate(t) for t in offs * FS):.3e} checks={offs.size}")
            for ts_k in snaps:                             # snapshots (Alg. 2 reuse)
                tau = (ts_k - t_a) * FS
                yk = basis.expv(tau) + y0 + tau * z1 - z2
                while k_out < t_out.size and t_out[k_out] == ts_k:
                    out[:, k_out] = yk[probe]
                    k_out += 1
            tau = (t_b - t_a) * FS
            y = basis.expv(tau) + y0 + tau * z1 - z2
            t_a = t_b
        return out, y

    def transient(self, prob, tol: float, m_max: int | None = None,
                  decompose: bool = True, safety: float = 1.0, h_min: int = 1,
                  shift_ratio: float = LADDER_LO, t_start: int = 0):
        """Full run with superposition over subtasks (Sec. 3.1-3.2). Returns
        (x at probes x t_out, y(t_end) summed)."""
        m_max = m_max or prob.m_max
        src = prob.sources
        groups = subtasks(src) if decompose else [np.arange(src.n_src)]
        y_out = np.zeros((prob.probe.size, prob.t_out.size))
        y_end = np.zeros(self.n)
        for idx in groups:
            o, ye = self.subtask(src, idx, prob.t_end, prob.t_out, prob.probe, tol,
                                 m_max, safety, h_min, shift_ratio, t_start)
            y_out += o
            y_end += ye
        return self.nl.vdd - y_out, y_end


class IMatex(RMatex):
    """I-MATEX (Sec. 3.3.1): the inverted Krylov subspace K_m(A^-1, v).

    Alg. 1 with X1 = G (factored once) and X2 = C: each step is
    w = G^-1 (C v_j) = -A^-1 v_j, so the Arnoldi matrix H' of this process is
    minus that of A^-1 and H_m = (-H')^-1 = -H'^-1. The stopping estimate is
    the empirical one of Sec. 3.3.3 with h_{m+1,m} = h'_{m+1,m} (the same
    estimate as R-MATEX, difference term included). There is no shift, so no
    ladder: a segment that does not converge within m_max is halved (Alg. 2).
    """

    def __init__(self, netlist):
        self.nl = netlist
        self.n = netlist.n
        self.gammas = [np.inf]          # one factor; pick_shift keeps whole segments
        self.c = np.asarray(netlist.c_node, dtype=np.float64)
        rp, ci, gv = assemble_G(netlist)
        self.G = (rp, ci, gv)
        self.Gf = Cholesky(rp, ci, gv)
        self.stats = Stats()
        self.trace = False

    def arnoldi(self, v: np.ndarray, check_taus, tol: float, m_max: int,
                safety: float = 1.0, breakdown: float = 1e-14, shift: int = 0):
        """Inverted Arnoldi on K_m(G^-1 C, v); returns (basis, converged) with
        the stopping rule applied as in RMatex.arnoldi."""
        n = v.size
        taus = np.sort(np.asarray(check_taus, dtype=np.float64))
        beta = float(np.linalg.norm(v))
        if beta == 0.0:
            return KrylovBasis(np.zeros((n, 0)), np.zeros((0, 0)), 0.0, 0.0, 0, True), True
        V = np.zeros((n, m_max + 1))
        Hp = np.zeros((m_max + 1, m_max))
        V[:, 0] = v / beta
        basis = None
        for j in range(m_max):
            w = self.Gf.solve(self.c * V[:, j])          # X1^-1 (X2 v_j), X1 = G
            self.stats.solve_pairs_M += 1
            for i in range(j + 1):                         # modified Gram-Schmidt
                Hp[i, j] = w @ V[:, i]
                w = w - Hp[i, j] * V[:, i]
            Hp[j + 1, j] = np.linalg.norm(w)
            m = j + 1
            Hprev = basis.Hm if basis is not None else None
            Hm = -np.linalg.inv(Hp[:m, :m])
            exact = Hp[j + 1, j] <= breakdown * np.abs(Hp[:m + 1, :m]).max()
            basis = KrylovBasis(V[:, :m].copy(), Hm, beta, float(Hp[j + 1, j]), m,
                                bool(exact), Hprev)
            if exact:
                self.stats.m_hist.append(m)
                return basis, True
            V[:, j + 1] = w / Hp[j + 1, j]
            ends = (taus[0], taus[-1])
            if all(safety * basis.estimate(t) < tol for t in ends):
                if all(safety * basis.estimate(t) < tol for t in taus):
                    self.stats.m_hist.append(m)
                    return basis, True
        self.stats.m_hist.append(basis.m)
        return basis, False
