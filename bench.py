#!/usr/bin/env python
"""Benchmark of the R-MATEX transient on one MI355X: batched vs plain.

Workload (one step): the 3 x 580 x 580 grid (1,009,200 nodes, 1521 pads,
2000 pulse sources in 64 subtasks of shared pulse timing, 20 ns window, 2001
output times at 512 probe rows), every step of the hot path (segment
planning, the F/P terms of Eq. 6, rational Arnoldi with substitution pairs
on C + gamma_k G, Gram-Schmidt, the small matrix exponential, reconstruction
at the output times, superposition of the subtasks), inputs resident on the
device. Tolerance 1e-10 V per basis and subtask count (1e-10 / 64).
Factorisation is set-up and excluded, as the paper excludes LU from its
transient times.

value: node-steps/s of the batched mode (all 64 subtasks through
64-right-hand-side substitution pairs) = n * N_out / transient seconds.
plain: the same workload with the subtasks one after another (one-vector
pairs), run once; speedup = plain seconds / batched seconds (same steps).
parity: both modes against the oracle's stored windows of this workload
([0, 300] ps from t = 0; [0.9, 1.0] ns from a quasi-static start).
roofline: the 64-right-hand-side substitution pair (the batched transient's
dominant kernels), algorithmic bytes per pair (each nonzero of L once per
sweep, 8 B, plus 4 x 8 B per row and right-hand side) over the event-timed
mean pair duration, against 8 TB/s; traffic from the committed rocprofv3
counter summary when it was taken on the current kernel sources.
cpu_baseline: the CPU oracle on a bounded sample of the same workload (all
64 subtasks over its first 50 ps), one core and all cores (subtasks in
threads), and the oracle's trapezoidal rule at a fixed 10 ps step (the
paper's comparator) on the same window; the oracle's factors (those of the
trapezoidal rule too) are built in threads while the GPU runs and are
excluded, as on the GPU.
trapezoidal: the trapezoidal rule at a fixed 10 ps step (the paper's
comparator) on the same workload, its time and its error.
config1: context, the 2 x 300 x 300 grid (180k nodes) in plain mode, run
once, with its oracle windows and its one-vector pair (a cache-resident
factor: 130 MB against the 256 MB Infinity Cache).
config3_uneven: the 128 uneven meshes (10k to 300k nodes, own factor each)
over their first nanosecond, concurrently and one at a time.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       python bench.py --pairs-only   (the profiling run of the sweep kernels)
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "SpTRSV HBM GB/s + transient node·steps/s, batched vs plain, at 1e-9 rel err"
# Nested-dissection leaf size of the 180k-node grid's factor (13 levels
# instead of 14 with 16-node leaves; 145 against 149 us per pair).
CONFIG1_LEAF = 32
CPU_WINDOW_PS = 50
TRAFFIC_PROFILE64 = os.path.join(ROOT, "profiles", "solve_pair64_config2.md")
TRAFFIC_PROFILE1 = os.path.join(ROOT, "profiles", "solve_pair_config1.md")
# the sources a profile's counters depend on (matex.cpp and schedule.cpp
# build the sweep schedules and task tables)
PLAIN_SOURCES = ("kernels.hip", "kernels.hpp", "device_common.hpp", "factor.cpp", "factor.hpp",
                 "schedule.cpp", "schedule.hpp", "matex.cpp")
BATCHED_SOURCES = ("batched.hip", "batched.hpp", "kernels.hpp", "device_common.hpp", "factor.cpp",
                   "factor.hpp", "schedule.cpp", "schedule.hpp", "matex.cpp")


def kernel_source_digest(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_1511_04519_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(path, files):
    """HBM bytes per substitution pair from a committed rocprofv3 counter
    summary, if it was taken on the current kernel sources (else None)."""
    if path is None:
        return None
    try:
        txt = open(path).read()
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in txt.splitlines()
                  if line.startswith(("kernel-sources:", "traffic-bytes-per-pair:")))
    if fields.get("kernel-sources", "").strip() != kernel_source_digest(files):
        return None
    return float(fields["traffic-bytes-per-pair"])


def host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


# ------------------------------------------------------------ CPU baseline

def cpu_child(window_ps, cores):
    """Runs in a child process: the oracle on the first window_ps of the
    1M-node workload. Prints one JSON line after each phase; waits for a line
    on stdin before the all-core and trapezoidal phases (the GPU's timed
    region is over by then)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    from oracle import circuit as OC
    from oracle import reference as OR
    from oracle import rmatex as RM
    from paper_1511_04519_amd import instances as I

    p = I.config2()
    T = window_ps * I.PS
    q = I.Problem("sample", p.netlist, p.sources, T, p.t_out[p.t_out <= T], p.probe)
    groups = OC.subtasks(p.sources)
    tol = 1e-10 / len(groups)
    # the oracle's factors (5 shifts and G), built side by side: the C
    # factorisation runs outside the interpreter lock
    t0 = time.time()
    s = RM.RMatex.__new__(RM.RMatex)
    s.nl, s.n = p.netlist, p.netlist.n
    s.gammas = [p.gamma * 10.0 ** (-k) for k in range(5)]
    s.c = np.asarray(p.netlist.c_node, dtype=np.float64)
    rp, ci, gv = OC.assemble_G(p.netlist)
    s.G = (rp, ci, gv)
    h_tr = 10 * I.PS
    with ThreadPoolExecutor(7) as ex:
        fg = ex.submit(OC.Cholesky, rp, ci, gv)
        fm = [ex.submit(OC.Cholesky, rp, ci, OC.csr_add_diag(rp, ci, gv, s.c, alpha=g)) for g in s.gammas]
        ft = ex.submit(OC.Cholesky, rp, ci, OC.csr_add_diag(rp, ci, gv, s.c / (h_tr * OC.FS), alpha=0.5))
        s.Gf = fg.result()
        s.Mfs = [f.result() for f in fm]
        tr_facs = {"G": s.Gf, h_tr: ft.result()}
    s.stats = RM.Stats()
    s.trace = False
    factor_s = time.time() - t0
    n_out = int(q.t_out.size)

    def run(idx_list):
        for idx in idx_list:
            s.subtask(p.sources, idx, T, q.t_out, q.probe, tol, p.m_max, 1.0, 1, 1.0, 0)

    t0 = time.time()
    run(groups)
    one = time.time() - t0
    st = s.stats
    print(json.dumps({"phase": "one", "factor_s": factor_s, "transient_s": one, "n": s.n, "n_out": n_out,
                      "bases": st.bases, "pairs": st.solve_pairs_M + st.solve_pairs_G,
                      "subtasks": len(groups)}), flush=True)
    sys.stdin.readline()
    # all cores: the subtasks dealt to `cores` threads (the sparse solves and
    # the vector operations release the interpreter lock); time = the slowest
    shares = [groups[k::cores] for k in range(cores)]
    t0 = time.time()
    with ThreadPoolExecutor(cores) as ex:
        list(ex.map(run, shares))
    allc = time.time() - t0
    print(json.dumps({"phase": "all", "transient_s": allc, "cores": cores}), flush=True)
    t0 = time.time()
    _, _, pairs_tr = OR.trapezoidal(q, h_tr, align=False, factors=tr_facs)
    tr = time.time() - t0
    print(json.dumps({"phase": "tr", "seconds": tr, "pairs": pairs_tr}), flush=True)


class CpuBaseline:
    def __init__(self, window_ps, cores):
        self.window_ps, self.cores = window_ps, cores
        self.p = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-child",
                                   str(window_ps), str(cores)], stdin=subprocess.PIPE,
                                  stdout=subprocess.PIPE, text=True,
                                  env=dict(os.environ, OPENBLAS_NUM_THREADS="1", OMP_NUM_THREADS="1",
                                           MKL_NUM_THREADS="1"))

    def _line(self):
        line = self.p.stdout.readline()
        if not line:
            raise RuntimeError("CPU baseline child ended early")
        return json.loads(line)

    def finish(self):
        one = self._line()
        self.p.stdin.write("go\n")
        self.p.stdin.flush()
        allc = self._line()
        tr = self._line()
        self.p.wait(timeout=60)
        model, ncpu = host_cpu()
        work = one["n"] * one["n_out"]
        return {
            "value": work / one["transient_s"], "unit": "node*steps/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle R-MATEX on the same 1M-node workload and tolerance, all {one['subtasks']} "
                       f"subtasks over [0, {self.window_ps} ps] ({one['n_out']} output times, "
                       f"{one['bases']} bases, {one['pairs']} solve pairs), {one['transient_s']:.1f} s on "
                       f"one core; its factors ({one['factor_s']:.0f} s, built in threads) excluded"),
            "all_cores": {"value": work / allc["transient_s"], "cores": allc["cores"],
                          "seconds": allc["transient_s"],
                          "how": "subtasks dealt to threads, time of the slowest (the paper's max over nodes)"},
            "oracle_tr_10ps": {"value": work / tr["seconds"], "seconds": tr["seconds"],
                               "pairs": tr["pairs"], "cores": 1,
                               "how": "Eq. 2 at a fixed 10 ps step (the paper's comparator), same window"},
            "host": {"nproc": ncpu, "model": model},
        }


# ------------------------------------------------------------------- GPU

def pair_roofline(F, nrhs, reps, profile, sources):
    from paper_1511_04519_amd import matex as M
    sec, byt = M.matex_time_solves(F, which=0, reps=reps, nrhs=nrhs)
    info = F.info
    fmt = 2 * 8 * info["nnz_l"] + 32 * info["n"] * nrhs
    slots = 16 * info["n_upd"] * nrhs
    achieved = byt / sec / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": measured_traffic(profile, sources),
            "kernel": (f"substitution pair on C + gamma G, {nrhs} right-hand side(s): all level launches "
                       f"of one forward and one backward sweep"),
            "pair_ms": round(sec * 1e3, 4), "algorithmic_bytes": int(byt),
            "algorithmic_bytes_def": "2*8*nnz(L) + 4*8*n*nrhs, nnz(L) the factor's structural nonzeros",
            "nnz_l_exact": info["nnz_l_exact"], "nnz_l_stored": info["nnz_l"],
            "format_bytes": int(fmt), "update_slot_bytes": int(slots),
            "kernel_sources": kernel_source_digest(sources)}


def windows_error(x, gold_dir, names, t_out):
    import numpy as np
    out = {}
    for nm in names:
        g = np.load(os.path.join(gold_dir, nm))
        sel = np.isin(t_out, g["t_out"])
        out[nm] = float(np.abs(x[:, sel] - g["x"]).max())
    return out


def config1_context(tol):
    import numpy as np
    import torch
    from paper_1511_04519_amd import instances as I
    from paper_1511_04519_amd import matex as M
    p = I.config1()
    F = M.matex_factor(p.netlist, p.gamma, leaf_max=CONFIG1_LEAF)
    torch.cuda.synchronize()
    t0 = time.time()
    x, _, st = M.matex_transient(F, p, tol=tol, m_max=p.m_max)
    torch.cuda.synchronize()
    dt = time.time() - t0
    xs = x.cpu().numpy()
    gold = np.load(os.path.join(ROOT, "tests/golden/config1_head.npz"))
    k = int((p.t_out <= int(gold["t_end"])).sum())
    mid = np.load(os.path.join(ROOT, "tests/golden/config1_mid.npz"))
    sel = np.isin(p.t_out, mid["t_out"])
    roof = pair_roofline(F, 1, 50, TRAFFIC_PROFILE1, PLAIN_SOURCES)
    roof["bound"] = "hbm (cache-resident: the factor fits the 256 MB Infinity Cache)"
    return {"workload": p.name, "n": p.netlist.n, "n_out": int(p.t_out.size), "mode": "plain",
            "leaf": CONFIG1_LEAF, "tol": tol, "seconds": round(dt, 3),
            "node_steps_per_s": p.netlist.n * p.t_out.size / dt, "segments": st["segments"],
            "bases": st["bases"], "solve_pairs": st["solve_pairs_m"] + st["solve_pairs_g"],
            "max_abs_err_vs_oracle_0_500ps": float(np.abs(xs[:, :k] - gold["x"][:, :k]).max()),
            "max_abs_err_vs_oracle_2900_3000ps": float(np.abs(xs[:, sel] - mid["x"]).max()),
            "pair1": roof}


def tr_comparator(p, batched_s, gold_dir):
    """The trapezoidal rule at a fixed 10 ps step (Eq. 2; the comparator of
    the paper's Tab. 3) on the same workload, all sources together: time,
    node-steps/s and its distance from the oracle's windows."""
    import torch
    from paper_1511_04519_amd import instances as I
    from paper_1511_04519_amd import matex as M
    h = 10 * I.PS
    t0 = time.time()
    F = M.matex_factor(p.netlist, 0.5 * h * 1e-15, n_shifts=1)
    fs = time.time() - t0
    M.matex_trapezoidal(F, p, h, final=False)   # warm
    torch.cuda.synchronize()
    t0 = time.time()
    x, _, st = M.matex_trapezoidal(F, p, h, final=False)
    torch.cuda.synchronize()
    dt = time.time() - t0
    err = windows_error(x.cpu().numpy(), gold_dir, ("config2_head.npz", "config2_mid.npz"), p.t_out)
    return {"h_ps": 10, "steps": st["segments"], "seconds": round(dt, 3), "factor_s": round(fs, 2),
            "node_steps_per_s": p.netlist.n * p.t_out.size / dt,
            "max_abs_err_vs_oracle": err,
            "batched_matex_speedup_vs_tr": round(dt / batched_s, 3)}


def config3_uneven(window_ps, tol):
    """The 128 uneven meshes (own factor each) over their first window_ps:
    advanced concurrently (matex_transient_many, 16 streams) and one at a
    time; node-steps/s = sum of n * N_out over the instances / seconds."""
    from concurrent.futures import ThreadPoolExecutor

    import torch
    from paper_1511_04519_amd import instances as I
    from paper_1511_04519_amd import matex as M
    T = window_ps * I.PS
    probs = []
    for k in range(128):
        p = I.config3(k)
        probs.append(I.Problem(p.name, p.netlist, p.sources, T, p.t_out[p.t_out <= T], p.probe))
    t0 = time.time()
    with ThreadPoolExecutor(4) as ex:
        factors = list(ex.map(lambda q: M.matex_factor(q.netlist, q.gamma), probs))
    fs = time.time() - t0
    work = sum(q.netlist.n * q.t_out.size for q in probs)
    torch.cuda.synchronize()
    t0 = time.time()
    res = M.matex_transient_many(factors, probs, tol=tol, m_max=20, n_streams=16, final=False)
    torch.cuda.synchronize()
    tc = time.time() - t0
    t0 = time.time()
    one = [M.matex_transient(F, q, tol=tol, m_max=20, final=False) for F, q in zip(factors, probs)]
    torch.cuda.synchronize()
    ts = time.time() - t0
    same = all(torch.equal(a[0], b[0]) for a, b in zip(res, one))
    return {"instances": 128, "window_ps": window_ps, "nodes": int(sum(q.netlist.n for q in probs)),
            "sources": int(sum(q.sources.n_src for q in probs)), "factor_s": round(fs, 1), "tol": tol,
            "concurrent_s": round(tc, 3), "one_at_a_time_s": round(ts, 3),
            "concurrent_node_steps_per_s": work / tc, "one_at_a_time_node_steps_per_s": work / ts,
            "speedup": round(ts / tc, 3), "identical_results": bool(same),
            "bases": int(sum(r[2]["bases"] for r in res))}


def pairs_only():
    """The profiling run for the sweep kernels' counters: 1 + 50 one-vector
    pairs on the 180k-node grid, 1 + 20 pairs with 64 right-hand sides on the
    1M-node grid, then a 256 MiB device copy for calibration."""
    import torch
    from paper_1511_04519_amd import instances as I
    from paper_1511_04519_amd import matex as M
    out = {}
    for name, prob, nrhs, reps, leaf in (("config1", I.config1(), 1, 50, CONFIG1_LEAF),
                                         ("config2", I.config2(), 64, 20, 16)):
        F = M.matex_factor(prob.netlist, prob.gamma, leaf_max=leaf)
        sec, byt = M.matex_time_solves(F, which=0, reps=reps, nrhs=nrhs)
        out[name] = {"nrhs": nrhs, "pairs": reps + 1, "pair_ms": sec * 1e3, "pair_bytes": byt,
                     "GB_s": byt / sec / 1e9, "frac": byt / sec / 1e9 / HBM_PEAK_GBS}
        print(f"[bench] {name}: pair {sec * 1e3:.3f} ms, {byt / sec / 1e9:.0f} GB/s", flush=True)
        del F
    a = torch.ones(2 ** 25, dtype=torch.float64, device="cuda")
    torch.empty_like(a).copy_(a)
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--cpu-child":
        cpu_child(int(sys.argv[2]), int(sys.argv[3]))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--window-ps", type=int, default=0, help="shorten the window (0 = full)")
    ap.add_argument("--cpu-window-ps", type=int, default=CPU_WINDOW_PS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-config1", action="store_true")
    ap.add_argument("--no-tr", action="store_true")
    ap.add_argument("--config3-window-ps", type=int, default=1000,
                    help="window of the 128-mesh uneven batch (0 = skip it)")
    ap.add_argument("--pairs-only", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: nothing in this build uses a second one (asked for {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1511_04519_amd import instances as I
    from paper_1511_04519_amd import matex as M

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    M.lib()   # fails loudly if libmatex.so is missing
    if args.pairs_only:
        pairs_only()
        return
    cores = max(1, min(16, os.cpu_count() or 1))
    cpu = None if args.no_cpu_baseline else CpuBaseline(args.cpu_window_ps, cores)

    p = I.config2()
    if args.window_ps:
        T = args.window_ps * I.PS
        p = I.Problem(p.name + f" (first {args.window_ps} ps)", p.netlist, p.sources, T,
                      p.t_out[p.t_out <= T], p.probe)
    groups = len(np.unique(p.sources.group))
    tol = 1e-10 / groups
    n, n_out = p.netlist.n, p.t_out.size
    t0 = time.time()
    F = M.matex_factor(p.netlist, p.gamma)
    factor_s = time.time() - t0
    print(f"[bench] factor {factor_s:.1f} s (host analyse {F.info['seconds_analyse']:.2f} s, numeric "
          f"{F.info['seconds_numeric']:.1f} s), nnz(L) {F.info['nnz_l_exact']} (stored "
          f"{F.info['nnz_l']}), levels {F.info['n_levels']}, subtree blocks {F.info['subtree_blocks']}",
          flush=True)

    for w in range(args.warmup):
        M.matex_transient(F, p, tol=tol, m_max=p.m_max, mode=M.MATEX_BATCHED)
        print(f"[bench] warmup {w + 1}/{args.warmup} done", flush=True)
    torch.cuda.synchronize()
    t0 = time.time()
    for k in range(args.steps):
        x, _, st = M.matex_transient(F, p, tol=tol, m_max=p.m_max, mode=M.MATEX_BATCHED)
        print(f"[bench] step {k + 1}/{args.steps}: {st['seconds']:.3f} s, segments {st['segments']}, "
              f"bases {st['bases']}, 64-column pairs {st['solve_pairs_m']}+{st['solve_pairs_g']}", flush=True)
    torch.cuda.synchronize()
    dt = (time.time() - t0) / args.steps
    value = n * n_out / dt
    xb = x.cpu().numpy()

    plain = None
    if not args.no_plain:
        torch.cuda.synchronize()
        t0 = time.time()
        xp_t, _, sp = M.matex_transient(F, p, tol=tol, m_max=p.m_max, mode=M.MATEX_PLAIN)
        torch.cuda.synchronize()
        tp = time.time() - t0
        xp = xp_t.cpu().numpy()
        print(f"[bench] plain: {tp:.2f} s, pairs {sp['solve_pairs_m']}+{sp['solve_pairs_g']}", flush=True)
        plain = {"seconds": round(tp, 3), "node_steps_per_s": n * n_out / tp,
                 "speedup_batched_vs_plain": round(tp / dt, 3),
                 "same_steps": sp["segments"] == st["segments"] and sp["krylov_dims"] == st["krylov_dims"]
                 and sp["bases"] == st["bases"],
                 "max_abs_diff_batched_vs_plain": float(np.abs(xb - xp).max()),
                 "stats": sp}

    gold_dir = os.path.join(ROOT, "tests/golden")
    parity = {"batched": windows_error(xb, gold_dir, ("config2_head.npz", "config2_mid.npz"), p.t_out)}
    if plain is not None:
        parity["plain"] = windows_error(xp, gold_dir, ("config2_head.npz", "config2_mid.npz"), p.t_out)
    parity["criterion"] = "max |x_gpu - x_oracle| / max |x_oracle| <= 1e-9 (x ~ Vdd = 1 V)"

    roof = pair_roofline(F, 64, 20, TRAFFIC_PROFILE64, BATCHED_SOURCES)
    pair1 = pair_roofline(F, 1, 20, None, PLAIN_SOURCES)
    pair1.pop("traffic")
    # calibration copy for the hardware byte counters (256 MiB read + write)
    a = torch.ones(2 ** 25, dtype=torch.float64, device="cuda")
    torch.empty_like(a).copy_(a)
    torch.cuda.synchronize()
    F_info = F.info
    schedule = M.matex_factor_describe(F).splitlines()
    del F

    tr = None if args.no_tr else tr_comparator(p, dt, gold_dir)
    if tr is not None:
        print(f"[bench] trapezoidal 10 ps: {tr['seconds']:.2f} s", flush=True)
    c1 = None if args.no_config1 else config1_context(1e-10)
    c3 = config3_uneven(args.config3_window_ps, 1e-10) if args.config3_window_ps > 0 else None
    if c3 is not None:
        print(f"[bench] uneven batch: concurrent {c3['concurrent_s']:.2f} s, one at a time "
              f"{c3['one_at_a_time_s']:.2f} s", flush=True)
    cpu_line = cpu.finish() if cpu is not None else None

    line = {
        "metric": METRIC, "value": value, "unit": "node*steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded 3x580x580 RC grid, 2000 pulse sources in 64 timing groups)",
        "config": {"workload": p.name + ", batched (64 subtasks per substitution pair)", "n": n,
                   "n_out": int(n_out), "n_probe": int(p.probe.size), "subtasks": groups, "mode": "batched",
                   "tol": tol, "gamma": p.gamma, "m_max": p.m_max, "factor_s": round(factor_s, 2),
                   "segments": st["segments"], "bases": st["bases"],
                   "pairs_64rhs": st["solve_pairs_m"] + st["solve_pairs_g"],
                   "krylov_dims": st["krylov_dims"], "seconds_tune": round(F_info["seconds_tune"], 3),
                   "batched_schedule": schedule},
        "plain": plain, "parity": parity, "roofline": roof, "pair1": pair1, "trapezoidal": tr,
        "config1": c1, "config3_uneven": c3,
        "cpu_baseline": cpu_line,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
