"""Writes the stored expected values of the GPU parity tests.

Calls only the CPU oracle (R-MATEX at a tight tolerance, plus exact references
where they fit). Instances come from the seeded generator; their SHA-256 is
stored so a test can tell that it rebuilt the same instance.

  config1_head.npz  the 2x300x300 workload (180k nodes, 2000 sources) over
                    its first 500 ps: x at the 512 probe rows for t = 0..500 ps
                    every 10 ps, and x(500 ps) at every node. Oracle R-MATEX,
                    tol 1e-13 (every basis) with the 4-shift ladder.
Run:  python tests/golden/make_golden.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import rmatex as RM  # noqa: E402
from paper_1511_04519_amd import instances as I  # noqa: E402


def config1_head(t_end=500 * I.PS):
    p = I.config1()
    digest = p.digest()
    q = I.Problem(p.name + " (head)", p.netlist, p.sources, t_end,
                  p.t_out[p.t_out <= t_end], p.probe)
    t0 = time.time()
    s = RM.RMatex(p.netlist, p.gamma)
    x, y_end = s.transient(q, tol=1e-13, m_max=p.m_max)
    print(f"config1 head: {time.time() - t0:.1f} s, bases {s.stats.bases}, "
          f"pairs {s.stats.solve_pairs_M}+{s.stats.solve_pairs_G}", flush=True)
    np.savez_compressed(os.path.join(HERE, "config1_head.npz"), x=x,
                        x_end=p.netlist.vdd - y_end, t_end=t_end, digest=digest,
                        tol=1e-13)


if __name__ == "__main__":
    config1_head()
