"""Tiny hand-made circuits for the oracle pins."""
import numpy as np

from paper_1511_04519_amd.instances import NS, PS, Netlist, Problem, Sources


def single_rc(c=2e-14, g=0.5):
    """One node, capacitance c to ground, conductance g to the supply."""
    return Netlist(n=1, br_a=np.zeros(0, np.int32), br_b=np.zeros(0, np.int32),
                   br_g=np.zeros(0), c_node=np.array([c]), pad_node=np.array([0], np.int32),
                   pad_g=np.array([g]), vdd=1.0, coord=np.zeros((1, 3), np.int32))


def uniform_mesh(k, R=1.0, c=1e-14, g0=0.05):
    """k x k mesh, equal R and C, ground conductance g0 at every node."""
    ii, jj = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
    base = ii * k + jj
    a = np.concatenate([base[:, :-1].ravel(), base[:-1, :].ravel()]).astype(np.int32)
    b = np.concatenate([base[:, 1:].ravel(), base[1:, :].ravel()]).astype(np.int32)
    n = k * k
    coord = np.stack([np.zeros(n, np.int32), ii.ravel(), jj.ravel()], 1).astype(np.int32)
    return Netlist(n=n, br_a=a, br_b=b, br_g=np.full(a.size, 1.0 / R), c_node=np.full(n, c),
                   pad_node=np.arange(n, dtype=np.int32), pad_g=np.full(n, g0), vdd=1.0,
                   coord=coord)


def sources(node, amp, delay, rise, width, fall, group=None):
    k = len(node)
    return Sources(node=np.asarray(node, np.int32), amp=np.asarray(amp, float),
                   delay=np.asarray(delay, np.int64), rise=np.asarray(rise, np.int64),
                   width=np.asarray(width, np.int64), fall=np.asarray(fall, np.int64),
                   group=np.zeros(k, np.int32) if group is None else np.asarray(group, np.int32))


def problem(nl, src, t_end, step=10 * PS, probe=None):
    t_out = np.arange(0, t_end + 1, step, dtype=np.int64)
    return Problem("hand-made", nl, src, t_end, t_out,
                   np.arange(nl.n, dtype=np.int32) if probe is None else np.asarray(probe, np.int32))
