"""Seeded synthetic power-distribution-network instances.

This module is shared by the CPU oracle's tests and by the GPU path. It holds
none of the method's arithmetic: it draws mesh topology, element values, pad
placement, pulse timings and probe sets, and nothing else. Assembling the
conductance matrix, deciding transition spots and every other step of the
method are done separately by each side.

The workloads follow the paper's setting (Sec. 2.1, Eq. 1; pulse sources of
Fig. 3): a multi-layer resistive mesh with node-to-ground capacitance, Norton
supply pads, and trapezoidal current pulses drawn from the mesh nodes. The
paper measures on the IBM power-grid benchmarks (Sec. 4.2-4.3), which are not
available here; these seeded meshes stand in for them.

Units: conductance in S, capacitance in F, current in A, time in integer
femtoseconds (1 ps = 1000 fs).
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

PS = 1000
NS = 1000 * PS


@dataclass
class Netlist:
    """A linear RC power grid.

    br_a/br_b/br_g: resistive branches between two nodes, conductance in S.
    c_node: node-to-ground capacitance (F), one per node.
    pad_node/pad_g: Norton supply pads (conductance to the Vdd rail, S).
    coord: int32 (n, 3) grid coordinates (layer, i, j) of every node.
    """
    n: int
    br_a: np.ndarray
    br_b: np.ndarray
    br_g: np.ndarray
    c_node: np.ndarray
    pad_node: np.ndarray
    pad_g: np.ndarray
    vdd: float
    coord: np.ndarray


@dataclass
class Sources:
    """Trapezoidal current pulses drawn from mesh nodes to ground.

    Timing follows the pulse description of Fig. 3 (delay, rise, width, fall),
    single pulse, no period. group[k] is the subtask a source belongs to.
    """
    node: np.ndarray
    amp: np.ndarray
    delay: np.ndarray
    rise: np.ndarray
    width: np.ndarray
    fall: np.ndarray
    group: np.ndarray

    @property
    def n_src(self) -> int:
        return int(self.node.shape[0])


@dataclass
class Problem:
    name: str
    netlist: Netlist
    sources: Sources
    t_end: int                 # fs
    t_out: np.ndarray          # int64 fs, increasing, output grid
    probe: np.ndarray          # int32 node ids whose voltages are reported
    gamma: float = 1e-11
    m_max: int = 20
    extra: dict = field(default_factory=dict)

    def digest(self) -> str:
        """SHA-256 of every array of the instance (reproducibility check)."""
        h = hashlib.sha256()
        nl, s = self.netlist, self.sources
        for a in (nl.br_a, nl.br_b, nl.br_g, nl.c_node, nl.pad_node, nl.pad_g,
                  nl.coord, s.node, s.amp, s.delay, s.rise, s.width, s.fall,
                  s.group, self.t_out, self.probe):
            h.update(np.ascontiguousarray(a).tobytes())
        h.update(repr((nl.n, nl.vdd, self.t_end, self.gamma, self.m_max)).encode())
        return h.hexdigest()


def _log_uniform(rng, lo, hi, size):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size))


def mesh(rng, layers: int, nx: int, ny: int, r_lo: float, r_hi: float,
         c_lo: float, c_hi: float, via_r: float = 0.05, via_pitch: int = 10,
         pad_nodes=None, pad_pitch: int = 15, pad_offset: int = 7,
         pad_r: float = 0.01, vdd: float = 1.0) -> Netlist:
    """Multi-layer rectangular mesh.

    Node id = layer * nx * ny + i * ny + j. In-layer branches join 4-neighbours
    with R log-uniform in [r_lo, r_hi]; vias of resistance via_r join layer L
    and L+1 wherever i % via_pitch == 0 and j % via_pitch == 0. Pads sit on
    the top layer (layers - 1) on a pitch x pitch lattice unless pad_nodes
    is given.
    """
    per = nx * ny
    n = layers * per
    a_list, b_list = [], []
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    base = ii * ny + jj
    for L in range(layers):
        off = L * per
        a_list.append((off + base[:, :-1]).ravel())   # horizontal
        b_list.append((off + base[:, 1:]).ravel())
        a_list.append((off + base[:-1, :]).ravel())   # vertical
        b_list.append((off + base[1:, :]).ravel())
    n_layer_br = sum(x.size for x in a_list)
    r_layer = _log_uniform(rng, r_lo, r_hi, n_layer_br)
    via_mask = (ii % via_pitch == 0) & (jj % via_pitch == 0)
    vias = base[via_mask]
    va, vb = [], []
    for L in range(layers - 1):
        va.append(L * per + vias)
        vb.append((L + 1) * per + vias)
    br_a = np.concatenate(a_list + va).astype(np.int32)
    br_b = np.concatenate(b_list + vb).astype(np.int32)
    r_all = np.concatenate([r_layer, np.full(sum(x.size for x in va), via_r)])
    br_g = 1.0 / r_all
    c_node = _log_uniform(rng, c_lo, c_hi, n)
    if pad_nodes is None:
        pi = np.arange(pad_offset, nx, pad_pitch)
        pj = np.arange(pad_offset, ny, pad_pitch)
        PI, PJ = np.meshgrid(pi, pj, indexing="ij")
        pad_nodes = (layers - 1) * per + (PI * ny + PJ).ravel()
    pad_nodes = np.asarray(pad_nodes, dtype=np.int32)
    pad_g = np.full(pad_nodes.size, 1.0 / pad_r)
    L_, I_, J_ = np.meshgrid(np.arange(layers), np.arange(nx), np.arange(ny), indexing="ij")
    coord = np.stack([L_.ravel(), I_.ravel(), J_.ravel()], axis=1).astype(np.int32)
    return Netlist(n=n, br_a=br_a, br_b=br_b, br_g=br_g, c_node=c_node,
                   pad_node=pad_nodes, pad_g=pad_g, vdd=vdd, coord=coord)


def pulse_timings(rng, size):
    """Delay U[0, 5] ns, rise and fall U[20, 100] ps, width U[0.2, 1] ns, in fs."""
    delay = np.rint(rng.uniform(0.0, 5.0 * NS, size)).astype(np.int64)
    rise = np.rint(rng.uniform(20.0 * PS, 100.0 * PS, size)).astype(np.int64)
    width = np.rint(rng.uniform(0.2 * NS, 1.0 * NS, size)).astype(np.int64)
    fall = np.rint(rng.uniform(20.0 * PS, 100.0 * PS, size)).astype(np.int64)
    return delay, rise, width, fall


def pick_source_nodes(rng, candidates: np.ndarray, count: int) -> np.ndarray:
    return rng.choice(candidates, size=count, replace=False).astype(np.int32)


def make_sources(rng, nodes: np.ndarray, n_groups: int = 0) -> Sources:
    """Per-source amplitude U[0, 1] mA. With n_groups > 0, the timing is one of
    n_groups seeded tuples (delay, rise, width, fall), chosen uniformly per
    source; group = tuple index. Otherwise every source draws its own timing
    and all sources form subtask 0."""
    k = nodes.size
    amp = rng.uniform(0.0, 1e-3, k)
    if n_groups > 0:
        d, r, w, f = pulse_timings(rng, n_groups)
        g = rng.integers(0, n_groups, k).astype(np.int32)
        delay, rise, width, fall = d[g], r[g], w[g], f[g]
    else:
        delay, rise, width, fall = pulse_timings(rng, k)
        g = np.zeros(k, dtype=np.int32)
    return Sources(node=nodes.astype(np.int32), amp=amp, delay=delay, rise=rise,
                   width=width, fall=fall, group=g)


def output_grid(t_end: int, step: int = 10 * PS) -> np.ndarray:
    return np.arange(0, t_end + 1, step, dtype=np.int64)


def non_pad(netlist: Netlist, layer: int | None = None) -> np.ndarray:
    ids = np.arange(netlist.n)
    if layer is not None:
        ids = ids[netlist.coord[:, 0] == layer]
    return np.setdiff1d(ids, netlist.pad_node).astype(np.int32)


# --------------------------------------------------------------------------
# Named workloads.
# --------------------------------------------------------------------------

def config0(instance: int = 0) -> Problem:
    """32x32 single-layer RC mesh, 4 corner pads, 50 pulse sources, 10 ns."""
    rng = np.random.Generator(np.random.PCG64(1000 * 0 + instance))
    nx = ny = 32
    corners = np.array([0, ny - 1, (nx - 1) * ny, nx * ny - 1], dtype=np.int32)
    nl = mesh(rng, 1, nx, ny, 0.5, 2.0, 1e-15, 1e-13, pad_nodes=corners)
    nodes = pick_source_nodes(rng, non_pad(nl), 50)
    src = make_sources(rng, nodes)
    t_end = 10 * NS
    return Problem("config0: 32x32 RC mesh, 50 sources, 10 ns", nl, src, t_end,
                   output_grid(t_end), np.arange(nl.n, dtype=np.int32))


def config1(instance: int = 0) -> Problem:
    """2x300x300 mesh (180k nodes), 400 pads, 2000 bottom-layer sources, 20 ns,
    512 probe rows, single subtask."""
    rng = np.random.Generator(np.random.PCG64(1000 * 1 + instance))
    nl = mesh(rng, 2, 300, 300, 0.1, 1.0, 1e-15, 1e-13)
    nodes = pick_source_nodes(rng, non_pad(nl, 0), 2000)
    src = make_sources(rng, nodes)
    probe = np.sort(pick_source_nodes(rng, non_pad(nl, 0), 512))
    t_end = 20 * NS
    return Problem("config1: 2x300x300 mesh, 2000 sources, 20 ns", nl, src,
                   t_end, output_grid(t_end), probe)


def config2(instance: int = 0) -> Problem:
    """3x580x580 mesh (~1M nodes), 1521 pads, 2000 sources in 64 timing groups."""
    rng = np.random.Generator(np.random.PCG64(1000 * 2 + instance))
    nl = mesh(rng, 3, 580, 580, 0.1, 1.0, 1e-15, 1e-13)
    nodes = pick_source_nodes(rng, non_pad(nl, 0), 2000)
    src = make_sources(rng, nodes, n_groups=64)
    probe = np.sort(pick_source_nodes(rng, non_pad(nl, 0), 512))
    t_end = 20 * NS
    return Problem("config2: 3x580x580 mesh, 2000 sources, 64 subtasks, 20 ns",
                   nl, src, t_end, output_grid(t_end), probe)


def config3(instance: int) -> Problem:
    """One of 128 uneven 2-layer meshes: n log-uniform in [1e4, 3e5], aspect
    ratio log-uniform in [0.5, 2], 100-1000 sources."""
    rng = np.random.Generator(np.random.PCG64(1000 * 3 + instance))
    n_tot = float(_log_uniform(rng, 1e4, 3e5, 1)[0])
    ar = float(_log_uniform(rng, 0.5, 2.0, 1)[0])
    nx = max(16, int(round(np.sqrt(n_tot / 2 * ar))))
    ny = max(16, int(round(n_tot / 2 / nx)))
    nl = mesh(rng, 2, nx, ny, 0.1, 1.0, 1e-15, 1e-13)
    k = int(rng.integers(100, 1001))
    nodes = pick_source_nodes(rng, non_pad(nl, 0), k)
    src = make_sources(rng, nodes)
    probe = np.sort(pick_source_nodes(rng, non_pad(nl, 0), min(512, nl.n // 4)))
    t_end = 20 * NS
    return Problem(f"config3[{instance}]: 2x{nx}x{ny} mesh, {k} sources", nl, src,
                   t_end, output_grid(t_end), probe)


def small(seed: int, layers: int = 1, nx: int = 8, ny: int = 8, n_src: int = 6,
          t_end: int = 2 * NS, n_groups: int = 0, n_pads: int | None = None,
          out_step: int = 10 * PS) -> Problem:
    """Small seeded grid for tests, with config-0 element statistics."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if layers == 1 and n_pads is None:
        pads = np.array([0, ny - 1, (nx - 1) * ny, nx * ny - 1], dtype=np.int32)
        nl = mesh(rng, 1, nx, ny, 0.5, 2.0, 1e-15, 1e-13, pad_nodes=pads)
    else:
        nl = mesh(rng, layers, nx, ny, 0.1, 1.0, 1e-15, 1e-13,
                  pad_pitch=max(2, min(nx, ny) // 3), pad_offset=1)
    nodes = pick_source_nodes(rng, non_pad(nl, 0), n_src)
    src = make_sources(rng, nodes, n_groups=n_groups)
    # squeeze pulse timings into the window
    scale = t_end / (7 * NS)
    for name in ("delay", "width"):
        v = getattr(src, name)
        setattr(src, name, np.maximum(1, np.rint(v * scale)).astype(np.int64))
    return Problem(f"small(seed={seed}, {layers}x{nx}x{ny}, {n_src} src)", nl, src,
                   t_end, output_grid(t_end, out_step), np.arange(nl.n, dtype=np.int32))


CONFIGS = {0: config0, 1: config1, 2: config2}
