"""CPU-only checks of the library's host side: the factor layout (emulated
sweeps against a dense solve, in a standalone C++ program built with g++), a
replay of the subtree sweeps on the schedule the library builds (every
address bounds-checked, see tests/native/tree_check.cpp) and that
libmatex.so loads and exports every symbol matex.h declares.

MATEX_TREE_CHECK_FULL=1 also replays the 3 x 580 x 580 grid's schedule
(2048 subtree blocks, about a minute)."""
import os
import re
import subprocess

import pytest

from paper_1511_04519_amd import matex as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def factor_check(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("fc") / "factor_check")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-o", exe,
                           os.path.join(ROOT, "tests/native/factor_check.cpp"),
                           os.path.join(ROOT, "paper_1511_04519_amd/csrc/factor.cpp")])
    return exe


@pytest.fixture(scope="module")
def tree_check(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("tc") / "tree_check")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-o", exe,
                           os.path.join(ROOT, "tests/native/tree_check.cpp"),
                           os.path.join(ROOT, "paper_1511_04519_amd/csrc/factor.cpp"),
                           os.path.join(ROOT, "paper_1511_04519_amd/csrc/schedule.cpp")])
    return exe


def _write_netlist(nl, path):
    import numpy as np
    with open(path, "wb") as f:
        f.write(np.int64(nl.n).tobytes())
        f.write(np.int64(len(nl.br_a)).tobytes())
        f.write(np.int32(len(nl.pad_node)).tobytes())
        f.write(np.float64(nl.vdd).tobytes())
        for a, t in ((nl.br_a, np.int32), (nl.br_b, np.int32), (nl.br_g, np.float64),
                     (nl.c_node, np.float64), (nl.pad_node, np.int32), (nl.pad_g, np.float64),
                     (nl.coord, np.int32)):
            f.write(np.ascontiguousarray(a, t).tobytes())


# (layers, nx, ny, leaf, seed): subtrees of 1 to 7 levels, 2 to 512 blocks
@pytest.mark.parametrize("args", ["2 64 64 16 1", "1 40 33 8 2", "3 50 47 16 3", "2 120 120 16 4",
                                  "2 150 150 32 5", "2 400 400 16 6"])
def test_subtree_sweeps_stay_in_bounds(tree_check, args):
    r = subprocess.run([tree_check, *args.split()], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 out-of-range accesses" in r.stdout


def test_subtree_sweeps_stay_in_bounds_on_the_180k_node_grid(tree_check, tmp_path):
    from paper_1511_04519_amd import instances as I
    path = str(tmp_path / "c1.bin")
    _write_netlist(I.config1().netlist, path)
    for leaf in ("16", "32"):
        r = subprocess.run([tree_check, "--file", path, leaf], capture_output=True, text=True)
        assert r.returncode == 0, r.stdout + r.stderr


@pytest.mark.skipif(os.environ.get("MATEX_TREE_CHECK_FULL") != "1",
                    reason="about a minute; MATEX_TREE_CHECK_FULL=1 runs it")
def test_subtree_sweeps_stay_in_bounds_on_the_1m_node_grid(tree_check, tmp_path):
    from paper_1511_04519_amd import instances as I
    path = str(tmp_path / "c2.bin")
    _write_netlist(I.config2().netlist, path)
    r = subprocess.run([tree_check, "--file", path, "16"], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "blocks 2048" in r.stdout


@pytest.mark.parametrize("args", ["1 8 8 4 1", "2 12 9 8 2", "3 10 14 16 3", "2 20 20 1 4",
                                  "1 1 30 4 5", "2 17 23 16 6", "1 2 2 16 7"])
def test_supernodal_panels_solve_exactly(factor_check, args):
    r = subprocess.run([factor_check, *args.split()], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include/matex.h")).read()
    declared = set(re.findall(r"^\s*(?:matex_status|size_t|const char\*)\s+(matex_\w+)\(", hdr, re.M))
    assert declared >= {"matex_factor", "matex_krylov_step", "matex_transient", "matex_adjoint"}
    L = M.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert set(M.EXPORTS) == declared
    assert b"gfx950" in L.matex_version()


def test_invalid_arguments_are_rejected_without_gpu():
    # argument checks run before any device work
    from paper_1511_04519_amd import instances as I
    p = I.small(1, nx=4, ny=4, n_src=2)
    with pytest.raises(M.MatexError) as e:
        M.matex_factor(p.netlist, -1.0)
    assert e.value.status == M.MATEX_E_INVALID
    p.netlist.c_node[3] = 0.0
    with pytest.raises(M.MatexError) as e:
        M.matex_factor(p.netlist, 1e-11)
    assert e.value.status == M.MATEX_E_INVALID
