"""CPU-only checks of the library's host side: the factor layout (emulated
sweeps against a dense solve, in a standalone C++ program built with g++) and
that libmatex.so loads and exports every symbol matex.h declares."""
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
