"""CPU checks of the C-ABI library: it loads and exports every symbol declared
in include/kdmg.h (no compute calls without a GPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kdmg.h")
LIB = os.path.join(ROOT, "paper_1801_07823_amd", "libkdmg.so")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(kdmg_[A-Za-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("kdmg_apply_D", "kdmg_hierarchy_build", "kdmg_solve",
                     "kdmg_coarse_apply", "kdmg_restrict", "kdmg_prolong"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s+(kdmg_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_loads_and_matches_header():
    from paper_1801_07823_amd import kdmg
    assert sorted(kdmg.EXPORTED) == declared_functions()
    p = kdmg.default_params()
    # Table 1 defaults
    assert p.nlevels == 3 and p.lvl[0].nvec == 8 and p.lvl[1].nvec == 12
    assert p.setup_maxit == 250 and abs(p.setup_tol - 1e-4) < 1e-18
    assert p.outer_restart == 32 and p.mr_its == 2 and abs(p.mr_omega - 0.85) < 1e-15
    assert p.inter_restart == 8 and p.inter_maxit == 16 and abs(p.inter_tol - 0.2) < 1e-15
    assert p.coarse_maxit == 256 and abs(p.coarse_tol - 0.2) < 1e-15
    assert p.outer_stall == 0  # the serving stall rule is off unless asked for
    assert p.coarse_tail == 16
    assert p.coarse_solver == 0  # Table 1: CGNE on the coarsest level
    assert p.fine_op == 0 and p.asymmetric == 0


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_params_layout_reaches_the_last_field():
    """The library's kdmg_default_params writes every field of the binding's
    struct, up to the last one: filled with a byte pattern first, no field
    keeps it."""
    import ctypes
    from paper_1801_07823_amd import kdmg
    p = kdmg.kdmg_mg_params()
    ctypes.memset(ctypes.byref(p), 0x55, ctypes.sizeof(p))
    kdmg._lib.kdmg_default_params(ctypes.byref(p))
    assert p.coarse_tail == 16 and p.coarse_solver == 0 and p.fine_op == 0 and p.asymmetric == 0
    last = kdmg.kdmg_mg_params._fields_[-1][0]
    assert last == "asymmetric"
    assert kdmg._lib.kdmg_status_string(kdmg.KDMG_ENOCONV) == b"solver did not converge"
