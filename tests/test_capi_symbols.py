"""The C-ABI library loads (all symbols resolved) and exports every entry point that
include/mhd25.h declares; no compute call is made, so this runs without a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mhd25.h")
LIB = os.path.join(ROOT, "paper_2609_10849_amd", "libmhd25.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mhd25_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared()
    for must in ("mhd25_init", "mhd25_rhs_hydro", "mhd25_hydro_substep", "mhd25_step_magnetic",
                 "mhd25_strang_step", "mhd25_rhs_hydro_vjp", "mhd25_rhs_magnetic_vjp", "mhd25_batch_strang_step"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_loads_and_exports_every_symbol():
    lib = ctypes.CDLL(LIB, mode=os.RTLD_NOW | os.RTLD_LOCAL)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if " T " in l)
    assert set(declared()) <= exported


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_python_binding_covers_header():
    import paper_2609_10849_amd as pk
    assert set(declared()) <= set(pk._SIGS)


def test_default_options_without_gpu():
    import paper_2609_10849_amd as pk
    lib = pk.load_library()
    o = pk.Options()
    lib.mhd25_default_options(ctypes.byref(o))
    assert o.s_H == 0.02 and o.C_s == 5.0 and o.C_eta == 0.2 and o.max_halvings == 10 and o.pp == 0
