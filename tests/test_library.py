"""Host-side checks of the C-ABI library (no GPU): it loads and exports every
function include/apic.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "apic.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(apic_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_five_entry_points():
    names = declared_functions()
    for n in ("apic_sort_by_cell", "apic_deposit", "apic_gather_push", "apic_step", "apic_step_adjoint"):
        assert n in names, n


def test_library_exports_every_declared_symbol():
    from paper_2608_15249_amd import apic
    path = apic.LIB_PATH
    if not os.path.exists(path):
        pytest.fail("libapic.so not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares a signature for each of them
    L = apic.load_library()
    for n in declared_functions():
        assert getattr(L, n).argtypes is not None or n in ("apic_destroy",), n


def test_struct_layouts_match_header():
    from paper_2608_15249_amd import apic
    # apic_grid_desc: 4 ints, 7 doubles, 4 ints -> 88 bytes; apic_particles: int64 + 10 pointers
    assert ctypes.sizeof(apic.GridDesc) == 88
    assert ctypes.sizeof(apic.ParticlesC) == 8 + 10 * 8
