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


def test_struct_layouts_match_header(tmp_path):
    """Size and every field offset of the binding's ctypes structs equal what
    a C compiler gives for the structs of include/apic.h."""
    import subprocess
    from paper_2608_15249_amd import apic
    structs = {"apic_grid_desc": apic.GridDesc, "apic_particles": apic.ParticlesC,
               "apic_replica": apic.ReplicaC, "apic_batch_state": apic.BatchStateC}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "apic.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('printf("%s sizeof %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = {}
    for ln in subprocess.check_output([str(exe)]).decode().split("\n"):
        if ln.strip():
            a, b, v = ln.split()
            got[(a, b)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_kernel_source_hash_ignores_comments_only():
    """The hash a stored counter run is checked against changes with the
    kernels' code, not with their comments or blank lines."""
    from paper_2608_15249_amd.rocprof_summary import _code_only
    a = 'int f(int x) {  // doubled\n    return 2 * x; /* "x" */\n}\nconst char *s = "a // b /* c";\nchar q = \'\\\'\';\n'
    b = '// header\n\nint f(int x) {\n    return 2 * x;   \n}\n/* a\n   block */\nconst char *s = "a // b /* c";\nchar q = \'\\\'\';\n'
    assert _code_only(a) == _code_only(b)
    assert '"a // b /* c"' in _code_only(a)
    assert _code_only(a) != _code_only(a.replace("2 * x", "3 * x"))
