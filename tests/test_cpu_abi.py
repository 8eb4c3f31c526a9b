"""The C-ABI library loads on a machine without a GPU and exports every
symbol that include/dagrt.h declares."""

import os
import re
import subprocess

from paper_2012_09646_amd import dagrt as D

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    txt = open(os.path.join(ROOT, "include", "dagrt.h")).read()
    return set(re.findall(r"^(?:dag_status|const char\*)\s+(dag_\w+)\s*\(", txt, re.M))


def test_library_exports_header_symbols():
    L = D.lib()
    names = declared()
    assert len(names) >= 28
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", D.LIB_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.split()[-1].startswith("dag_")}
    assert exported == names


def test_binding_covers_every_symbol():
    assert set(D._SIGS) == declared()
    for n in declared():
        assert callable(getattr(D, n)), n


def test_status_strings():
    assert D.dag_status_string(0) == "ok"
    assert "poisoned" in D.dag_status_string(-5)
