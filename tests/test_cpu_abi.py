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


def test_static_launch_rejects_bad_calls_before_touching_the_gpu():
    """dag_launch_static checks its arguments and its scratch limit on the
    host: these calls fail without any HIP call (the addresses are never
    dereferenced)."""
    fake = [0x10000 + 256 * i for i in range(5)]
    n = 1 << 20
    # nrows + nnz just under 2^31: more tile carries than the fixed array holds
    # at any items-per-thread setting
    nnz = (1 << 31) - 1 - n - 16
    sizes = [4 * (n + 1), 4 * nnz, 4 * nnz, 4 * n, 4 * n]
    cases = [
        (D.KERNEL_IDS["spmv"], D.dag_p_csr(n, n, nnz), fake, sizes, D.DAG_E_RANGE, "static scratch"),
        (999, D.dag_p_n(4), fake[:1], [16], D.DAG_E_INVAL, "unknown"),
        (D.KERNEL_IDS["sumsq"], D.dag_p_csr(1, 1, 1), fake[:2], [16, 8], D.DAG_E_INVAL, "parameter block"),
        (D.KERNEL_IDS["sumsq"], D.dag_p_n(4), fake[:1], [16], D.DAG_E_INVAL, "arguments"),
        (D.KERNEL_IDS["sumsq"], D.dag_p_n(4), [fake[0], 0], [16, 8], D.DAG_E_INVAL, "NULL"),
        (D.KERNEL_IDS["sumsq"], D.dag_p_n(8), fake[:2], [16, 8], D.DAG_E_INVAL, "smaller"),
    ]
    for kid, prm, ptrs, sz, status, text in cases:
        try:
            D.dag_launch_static(kid, prm, ptrs, sz)
        except D.DagError as e:
            assert e.status == status, (kid, e)
            assert text in str(e), (text, str(e))
        else:
            raise AssertionError("call was accepted: kernel %d" % kid)
