"""The C-ABI library loads and exports every entry point include/qk.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qk.h")
LIB = os.path.join(ROOT, "paper_2602_01330_amd", "libqk.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"QK_API\s+[\w\s\*]+?\b(qk_\w+)\s*\(", text)))


def test_header_declares_the_four_operations():
    names = declared()
    for n in ("qk_mps_build", "qk_overlap_gram", "qk_rbf_gram", "qk_dual_mix"):
        assert n in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libqk.so not built (python -m paper_2602_01330_amd.build_lib)"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.qk_status_string.restype = ctypes.c_char_p
    assert lib.qk_status_string(0) == b"ok"
    assert lib.qk_status_string(-1) == b"invalid argument"


def test_binding_covers_the_abi():
    import paper_2602_01330_amd.qk as qk
    for n in declared():
        assert n in qk.EXPORTED and hasattr(qk, n), n


def test_tuning_table_round_trip_without_gpu():
    """qk_tune_import / qk_tune_export parse and print the table on the host."""
    import paper_2602_01330_amd.qk as qk
    qk.qk_tune_import("4 10 5 1 12.5\n2 1 1 3 0.25\n")
    text = qk.qk_tune_export()
    rows = {tuple(l.split()[:4]) for l in text.strip().splitlines()}
    assert ("4", "10", "5", "1") in rows and ("2", "1", "1", "3") in rows
    import pytest
    with pytest.raises(qk.QkError):
        qk.qk_tune_import("4 10 99 1 1.0\n")  # unknown form
    with pytest.raises(qk.QkError):
        qk.qk_tune_import("garbage")
