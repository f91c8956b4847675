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


def test_argument_checks_of_the_svm_and_path_sum_entry_points_without_gpu():
    """Host-side validation returns before any device call: bad labels,
    class counts, box bound and step cap of qk_svm_fit_ovo; sizes and
    outputs of qk_svm_predict_ovo; layer count and outputs of
    qk_pathsum_gram. The pointers are never dereferenced."""
    lib = ctypes.CDLL(LIB)
    P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.qk_svm_fit_ovo.argtypes = [P, I64, I64, P, I32, D, D, I64, P, I64, P, P, P]
    lib.qk_svm_predict_ovo.argtypes = [P, I64, I64, I64, P, I64, P, I32, P, I64, P, P]
    lib.qk_pathsum_gram.argtypes = [P, I64, I64, P, I64, I64, I32, I32, I32, I32, P, I64, P,
                                    I64, P, P]
    INVALID, UNSUPPORTED = -1, -4
    fake = P(0x1000)
    labels = (ctypes.c_int32 * 4)(0, 1, 2, 1)

    def fit(lab, n_classes=3, C=1.0, eps=1e-3, max_iter=10):
        return lib.qk_svm_fit_ovo(fake, 4, 4, ctypes.cast(lab, P), n_classes, C, eps, max_iter,
                                  fake, 4, fake, fake, None)

    assert fit((ctypes.c_int32 * 4)(0, 1, 3, 1)) == INVALID   # label >= n_classes
    assert fit((ctypes.c_int32 * 4)(0, -2, 2, 1)) == INVALID  # label below -1
    assert fit(labels, n_classes=1) == INVALID
    assert fit(labels, n_classes=65) == INVALID
    assert fit(labels, C=0.0) == INVALID
    assert fit(labels, C=float("inf")) == INVALID
    assert fit(labels, eps=0.0) == INVALID
    assert fit(labels, max_iter=0) == INVALID
    assert lib.qk_svm_predict_ovo(fake, 3, 4, 4, fake, 4, fake, 3, None, 3, None, None) == INVALID
    assert lib.qk_svm_predict_ovo(fake, 3, 4, 4, fake, 4, fake, 3, fake, 2, None, None) == INVALID
    assert lib.qk_svm_predict_ovo(fake, 3, 4, 3, fake, 4, fake, 3, fake, 3, None, None) == INVALID
    ln = fake
    assert lib.qk_pathsum_gram(fake, 4, 8, fake, 4, 8, 8, 4, 1, 1, None, 0, ln, 4, None,
                               None) == UNSUPPORTED
    assert lib.qk_pathsum_gram(fake, 4, 8, fake, 4, 8, 8, 2, 1, 1, None, 0, None, 0, None,
                               None) == INVALID  # no output
    assert lib.qk_pathsum_gram(fake, 4, 8, P(0x2000), 4, 8, 8, 2, 1, 1, None, 0, ln, 4, None,
                               None) == INVALID  # symmetric with different features
    assert lib.qk_pathsum_gram(fake, 4, 7, fake, 4, 7, 8, 2, 1, 0, None, 0, ln, 4, None,
                               None) == INVALID  # leading dimension below d


def test_pathsum_rejects_a_negative_gamma_and_sweep_limit_range():
    """A fused path-sum call with gamma < 0 would give K_c > 1 (outside the
    kernel range of Eq. (3)); it is rejected before any launch, as the MPS
    route's fusion and qk_rbf_gram do. The SVD sweep limit accepts [0, 1000]."""
    from paper_2602_01330_amd.qk import qk_fuse_desc
    lib = ctypes.CDLL(LIB)
    P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.qk_pathsum_gram.argtypes = [P, I64, I64, P, I64, I64, I32, I32, I32, I32, P, I64, P,
                                    I64, ctypes.POINTER(qk_fuse_desc), P]
    fake = P(0x1000)
    for gamma, want in ((-0.5, -1), (float("nan"), -1), (float("inf"), -1)):
        f = qk_fuse_desc(gamma=gamma, w=0.5, k_dev=0x3000, ld_k=4)
        assert lib.qk_pathsum_gram(fake, 4, 8, fake, 4, 8, 8, 2, 1, 1, None, 0, None, 0,
                                   ctypes.byref(f), None) == want
    lib.qk_set_svd_sweep_limit.argtypes = [I32]
    assert lib.qk_set_svd_sweep_limit(-1) == -1
    assert lib.qk_set_svd_sweep_limit(1001) == -1
    assert lib.qk_set_svd_sweep_limit(60) == 0


def test_argument_checks_of_preprocessing_and_the_allocation_free_call_without_gpu():
    """qk_preproc_fit / qk_preproc_apply reject bad sizes, leading dimensions,
    component counts and scales before any allocation or launch; the
    allocation-free Gram call rejects a NULL batch first. Pointers are never
    dereferenced."""
    lib = ctypes.CDLL(LIB)
    P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.qk_preproc_fit.argtypes = [P, I64, I64, I32, I32, P, ctypes.POINTER(P)]
    lib.qk_preproc_apply.argtypes = [P, P, I64, I64, D, P, I64, P]
    lib.qk_overlap_gram_noalloc.argtypes = [P, P, I32, I32, P, I64, P, I64, P, P]
    INVALID = -1
    fake = P(0x1000)
    out = P()
    fit = lambda x, n, ld, d, k: lib.qk_preproc_fit(x, n, ld, d, k, None, ctypes.byref(out))
    assert fit(None, 10, 8, 8, 2) == INVALID          # no features
    assert fit(fake, 1, 8, 8, 2) == INVALID           # one row: no covariance
    assert fit(fake, 10, 8, 0, 1) == INVALID          # d < 1
    assert fit(fake, 10, 9000, 8193, 2) == INVALID    # d above 8192
    assert fit(fake, 10, 7, 8, 2) == INVALID          # ld_x < d
    assert fit(fake, 10, 8, 8, 0) == INVALID          # no component
    assert fit(fake, 10, 8, 8, 9) == INVALID          # more components than features
    assert fit(fake, 2 ** 31, 8, 8, 2) == INVALID     # rows beyond int32
    assert lib.qk_preproc_fit(fake, 10, 8, 8, 2, None, None) == INVALID  # no out pointer
    assert not out.value
    # apply: NULL handle first, then the arguments
    assert lib.qk_preproc_apply(None, fake, 4, 8, 1.0, fake, 2, None) == INVALID
    assert lib.qk_preproc_release(None) == 0
    assert lib.qk_overlap_gram_noalloc(None, None, 1, 5, fake, 4, None, 0, None, None) == INVALID


def test_tuning_table_launch_shape_fields_without_gpu():
    """Entries carry the launch shape: 'T bucket form wg_per_cu band us'.
    A five-field entry imports with band 4; a band outside 1..64 or a
    workgroup count below 1 is rejected; export prints six fields."""
    import pytest

    import paper_2602_01330_amd.qk as qk
    mfma = qk.PREC["fp32_mfma"]
    qk.qk_tune_import(f"4 9 {mfma} 1 8 2.5\n2 3 {mfma} 2 1.25\n")
    rows = {tuple(l.split()[:2]): l.split() for l in qk.qk_tune_export().strip().splitlines()}
    assert rows[("4", "9")][2:5] == [str(mfma), "1", "8"] and len(rows[("4", "9")]) == 6
    assert rows[("2", "3")][2:5] == [str(mfma), "2", "4"]
    for bad in (f"4 9 {mfma} 1 0 1.0\n", f"4 9 {mfma} 1 65 1.0\n", f"4 9 {mfma} 0 4 1.0\n"):
        with pytest.raises(qk.QkError):
            qk.qk_tune_import(bad)
