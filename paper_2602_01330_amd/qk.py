"""Thin ctypes binding of libqk (include/qk.h), same names as the C ABI.

Argument marshalling only: every step of the computation runs in the HIP
kernels of libqk. PyTorch supplies device memory (``tensor.data_ptr()``) and
streams (``torch.cuda.current_stream().cuda_stream``). There is no CPU
fallback: a missing library raises at import.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqk.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"libqk.so not found at {LIB_PATH}; build it with "
        "`python -m paper_2602_01330_amd.build_lib` (no CPU fallback exists)")

_lib = C.CDLL(LIB_PATH)

# ---- enums (qk.h) -----------------------------------------------------------
QK_OK = 0
STATUS = {0: "QK_OK", -1: "QK_ERR_INVALID_ARG", -2: "QK_ERR_OUT_OF_MEMORY",
          -3: "QK_ERR_HIP", -4: "QK_ERR_UNSUPPORTED", -5: "QK_ERR_BUSY",
          -6: "QK_ERR_CANCELLED", -7: "QK_ERR_DEVICE", -8: "QK_ERR_NOT_FOUND"}
QK_PREC_FP64, QK_PREC_FP32, QK_PREC_BF16X2, QK_PREC_BF16X3, QK_PREC_AUTO, \
    QK_PREC_FP32_MFMA = 0, 1, 2, 3, 4, 5
PREC = {"fp64": 0, "fp32": 1, "bf16x2": 2, "bf16x3": 3, "auto": 4, "fp32_mfma": 5}
PREC_NAME = {v: k for k, v in PREC.items()}
QK_STORE_FP64, QK_STORE_FP32, QK_STORE_ALL = 1, 2, 3


class QkError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class qk_circuit_desc(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("n_layers", C.c_int32),
                ("chi_max", C.c_int32), ("entangle", C.c_int32),
                ("cutoff_rel", C.c_double)]


class qk_fuse_desc(C.Structure):
    _fields_ = [("x_rows_dev", C.c_void_p), ("ld_xr", C.c_int64),
                ("x_cols_dev", C.c_void_p), ("ld_xc", C.c_int64),
                ("gamma", C.c_double), ("w", C.c_double),
                ("kc_dev", C.c_void_p), ("ld_kc", C.c_int64),
                ("k_dev", C.c_void_p), ("ld_k", C.c_int64)]


class qk_gram_task(C.Structure):
    _fields_ = [("rows", C.c_void_p), ("cols", C.c_void_p),
                ("symmetric", C.c_int32), ("kq_dev", C.c_void_p),
                ("ld_kq", C.c_int64), ("lnkq_dev", C.c_void_p),
                ("ld_ln", C.c_int64), ("fuse", qk_fuse_desc),
                ("use_fuse", C.c_int32)]


_P = C.c_void_p
_lib.qk_mps_build.argtypes = [C.POINTER(qk_circuit_desc), _P, C.c_int64, C.c_int64,
                              C.c_uint32, _P, C.POINTER(_P)]
_lib.qk_mps_import.argtypes = [C.POINTER(qk_circuit_desc), C.c_int64, C.c_int32, _P, _P,
                               C.c_uint32, _P, C.POINTER(_P)]
_lib.qk_mps_info.argtypes = [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                             C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                             C.POINTER(C.c_int64)]
_lib.qk_mps_chi.argtypes = [_P, _P]
_lib.qk_mps_release.argtypes = [_P]
_lib.qk_overlap_gram.argtypes = [_P, _P, C.c_int32, C.c_int, _P, C.c_int64, _P, C.c_int64,
                                 C.POINTER(qk_fuse_desc), _P]
_lib.qk_overlap_gram_multi.argtypes = [C.POINTER(qk_gram_task), C.c_int32, C.c_int, _P]
_lib.qk_rbf_gram.argtypes = [_P, C.c_int64, C.c_int64, _P, C.c_int64, C.c_int64, C.c_int32,
                             C.c_double, _P, C.c_int64, _P]
_lib.qk_dual_mix.argtypes = [_P, C.c_int64, _P, C.c_int64, C.c_int64, C.c_int64, C.c_double,
                             _P, C.c_int64, _P]
_lib.qk_resolve_precision.argtypes = [_P, _P, C.POINTER(C.c_int)]
_lib.qk_set_refine_threshold.argtypes = [C.c_int, C.c_double]
_lib.qk_status_string.restype = C.c_char_p
_lib.qk_status_string.argtypes = [C.c_int]
_lib.qk_last_error.restype = C.c_char_p
for _f in ("qk_mps_build", "qk_mps_import", "qk_mps_info", "qk_mps_chi", "qk_mps_release",
           "qk_overlap_gram", "qk_overlap_gram_multi", "qk_rbf_gram", "qk_dual_mix",
           "qk_resolve_precision", "qk_set_refine_threshold"):
    getattr(_lib, _f).restype = C.c_int

EXPORTED = ["qk_mps_build", "qk_mps_import", "qk_mps_info", "qk_mps_chi", "qk_mps_release",
            "qk_overlap_gram", "qk_overlap_gram_multi", "qk_rbf_gram", "qk_dual_mix",
            "qk_resolve_precision", "qk_set_refine_threshold", "qk_status_string",
            "qk_last_error"]


def _check(st):
    if st != QK_OK:
        raise QkError(st, _lib.qk_last_error().decode())


def _stream(stream):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _mat(t, name, dtype=torch.float64):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if t.dim() != 2 or (t.shape[1] > 1 and t.stride(1) != 1):
        raise ValueError(f"{name} must be a row-major 2-D tensor")
    return C.c_void_p(t.data_ptr()), max(t.stride(0), t.shape[1], 1)


def _opt(t, name):
    if t is None:
        return C.c_void_p(0), 0
    return _mat(t, name)


class MpsBatch:
    """Owns a qk_mps_batch handle; released on close() or garbage collection."""

    def __init__(self, handle, n_qubits, keepalive=None):
        self._h = handle
        self.n_qubits = n_qubits
        self._keep = keepalive

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("batch released")
        return self._h

    def close(self):
        if self._h is not None:
            _lib.qk_mps_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def circuit(n_qubits, n_layers, chi_max, cutoff=1e-10, entangle=True):
    return qk_circuit_desc(int(n_qubits), int(n_layers), int(chi_max), 1 if entangle else 0,
                           float(cutoff))


def qk_mps_build(x, n_layers, chi_max, cutoff=1e-10, entangle=True, store=QK_STORE_ALL,
                 stream=None) -> MpsBatch:
    """Build one MPS per row of x (float64 CUDA tensor, n x d)."""
    xp, ld = _mat(x, "x")
    desc = circuit(x.shape[1], n_layers, chi_max, cutoff, entangle)
    h = C.c_void_p()
    _check(_lib.qk_mps_build(C.byref(desc), xp, x.shape[0], ld, store, _stream(stream),
                             C.byref(h)))
    return MpsBatch(h, x.shape[1], keepalive=x)


def qk_mps_import(chi, tensors, n_layers, chi_max, cutoff=1e-10, entangle=True,
                  store=QK_STORE_ALL, stream=None) -> MpsBatch:
    """Upload host MPS: chi int32 (n, nq+1); tensors complex128 [nq][n][2][T][T]."""
    chi = np.ascontiguousarray(chi, dtype=np.int32)
    tensors = np.ascontiguousarray(tensors, dtype=np.complex128)
    nq, n, two, T, T2 = tensors.shape
    if two != 2 or T != T2 or chi.shape != (n, nq + 1):
        raise ValueError("bad import shapes")
    desc = circuit(nq, n_layers, chi_max, cutoff, entangle)
    h = C.c_void_p()
    _check(_lib.qk_mps_import(C.byref(desc), n, T, chi.ctypes.data_as(C.c_void_p),
                              tensors.ctypes.data_as(C.c_void_p), store, _stream(stream),
                              C.byref(h)))
    return MpsBatch(h, nq)


def qk_mps_info(batch: MpsBatch) -> dict:
    n, nq, T, cmax, nbytes = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
    _check(_lib.qk_mps_info(batch.handle, C.byref(n), C.byref(nq), C.byref(T), C.byref(cmax),
                            C.byref(nbytes)))
    return {"n_samples": n.value, "n_qubits": nq.value, "chi_pad": T.value,
            "chi_realized_max": cmax.value, "device_bytes": nbytes.value}


def qk_mps_chi(batch: MpsBatch) -> np.ndarray:
    info = qk_mps_info(batch)
    out = np.empty((info["n_samples"], info["n_qubits"] + 1), dtype=np.int32)
    _check(_lib.qk_mps_chi(batch.handle, out.ctypes.data_as(C.c_void_p)))
    return out


def qk_mps_release(batch: MpsBatch):
    batch.close()


def _fuse(fuse):
    if fuse is None:
        return None
    f = qk_fuse_desc()
    f.x_rows_dev, f.ld_xr = _mat(fuse["x_rows"], "x_rows")
    f.x_cols_dev, f.ld_xc = _mat(fuse["x_cols"], "x_cols")
    f.gamma = float(fuse["gamma"])
    f.w = float(fuse["w"])
    f.kc_dev, f.ld_kc = _opt(fuse.get("kc"), "kc")
    f.k_dev, f.ld_k = _opt(fuse.get("k"), "k")
    return f


def qk_overlap_gram(rows: MpsBatch, cols: MpsBatch, symmetric=False, prec="auto", kq=None,
                    lnkq=None, fuse=None, stream=None):
    """Fill kq / lnkq (and fused kc / k) in place; returns (kq, lnkq)."""
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    kp, ldk = _opt(kq, "kq")
    lp, ldl = _opt(lnkq, "lnkq")
    f = _fuse(fuse)
    _check(_lib.qk_overlap_gram(rows.handle, cols.handle, 1 if symmetric else 0, p, kp, ldk,
                                lp, ldl, C.byref(f) if f is not None else None,
                                _stream(stream)))
    return kq, lnkq


def qk_overlap_gram_multi(tasks, prec="auto", stream=None):
    """tasks: list of dicts with rows, cols, symmetric, kq, lnkq, fuse."""
    arr = (qk_gram_task * len(tasks))()
    for a, t in zip(arr, tasks):
        a.rows = t["rows"].handle
        a.cols = t["cols"].handle
        a.symmetric = 1 if t.get("symmetric") else 0
        a.kq_dev, a.ld_kq = _opt(t.get("kq"), "kq")
        a.lnkq_dev, a.ld_ln = _opt(t.get("lnkq"), "lnkq")
        f = _fuse(t.get("fuse"))
        if f is not None:
            a.fuse = f
            a.use_fuse = 1
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    _check(_lib.qk_overlap_gram_multi(arr, len(tasks), p, _stream(stream)))


def qk_rbf_gram(x, y, gamma, kc, stream=None):
    xp, ldx = _mat(x, "x")
    yp, ldy = _mat(y, "y")
    kp, ldk = _mat(kc, "kc")
    _check(_lib.qk_rbf_gram(xp, x.shape[0], ldx, yp, y.shape[0], ldy, x.shape[1],
                            float(gamma), kp, ldk, _stream(stream)))
    return kc


def qk_dual_mix(kq, kc, w, k, stream=None):
    qp, ldq = _mat(kq, "kq")
    cp, ldc = _mat(kc, "kc")
    kp, ldk = _mat(k, "k")
    _check(_lib.qk_dual_mix(qp, ldq, cp, ldc, kq.shape[0], kq.shape[1], float(w), kp, ldk,
                            _stream(stream)))
    return k


def qk_resolve_precision(rows: MpsBatch, cols: MpsBatch) -> str:
    out = C.c_int()
    _check(_lib.qk_resolve_precision(rows.handle, cols.handle, C.byref(out)))
    return PREC_NAME[out.value]


def qk_set_refine_threshold(prec, tau: float):
    """FP64 recomputation of tiles holding K_q > tau for a reduced form."""
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    _check(_lib.qk_set_refine_threshold(p, float(tau)))


REFINE_DEFAULT = {"fp32": 1e-2, "fp32_mfma": 1e-2, "bf16x3": 1e-2, "bf16x2": 1e-3}


def qk_status_string(s: int) -> str:
    return _lib.qk_status_string(s).decode()


def qk_last_error() -> str:
    return _lib.qk_last_error().decode()
