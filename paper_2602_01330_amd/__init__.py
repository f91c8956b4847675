"""MI355X-native quantum-classical dual kernel: MPS quantum kernel Gram
matrices, the RBF kernel and their linear mix, computed by the HIP library
libqk (C ABI in include/qk.h).

Import is lightweight; ``paper_2602_01330_amd.qk`` loads the native library
and raises if it has not been built (there is no CPU fallback).
"""
