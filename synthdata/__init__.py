"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This package holds input generators only: it draws feature vectors, labels and
request streams and contains none of the kernel arithmetic (no circuit, no
tensor network, no RBF, no mixing). Both the CPU oracle and the HIP library are
fed from these arrays, so the two sides never exchange code.
"""
from .generators import (  # noqa: F401
    CONFIGS,
    gen_clusters,
    gen_images,
    gen_isometry_mps,
    gen_requests,
    config_inputs,
)
