"""The benchmark's CPU-oracle leg forks worker processes, so it refuses to
run in a process that holds GPU state: here the library itself is mapped
(ctypes load, no device call), and the leg must raise before forking."""
import ctypes
import os

import numpy as np
import pytest

import bench

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2602_01330_amd", "libqk.so")


def test_cpu_baseline_refuses_once_the_library_is_loaded():
    ctypes.CDLL(LIB)
    assert any("libqk.so" in r for r in bench.gpu_state_held())
    with pytest.raises(RuntimeError, match="must run before anything touches the GPU"):
        bench.cpu_baseline(np.zeros((16, 784)))


def test_cpu_description_fields():
    info = bench.cpu_model()
    assert info["affinity_cpus"] >= 1
