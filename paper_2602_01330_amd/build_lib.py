"""Compile libqk.so for gfx950 in place (hipcc, no JIT cache).

Used by ``__graft_entry__.build()`` and runnable directly:
``python -m paper_2602_01330_amd.build_lib``.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libqk.so")

SOURCES = ["qk_api.cpp", "tune.cpp", "server.cpp", "preproc_api.cpp", "build.hip",
           "sweep_valu.hip", "sweep_mfma.hip", "sweep_big.hip", "sweep_wide.hip",
           "classical.hip", "svm.hip", "pathsum.hip", "preprocess.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(HERE, "_build", src + ".o")
        cmd = [hipcc] + [f for f in FLAGS if f != "-shared"] + [
            "-I", os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, src),
            "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc, "-x", "hip"] + cmd[1:]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{res.stderr}")
        if verbose and res.stderr.strip():
            errs = [l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l]
            if errs:
                print("\n".join(errs), file=sys.stderr)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
