"""The oracle and the device path share no code, and the oracle is test
infrastructure: nothing under oracle/ or synthdata/ imports the package;
synthdata/ (seeded inputs only) does not import the oracle; the package
(binding and sources) never refers to the oracle; bench.py imports the
oracle only in its CPU-baseline functions, and __graft_entry__.py only in
smoke()."""
import ast
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = "paper_2602_01330_amd"


def py_files(sub):
    for dp, _, fs in os.walk(os.path.join(ROOT, sub)):
        for f in fs:
            if f.endswith(".py"):
                yield os.path.join(dp, f)


def imported_roots(tree):
    """(root module name, enclosing top-level function or None) per import."""
    out = []

    def visit(node, func):
        for ch in ast.iter_child_nodes(node):
            f = func
            if isinstance(ch, (ast.FunctionDef, ast.AsyncFunctionDef)) and func is None:
                f = ch.name
            if isinstance(ch, ast.Import):
                out.extend((a.name.split(".")[0], f) for a in ch.names)
            elif isinstance(ch, ast.ImportFrom) and ch.module and ch.level == 0:
                out.append((ch.module.split(".")[0], f))
            visit(ch, f)

    visit(tree, None)
    return out


def roots_of(path):
    with open(path) as fh:
        return imported_roots(ast.parse(fh.read()))


@pytest.mark.parametrize("sub", ["oracle", "synthdata"])
def test_oracle_and_inputs_do_not_import_the_package(sub):
    for p in py_files(sub):
        assert all(r != PKG for r, _ in roots_of(p)), p


def test_inputs_do_not_import_the_oracle():
    for p in py_files("synthdata"):
        assert all(r != "oracle" for r, _ in roots_of(p)), p


def test_package_never_refers_to_the_oracle():
    for dp, _, fs in os.walk(os.path.join(ROOT, PKG)):
        if "_build" in dp:
            continue
        for f in fs:
            p = os.path.join(dp, f)
            if f.endswith(".py"):
                assert all(r != "oracle" for r, _ in roots_of(p)), p
            elif f.endswith((".hip", ".cpp", ".h")):
                with open(p) as fh:
                    src = fh.read()
                assert "oracle/" not in src and '#include "oracle' not in src, p


def test_bench_and_entry_point_confine_the_oracle():
    bench = [(r, f) for r, f in roots_of(os.path.join(ROOT, "bench.py")) if r == "oracle"]
    assert bench and all(f in ("cpu_baseline", "cpu_baseline_pathsum", "cpu_baseline_svm",
                                "_oracle_chunk") for _, f in bench), bench
    entry = [(r, f) for r, f in roots_of(os.path.join(ROOT, "__graft_entry__.py"))
             if r == "oracle"]
    assert entry and all(f == "smoke" for _, f in entry), entry


def test_binding_fails_loudly_without_the_library(tmp_path):
    """A copy of the binding next to no libqk.so raises ImportError at
    import: there is no CPU fallback for the product path."""
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / PKG
    pkg.mkdir()
    (pkg / "__init__.py").write_text("")
    shutil.copy(os.path.join(ROOT, PKG, "qk.py"), pkg / "qk.py")
    r = subprocess.run([sys.executable, "-c", f"import {PKG}.qk"], cwd=tmp_path,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "ImportError" in r.stderr and "libqk.so not found" in r.stderr
