"""The product path has no CPU fallback: the binding refuses to run without the
HIP library, and nothing in the package (or bench.py's GPU legs) reaches the
oracle."""
import ast
import os

import pytest

from paper_2602_09020_amd import cfh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2602_09020_amd")


def test_binding_raises_without_the_library(monkeypatch):
    monkeypatch.setattr(cfh, "_L", None)
    monkeypatch.setattr(cfh, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libcfh.so"))
    with pytest.raises(ImportError):
        cfh.lib()


def imported_modules(path):
    tree = ast.parse(open(path).read(), filename=path)
    out = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            out.update(a.name for a in node.names)
        elif isinstance(node, ast.ImportFrom):
            out.add(node.module or "")
    return out


def test_package_never_imports_the_oracle():
    files = []
    for d, _, names in os.walk(PKG):
        files += [os.path.join(d, f) for f in names if f.endswith(".py")]
    assert files
    for f in files:
        assert not any(m == "oracle" or m.startswith("oracle.") for m in imported_modules(f)), f
    for f in os.listdir(os.path.join(PKG, "csrc")):
        text = open(os.path.join(PKG, "csrc", f), errors="replace").read()
        assert "cfh_oracle" not in text and "oracle/" not in text, f


def test_bench_imports_the_oracle_only_in_its_cpu_baseline_leg():
    src = open(os.path.join(ROOT, "bench.py")).read()
    tree = ast.parse(src)
    top = {a.name for n in tree.body if isinstance(n, ast.Import) for a in n.names}
    top |= {n.module for n in tree.body if isinstance(n, ast.ImportFrom)}
    assert not any(m and (m == "oracle" or m.startswith("oracle.")) for m in top)
