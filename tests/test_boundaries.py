"""The product path fails loudly without its HIP library (no CPU fallback),
and the oracle and the product share no code: no product module imports the
oracle, and the oracle imports nothing from the product package."""
import ast
import os

import pytest

from paper_2004_07484_amd import _capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _imports(path):
    tree = ast.parse(open(path).read())
    out = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            out.update(a.name for a in node.names)
        elif isinstance(node, ast.ImportFrom) and node.module:
            out.add(node.module)
    return out


def _py_files(d):
    for base, _, files in os.walk(os.path.join(ROOT, d)):
        for f in files:
            if f.endswith(".py"):
                yield os.path.join(base, f)


def test_missing_library_raises(monkeypatch, tmp_path):
    monkeypatch.setattr(_capi, "LIB_PATH", str(tmp_path / "libpulsar.so"))
    monkeypatch.setattr(_capi, "_lib", None)
    with pytest.raises(_capi.PulsarLibraryMissing):
        _capi.load()
    params = _capi.make_params(0.1, 1e-5, 0.0, 5)
    with pytest.raises(_capi.PulsarLibraryMissing):
        _capi.pulsar_workspace_size(10, 64, 64, 3, params)


def test_product_does_not_import_the_oracle():
    for path in _py_files("paper_2004_07484_amd"):
        bad = {m for m in _imports(path) if m == "oracle" or m.startswith("oracle.")}
        assert not bad, f"{path} imports {bad}"


def test_oracle_imports_nothing_from_the_product():
    for path in _py_files("oracle"):
        bad = {m for m in _imports(path) if m.startswith("paper_2004_07484_amd")}
        assert not bad, f"{path} imports {bad}"
