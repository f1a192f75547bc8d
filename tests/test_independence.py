"""Separation of the oracle from the product path (CPU only).

* No module of the package, nor the seeded input generators, imports the oracle;
  the oracle imports neither of them.
* No HIP source or public header includes anything from the oracle's folder.
* bench.py imports the oracle only inside its CPU-baseline worker.
* The binding raises when the compiled library is missing: there is no
  fallback that would compute the path elsewhere.
"""
import ast
import pathlib

import pytest

from paper_2304_11002_amd import fmm

ROOT = pathlib.Path(__file__).resolve().parents[1]


def imported_modules(path):
    """(top-level module name, enclosing function name or None) for every import."""
    tree = ast.parse(path.read_text(), filename=str(path))
    found = []

    def visit(node, func):
        for child in ast.iter_child_nodes(node):
            if isinstance(child, (ast.FunctionDef, ast.AsyncFunctionDef)):
                visit(child, child.name)
                continue
            if isinstance(child, ast.Import):
                found.extend((a.name.split(".")[0], func) for a in child.names)
            elif isinstance(child, ast.ImportFrom) and child.level == 0 and child.module:
                found.append((child.module.split(".")[0], func))
            visit(child, func)

    visit(tree, None)
    return found


def py_files(folder):
    return sorted(p for p in (ROOT / folder).rglob("*.py") if "__pycache__" not in p.parts)


def test_package_and_generators_do_not_import_the_oracle():
    files = py_files("paper_2304_11002_amd") + py_files("synth")
    assert len(files) >= 4
    for f in files:
        mods = {m for m, _ in imported_modules(f)}
        assert "oracle" not in mods, "%s imports the oracle" % f.relative_to(ROOT)


def test_oracle_imports_neither_the_package_nor_the_generators():
    files = py_files("oracle")
    assert len(files) >= 3
    for f in files:
        mods = {m for m, _ in imported_modules(f)}
        assert not mods & {"paper_2304_11002_amd", "synth", "torch", "ctypes"}, \
            "%s imports %s" % (f.relative_to(ROOT), mods & {"paper_2304_11002_amd", "synth", "torch", "ctypes"})


def test_native_sources_do_not_include_oracle_files():
    srcs = sorted((ROOT / "paper_2304_11002_amd" / "csrc").glob("*")) + sorted((ROOT / "include").glob("*"))
    assert any(s.suffix == ".hip" for s in srcs)
    for s in srcs:
        for line in s.read_text().splitlines():
            if line.lstrip().startswith("#include"):
                assert "oracle" not in line, "%s: %s" % (s.relative_to(ROOT), line)


def test_bench_uses_the_oracle_only_in_the_cpu_baseline_worker():
    uses = [func for m, func in imported_modules(ROOT / "bench.py") if m == "oracle"]
    assert uses == ["_oracle_worker"]


def test_missing_library_raises(monkeypatch, tmp_path):
    monkeypatch.setattr(fmm, "_lib", None)
    with pytest.raises(ImportError, match="not found"):
        fmm.load_library(str(tmp_path / "libfmm.so"))
