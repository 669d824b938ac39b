"""The oracle is test infrastructure: nothing in the product package (Python
or native sources) imports, loads or names a file under ``oracle/``, and the
oracle imports nothing from the product.  Only the seeded input generators
(``synth``) serve both."""
import ast
import os
import re

from conftest import ROOT

PKG = os.path.join(ROOT, "paper_2608_15764_amd")
ORACLE = os.path.join(ROOT, "oracle")


def _py_files(top):
    for d, _, files in os.walk(top):
        if "__pycache__" in d:
            continue
        for f in files:
            if f.endswith(".py"):
                yield os.path.join(d, f)


def _imports(path):
    tree = ast.parse(open(path).read(), path)
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            for a in node.names:
                yield a.name
        elif isinstance(node, ast.ImportFrom) and node.module:
            yield node.module


def test_product_python_never_imports_the_oracle():
    for p in _py_files(PKG):
        for mod in _imports(p):
            assert mod.split(".")[0] != "oracle", (p, mod)


def test_native_sources_never_name_the_oracle():
    csrc = os.path.join(PKG, "csrc")
    for f in os.listdir(csrc):
        text = open(os.path.join(csrc, f), errors="replace").read()
        assert not re.search(r"\boracle/", text), f


def test_oracle_never_imports_the_product():
    for p in _py_files(ORACLE):
        for mod in _imports(p):
            root = mod.split(".")[0]
            assert root not in ("paper_2608_15764_amd", "bench", "__graft_entry__"), (p, mod)


def test_bench_reaches_the_oracle_only_in_its_cpu_baseline():
    """bench.py may call the oracle only inside its cpu_baseline leg: the
    leg itself, its worker-process helpers and the precision and batch
    checks whose oracle time it reports."""
    src = open(os.path.join(ROOT, "bench.py")).read()
    tree = ast.parse(src)
    allowed = {"cpu_baseline", "_oracle_cell", "cpu_oracle_worker", "cpu_precision_hook",
               "cpu_batch_verifier"}
    for fn in [n for n in tree.body if isinstance(n, ast.FunctionDef)]:
        uses = [m for m in _names_imported(fn) if m.split(".")[0] == "oracle"]
        if uses:
            assert fn.name in allowed or any(
                f.name in allowed for f in ast.walk(fn) if isinstance(f, ast.FunctionDef)), \
                (fn.name, uses)
    top = [m for n in tree.body if isinstance(n, (ast.Import, ast.ImportFrom))
           for m in _names_imported(n)]
    assert not any(m.split(".")[0] == "oracle" for m in top)


def _names_imported(node):
    for n in ast.walk(node):
        if isinstance(n, ast.Import):
            for a in n.names:
                yield a.name
        elif isinstance(n, ast.ImportFrom) and n.module:
            yield n.module
