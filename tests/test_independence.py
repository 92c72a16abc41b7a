"""The product path never reaches the oracle, and fails loudly without the
HIP library.

* No module of the package imports `oracle` (checked on the syntax tree, so
  a lazy import inside a function counts too), and no HIP source or public
  header includes an oracle header or names its functions.
* In bench.py only the host-core baseline (`cpu_baseline`) imports the oracle.
* With the shared library missing, the binding raises instead of falling back
  to anything else.
"""

import ast
import glob
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2602_23434_amd")


def _imports(tree):
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            for a in node.names:
                yield node, a.name.split(".")[0]
        elif isinstance(node, ast.ImportFrom) and node.module:
            yield node, node.module.split(".")[0]


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(PKG, "*.py"))), ids=os.path.basename)
def test_package_module_does_not_import_oracle(path):
    with open(path) as f:
        tree = ast.parse(f.read())
    assert not [n.lineno for n, mod in _imports(tree) if mod == "oracle"], path


def test_native_sources_do_not_reach_the_oracle():
    srcs = glob.glob(os.path.join(PKG, "csrc", "*")) + glob.glob(os.path.join(ROOT, "include", "*.h"))
    assert srcs
    for p in srcs:
        with open(p) as f:
            text = f.read()
        assert "orc.h" not in text and "orc_" not in text and "liborc" not in text, p


def test_bench_imports_oracle_only_in_cpu_baseline():
    with open(os.path.join(ROOT, "bench.py")) as f:
        tree = ast.parse(f.read())
    owners = []
    for fn in ast.walk(tree):
        if isinstance(fn, ast.FunctionDef):
            for node, mod in _imports(fn):
                if mod == "oracle":
                    owners.append(fn.name)
    top = [n.lineno for n, mod in _imports(ast.Module(body=[s for s in tree.body
                                                           if not isinstance(s, ast.FunctionDef)],
                                                     type_ignores=[]))
           if mod == "oracle"]
    assert not top
    assert set(owners) <= {"cpu_baseline"}, owners


def test_binding_raises_without_the_library(monkeypatch, tmp_path):
    from paper_2602_23434_amd import binding
    monkeypatch.setattr(binding, "_LIB", None)
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "libpl.so"))
    with pytest.raises(RuntimeError, match="missing"):
        binding.lib()
