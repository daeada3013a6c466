"""The oracle and the product path stay apart, and the product path fails
loudly without its compiled library (CPU only)."""
import ast
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _imports(path):
    tree = ast.parse(open(path).read(), filename=path)
    names = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            names.update(a.name.split(".")[0] for a in node.names)
        elif isinstance(node, ast.ImportFrom) and node.module and node.level == 0:
            names.add(node.module.split(".")[0])
    return names


def _py_files(folder):
    return [os.path.join(folder, f) for f in sorted(os.listdir(folder)) if f.endswith(".py")]


def test_product_modules_do_not_import_the_oracle():
    for path in _py_files(os.path.join(ROOT, "paper_2104_10785_amd")):
        assert "oracle" not in _imports(path), path


def test_oracle_imports_nothing_from_the_product():
    for path in _py_files(os.path.join(ROOT, "oracle")):
        assert "paper_2104_10785_amd" not in _imports(path), path


def test_device_sources_do_not_name_the_oracle():
    csrc = os.path.join(ROOT, "paper_2104_10785_amd", "csrc")
    for f in sorted(os.listdir(csrc)) + [os.path.join("..", "..", "include", h)
                                         for h in sorted(os.listdir(os.path.join(ROOT, "include")))]:
        text = open(os.path.join(csrc, f)).read()
        assert "oracle/" not in text and "import oracle" not in text, f


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2104_10785_amd import gkb
    monkeypatch.setattr(gkb, "_lib", None)
    monkeypatch.setattr(gkb, "LIB_PATH", str(tmp_path / "libgkb.so"))
    with pytest.raises(RuntimeError, match="missing"):
        gkb.lib()
    with pytest.raises(RuntimeError, match="missing"):
        gkb.gkb_host_dense_svd([[1.0]])
