"""The product path has no CPU fallback: without the built HIP library the
binding refuses to load, and nothing in the package reaches the oracle."""
import ast
import importlib.util
import os
import shutil

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1505_02100_amd")


def test_binding_refuses_to_load_without_the_library(tmp_path):
    pkg = tmp_path / "pkg_without_library"
    pkg.mkdir()
    shutil.copy(os.path.join(PKG, "kdeplugin.py"), pkg / "kdeplugin.py")
    spec = importlib.util.spec_from_file_location("kdeplugin_probe", pkg / "kdeplugin.py")
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError, match="libkdeplugin.so not found"):
        spec.loader.exec_module(mod)


def test_package_never_imports_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for name in files:
            if not name.endswith(".py"):
                continue
            path = os.path.join(dirpath, name)
            tree = ast.parse(open(path).read(), path)
            for node in ast.walk(tree):
                if isinstance(node, ast.Import):
                    mods = [a.name for a in node.names]
                elif isinstance(node, ast.ImportFrom):
                    mods = [node.module or ""]
                else:
                    continue
                assert not any(m == "oracle" or m.startswith("oracle.") for m in mods), (path, mods)


def test_native_sources_do_not_reference_the_oracle():
    csrc = os.path.join(PKG, "csrc")
    for name in os.listdir(csrc):
        if name.endswith((".hip", ".cpp", ".h")):
            text = open(os.path.join(csrc, name)).read()
            assert "oracle" not in text.lower(), name
