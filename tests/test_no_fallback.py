"""The product path has no CPU fallback and never touches the oracle (CPU).

Without libspinsum.so the package refuses to import; and neither the
binding nor the library sources name the oracle, so no computation of the
package can route through it.
"""
import importlib.util
import os
import re
import shutil

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1705_06661_amd")


def test_import_fails_without_the_library(tmp_path):
    probe = tmp_path / "spinsum_probe"
    probe.mkdir()
    shutil.copy(os.path.join(PKG, "__init__.py"), probe / "__init__.py")
    spec = importlib.util.spec_from_file_location("spinsum_probe", probe / "__init__.py")
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError, match="no CPU fallback"):
        spec.loader.exec_module(mod)


def test_package_never_names_the_oracle():
    pat = re.compile(r"\boracle\b")
    for dirpath, _, files in os.walk(PKG):
        if "_build" in dirpath:
            continue
        for f in files:
            if f.endswith((".py", ".h", ".hip", ".cpp")):
                text = open(os.path.join(dirpath, f), encoding="utf-8").read()
                assert not pat.search(text), os.path.join(dirpath, f)
    header = open(os.path.join(ROOT, "include", "spinsum.h"), encoding="utf-8").read()
    assert not pat.search(header)
