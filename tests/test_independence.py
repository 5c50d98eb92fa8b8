"""The product path and the oracle stay apart: the package neither imports
nor includes anything of the oracle, the oracle uses only the package's
seeded input generators (no pricing arithmetic), and the binding refuses to
run without the HIP library instead of falling back to anything else."""
import os
import re

import pytest

import paper_1110_2477_amd as bt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1110_2477_amd")
ORC = os.path.join(ROOT, "oracle")


def _sources(top, exts):
    for d, _, files in os.walk(top):
        if "__pycache__" in d:
            continue
        for f in files:
            if f.endswith(exts):
                yield os.path.join(d, f)


def test_package_does_not_reach_the_oracle():
    pat = re.compile(r"^\s*(import\s+oracle|from\s+oracle|#\s*include\s*[<\"].*oracle)", re.M)
    hits = [p for p in _sources(PKG, (".py", ".hip", ".hpp", ".h", ".cpp")) if pat.search(open(p).read())]
    assert hits == []
    for p in _sources(PKG, (".py",)):
        assert "liboracle" not in open(p).read(), p


def test_oracle_uses_only_the_input_generators():
    pat = re.compile(r"^\s*(?:from|import)\s+(paper_1110_2477_amd[\w.]*)", re.M)
    for p in _sources(ORC, (".py",)):
        for mod in pat.findall(open(p).read()):
            assert mod == "paper_1110_2477_amd", (p, mod)
        assert not re.search(r"from\s+paper_1110_2477_amd\s+import\s+(?!workloads\b)", open(p).read()), p
    for p in _sources(ORC, (".c", ".h")):
        assert "bt_" + "kernels" not in open(p).read() and "bt.h" not in open(p).read(), p
    assert "def price" not in open(os.path.join(PKG, "workloads.py")).read()


def test_missing_library_raises(monkeypatch):
    monkeypatch.setattr(bt, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libbtprice.so"))
    monkeypatch.setattr(bt, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        bt.lib()
