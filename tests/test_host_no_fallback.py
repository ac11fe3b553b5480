"""The product path has no CPU fallback: without the HIP library every entry point raises, and no
product source imports or loads the oracle."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2602_04103_amd")


def test_missing_library_raises(monkeypatch):
    import paper_2602_04103_amd as qr
    monkeypatch.setattr(qr, "LIB_PATH", os.path.join(PKG, "no-such-library.so"))
    monkeypatch.setattr(qr, "_lib", None)
    with pytest.raises(ImportError):
        qr.lib()
    with pytest.raises(ImportError):
        qr.qr_line_of(5, 0)


def product_sources():
    for d, _, files in os.walk(PKG):
        if "__pycache__" in d:
            continue
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                yield os.path.join(d, f)
    yield os.path.join(ROOT, "include", "quadrank.h")


def test_product_never_touches_the_oracle():
    pat = re.compile(r"^\s*(import\s+oracle|from\s+oracle\b)|liboracle|oracle\.(rank|count|suffix|bwt|locate|interval)",
                     re.M)
    offenders = [p for p in product_sources() if pat.search(open(p, errors="replace").read())]
    assert not offenders, offenders
