"""The C-ABI library builds for gfx950, loads, and exports every entry point declared in include/gpmg.h
(no GPU needed: nothing here launches a kernel)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gpmg.h")
HEADER3 = os.path.join(ROOT, "include", "gpmg3.h")
LIB = os.path.join(ROOT, "paper_1911_00994_amd", "libgpmg.so")


def declared_functions(header=HEADER):
    src = open(header).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*(gp3?_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("gp_setup_grid", "gp_set_levelset", "gp_cn_step", "gp_mg_vcycle", "gp_solve"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        from paper_1911_00994_amd import build
        build.build()
    lib = ctypes.CDLL(LIB)
    missing = [n for h in (HEADER, HEADER3) for n in declared_functions(h) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_1911_00994_amd import gpmg, gpmg3
    assert sorted(gpmg.EXPORTS) == declared_functions()
    assert sorted(gpmg3.EXPORTS) == declared_functions(HEADER3)


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1911_00994_amd import gpmg
    monkeypatch.setattr(gpmg, "LIBPATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(gpmg, "_lib", None)
    with pytest.raises(RuntimeError):
        gpmg.lib()
