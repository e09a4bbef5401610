"""Host-side checks of the C-ABI library: it loads and exports every entry
point that include/hd.h declares, and the binding covers the same names.
No compute calls (this runs without a GPU)."""
import ctypes
import os
import re

from tests.conftest import ROOT


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hd_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_0909_5215_amd import hd
    lib = ctypes.CDLL(hd.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 25
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_the_header():
    from paper_0909_5215_amd import hd
    assert sorted(hd.exported_symbols()) == declared_functions()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_0909_5215_amd import hd
    monkeypatch.setattr(hd, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(hd, "_lib", None)
    import pytest
    with pytest.raises(RuntimeError):
        hd.load()


def test_struct_sizes_match_header_layout():
    from paper_0909_5215_amd import hd
    # hd_system_desc: 2 ints, 3 doubles, 3 ints (+pad), 3 pointers, 1 double
    assert ctypes.sizeof(hd.hd_system_desc) == 8 + 24 + 16 + 24 + 8
    assert ctypes.sizeof(hd.hd_lj_params) == 8 * 10
    # hd_scalars: 11 doubles, step, flags + n_rebuilds, kappa, dv1, dv2, e_nhc, lambda
    assert ctypes.sizeof(hd.hd_scalars) == 8 * 11 + 8 + 8 + 8 * 5
