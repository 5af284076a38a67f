"""The C-ABI library loads without a GPU and exports every function include/mxn.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "mxn.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nb_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for core in ("nb_grid_sort", "nb_pairlist_build", "nb_forces", "nb_buffer_estimate"):
        assert core in names


def test_library_exports_every_declared_symbol():
    import paper_1306_1737_amd as mxn
    if not os.path.exists(mxn.LIB_PATH):
        pytest.fail("libmxn.so is not built (run python -m paper_1306_1737_amd.build)")
    lib = ctypes.CDLL(mxn.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps exactly the declared C names
    assert sorted(mxn.EXPORTS) == sorted(n for n in declared_functions() if n in mxn.EXPORTS)
    assert set(declared_functions()) <= set(mxn.EXPORTS)


def test_binding_refuses_to_run_without_library(tmp_path, monkeypatch):
    import paper_1306_1737_amd as mxn
    monkeypatch.setattr(mxn, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(mxn, "_lib", None)
    with pytest.raises(ImportError):
        mxn.lib()
