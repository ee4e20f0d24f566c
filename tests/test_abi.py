"""The C-ABI library loads and exports every symbol include/ditr.h declares
(no compute call: runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1202_6168_amd import ditr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "ditr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ditr_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for must in ["ditr_create", "ditr_destroy", "ditr_graph_create", "ditr_solve",
                 "ditr_residual", "ditr_partition", "ditr_abort", "ditr_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(ditr.LIB_PATH)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(declared_symbols()) <= set(ditr._SIGNATURES)


def test_version_and_defaults():
    assert ditr.version() == 1
    o = ditr.opts_default()
    assert o.alpha == 2.0 and o.refresh_at == 0 and o.part_type == ditr.PART_MINCUT
    with pytest.raises(KeyError):
        ditr.opts_default(no_such_field=1)


def test_null_arguments_are_errors_not_crashes():
    L = ditr.lib()
    assert L.ditr_opts_default(None) == ditr.EINVAL
    assert "NULL" in ditr.last_error()
    assert L.ditr_create(None, 0, None) == ditr.EINVAL
    assert L.ditr_abort(None) == ditr.EINVAL
    assert L.ditr_destroy(None) == ditr.OK
    assert L.ditr_graph_destroy(None) == ditr.OK
