"""The C-ABI library builds, loads and exports every symbol its header declares.

CPU only: no compute call is made (there is no GPU here).
"""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nb6.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nb6_[a-z0-9_]+)\s*\(", text)))


def _lib():
    from paper_1205_1222_amd import nb6
    if not os.path.exists(nb6.LIB_PATH):
        from paper_1205_1222_amd import build
        build.build()
    return nb6


def test_header_declares_the_hot_path():
    names = declared_functions()
    for n in ("nb6_load_particles", "nb6_predict_j", "nb6_regular_force",
              "nb6_create", "nb6_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    nb6 = _lib()
    lib = nb6.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    nb6 = _lib()
    assert set(declared_functions()) <= set(nb6.EXPORTED)
    for n in nb6.EXPORTED:
        assert n in declared_functions()


def test_binding_rejects_wrong_dtype_without_calling():
    import numpy as np
    nb6 = _lib()
    with pytest.raises(TypeError):
        nb6._ptr(np.zeros(3, np.float32), np.float64)
    with pytest.raises(ValueError):
        nb6._ptr(np.zeros((3, 3))[:, 0], np.float64)


def test_shared_object_is_gfx950():
    nb6 = _lib()
    data = open(nb6.LIB_PATH, "rb").read()
    assert b"gfx950" in data
