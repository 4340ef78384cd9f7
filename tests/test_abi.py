"""The C ABI library loads and exports every symbol that include/bs.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2506_10526_amd import bs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "bs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bs_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_binding_names():
    decl = declared_symbols()
    assert set(decl) == set(bs.EXPORTED)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(bs.LIBPATH):
        pytest.skip("libbs.so not built")
    lib = ctypes.CDLL(bs.LIBPATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_no_gpu_calls_fail_cleanly():
    """bs_create on a machine without a GPU returns an error code instead of crashing."""
    if not os.path.exists(bs.LIBPATH):
        pytest.skip("libbs.so not built")
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(bs.BsError):
        bs.bs_create(0)
