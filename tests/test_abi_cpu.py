"""The C-ABI library loads on a machine without a GPU and exports every entry
point that include/pcdn.h declares (no compute call is made here)."""
import ctypes
import os
import re

import paper_1306_4080_amd as pc
from paper_1306_4080_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pcdn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|int)\s+(pcdn_\w+)\s*\(", src, re.M)))


def test_header_declares_the_abi():
    names = _declared()
    for must in ("pcdn_create", "pcdn_load_csc", "pcdn_solve", "pcdn_step", "pcdn_destroy"):
        assert must in names
    assert sorted(binding.SYMBOLS) == names


def test_library_loads_and_exports_every_declared_symbol():
    pc.ensure_built()
    lib = ctypes.CDLL(pc.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_create_without_device_fails_cleanly():
    """With no GPU the library reports an error instead of crashing; on a GPU
    machine this is skipped."""
    import torch
    if torch.cuda.is_available():
        import pytest
        pytest.skip("a GPU is present")
    lib = binding.load_library()
    h = ctypes.c_void_p()
    rc = lib.pcdn_create(ctypes.byref(h), 0, None)
    assert rc == -4 and not h.value
    assert lib.pcdn_last_error(None)
    # destroy accepts NULL
    assert lib.pcdn_destroy(None) == 0
