"""The C-ABI library builds for gfx950, loads, and exports every declared entry
point; record layouts match the header. No compute call is made (no GPU here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1308_4011_amd import mm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mm.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:mm_status|const char \*)\s*(mm_\w+)\s*\(", text, re.M)))


def test_library_exists_and_loads():
    assert os.path.exists(mm.LIB_PATH), "run __graft_entry__.build() first"
    ctypes.CDLL(mm.LIB_PATH)


def test_every_declared_symbol_is_exported():
    L = ctypes.CDLL(mm.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # and the binding knows every one of them
    assert set(names) <= set(mm._SIGS), set(names) - set(mm._SIGS)


def test_record_layouts():
    assert mm.CLASS_METRICS.itemsize == 48
    assert mm.METHOD_METRICS.itemsize == 16
    assert mm.MOVE_SCORE.itemsize == 96
    assert ctypes.sizeof(mm.SystemDesc) == 4 * 3 + 4 + 6 * 8
    assert ctypes.sizeof(mm.SystemInfo) == 48


def test_context_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(mm.MMError) as e:
        mm.context_create(0)
    assert e.value.code in (mm.MM_EHIP, mm.MM_EINVAL)
    assert mm.lib().mm_last_error()


def test_null_arguments_rejected_without_gpu():
    L = mm.lib()
    n = ctypes.c_int64()
    assert L.mm_score_moves(None, 2, None, None, 0, 3, 0, 0, None, 0, ctypes.byref(n)) == mm.MM_EINVAL
    assert L.mm_apply_move(None, 0, 0) == mm.MM_EINVAL
    assert L.mm_free_system(None) == mm.MM_EINVAL
    assert L.mm_context_destroy(None) == mm.MM_EINVAL
    assert b"NULL" in L.mm_last_error()
