"""CPU checks of the C ABI: libgs3.so loads and exports every call that
include/gs3.h declares; the Python binding covers the same set.  No compute
calls (there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "gs3.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gs3_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_calls():
    names = declared()
    for must in ("gs3_create", "gs3_render", "gs3_render_backward", "gs3_ntc_forward", "gs3_ntc_backward",
                 "gs3_ntc_step", "gs3_loss", "gs3_warmup_loss", "gs3_adam"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2403_01444_amd import gs3
    if not os.path.exists(gs3.LIB_PATH):
        from paper_2403_01444_amd import build
        build.build()
    lib = ctypes.CDLL(gs3.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2403_01444_amd import gs3
    assert sorted(gs3.EXPORTED) == declared()
    for n in declared():
        assert callable(getattr(gs3, n)), n


def test_struct_layouts_match_header_sizes():
    from paper_2403_01444_amd import gs3
    # int32 x5 + int32[16] + float[6] = 27 words; config adds 2 int64 + 6 int32
    assert ctypes.sizeof(gs3.NtcConfigC) == 4 * 27
    assert ctypes.sizeof(gs3.ConfigC) == 16 + 24 + 4 * 27 + 4   # padded to 8
    assert ctypes.sizeof(gs3.CameraC) == 4 * (7 + 12 + 3 + 3)
    assert ctypes.sizeof(gs3.GradsC) == 8 * 13


def test_context_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2403_01444_amd import gs3
    with pytest.raises(RuntimeError):
        gs3.Context(10, 100, 16, 16)
