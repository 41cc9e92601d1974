"""C-ABI contract checks that need no GPU: the library loads, exports every
entry point declared in include/r3m.h, its size queries follow the documented
layouts, and context creation without a visible GPU returns R3M_ERR_HIP."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "r3m.h")
LIB = os.path.join(ROOT, "paper_2112_05082_amd", "libr3m.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(r3m_[a-z0-9_]+)\s*\(", text)))


def lib_or_skip():
    if not os.path.exists(LIB):
        pytest.skip("libr3m.so not built (run __graft_entry__.build())")
    from paper_2112_05082_amd import r3m
    return r3m.load()


def test_every_declared_symbol_exported():
    lib = lib_or_skip()
    names = declared()
    assert len(names) >= 16
    for name in names:
        assert hasattr(lib, name), name
    from paper_2112_05082_amd import r3m
    assert set(r3m.EXPORTED) == set(names)


def test_version_and_size_queries():
    lib = lib_or_skip()
    from paper_2112_05082_amd import r3m
    assert b"gfx950" in lib.r3m_version()
    assert r3m.blocks_bytes(80, 5, 5, r3m.C128) == 121 * 80 * 80 * 16
    assert r3m.blocks_bytes(160, 2, 2, r3m.C64) == 25 * 160 * 160 * 8
    assert r3m.far_count(31, 31, 2) == 3969 - 25
    assert r3m.far_count(127, 127, 2) == 65025 - 25
    assert r3m.far_count(5, 5, 5) == 0
    head = ((3944 * 4 + 255) // 256) * 256
    assert r3m.far_bytes(160, 3944, 12, r3m.C64) == head + 3944 * 2 * 12 * 160 * 8
    assert r3m.blocks_bytes(0, 1, 1, r3m.C128) == 0
    # spectra: n^2 grids of next_pow2(2D + 1) per axis
    assert r3m.spectral_bytes(160, 31, 31, r3m.SPEC_C64) == 160 * 160 * 64 * 64 * 8
    assert r3m.spectral_bytes(80, 3, 2, r3m.SPEC_C128) == 80 * 80 * 8 * 8 * 16
    assert r3m.spectral_bytes(80, 0, 4, r3m.SPEC_C64) == 80 * 80 * 2 * 16 * 8
    assert r3m.spectral_bytes(80, 3, 3, r3m.C64) == 0
    assert r3m.static_scratch_bytes() == 64 << 20


def test_ctx_create_without_gpu_reports_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    lib = lib_or_skip()
    from paper_2112_05082_amd import r3m
    h = C.c_void_p()
    rc = lib.r3m_ctx_create(C.byref(h), 0)
    assert rc == r3m.R3M_ERR_HIP
    assert lib.r3m_last_error(None)
    with pytest.raises(r3m.R3MError):
        r3m.Context(0)


def test_null_ctx_is_invalid_arg():
    lib = lib_or_skip()
    from paper_2112_05082_amd import r3m
    rc = lib.r3m_fill_unique_blocks(None, None, 1, 1, r3m.C128, None, 0, None)
    assert rc == r3m.R3M_ERR_INVALID_ARG
