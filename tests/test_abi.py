"""The C-ABI library loads and exports every symbol include/cpm.h declares
(no compute call: this runs without a GPU)."""

import ctypes
import os
import re

import pytest

from paper_2305_04711_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "cpm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cpm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("cpm_build_band", "cpm_apply", "cpm_solve", "cpm_solve_adjoint"):
        assert required in names
    assert set(names) == set(capi.EXPORTED)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(capi.LIB_PATH):
        pytest.fail("libcpm.so is not built; run python -m paper_2305_04711_amd.build")
    lib = ctypes.CDLL(capi.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    capi.load()


def test_struct_layouts_match_header_sizes():
    # the Python mirrors of the C structs: field order and padding
    assert ctypes.sizeof(capi.Surface) == 4 + 4 + 3 * 8 + 8 + 8
    assert ctypes.sizeof(capi.IBC) == 8 + 3 * 8 + 3 * 8 + 8 + 2 * 8 + 2 * 4 + 4 * 8
    assert ctypes.sizeof(capi.Grid) == 4 * 4 + 3 * 8 + 4 + 4
    assert ctypes.sizeof(capi.SolveOpts) == 3 * 8 + 2 * 4 + 8 + 2 * 4 + 8 + 8
    assert ctypes.sizeof(capi.SolveStats) == 5 * 4 + 4 + 2 * 8
    assert ctypes.sizeof(capi.Allocator) == 3 * 8
    assert ctypes.sizeof(capi.BandInfo) == 4 * 4 + 9 * 8 + 3 * 8 + 2 * 8


def test_device_memory_only_through_the_allocator():
    # hipMalloc / hipFree appear only in the default provider of cpm::DevAlloc;
    # every other device allocation goes through a band's or batch's allocator
    csrc = os.path.join(ROOT, "paper_2305_04711_amd", "csrc")
    hits = []
    for f in sorted(os.listdir(csrc)):
        text = open(os.path.join(csrc, f)).read()
        for m in re.finditer(r"\bhip(Malloc|Free|MallocAsync|FreeAsync|MallocManaged)\s*\(", text):
            line = text[:m.start()].count("\n") + 1
            hits.append((f, line))
    assert [f for f, _ in hits] == ["common.hip", "common.hip"], hits
    text = open(os.path.join(csrc, "common.hip")).read()
    body = text[text.index("void* DevAlloc::get("):text.index("void* Workspace::get(")]
    assert body.count("hipMalloc(") == 1 and body.count("hipFree(") == 1


def test_errors_without_gpu_are_reported_not_raised():
    lib = capi.load()
    out = ctypes.c_void_p()
    # a null surface is rejected before any device work
    st = lib.cpm_build_band(None, None, 0, None, None, None, ctypes.byref(out))
    assert st == capi.E_INVALID
    assert b"null" in lib.cpm_last_error()
