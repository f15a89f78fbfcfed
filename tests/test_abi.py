"""The C-ABI library loads and exports every entry point include/vd.h declares
(host-only checks: no compute calls, no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vd.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"VD_API\s+[\w\s\*]+?\b(vd_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2605_06408_amd as vd
    if not os.path.exists(vd.LIB_PATH):
        vd.build_library()
    return vd.load_library()


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ["vd_create", "vd_destroy", "vd_build", "vd_write", "vd_backward", "vd_get_sizes", "vd_last_error",
              "vd_version"]:
        assert s in syms


def test_library_exports_every_declared_symbol(lib):
    import paper_2605_06408_amd as vd
    for s in declared_symbols():
        assert hasattr(lib, s), s
    out = subprocess.run(["nm", "-D", "--defined-only", vd.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT\s+(vd_\w+)", out))
    assert exported == set(declared_symbols())  # nothing else leaks out


def test_version_and_empty_error(lib):
    assert b"gfx950" in lib.vd_version()
    assert lib.vd_last_error() == b""


def test_null_arguments_are_rejected_on_the_host(lib):
    import paper_2605_06408_amd as vd
    sz = vd.Sizes()
    assert lib.vd_build(None, None, None, 10, None, None, None, ctypes.byref(sz)) == 1
    assert b"null" in lib.vd_last_error()
    assert lib.vd_write(None, None, None) == 1
    assert lib.vd_get_sizes(None, None) == 1
    assert lib.vd_create(0, None) == 1
    assert lib.vd_backward(None, None, None, None, None, None, None) == 1
    assert lib.vd_backward_noalloc(None, None, None, None, None, None, None) == 1
    lib.vd_destroy(None)  # no-op


def test_struct_layouts_match_header():
    import paper_2605_06408_amd as vd
    assert ctypes.sizeof(vd.Options) == 32
    # one int64 per field the header declares in vd_sizes, in the same order
    hdr = open(HEADER).read()
    body = re.search(r"typedef struct vd_sizes \{(.*?)\} vd_sizes;", hdr, re.S).group(1)
    names = re.findall(r"int64_t\s+(\w+);", body)
    assert [f[0] for f in vd.Sizes._fields_] == names
    assert ctypes.sizeof(vd.Sizes) == 8 * len(names)
    assert ctypes.sizeof(vd.Outputs) == 12 * 8
