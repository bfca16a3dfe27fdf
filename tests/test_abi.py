"""Host-side checks of the C ABI: the library loads, exports what the header
declares, and its host logic (options, status strings, argument checks)
behaves, all without a GPU."""
import ctypes
import os
import re

import pytest

from paper_2601_17707_amd import bbc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bbc.h")


def _lib():
    if not os.path.exists(bbc.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    return bbc.load_library()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bbc_[a-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("bbc_create", "bbc_destroy", "bbc_count", "bbc_options_init", "bbc_last_stats",
                     "bbc_status_string", "bbc_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    for name in declared_functions():
        assert hasattr(lib, name), f"libbbc.so does not export {name}"


def test_struct_layouts_match_header():
    lib = _lib()
    o = bbc.Options()
    lib.bbc_options_init(ctypes.byref(o))
    assert o.struct_size == ctypes.sizeof(bbc.Options)
    assert o.side == bbc.SIDE_AUTO and o.checks == bbc.CHECK_ALL and o.timing == 0
    assert o.schedule == bbc.SCHED_DYNAMIC and o.no_tuning == 0 and o.n_blocks == 0
    st = bbc.Stats()
    assert ctypes.sizeof(st) > 0


def test_status_strings():
    lib = _lib()
    for s in range(10):
        txt = lib.bbc_status_string(s).decode()
        assert txt and txt != "unknown status"
    assert lib.bbc_status_string(99).decode() == "unknown status"


def test_host_argument_checks():
    lib = _lib()
    out = ctypes.c_uint64(7)
    # NULL context
    assert lib.bbc_count(None, 1, 1, 0, None, None, None, ctypes.byref(out), None, None, None) == bbc.EINVAL
    assert out.value == 7
    assert lib.bbc_destroy(None) == bbc.OK
    assert lib.bbc_create(0, None) == bbc.EINVAL
    assert lib.bbc_last_stats(None, None) == bbc.EINVAL
    assert lib.bbc_last_error(None).decode() == "no context"
    # the extension entry points reject a NULL context before touching anything
    cls = (ctypes.c_uint64 * 6)(*range(6))
    assert lib.bbc_count_classes(None, 1, 1, 0, None, None, None, cls, None, None) == bbc.EINVAL
    assert list(cls) == list(range(6))
    two = (ctypes.c_uint64 * 2)(5, 6)
    assert lib.bbc_count_bicliques(None, 1, 1, 0, None, None, None, 3, two, None, None) == bbc.EINVAL
    assert list(two) == [5, 6]
    d = ctypes.c_int64(9)
    assert lib.bbc_update_delta(None, 1, 1, 0, None, None, None, 0, None, None, None, ctypes.byref(d), None,
                                None) == bbc.EINVAL
    assert d.value == 9


def test_no_gpu_means_device_error():
    """Without a gfx950 device bbc_create reports BBC_EDEVICE (never a CPU path)."""
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = _lib()
    h = ctypes.c_void_p()
    assert lib.bbc_create(0, ctypes.byref(h)) == bbc.EDEVICE
    with pytest.raises(bbc.BbcError):
        bbc.Context(0)


def test_binding_has_no_cpu_fallback():
    src = open(os.path.join(ROOT, "paper_2601_17707_amd", "bbc.py")).read()
    assert "import oracle" not in src and "from oracle" not in src
    for f in os.listdir(os.path.join(ROOT, "paper_2601_17707_amd", "csrc")):
        assert "oracle" not in open(os.path.join(ROOT, "paper_2601_17707_amd", "csrc", f)).read()
