"""CPU-side checks of the C ABI: the library loads and exports every function
include/gheap.h declares; host-only calls (no device work) behave as
documented; the Python binding mirrors the header's struct layouts."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gheap.h")
LIB = os.path.join(ROOT, "paper_1906_06504_amd", "libgheap.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*\*?\s*\b(heap_[a-z_]+)\s*\(",
                      text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1906_06504_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), "missing export " + n


def test_binding_lists_every_export():
    from paper_1906_06504_amd import gheap
    assert sorted(gheap.EXPORTS) == declared_functions()


def test_host_only_calls(lib):
    lib.heap_arena_bytes.restype = ctypes.c_uint64
    lib.heap_arena_bytes.argtypes = [ctypes.c_uint32, ctypes.c_int, ctypes.c_uint32,
                                     ctypes.c_void_p, ctypes.c_uint64]
    f = lambda *a: lib.heap_arena_bytes(a[0], 0, *a[1:])     # 8-byte entries  # noqa: E731
    assert f(1000, 1, None, 100) == 0          # unsupported k
    a = f(1024, 1, None, 1 << 22)
    b = f(1024, 1, None, 1 << 23)
    assert a > (1 << 22) * 8 and b > a
    assert f(1024, 0, None, 1024) == 0
    assert f(64, 1 << 20, None, 64) > 0
    assert f(64, (1 << 20) + 1, None, 64) == 0     # heaps per set
    assert f(64, 0xFFFFFFFF, None, 1 << 40) == 0
    assert f(32, 1, None, ((1 << 30) - 2) * 32) == 0   # 2^30 - 1 nodes
    assert f(32, 1, None, ((1 << 30) - 3) * 32) > (1 << 37)
    # 16-byte entries: nodes and partial buffer take twice the bytes
    w = lib.heap_arena_bytes(1024, 1, 1, None, 1 << 22)
    assert w > (1 << 22) * 16 and w - (1 << 22) * 16 < a - (1 << 22) * 8 + (1 << 16)
    assert lib.heap_arena_bytes(1024, 2, 1, None, 1 << 22) == 0    # unknown key type
    assert lib.heap_arena_bytes(1024, -1, 1, None, 1 << 22) == 0
    f = lib.heap_serve_workspace_bytes
    f.restype = ctypes.c_uint64
    f.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64]
    assert f(256, 1000, 4000) > 4000 * 32
    assert f(256, 1000, 0) == 0 and f(0, 1000, 4000) == 0
    assert f(256, 1000, 1 << 24) == 0 and f(256, 1000, (1 << 24) - 1) > 0
    assert f(256, 1000, (1 << 64) - 1) == 0
    lib.heap_supported_shape.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    assert lib.heap_supported_shape(1024, 256) == 1
    assert lib.heap_supported_shape(1024, 64) == 0
    assert lib.heap_supported_shape(32, 64) == 1
    assert lib.heap_supported_shape(48, 64) == 0
    lib.heap_strerror.restype = ctypes.c_char_p
    assert b"capacity" in lib.heap_strerror(-2)
    for fn in ("heap_insert", "heap_sync", "heap_destroy"):
        f = getattr(lib, fn)
        f.restype = ctypes.c_int
    lib.heap_insert.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64]
    assert lib.heap_insert(None, None, 5) == -1
    lib.heap_destroy.argtypes = [ctypes.c_void_p]
    assert lib.heap_destroy(None) == -1


def test_binding_checks_tensors_before_the_library():
    """The library takes counts and trusts the buffers; the binding refuses a
    tensor of the wrong dtype or too few bytes before any call."""
    import torch
    from paper_1906_06504_amd import gheap
    assert gheap._ptr(None) is None
    with pytest.raises(TypeError):
        gheap._ptr(torch.zeros(4, dtype=torch.int32), gheap._U64, what="keys")
    with pytest.raises(ValueError, match="at least 32"):
        gheap._ptr(torch.zeros(3, dtype=torch.int64), gheap._U64, 32, "out")
    with pytest.raises(ValueError, match="device tensor"):
        gheap._ptr(torch.zeros(4, dtype=torch.int64), gheap._U64, 32, "out")


def _header_structs():
    """{struct name: [(field, C type)]} of every typedef struct in the header."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct \w+ \{(.*?)\} (\w+);", text, flags=re.S):
        fields = []
        for line in body.split(";"):
            line = line.strip()
            if line:
                typ, field = line.rsplit(None, 1)
                fields.append((field.lstrip("*"), typ))
        out[name] = fields
    return out


_CTYPE = {"uint64_t": "<u8", "uint32_t": "<u4", "uint16_t": "<u2", "uint8_t": "|u1"}


def test_struct_layouts_match_header():
    """Every struct the binding mirrors has the header's fields, in order,
    with the same widths."""
    from paper_1906_06504_amd import gheap
    structs = _header_structs()
    pairs = {"gh_op": gheap.OP_DTYPE, "gh_logrec": gheap.LOG_DTYPE, "gh_reqrec": gheap.REQ_DTYPE,
             "gh_knapres": gheap.KNAP_DTYPE, "gh_ssspstats": gheap.SSSP_DTYPE,
             "gh_ssspop": gheap.SSSPOP_DTYPE}
    for name, dt in pairs.items():
        fields = structs[name]
        assert list(dt.names) == [f for f, _ in fields], name
        for f, typ in fields:
            assert dt.fields[f][0].str.replace("=", "<") in (_CTYPE[typ], _CTYPE[typ].replace("|", "<")), (name, f)


def test_oplist_seq_ranks():
    from paper_1906_06504_amd import workloads as W
    ops = W.OpList(np.zeros(6, np.uint8), np.ones(6, np.uint32), np.zeros(6, np.uint64),
                   np.zeros(6, np.uint64), 0, heap=np.array([2, 0, 2, 1, 0, 2], np.uint32))
    assert list(ops.seq()) == [0, 0, 1, 0, 1, 2]
