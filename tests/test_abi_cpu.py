"""Host-side checks of the C-ABI library (no GPU needed, no compute calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2103_08053_amd import tc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "trust_tc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\*?\s+\**(tc_[a-z_]+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = tc.load_library()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(tc.EXPORTS) == names


def test_static_scratch_size_matches_header():
    text = open(HEADER).read()
    m = re.search(r"#define TC_STATIC_SCRATCH_BYTES \((\d+)ull << (\d+)\)", text)
    assert m, "TC_STATIC_SCRATCH_BYTES not found"
    assert tc.TC_STATIC_SCRATCH_BYTES == int(m.group(1)) << int(m.group(2))


def _header_fields(struct):
    """(type, name) of every field of `typedef struct <struct> { ... }` in the public header."""
    text = open(HEADER).read()
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (struct, struct), text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    return re.findall(r"(uint32_t|uint64_t)\s+(\w+);", body)


def test_struct_layouts_match_header():
    for struct, cls in (("tc_params", tc._Params), ("tc_graph_info", tc._GraphInfo)):
        fields = _header_fields(struct)
        want = [(name, ctypes.c_uint64 if t == "uint64_t" else ctypes.c_uint32) for t, name in fields]
        assert [(n, c) for n, c in cls._fields_] == want, struct
        assert ctypes.sizeof(cls) == sum(8 if t == "uint64_t" else 4 for t, _ in fields)


def test_default_params():
    lib = tc.load_library()
    p = tc._Params()
    assert lib.tc_default_params(ctypes.byref(p)) == tc.TC_OK
    assert p.struct_size == ctypes.sizeof(tc._Params)
    d = tc.Params.from_c(p)
    assert d == tc.Params()  # the binding's defaults mirror the library's
    assert lib.tc_default_params(None) == tc.TC_E_INVALID


def test_status_strings():
    lib = tc.load_library()
    for s in range(7):
        assert lib.tc_status_str(s)
    assert lib.tc_status_str(99) == b"unknown status"
    assert lib.tc_last_error(None) == b""


@pytest.mark.parametrize("field,value", [
    ("struct_size", 3), ("wg_waves", 0), ("wg_waves", 17), ("wg_lds_bytes", 1024),
    ("wg_lds_bytes", 4100), ("slots_per_bucket", 3), ("load_factor_pct", 5), ("load_factor_pct", 101),
    ("hash_kind", 2), ("light_chunk", 0), ("light_chunk", 300), ("flags", 0x8000), ("flags", 0xC0), ("flags", 0x300),
])
def test_create_rejects_bad_params_before_touching_a_device(field, value):
    lib = tc.load_library()
    p = tc._Params()
    lib.tc_default_params(ctypes.byref(p))
    setattr(p, field, value)
    h = ctypes.c_void_p()
    assert lib.tc_create(0, ctypes.byref(p), ctypes.byref(h)) == tc.TC_E_INVALID
    assert not h.value


def test_null_arguments_are_invalid():
    lib = tc.load_library()
    b = ctypes.c_uint64()
    assert lib.tc_workspace_bytes(None, 10, 10, ctypes.byref(b)) == tc.TC_E_INVALID
    assert lib.tc_create(0, None, None) == tc.TC_E_INVALID
    assert lib.tc_count(None, 1, 1, None, None, None, None, 0, None, None) == tc.TC_E_INVALID
    assert lib.tc_graph_count(None, None, None, None, None, 0, None) == tc.TC_E_INVALID
    assert lib.tc_graph_info_get(None, None, None) == tc.TC_E_INVALID
    assert lib.tc_destroy(None) == tc.TC_OK
    assert lib.tc_graph_release(None) == tc.TC_OK


def test_no_device_is_reported(monkeypatch):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    lib = tc.load_library()
    h = ctypes.c_void_p()
    assert lib.tc_create(0, None, ctypes.byref(h)) == tc.TC_E_DEVICE
    with pytest.raises(tc.TCError):
        tc.Context(0)


def read_fixture(name):
    """key -> list of ints from a tests/golden text fixture (comment lines start with '#')."""
    out = {}
    for line in open(os.path.join(ROOT, "tests", "golden", name)):
        line = line.strip()
        if line and not line.startswith("#"):
            key, *vals = line.split()
            out[key] = [int(v) for v in vals]
    return out


def test_virtual_combination_worked_example():
    """The worked example of Section 4.2, through the index-map code the count kernels run
    (tc_vc_locate evaluates the same template on the host): neighbours {2,3,4,5,7} with 2-hop list
    lengths {7,3,2,6,5}; flattened index 11 is the second entry (offset 1) of neighbour 4's list."""
    fx = read_fixture("paper_vc_example.txt")
    nbrs, lens = fx["neighbours"], fx["degrees"]
    incl = list(np.cumsum(lens))
    assert incl == fx["inclusive_prefix"]
    k, off = tc.vc_locate(incl, fx["query_index"][0])
    assert nbrs[k] == fx["owner"][0] and off == fx["local_offset"][0]


def test_virtual_combination_map_is_the_concatenation():
    """Every flattened index maps to the list and position it has in the concatenation of the
    lists, empty lists included (they own no index); indices past the end are rejected."""
    for lens in ([7, 3, 2, 6, 5], [1], [0, 0, 4, 0, 1, 0], [5, 0, 0], [64] * 9, [3, 65, 1, 128]):
        incl = list(np.cumsum(lens))
        flat = [(k, j) for k, ln in enumerate(lens) for j in range(ln)]
        assert [tc.vc_locate(incl, i) for i in range(len(flat))] == flat
        with pytest.raises(tc.TCError):
            tc.vc_locate(incl, incl[-1])
    with pytest.raises(tc.TCError):
        tc.vc_locate([], 0)


def test_list_addressing_threshold():
    """32-bit byte cursors while 4 m_in + 256 < 2^32 (a lane may step 256 bytes past its last list);
    64-bit addressing from m_in = 2^30 - 64 on, or when forced."""
    edge = (1 << 30) - 64
    assert not tc.wide_list_addressing(edge - 1)
    assert tc.wide_list_addressing(edge)
    assert tc.wide_list_addressing(1 << 30)
    assert not tc.wide_list_addressing(0) and not tc.wide_list_addressing(67108864)
    assert tc.wide_list_addressing(100, flags=tc.TC_F_WIDE_ADDR)
    for m in (edge - 1, edge):  # the rule itself: the largest byte offset a cursor reaches fits in 32 bits
        assert (4 * m + 256 < 2**32) == (not tc.wide_list_addressing(m))
