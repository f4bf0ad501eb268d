"""The C-ABI library loads and exports every symbol include/skim.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "skim.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(skim_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = _declared()
    for want in ("skim_build_sketches", "skim_query_batch", "skim_greedy"):
        assert want in names


def test_library_exports_every_declared_symbol():
    import paper_1408_6282_amd as sk
    if not os.path.exists(sk.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(sk.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(_declared()) == sorted(sk.EXPORTS)
    lib.skim_abi_version.restype = ctypes.c_uint32
    import re
    with open(os.path.join(ROOT, "include", "skim.h")) as f:
        want = int(re.search(r"#define SKIM_ABI_VERSION (\d+)u", f.read()).group(1))
    assert lib.skim_abi_version() == want


def test_binding_fails_loudly_without_library(tmp_path):
    import paper_1408_6282_amd as sk
    saved = sk._lib
    try:
        sk._lib = None
        with pytest.raises(RuntimeError, match="not built"):
            sk.load_library(str(tmp_path / "missing.so"))
    finally:
        sk._lib = saved


def _header_structs():
    """typedef struct { ... } name; blocks of the header: name -> [(field, C type)]."""
    text = open(os.path.join(ROOT, "include", "skim.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct\s*\{(.*?)\}\s*(\w+)\s*;", text, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            m = re.match(r"(?:const\s+)?(\w+)\s*(\*?)\s*(\w+)$", decl)
            assert m, decl
            fields.append((m.group(3), "pointer" if m.group(2) else m.group(1)))
        out[name] = fields
    return out


def test_binding_structs_mirror_the_header():
    """The ctypes structures the binding passes across the ABI have the
    header's fields in the header's order, with matching widths."""
    import ctypes as C
    import paper_1408_6282_amd as sk
    structs = _header_structs()
    assert {"skim_graph", "skim_build_params", "skim_server_config"} <= set(structs)
    for name, fields in structs.items():
        cls = getattr(sk, name)
        assert [f for f, _ in cls._fields_] == [f for f, _ in fields], name
        for (fname, ctype), (_, py) in zip(fields, cls._fields_):
            if ctype == "pointer":
                assert C.sizeof(py) == C.sizeof(C.c_void_p), (name, fname)
            else:
                assert C.sizeof(py) == {"uint32_t": 4, "uint64_t": 8}[ctype], (name, fname)
