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
