"""The C-ABI library loads and exports every entry point its header declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]


def _declared():
    names = set()
    for h in HEADERS:
        src = open(h).read()
        names.update(re.findall(r"TSNE_API\s+[\w\s\*]*?\b(tsne_\w+)\s*\(", src))
    return sorted(names)


def test_header_declares_entry_points():
    names = _declared()
    for required in ("tsne_affinities", "tsne_step", "tsne_cost", "tsne_workspace_bytes"):
        assert required in names


def test_library_exports_all_declared_symbols():
    from paper_1812_09869_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libtsne355.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_lib.EXPORTED) >= set(_declared())


def test_workspace_bytes_host_only():
    """Size query is pure host arithmetic: no device needed."""
    from paper_1812_09869_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libtsne355.so not built")
    n2 = _lib.workspace_bytes(2000, 10)
    n65 = _lib.workspace_bytes(65536, 50)
    assert n2 > 8 * 36 * 256 * 256 // 8  # holds 36 tiles of FP32 P
    assert n65 > 32896 * 256 * 256 * 4
    assert _lib.workspace_bytes(1, 10) == 0
    assert _lib.workspace_bytes(100, 0) == 0
