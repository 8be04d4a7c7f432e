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


def test_pt_host_logic_matches_the_paper_examples():
    """Iterations per epoch and option checks of the ptSNE entry points are
    host arithmetic; the iteration count follows the paper's worked numbers
    (the same fixture that pins the oracle)."""
    import json
    from paper_1812_09869_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libtsne355.so not built")
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "ptsne_paper_examples.json")))
    g = gold["rounds_digits"]
    opts = _lib.pt_opts(g["threads"], g["layers"], 400.0)
    assert _lib.pt_iterations(g["n"], opts) == g["iterations"]
    assert _lib.pt_iterations(g["n"], _lib.pt_opts(120, 2, 400.0, iters=7)) == 7
    lib = _lib.load()
    ok = lib.tsne_pt_workspace_bytes(2000, 10, ctypes.byref(_lib.pt_opts(5, 2, 20.0)))
    assert ok > 5 * _lib.workspace_bytes(800, 10)  # five partial workspaces of 800 points
    for bad in (_lib.pt_opts(5, 6, 20.0),        # layers > threads
                _lib.pt_opts(0, 1, 20.0),        # no threads
                _lib.pt_opts(5, 2, 799.5),       # perplexity >= z - 1
                _lib.pt_opts(5, 2, 1.0)):        # perplexity <= 1
        assert lib.tsne_pt_workspace_bytes(2000, 10, ctypes.byref(bad)) == 0


def test_implicit_workspace_is_small():
    """An implicit-P workspace holds a bounded buffer of P tiles instead of the triangle."""
    from paper_1812_09869_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libtsne355.so not built")
    lib = _lib.load()
    full = _lib.workspace_bytes(65536, 50)
    imp = lib.tsne_workspace_bytes_implicit(65536, 50, 0)
    assert 0 < imp < full / 5
    assert lib.tsne_workspace_bytes_implicit(1, 50, 0) == 0
    # a reduced distance mode keeps its contraction operands as well
    for mode in range(1, 6):
        assert imp < lib.tsne_workspace_bytes_implicit(65536, 50, mode) < full / 5
    assert lib.tsne_workspace_bytes_implicit(65536, 50, 6) == 0
    assert lib.tsne_workspace_bytes_implicit(65536, 50, -1) == 0
