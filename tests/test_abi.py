"""The C-ABI library loads and exports every entry point include/hk.h declares
(no compute calls: runs without a GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "hk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hk_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_0902_0852_amd as pkg
    L = pkg.lib()
    decl = declared_symbols()
    assert len(decl) >= 14
    missing = [s for s in decl if not hasattr(L, s)]
    assert missing == []
    assert sorted(pkg.EXPORTS) == decl


def test_workspace_planning_is_consistent():
    import paper_0902_0852_amd as pkg
    a = pkg.workspace_bytes(32, (1, 1), 512)
    b = pkg.workspace_bytes(200, (7, 4), 2048)
    c = pkg.workspace_bytes(500, (1, 2), 6144)
    assert 0 < a < b < c
    assert pkg.workspace_bytes(32, (1, 1), 511) == 0      # K odd
    assert pkg.workspace_bytes(0, (1, 1), 512) == 0
    assert pkg.workspace_bytes(32, (0, 1), 512) == 0
