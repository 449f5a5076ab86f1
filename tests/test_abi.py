"""The C-ABI library loads and exports every symbol include/phasorpic.h
declares (no GPU needed); configuration errors are caught on the host."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "phasorpic.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:pic_status|void|const char \*)\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_header_symbols():
    import paper_2609_15043_amd.phasorpic as pp
    L = pp.lib()
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    assert sorted(pp.SYMBOLS) == names


def test_workspace_query_and_config_validation():
    import paper_2609_15043_amd.phasorpic as pp
    from paper_2609_15043_amd import workloads as W
    wl = W.small()
    for prec in ("fp64", "mixed"):
        cfg, keep = pp.config_from_workload(wl, precision=prec)
        n = pp.pic_workspace_bytes(cfg)
        assert n > 0
    cfg64, _ = pp.config_from_workload(wl, precision="fp64")
    cfg32, _ = pp.config_from_workload(wl, precision="mixed")
    assert pp.pic_workspace_bytes(cfg64) > pp.pic_workspace_bytes(cfg32)
    bad, keep = pp.config_from_workload(wl)
    bad.ip = 0
    with pytest.raises(pp.PicError):
        pp.pic_workspace_bytes(bad)
    bad, keep = pp.config_from_workload(wl)
    bad.sort_every = 0
    with pytest.raises(pp.PicError):
        pp.pic_workspace_bytes(bad)
