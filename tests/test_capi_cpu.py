"""C-ABI library on the CPU: it loads, exports every function include/rsoc.h
declares, and its host-only entry points behave (no GPU calls here)."""
import os
import re

import numpy as np
import pytest

import graphgen as gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "rsoc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rsoc_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    import ctypes
    import paper_1505_04086_amd as rsoc
    names = _declared()
    assert len(names) >= 15
    lib = ctypes.CDLL(rsoc.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(rsoc.EXPORTED)


def test_check_csr_host():
    import paper_1505_04086_amd as rsoc
    rp, ci = gg.tri_grid(9, 7)
    assert rsoc.rsoc_check_csr(rp, ci, flags=3) == rsoc.RSOC_OK
    bad = rp.copy(); bad[0] = 1
    assert rsoc.rsoc_check_csr(bad, ci) == rsoc.RSOC_ECSR
    bad = rp.copy(); bad[5], bad[6] = bad[6], bad[5]
    assert rsoc.rsoc_check_csr(bad, ci) == rsoc.RSOC_ECSR
    bad = ci.copy(); bad[3] = 63
    assert rsoc.rsoc_check_csr(rp, bad) == rsoc.RSOC_ECSR
    bad = ci.copy(); bad[0] = 0
    assert rsoc.rsoc_check_csr(rp, bad) == rsoc.RSOC_ESELFLOOP
    # one direction of an edge removed
    r2, c2 = gg.from_edges(4, [(0, 1), (1, 2), (2, 3)])
    c3 = c2.copy(); c3[-1] = 1  # row 3 lists 1 instead of 2
    assert rsoc.rsoc_check_csr(r2, c3, flags=1) == rsoc.RSOC_OK
    assert rsoc.rsoc_check_csr(r2, c3, flags=3) == rsoc.RSOC_EASYM
    assert rsoc.rsoc_check_csr(rp, ci, flags=8) == rsoc.RSOC_EINVAL


def test_strerror_and_options():
    import paper_1505_04086_amd as rsoc
    for code in range(0, -10, -1):
        assert rsoc.rsoc_strerror(code)
    o = rsoc.make_options("deterministic", "higher", max_rounds=3, t_thread=5)
    assert (o.mode, o.tie, o.max_rounds, o.t_thread) == (1, 1, 3, 5)


def test_product_does_not_reference_oracle():
    """The product package never imports, links or names the oracle."""
    pkg = os.path.join(ROOT, "paper_1505_04086_amd")
    for dp, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dp, f)).read()
                assert "import oracle" not in text and "from oracle" not in text and "orc_" not in text, f
