"""The C-ABI library loads and exports every entry point include/apd.h
declares (no GPU needed: nothing here launches a kernel)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "apd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(apd_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_paper_calls():
    names = _declared()
    for n in ("apd_assign", "apd_dual_objective_grad", "apd_fit_weights", "apd_lloyd_step"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2403_03571_amd as apd
    L = apd.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(apd.EXPORTS) == _declared()


def test_choose_resolution_matches_the_rule():
    """eq. (2.10) on the host side of the library (no kernel)."""
    import paper_2403_03571_amd as apd
    assert apd.apd_choose_resolution(2, 0.01, 1e-4) == 2001
    assert apd.apd_choose_resolution(3, 0.01, 1e-4) == 201
    assert apd.apd_choose_resolution(2, 0.01, 1.0 / 25) == 101
    with pytest.raises(apd.ApdError):
        apd.apd_choose_resolution(4, 0.01, 1e-4)


def test_library_has_no_oracle_dependency():
    """The product library links neither the oracle nor any CPU fallback."""
    import paper_2403_03571_amd as apd
    data = open(apd.LIB_PATH, "rb").read()
    assert b"orc_" not in data
    assert b"liboracle" not in data
    src = open(os.path.join(ROOT, "paper_2403_03571_amd", "__init__.py")).read()
    assert "import oracle" not in src and "from oracle" not in src


def test_null_context_is_rejected():
    import paper_2403_03571_amd as apd
    L = apd.lib()
    p = apd.apd_problem()
    assert L.apd_assign(None, ctypes.byref(p), None, None, 0) == 1
    assert L.apd_last_error(None) == b"no context"
