"""The C-ABI library loads and exports every function include/ccmg.h declares
(no GPU needed: nothing here launches work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1306_6883_amd", "libccmg.so")


def declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(ccmg_\w+)\s*\(", txt))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared()
    for must in ("ccmg_solve", "ccmg_plan_create", "ccmg_workspace_bytes", "ccmg_vcycle",
                 "ccmg_smooth", "ccmg_residual", "ccmg_restrict_residual", "ccmg_prolong_add",
                 "ccmg_fill_ghosts"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB, mode=os.RTLD_NOW)  # resolve every symbol now: a missing one fails here
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_validation_without_gpu():
    """Problem checks and workspace sizing are host-only and run without a GPU."""
    import paper_1306_6883_amd as cc
    assert cc.ccmg_problem_check(cc.Problem(n=64)) == cc.OK
    assert cc.ccmg_problem_check(cc.Problem(n=48)) == cc.ESIZE
    assert cc.ccmg_problem_check(cc.Problem(n=1)) == cc.ESIZE
    assert cc.ccmg_problem_check(cc.Problem(n=64, bc=("P", "D", "D", "D"))) == cc.EBC
    assert cc.ccmg_problem_check(cc.Problem(n=64, bc=(0, 0, 0, 7))) == cc.EBC
    assert cc.ccmg_problem_check(cc.Problem(n=64, ymax=2.0)) == cc.EINVAL
    assert cc.ccmg_problem_check(cc.Problem(n=64, alpha=0.0, beta=0.0)) == cc.EINVAL
    assert cc.ccmg_problem_check(cc.Problem(n=64, max_cycles=cc.HISTORY)) == cc.EINVAL
    assert cc.ccmg_problem_check(cc.Problem(n=64, rtol=float("nan"))) == cc.EINVAL
    assert cc.ccmg_workspace_bytes(cc.Problem(n=48)) == 0
    w1 = cc.ccmg_workspace_bytes(cc.Problem(n=1024))
    w2 = cc.ccmg_workspace_bytes(cc.Problem(n=2048))
    assert 0 < w1 < w2
    # the finest level needs one extra phi buffer of (n+2) rows: the rest is smaller
    assert w2 >= 8 * 2050 * 2050
    for s in (cc.OK, cc.NOT_CONVERGED, cc.EINVAL, cc.ESIZE, cc.EBC, cc.EINCOMPAT, cc.ENONFINITE,
              cc.EHIP, cc.EWORKSPACE):
        assert cc.ccmg_status_str(s) != "unknown status"
