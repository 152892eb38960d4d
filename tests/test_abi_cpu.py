"""CPU checks of the shared library: it loads and exports every entry point
that include/rid.h declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rid.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rid_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2310_09417_amd import binding
    lib = binding.library()
    names = _declared()
    assert {"rid_lupp_fixed_rank", "rid_lupp_adaptive", "rid_workspace_bytes"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings():
    from paper_2310_09417_amd import binding
    assert binding.rid_status_string(0) == "RID_OK"
    assert binding.rid_status_string(-4) == "RID_ERR_WORKSPACE"
    assert binding.rid_status_string(99) == "RID_UNKNOWN"


def test_flop_model():
    from paper_2310_09417_amd import flops_id
    # sketch 2*l*m*n dominates; hand count for a tiny case
    # m=2,n=3,k=1,l=2: 2*2*2*3=24, LU t=0: 2*(3-1)*(2-1)=4, solve 1*1*2=2
    assert flops_id(2, 3, 1, 2) == 30.0
