"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
entry point the header declares, and rejects invalid arguments before touching
the device."""
import ctypes
import os
import re

import pytest

from paper_2203_12126_amd import ibdl

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "ibdl.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ibdl_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = ibdl.lib()
    names = _declared()
    assert "ibdl_apply" in names and "ibdl_solve" in names and "ibdl_plan_create" in names
    for n in names:
        assert hasattr(L, n), n


@pytest.mark.parametrize("field,value,msg", [
    ("dim", 4, "dim"), ("n", 1000, "n must be"), ("n", 4, "n must be"), ("length", -1.0, "length"),
    ("alpha", -2.0, "alpha"), ("bc", 7, "bc"), ("delta", 9, "delta"), ("prec", 3, "precision"),
    ("npts", 0, "npts"),
])
def test_plan_create_rejects_bad_desc(field, value, msg):
    d = ibdl.make_desc(2, 64, (0, 0), 1.0, 1.0, 0, 0, 0, 16)
    d.X = d.normal = d.weight = 8
    setattr(d, field, value)
    h = ctypes.c_void_p()
    st = ibdl.lib().ibdl_plan_create(ctypes.byref(d), None, ctypes.byref(h))
    assert st == ibdl.ERR_ARG and msg in ibdl.last_error()
    assert h.value is None


def test_plan_create_rejects_null_pointers_and_3d_size():
    d = ibdl.make_desc(2, 64, (0, 0), 1.0, 1.0, 0, 0, 0, 16)
    h = ctypes.c_void_p()
    assert ibdl.lib().ibdl_plan_create(ctypes.byref(d), None, ctypes.byref(h)) == ibdl.ERR_ARG
    d = ibdl.make_desc(3, 1024, (0, 0, 0), 1.0, 1.0, 0, 0, 0, 16)
    d.X = d.normal = d.weight = 8
    assert ibdl.lib().ibdl_plan_create(ctypes.byref(d), None, ctypes.byref(h)) == ibdl.ERR_ARG


def test_null_plan_calls_fail_cleanly():
    L = ibdl.lib()
    assert L.ibdl_apply(None, 1, None, None, None) == ibdl.ERR_ARG
    assert L.ibdl_plan_destroy(None) == ibdl.ERR_ARG
    assert "plan" in ibdl.last_error()


def test_footprint_grows_with_size():
    a = ibdl.footprint(2, 256, 1000)
    b = ibdl.footprint(2, 1024, 4096)
    c = ibdl.footprint(2, 1024, 4096, nrhs=4)
    d = ibdl.footprint(3, 256, 40000, prec=ibdl.MIXED)
    assert 0 < a < b < c and d > c
    assert ibdl.footprint(2, 1000, 10) == 0


def test_info_list_reads_the_c_array():
    """Solve reports: one dict per right-hand side, read from the C array the
    library fills; slices give lists of dicts, field() whole columns."""
    info = (ibdl.SolveInfo * 5)()
    for r in range(5):
        info[r].iters = 10 + r
        info[r].rel_resid_est = 0.25 * r
        info[r].rel_resid_true = 0.5 * r
        info[r].status = ibdl.ERR_NOCONV if r == 3 else ibdl.OK
        info[r].fp64_applies = 2 * r
    lst = ibdl.InfoList(info)
    assert len(lst) == 5
    assert lst[2] == dict(iters=12, rel_resid_est=0.5, rel_resid_true=1.0, status=ibdl.OK, fp64_applies=4)
    assert lst[-1]["iters"] == 14 and lst[3]["status"] == ibdl.ERR_NOCONV
    assert [x["iters"] for x in lst] == [10, 11, 12, 13, 14]
    assert [x["fp64_applies"] for x in lst[1:4]] == [2, 4, 6]
    assert type(lst[0]["iters"]) is int and type(lst[0]["rel_resid_true"]) is float
    assert lst.field("iters").tolist() == [10, 11, 12, 13, 14]
    assert lst.field("rel_resid_est").tolist() == [0.0, 0.25, 0.5, 0.75, 1.0]
    with pytest.raises(IndexError):
        lst[5]
    # a view of the array: later writes by the library show through
    info[0].iters = 99
    assert lst[0]["iters"] == 99
