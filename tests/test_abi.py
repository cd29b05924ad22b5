"""The C-ABI library loads, exports every declared entry point, and rejects bad
arguments on the host before any device call (runs without a GPU)."""
import ctypes
import glob
import math
import os
import re

import numpy as np
import pytest

import paper_1409_4441_amd as cr

INCLUDE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")


def declared_functions(header=None):
    names = set()
    headers = [header] if header else sorted(glob.glob(os.path.join(INCLUDE, "*.h")))
    for h in headers:
        text = open(os.path.join(INCLUDE, h) if header else h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(conv_\w+)\s*\(", text))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    from paper_1409_4441_amd import learn, sht, split
    names = declared_functions()
    assert len(names) >= 30
    for n in names:
        assert hasattr(cr.lib, n), n
    assert sorted(cr.EXPORTS) == declared_functions("convreal.h")
    assert sorted(split.EXPORTS) == declared_functions("convsplit.h")
    assert sorted(learn.EXPORTS) == declared_functions("convlearn.h")
    assert sorted(sht.EXPORTS) == declared_functions("convsht.h")
    assert sorted(set(cr.EXPORTS) | set(split.EXPORTS) | set(learn.EXPORTS) | set(sht.EXPORTS)) == names


def test_strerror():
    for code in [cr.OK, cr.EINVAL, cr.ENOMEM, cr.EHIP, cr.EALIAS, cr.ENODEV]:
        assert cr.lib.conv_real_strerror(code)
    assert cr.lib.conv_real_strerror(-99) == b"unknown error"


def _init(nside, table, n_tab, theta_cut, precision):
    h = ctypes.c_void_p()
    t = None if table is None else np.ascontiguousarray(table, dtype=np.float64)
    tp = None if t is None else t.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    rc = cr.lib.conv_real_init(ctypes.byref(h), nside, tp, n_tab, theta_cut, precision)
    return rc, h


@pytest.mark.parametrize("nside,n_tab,theta_cut,precision", [
    (0, 16, 0.1, 0), (-3, 16, 0.1, 0), (8193, 16, 0.1, 0),
    (8, 3, 0.1, 0), (8, 8193, 0.1, 0),
    (8, 16, 0.0, 0), (8, 16, -0.1, 0), (8, 16, 3.2, 0), (8, 16, float("nan"), 0),
    (8, 16, 0.1, 7), (8, 16, 0.1, -1),
])
def test_init_rejects_bad_arguments(nside, n_tab, theta_cut, precision):
    rc, h = _init(nside, np.ones(max(n_tab, 4)), n_tab, theta_cut, precision)
    assert rc == cr.EINVAL
    assert h.value is None


def test_init_rejects_null_and_nonfinite():
    rc, _ = _init(8, None, 16, 0.1, 0)
    assert rc == cr.EINVAL
    t = np.ones(16)
    t[5] = np.inf
    rc, _ = _init(8, t, 16, 0.1, 0)
    assert rc == cr.EINVAL
    assert b"non-finite" in cr.lib.conv_real_last_error()
    assert cr.lib.conv_real_init(None, 8, None, 16, 0.1, 0) == cr.EINVAL


def test_apply_and_pairs_reject_bad_plan():
    x = ctypes.c_void_p(16)
    assert cr.lib.conv_real_apply(None, x, ctypes.c_void_p(32), 1, None) == cr.EINVAL
    n = ctypes.c_longlong()
    assert cr.lib.conv_real_pairs(None, ctypes.byref(n)) == cr.EINVAL
    assert cr.lib.conv_real_destroy(None) == cr.OK
    m = ctypes.c_int()
    assert cr.lib.conv_real_set_method(None, 1) == cr.EINVAL
    assert cr.lib.conv_real_get_method(None, ctypes.byref(m)) == cr.EINVAL


def test_tabulate_rejects_bad_arguments():
    k = np.ones(10)
    out = np.empty(16)
    kp = k.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    op = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert cr.lib.conv_real_tabulate(kp, -1, 0.1, 16, op) == cr.EINVAL
    assert cr.lib.conv_real_tabulate(kp, 9, 0.0, 16, op) == cr.EINVAL
    assert cr.lib.conv_real_tabulate(kp, 9, math.pi + 0.1, 16, op) == cr.EINVAL
    assert cr.lib.conv_real_tabulate(kp, 9, 0.1, 2, op) == cr.EINVAL
    assert cr.lib.conv_real_tabulate(None, 9, 0.1, 16, op) == cr.EINVAL
    assert cr.lib.conv_real_tabulate(kp, 9, 0.1, 16, None) == cr.EINVAL


def test_python_binding_validates():
    with pytest.raises(ValueError):
        cr.Plan(8, np.ones(16), 0.1, "f16")
    with pytest.raises(cr.ConvRealError) as e:
        cr.Plan(0, np.ones(16), 0.1, "f64")
    assert e.value.code == cr.EINVAL


def test_sht_rejects_bad_arguments():
    from paper_1409_4441_amd import sht
    h = ctypes.c_void_p()
    for nside, lmax in [(0, 8), (4096, 8), (16, -1), (16, 8193)]:
        assert cr.lib.conv_sht_init(ctypes.byref(h), nside, lmax) == cr.EINVAL
    assert cr.lib.conv_sht_init(None, 16, 8) == cr.EINVAL
    n = ctypes.c_longlong()
    assert cr.lib.conv_sht_alm_size(10, ctypes.byref(n)) == cr.OK and n.value == 66
    assert cr.lib.conv_sht_alm_size(-1, ctypes.byref(n)) == cr.EINVAL
    for f, args in [("conv_sht_analysis", (None, None, 0, None, None)),
                    ("conv_sht_synthesis", (None, None, None, 0, 0, None)),
                    ("conv_sht_almxfl", (None, None, None, None, None)),
                    ("conv_sht_convolve", (None, None, None, None, 0, 0, None)),
                    ("conv_sht_power_spectrum", (None, None, None, None)),
                    ("conv_hybrid_apply", (None, None, None, None, None, 1, None, None))]:
        assert getattr(cr.lib, f)(*args) == cr.EINVAL, f
    assert cr.lib.conv_sht_destroy(None) == cr.OK
    assert sht.alm_size(4) == 15
