"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every symbol include/wvl.h declares, builds localization regions bit-exactly
like the oracle, and rejects malformed plans before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import inputs
import paper_1401_7441_amd as W
from oracle import locreg as LR
from tests.abi_helpers import to_abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "wvl.h")).read()
    declared = set(re.findall(r"\b(wvl_[a-z_]+)\s*\(", header))
    assert declared == set(W.EXPORTED), declared ^ set(W.EXPORTED)
    lib = ctypes.CDLL(W.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name


def test_struct_layouts_match_header():
    assert W.SEG_DTYPE.itemsize == 24
    assert W.LOCREG_DTYPE.itemsize == 184
    assert W.LOCREG_DTYPE.fields["seg_c"][1] == 72


@pytest.mark.parametrize("workload,nsf", [("batch1k", 25), ("sweep2k", 12), ("serve", 30)])
def test_sphere_locregs_bit_exact_against_oracle(workload, nsf):
    g = inputs.geometry(workload, nsf=nsf)
    lr, segs = W.build_locregs(g.h, g.grid_n, g.centers, g.radii, g.fine_radii, g.ext)
    olr = LR.sphere_locregs(g.h, g.grid_n, g.centers, g.radii, g.fine_radii, g.ext)
    rec, oseg = to_abi(olr)
    for f in ("lo", "dims", "ext", "n_c", "n_f", "on_c", "on_f", "coef_off", "ocoef_off",
              "seg_c", "nseg_c", "seg_f", "nseg_f", "oseg_c", "noseg_c", "oseg_f", "noseg_f"):
        assert np.array_equal(lr[f], rec[f]), f
    assert np.array_equal(segs, oseg)


def _raw_ctx(h, n):
    ctx = ctypes.c_void_p()
    g = W._grid(h, n)
    assert W.lib().wvl_create(ctypes.byref(ctx), ctypes.byref(g), None) == 0
    return ctx


def _plan_status(ctx, rec, segs):
    plan = ctypes.c_void_p()
    ws = ctypes.c_size_t(0)
    st = W.lib().wvl_plan_create(ctx, len(rec), rec.ctypes.data, segs.ctypes.data, len(segs), 0,
                                 ctypes.byref(plan), ctypes.byref(ws))
    return st, W.lib().wvl_last_error(ctx).decode()


@pytest.fixture(scope="module")
def small_case():
    g = inputs.geometry("batch1k", nsf=4)
    olr = LR.sphere_locregs(g.h, g.grid_n, g.centers, np.full(4, 2.0), np.full(4, 1.0), 2)
    rec, segs = to_abi(olr)
    return g, rec, segs


@pytest.mark.parametrize("mutation,needle", [
    ("unsorted", "not sorted"),
    ("bad_off", "running sum"),
    ("outside_box", "outside"),
    ("fine_not_in_coarse", "not inside a coarse"),
    ("count_mismatch", "point counts"),
    ("ext_range", "ext outside"),
    ("box_outside_grid", "outside the grid"),
    ("overlapping_outputs", "overlap"),
])
def test_plan_rejects_malformed_input(small_case, mutation, needle):
    g, rec0, segs0 = small_case
    rec, segs = rec0.copy(), segs0.copy()
    r = rec[1]
    if mutation == "unsorted":
        a = int(r["seg_c"])
        for f in ("i1s", "i1e", "i2", "i3"):          # swap positions, keep offsets
            segs[a][f], segs[a + 1][f] = segs0[a + 1][f], segs0[a][f]
    elif mutation == "bad_off":
        segs[int(r["seg_c"]) + 1]["off"] += 1
    elif mutation == "outside_box":
        segs[int(r["seg_c"])]["i3"] = int(r["lo"][2]) - 1
    elif mutation == "fine_not_in_coarse":
        q = int(r["seg_f"])              # move the first fine run to the box corner row
        ln = int(segs[q]["i1e"]) - int(segs[q]["i1s"])
        segs[q]["i1s"] = int(r["lo"][0])
        segs[q]["i1e"] = int(r["lo"][0]) + ln
        segs[q]["i2"] = int(r["lo"][1])
        segs[q]["i3"] = int(r["lo"][2])
    elif mutation == "count_mismatch":
        rec[1]["n_c"] += 1
    elif mutation == "ext_range":
        rec[1]["ext"] = 17
    elif mutation == "box_outside_grid":
        rec[1]["lo"][0] = g.grid_n[0] - 1
    elif mutation == "overlapping_outputs":
        rec[2]["ocoef_off"] = rec[1]["ocoef_off"] + 1
    ctx = _raw_ctx(g.h, g.grid_n)
    try:
        st, msg = _plan_status(ctx, rec, segs)
    finally:
        W.lib().wvl_destroy(ctx)
    assert st == W.WVL_EINVAL, (st, msg)
    assert needle in msg, msg


def test_build_locregs_rejects_bad_arguments():
    g = W._grid(0.45, (40, 40, 40))
    n = ctypes.c_int64(0)
    lr = np.zeros(1, W.LOCREG_DTYPE)
    c = np.array([[5.0, 5.0, 5.0]])
    far = np.array([[-50.0, 5.0, 5.0]])
    neg = np.array([-1.0])
    one = np.array([1.0])
    st = W.lib().wvl_build_locregs(ctypes.byref(g), 1, c.ctypes.data, neg.ctypes.data,
                                   one.ctypes.data, 8, lr.ctypes.data, None, ctypes.byref(n))
    assert st == W.WVL_EINVAL
    st = W.lib().wvl_build_locregs(ctypes.byref(g), 1, far.ctypes.data, one.ctypes.data,
                                   one.ctypes.data, 8, lr.ctypes.data, None, ctypes.byref(n))
    assert st == W.WVL_EINVAL and "empty" in W.lib().wvl_last_error(None).decode()
