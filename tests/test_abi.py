"""CPU-side checks of the C-ABI library: it loads, exports every entry point
that include/hgp.h declares, and rejects invalid input before any device
work (these paths make no HIP call, so they run without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "hgp.h")).read()
    return sorted(set(re.findall(r"\b(hgp_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("hgp_basis_create", "hgp_plan_create", "hgp_jk", "hgp_eri_shell_quartets",
                 "hgp_eri_prim_quartets", "hgp_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2605_10312_amd as hgp
    h = hgp.lib()
    for name in _declared():
        assert hasattr(h, name), name
    assert set(_declared()) == set(hgp.SIGNATURES)


def test_version_and_built_l():
    import paper_2605_10312_amd as hgp
    assert hgp.lib().hgp_version() >= 1
    assert 2 <= hgp.max_l() <= 4


def _create(l, nprim, cen, exps, coefs):
    import paper_2605_10312_amd as hgp
    h = ctypes.c_void_p()
    arrs = [np.ascontiguousarray(l, np.int32), np.ascontiguousarray(nprim, np.int32),
            np.ascontiguousarray(cen, np.float64), np.ascontiguousarray(exps, np.float64),
            np.ascontiguousarray(coefs, np.float64)]
    rc = hgp.lib().hgp_basis_create(len(arrs[0]), *[a.ctypes.data_as(ctypes.c_void_p) for a in arrs], 1, ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("case,status", [
    ("l5", -2), ("lneg", -1), ("nprim0", -1), ("nan_exp", -1), ("neg_exp", -1), ("inf_centre", -1)])
def test_basis_validation(case, status):
    import paper_2605_10312_amd as hgp
    l, nprim, cen, exps, coefs = [0, 1], [1, 2], np.zeros((2, 3)), [1.0, 2.0, 3.0], [1.0, 1.0, 1.0]
    if case == "l5":
        l = [5, 1]
    elif case == "lneg":
        l = [-1, 1]
    elif case == "nprim0":
        nprim, exps, coefs = [0, 2], [2.0, 3.0], [1.0, 1.0]
    elif case == "nan_exp":
        exps = [1.0, float("nan"), 3.0]
    elif case == "neg_exp":
        exps = [1.0, -2.0, 3.0]
    elif case == "inf_centre":
        cen = np.array([[0, 0, 0], [0, np.inf, 0]], float)
    rc, h = _create(l, nprim, cen, exps, coefs)
    assert rc == status
    assert h.value is None
    assert len(hgp.lib().hgp_last_error()) > 0


def test_null_arguments_rejected():
    import paper_2605_10312_amd as hgp
    L = hgp.lib()
    assert L.hgp_basis_create(1, None, None, None, None, None, 1, ctypes.byref(ctypes.c_void_p())) == -1
    one = np.ones(1)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    zi = np.zeros(1, np.int32)
    assert L.hgp_basis_create(1, ptr(zi), ptr(np.ones(1, np.int32)), ptr(np.zeros(3)), ptr(one), ptr(one), 7,
                              ctypes.byref(ctypes.c_void_p())) == -1          # unknown flags
    assert L.hgp_plan_create(None, 1e-12, 0, 0, None, ctypes.byref(ctypes.c_void_p())) == -1
    assert L.hgp_jk(None, None, None, None, None) == -1
    assert L.hgp_eri_prim_quartets(5, 0, 0, 0, 1, None, None, None, 0, None) == -2
    assert L.hgp_eri_prim_quartets(0, 0, 0, 0, -1, None, None, None, 0, None) == -1
    assert L.hgp_eri_prim_quartets(0, 0, 0, 0, 0, None, None, None, 0, None) == 0


def test_noalloc_rejections_before_device_work():
    """The allocation-free integrals entry rejects, with no HIP call: l > 4, a
    class on an op-table tier, and more quartets than its fixed buffer holds."""
    import paper_2605_10312_amd as hgp
    h = hgp.lib()
    fake = ctypes.c_void_p(16)        # never dereferenced: every case fails validation first
    assert h.hgp_eri_prim_quartets_noalloc(5, 0, 0, 0, 1, fake, fake, fake, 0, None) == -2
    assert h.hgp_eri_prim_quartets_noalloc(0, 0, 0, 0, -1, fake, fake, fake, 0, None) == -1
    assert h.hgp_eri_prim_quartets_noalloc(0, 0, 0, 0, 4, fake, fake, fake, 2, None) == -1   # no such precision
    nmax = h.hgp_eri_prim_quartets_noalloc_max(0, 0, 0, 0)
    assert 100_000 <= nmax <= 1 << 20
    assert h.hgp_eri_prim_quartets_noalloc(0, 0, 0, 0, nmax + 1, fake, fake, fake, 0, None) == -1
    assert "quartets of this class per call" in h.hgp_last_error().decode()
    assert h.hgp_eri_prim_quartets_noalloc_max(2, 2, 2, 2) > 0
    assert h.hgp_eri_prim_quartets_noalloc_max(5, 0, 0, 0) == -1
    assert h.hgp_eri_prim_quartets_noalloc(0, 0, 0, 0, 0, fake, fake, fake, 0, None) == 0


def test_class_form_query():
    """hgp_class_form reports each class's tier and FP32 form (host-only;
    the four l in any order name the same class)."""
    import paper_2605_10312_amd as hgp
    assert hgp.class_form((0, 0, 0, 0)) == (0, True)           # register tier, FP32 form for mixed plans
    assert hgp.class_form((1, 0, 0, 0)) == hgp.class_form((0, 0, 0, 1)) == hgp.class_form((0, 0, 1, 0))
    tier, f32 = hgp.class_form((2, 2, 2, 2))
    assert tier == 1 and f32                                    # row form: Phase 1 in FP32 for mixed
    tier, f32 = hgp.class_form((4, 4, 4, 4))
    assert tier in (2, 3) and not f32                           # op tables: FP64 only
    h = hgp.lib()
    t = ctypes.c_int32()
    assert h.hgp_class_form(5, 0, 0, 0, ctypes.byref(t), None) == -2
    assert h.hgp_class_form(-1, 0, 0, 0, None, None) == -1
    assert h.hgp_class_form(1, 1, 0, 0, None, None) == 0


def test_deriv_entry_host_checks():
    """The derivative integrals entry: built for l <= 2, argument errors
    before any device work."""
    import paper_2605_10312_amd as hgp
    h = hgp.lib()
    assert hgp.deriv_max_l() == 2
    assert h.hgp_eri_deriv_shell_quartets(None, 1, None, None, None, None) == -1
    assert h.hgp_eri_deriv_shell_quartets(None, -1, None, None, None, None) == -1
