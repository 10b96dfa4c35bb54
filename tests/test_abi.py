"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/wos.h declares, and rejects bad arguments before it
touches the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wos.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wos_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def B():
    from paper_2406_01713_amd import binding
    return binding


def test_header_declares_the_paper_calls():
    names = declared_functions()
    for f in ["wos_create_domain", "wos_estimate", "wos_backward", "wos_estimate_batch",
              "wos_plan_create", "wos_plan_step", "wos_autotune", "wos_last_error"]:
        assert f in names


def test_library_exports_every_declared_symbol(B):
    names = declared_functions()
    missing = [n for n in names if not hasattr(B.lib, n)]
    assert not missing, missing
    assert sorted(B.EXPORTED) == names


def _bdata(B):
    return B.BData(0, 1.0, 0.0, 0.0, None, 0.0)


def _outer(B, d):
    lo = np.full(d, -1.0)
    hi = np.full(d, 1.0)
    return B.Outer(B.WOS_OUTER_BOX, lo.ctypes.data_as(C.POINTER(C.c_double)),
                   hi.ctypes.data_as(C.POINTER(C.c_double)), None, 0.0), (lo, hi)


def test_create_domain_rejects_bad_dimension(B):
    h = C.c_void_p()
    o, keep = _outer(B, 8)
    bd = _bdata(B)
    for d in (0, 1, 9, 100):
        rc = B.lib.wos_create_domain(d, None, None, None, None, C.byref(o), C.byref(bd), None, C.byref(h))
        assert rc == B.WOS_EDIM
        assert b"outside" in B.lib.wos_last_error()
    assert B.lib.wos_create_domain(3, None, None, None, None, None, C.byref(bd), None, C.byref(h)) == B.WOS_EINVAL
    assert B.lib.wos_create_domain(3, None, None, None, None, C.byref(o), None, None, C.byref(h)) == B.WOS_EINVAL
    assert B.lib.wos_create_domain(3, None, None, None, None, C.byref(o), C.byref(bd), None, None) == B.WOS_EINVAL


def test_create_domain_rejects_bad_obstacles(B):
    d = 2
    h = C.c_void_p()
    o, keep = _outer(B, d)
    bd = _bdata(B)
    c = np.zeros((1, d))
    r = np.array([-0.5])
    sp = B.Spheres(1, c.ctypes.data_as(C.POINTER(C.c_double)), r.ctypes.data_as(C.POINTER(C.c_double)))
    assert B.lib.wos_create_domain(d, C.byref(sp), None, None, None, C.byref(o), C.byref(bd), None, C.byref(h)) == B.WOS_EINVAL
    r2 = np.array([np.nan])
    sp2 = B.Spheres(1, c.ctypes.data_as(C.POINTER(C.c_double)), r2.ctypes.data_as(C.POINTER(C.c_double)))
    assert B.lib.wos_create_domain(d, C.byref(sp2), None, None, None, C.byref(o), C.byref(bd), None, C.byref(h)) == B.WOS_EINVAL
    sp3 = B.Spheres(1, None, None)
    assert B.lib.wos_create_domain(d, C.byref(sp3), None, None, None, C.byref(o), C.byref(bd), None, C.byref(h)) == B.WOS_EINVAL
    bad = B.BData(7, 1.0, 0.0, 0.0, None, 0.0)
    assert B.lib.wos_create_domain(d, None, None, None, None, C.byref(o), C.byref(bad), None, C.byref(h)) == B.WOS_EINVAL
    lo = np.array([1.0, -1.0])
    hi = np.array([-1.0, 1.0])
    ob = B.Outer(B.WOS_OUTER_BOX, lo.ctypes.data_as(C.POINTER(C.c_double)),
                 hi.ctypes.data_as(C.POINTER(C.c_double)), None, 0.0)
    assert B.lib.wos_create_domain(d, None, None, None, None, C.byref(ob), C.byref(bd), None, C.byref(h)) == B.WOS_EINVAL


def test_create_domain_rejects_bad_extrusion(B):
    """geom_d outside [0, d] and box obstacles in extruded geometry are
    rejected before any device call."""
    d = 3
    h = C.c_void_p()
    bd = _bdata(B)
    oc = np.zeros(d)
    for gd in (-1, 4, 9):
        ob = B.Outer(B.WOS_OUTER_BALL, None, None, oc.ctypes.data_as(C.POINTER(C.c_double)), 2.0, gd)
        assert B.lib.wos_create_domain(d, None, None, None, None, C.byref(ob), C.byref(bd), None, C.byref(h)) == B.WOS_EINVAL
        assert b"geom_d" in B.lib.wos_last_error()
    ob = B.Outer(B.WOS_OUTER_BALL, None, None, oc.ctypes.data_as(C.POINTER(C.c_double)), 2.0, 2)
    bc = np.zeros((1, d))
    bh = np.full((1, d), 0.1)
    bx = B.Boxes(1, bc.ctypes.data_as(C.POINTER(C.c_double)), bh.ctypes.data_as(C.POINTER(C.c_double)))
    assert B.lib.wos_create_domain(d, None, C.byref(bx), None, None, C.byref(ob), C.byref(bd), None, C.byref(h)) == B.WOS_EINVAL
    assert b"full space" in B.lib.wos_last_error()
    # an outer box whose bounds are only given for the leading coordinates
    lo = np.array([-1.0, -1.0, np.nan])
    hi = np.array([1.0, 1.0, np.nan])
    ob2 = B.Outer(B.WOS_OUTER_BOX, lo.ctypes.data_as(C.POINTER(C.c_double)),
                  hi.ctypes.data_as(C.POINTER(C.c_double)), None, 0.0, 3)
    assert B.lib.wos_create_domain(d, None, None, None, None, C.byref(ob2), C.byref(bd), None, C.byref(h)) == B.WOS_EINVAL


def test_create_domain_rejects_bad_arm(B):
    """Arm descriptions are checked before any device call: points, lengths,
    extrusion, and boundary data that would need a boundary point."""
    d = 2
    h = C.c_void_p()
    o, keep = _outer(B, d)
    bd = _bdata(B)
    pts = np.array([[0.0, 1.3]])
    P = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))

    def make(lengths, n=1, points=pts):
        return B.Arm(P(lengths), n, P(points))

    good = np.array([1.0, 1.0])
    for arm in (make(good, 0), make(np.array([1.0, -0.5])), make(np.array([0.0, 0.0])),
                make(good, 1, np.array([[np.nan, 1.0]])), make(np.array([np.inf, 1.0]))):
        rc = B.lib.wos_create_domain(d, None, None, C.byref(arm), None, C.byref(o), C.byref(bd), None, C.byref(h))
        assert rc == B.WOS_EINVAL, B.lib.wos_last_error()
    nul = B.Arm(None, 1, P(pts))
    assert B.lib.wos_create_domain(d, None, None, C.byref(nul), None, C.byref(o), C.byref(bd), None,
                                   C.byref(h)) == B.WOS_EINVAL
    a = np.array([0.1, 0.2])
    aff = B.BData(1, 0.0, 0.0, 0.0, P(a), 0.0)
    assert B.lib.wos_create_domain(d, None, None, C.byref(make(good)), None, C.byref(o), C.byref(aff), None,
                                   C.byref(h)) == B.WOS_ENOTSUP
    oc = np.zeros(3)
    ob = B.Outer(B.WOS_OUTER_BALL, None, None, P(oc), 2.0, 2)
    g3 = np.ones(3)
    assert B.lib.wos_create_domain(3, None, None, C.byref(make(g3)), None, C.byref(ob), C.byref(bd), None,
                                   C.byref(h)) == B.WOS_EINVAL
    assert b"full space" in B.lib.wos_last_error()


def test_calls_reject_null_handles(B):
    assert B.lib.wos_estimate(None, None, 1, 16, 1.0, 1e-3, 0, None, None, None, None, None) == B.WOS_EINVAL
    assert B.lib.wos_backward(None, None, 1, 16, 1.0, 1e-3, 0, None, None, None, None, None, None,
                              None) == B.WOS_EINVAL
    assert B.lib.wos_plan_step(None, 1) == B.WOS_EINVAL
    assert B.lib.wos_domain_dim(None) == B.WOS_EINVAL
    assert B.lib.wos_autotune(1, 10, 10, 64, b"/tmp/x.json") == B.WOS_EDIM
    assert B.lib.wos_estimate_batch(None, 0, None, None, None, None, None, 0, None, None, None, None,
                                    None, None, None, None, None) == B.WOS_OK
    opt = B.Options(B.WOS_FP64, 0, 0, 0)
    assert B.lib.wos_estimate_batch(None, 1, None, None, None, None, None, 0, None, None, None, None,
                                    None, None, None, C.byref(opt), None) == B.WOS_ENOTSUP
    B.lib.wos_destroy_domain(None)
    B.lib.wos_plan_destroy(None)


def test_product_path_imports_no_oracle():
    """The library package never imports, links or runs the oracle."""
    pkg = os.path.join(ROOT, "paper_2406_01713_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                for pat in (r"^\s*(from|import)\s+oracle\b", r"wos_oracle", r"libwos_oracle",
                            r"#include\s+[<\"].*oracle"):
                    assert not re.search(pat, src, flags=re.M), (f, pat)


def test_create_domain_rejects_bad_source(B):
    d = 3
    h = C.c_void_p()
    o, keep = _outer(B, d)
    bd = _bdata(B)
    zn = np.array([0.0, np.nan, 0.0])
    z0 = np.zeros(d)
    for src in (B.Source(zn.ctypes.data_as(C.POINTER(C.c_double)), 1.0, 1.0),
                B.Source(None, 1.0, 1.0),
                B.Source(z0.ctypes.data_as(C.POINTER(C.c_double)), 1.0, -1.0),
                B.Source(z0.ctypes.data_as(C.POINTER(C.c_double)), np.inf, 1.0)):
        rc = B.lib.wos_create_domain(d, None, None, None, None, C.byref(o), C.byref(bd), C.byref(src), C.byref(h))
        assert rc == B.WOS_EINVAL
        assert b"source" in B.lib.wos_last_error()


def test_varadhan_rejects_bad_arguments(B):
    vp = C.c_void_p(1)
    assert B.lib.wos_varadhan(vp, None, 4, 0, 0, 0.0, vp, None, None, None) == B.WOS_EINVAL
    assert B.lib.wos_varadhan(vp, None, 4, 0, 0, -1.0, vp, None, None, None) == B.WOS_EINVAL
    assert B.lib.wos_varadhan(None, None, 4, 0, 0, 1.0, vp, None, None, None) == B.WOS_EINVAL
    assert B.lib.wos_varadhan(vp, vp, 4, 3, 3, 1.0, vp, None, None, None) == B.WOS_EINVAL
    assert B.lib.wos_varadhan(vp, vp, 4, 9, 9, 1.0, vp, vp, None, None) == B.WOS_EDIM
    assert B.lib.wos_varadhan(vp, vp, 4, 3, 2, 1.0, vp, vp, None, None) == B.WOS_EINVAL
    assert B.lib.wos_varadhan(None, None, 0, 0, 0, 1.0, None, None, None, None) == B.WOS_OK


def test_binding_constants_match_the_header(B):
    """Every integer #define of include/wos.h that the binding also names
    has the same value there."""
    src = open(HEADER).read()
    defs = dict(re.findall(r"^#define\s+(WOS_[A-Z0-9_]+)\s+\(?(-?\d+)u?\)?", src, flags=re.M))
    shared = [k for k in defs if hasattr(B, k)]
    assert {"WOS_FP64", "WOS_FULL_SCAN", "WOS_SCALAR_CULL", "WOS_WAVE_SCAN", "WOS_OUT_FP64", "WOS_NO_BOX_TEST", "WOS_BOX_TEST",
            "WOS_EINVAL", "WOS_ENOTSUP", "WOS_OUTER_BOX", "WOS_NOALLOC_SCRATCH_BYTES",
            "WOS_NOALLOC_MAX_ENVS", "WOS_CLUSTER_ROWS", "WOS_BATCH_STATS",
            "WOS_BATCH_STRIDE"} <= set(shared)
    for k in shared:
        assert int(defs[k]) == getattr(B, k), k


def test_option_flags_are_checked_before_device_work(B):
    """Unknown flag bits, and the box test both forced on and off, are
    rejected; the read-out, which takes u as given, rejects WOS_OUT_FP64 (it
    applies to wos_estimate only)."""
    opt = B.Options(1 << 10, 0, 0, 0)
    assert B.lib.wos_varadhan(None, None, 0, 2, 2, 1.0, None, None, C.byref(opt), None) == B.WOS_EINVAL
    assert b"unknown flags" in B.lib.wos_last_error()
    opt = B.options(box_test=True, no_box_test=True)
    assert B.lib.wos_varadhan(None, None, 0, 2, 2, 1.0, None, None, C.byref(opt), None) == B.WOS_EINVAL
    assert b"together" in B.lib.wos_last_error()
    opt = B.options(out_fp64=True)
    assert B.lib.wos_varadhan(None, None, 0, 2, 2, 1.0, None, None, C.byref(opt), None) == B.WOS_ENOTSUP


def test_noalloc_batch_rejects_too_many_envs_on_the_host(B):
    """The no-allocation batch call takes at most WOS_NOALLOC_MAX_ENVS
    environments and says so before any device work (the handles are not
    even read)."""
    n = B.WOS_NOALLOC_MAX_ENVS + 1
    hs = (C.c_void_p * n)()
    qo = np.zeros(n + 1, dtype=np.int64)
    f = np.ones(n)
    nw = np.ones(n, dtype=np.int64)
    rc = B.lib.wos_estimate_batch_noalloc(hs, n, None, qo.ctypes.data_as(C.POINTER(C.c_int64)),
                                          f.ctypes.data_as(C.POINTER(C.c_double)),
                                          f.ctypes.data_as(C.POINTER(C.c_double)),
                                          nw.ctypes.data_as(C.POINTER(C.c_int64)), 0, None, None, None, None,
                                          None, None, None, None, None)
    assert rc == B.WOS_EINVAL
    assert b"at most 1024" in B.lib.wos_last_error()
