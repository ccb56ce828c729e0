"""The C-ABI library: loads, exports every declared symbol, rejects bad
arguments before touching a device (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nlfem.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nlfem_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def nl():
    import paper_2207_03921_amd as nl
    if not os.path.exists(nl.LIB_PATH):
        from paper_2207_03921_amd import build
        build.build()
    return nl


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("nlfem_build_pairs", "nlfem_assemble", "nlfem_rhs", "nlfem_pairs_info",
              "nlfem_pairs_export", "nlfem_csr_pattern", "nlfem_pairs_free", "nlfem_version",
              "nlfem_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(nl):
    L = nl.lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert nl.nlfem_version() == nl.ABI_VERSION == 5


def _cfg(nl, **over):
    from inputs import gauss7
    r = gauss7()
    d = dict(kernel="inv_dist", c=1.0, delta=0.1, outer_xi=r.xi, outer_w=r.w, inner_xi=r.xi,
             inner_w=r.w, singular_n=5)
    d.update(over)
    return nl.Config(**d)


def _fake_mesh(nl, K=4, M=6, null=False):
    # host pointers stand in for device arrays: validation rejects the call
    # before any device access
    return nl._Mesh(M, K, None if null else 1, 1, 1)


@pytest.mark.parametrize("bad,msg", [
    (dict(delta=0.0), "delta"),
    (dict(delta=-1.0), "delta"),
    (dict(kernel="frac_half", singular_n=0), "singular_n > 0"),
    (dict(outer_w=np.array([0.1] * 7)), "sum to 1/2"),
    (dict(singular_n=40), "singular_n"),
    (dict(approach="poly", polygon_dirs=None), "polygon"),
    (dict(approach="poly", polygon_dirs=np.array([[1.0, 0.0], [0.0, 1.0]])), "polygon_n"),
    (dict(approach="poly", polygon_dirs=np.array([[1.0, 0.0], [-1.0, 0.0], [0.0, 1.0], [0.0, -1.0]])),
     "convex"),
])
def test_build_rejects_bad_config(nl, bad, msg):
    cfg = _cfg(nl, **bad)
    cm = _fake_mesh(nl)
    h = C.c_void_p(None)
    cc = cfg.c_struct()
    rc = nl.lib().nlfem_build_pairs(C.byref(cm), C.byref(cc), C.byref(h), None)
    assert rc == -1
    assert msg in nl.nlfem_last_error()
    assert h.value is None


def test_build_rejects_bad_mesh(nl):
    cfg = _cfg(nl)
    cc = cfg.c_struct()
    h = C.c_void_p(None)
    L = nl.lib()
    assert L.nlfem_build_pairs(None, C.byref(cc), C.byref(h), None) == -1
    cm = _fake_mesh(nl, null=True)
    assert L.nlfem_build_pairs(C.byref(cm), C.byref(cc), C.byref(h), None) == -1
    cm = nl._Mesh(0, 4, 1, 1, 1)
    assert L.nlfem_build_pairs(C.byref(cm), C.byref(cc), C.byref(h), None) == -1
    cm = nl._Mesh(2 ** 31, 4, 1, 1, 1)
    assert L.nlfem_build_pairs(C.byref(cm), C.byref(cc), C.byref(h), None) == -5
    assert L.nlfem_build_pairs(C.byref(_fake_mesh(nl)), C.byref(cc), None, None) == -1


def test_other_entry_points_reject_null(nl):
    L = nl.lib()
    cfg = _cfg(nl)
    cc = cfg.c_struct()
    cm = _fake_mesh(nl)
    info = nl._Info()
    assert L.nlfem_pairs_info(None, C.byref(info)) == -1
    assert L.nlfem_assemble(C.byref(cm), C.byref(cc), None, None, None) == -1
    assert L.nlfem_pairs_export(None, None, None, None, None) == -1
    assert L.nlfem_csr_pattern(None, None, None, None) == -1
    assert L.nlfem_rhs(C.byref(cm), C.byref(cc), None, None, None, None) == -1
    assert "b is NULL" in nl.nlfem_last_error()
    L.nlfem_pairs_free(None)


def test_binding_fails_loudly_without_library(monkeypatch, nl):
    monkeypatch.setattr(nl, "_lib", None)
    monkeypatch.setattr(nl, "LIB_PATH", "/nonexistent/libnlfem.so")
    with pytest.raises(nl.NlfemError):
        nl.lib()


def test_timing_mask_validation(nl):
    L = nl.lib()
    assert L.nlfem_timing_enable(-1) == -1
    assert L.nlfem_timing_enable(1 << 9) == -1
    assert "mask" in nl.nlfem_last_error()
    assert L.nlfem_timing_enable(0) == 0          # off while off: nothing to do
    ms = np.zeros(9)
    n = np.zeros(9, np.int64)
    assert L.nlfem_timing_read(ms.ctypes.data, n.ctypes.data, 1) == 0
    assert not n.any()
    assert L.nlfem_timing_read(None, None, 1) == -1


def test_batch_entry_points_validate_without_device(nl):
    L = nl.lib()
    h = C.c_void_p(None)
    assert L.nlfem_batch_create(0, None, None, None, None, None, 0, C.byref(h), None) == -1
    assert "batch size" in nl.nlfem_last_error()
    assert L.nlfem_batch_create(1, None, None, None, None, None, 0, C.byref(h), None) == -1
    assert L.nlfem_batch_create(1, None, None, None, None, None, 0, None, None) == -1
    assert L.nlfem_batch_assemble(None, None) == -1
    assert L.nlfem_batch_launch_graph(None, None) == -1
    g = C.c_int32(0)
    sh = (C.c_int32 * 8)()
    assert L.nlfem_batch_info(None, C.byref(g), sh) == -1
    assert L.nlfem_assemble_batched(0, None, None, None, None, None, None) == -1
    L.nlfem_batch_free(None)


def test_allocator_and_capacity_validation(nl):
    """The allocator hooks come in pairs; the capacity limit is >= 0.  Both
    are host settings, checked without a device."""
    L = nl.lib()
    keep = nl.ALLOC_FN(lambda n, s, c: None)
    assert L.nlfem_set_allocator(keep, nl.FREE_FN(), None) == -1
    assert "both" in nl.nlfem_last_error()
    assert L.nlfem_set_allocator(nl.ALLOC_FN(), nl.FREE_FN(), None) == 0   # default
    with pytest.raises(ValueError):
        nl.nlfem_set_allocator(alloc=lambda n, s: 0)
    assert L.nlfem_set_capacity(-1) == -1
    assert L.nlfem_set_capacity(0) == 0
