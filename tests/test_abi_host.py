"""CPU-side checks of the C ABI: the library loads, exports every function
declared in include/adi.h, and rejects invalid arguments before touching a
device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "adi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(adi_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def native():
    from paper_1912_03744_amd import native
    return native


def test_library_exports_every_declared_function(native):
    lib = native.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    # the binding wraps exactly the declared set
    assert set(native.exported_symbols()) <= set(names)


def test_launch_shapes_listed(native):
    shapes = native.launch_shapes()
    assert len(shapes) >= 10
    for m, lpw, wpl, r, ngw in shapes:
        assert m >= 3 and lpw in (1, 2, 4, 8, 16) and wpl in (1, 2, 4, 8, 16)
        assert r >= 1 and 64 * wpl * ngw <= 1024


def test_batch_z_shapes_listed(native):
    """Every candidate z shape of the batched sweep launches covers the
    longest columns of its class, the batch's largest grid included."""
    classes = native.batch_zshapes()
    assert [c["max_rows"] for c in classes] == [192, 256, 320, 512]
    for cl in classes:
        assert len(cl["shapes"]) >= 2 and len(set(cl["shapes"])) == len(cl["shapes"])
        for waves, cells in cl["shapes"]:
            assert waves in (1, 2, 3) and cells >= 3
            assert 64 * waves * cells >= min(cl["max_rows"], 480)
    w = ctypes.c_int32(-7)
    assert native.lib().adi_batch_zshape_info(0, 9, ctypes.byref(w), ctypes.byref(ctypes.c_int32()),
                                              ctypes.byref(ctypes.c_int32())) == native.ADI_EINVAL
    assert w.value == -7
    assert native.lib().adi_batch_zshape_info(1, 0, None, None, None) == native.ADI_EINVAL


def test_status_strings(native):
    lib = native.lib()
    for code in range(0, -8, -1):
        assert lib.adi_status_string(code)
    assert b"gfx950" in lib.adi_version()


def _create(native, **kw):
    g = dict(r0=2.0, r1=3.0, r2=4.0, rmax=4.2, z0=8.0, zmax=10.0, ztop=10.2, nr=64, nz=160)
    g.update(kw)
    geom = native.Geometry(g["r0"], g["r1"], g["r2"], g["rmax"], g["z0"], g["zmax"], g["ztop"],
                           g["nr"], g["nz"], None, None)
    bc = native.BC((ctypes.c_double * 4)(0, 0.1, 0.1, 0.1), (ctypes.c_double * 4)(0, 0, 0, 0))
    h = ctypes.c_void_p()
    return native.lib().adi_create_problem(ctypes.byref(geom), ctypes.byref(bc), 0, None,
                                           ctypes.byref(h))


@pytest.mark.parametrize("kw", [dict(r0=-1.0), dict(r1=1.0), dict(rmax=3.9), dict(z0=0.0),
                                dict(zmax=11.0), dict(nr=0), dict(nz=-3), dict(r2=float("nan")),
                                dict(nr=100000, nz=100000)])
def test_invalid_geometry_rejected(native, kw):
    assert _create(native, **kw) == native.ADI_EINVAL
    assert native.lib().adi_last_error()


def test_invalid_bc_and_handles(native):
    lib = native.lib()
    geom = native.Geometry(2, 3, 4, 4.2, 8, 10, 10.2, 8, 8, None, None)
    bc = native.BC((ctypes.c_double * 4)(0, -1.0, 0, 0), (ctypes.c_double * 4)(0, 0, 0, 0))
    h = ctypes.c_void_p()
    assert lib.adi_create_problem(ctypes.byref(geom), ctypes.byref(bc), 0, None, ctypes.byref(h)) == native.ADI_EINVAL
    bc = native.BC((ctypes.c_double * 4)(0, 1.0, 0, 0), (ctypes.c_double * 4)(0, float("inf"), 0, 0))
    assert lib.adi_create_problem(ctypes.byref(geom), ctypes.byref(bc), 0, None, ctypes.byref(h)) == native.ADI_EINVAL
    bc = native.BC((ctypes.c_double * 4)(0, 1.0, 0, 0), (ctypes.c_double * 4)(0, 0, 0, 0))
    assert lib.adi_create_problem(ctypes.byref(geom), ctypes.byref(bc), 7, None, ctypes.byref(h)) == native.ADI_EINVAL
    # null handles are rejected without a device
    assert lib.adi_step(None, 1e-3, 1) == native.ADI_EINVAL
    assert lib.adi_set_sources(None, None) == native.ADI_EINVAL
    lib.adi_destroy(None)


def test_allocator_hook_arguments(native):
    """adi_set_allocator takes both functions or neither (no device call)."""
    lib = native.lib()
    assert lib.adi_set_allocator(native.ALLOC_FN(), native.FREE_FN(), None) == 0
    bad = native.ALLOC_FN(lambda n, ctx: 0)
    assert lib.adi_set_allocator(bad, native.FREE_FN(), None) == -1
    assert b"both" in lib.adi_last_error()
    with pytest.raises(ValueError):
        native.set_allocator(alloc=lambda n: 0)
    native.set_allocator()  # back to hipMalloc / hipFree
