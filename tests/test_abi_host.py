"""CPU tests of the C ABI: the library loads, exports every symbol the header
declares, validates its inputs and builds the offset-array tables. No compute
call is made (host-only plans), so these run without a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
import paper_2406_05577_amd as pk
from paper_2406_05577_amd import fftb as fb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fftb.h")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fftb_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = pk.lib()
    names = header_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert sorted(pk.EXPORTS) == names


def host_plan(dims, maps, nb=2, dtype="c128", tuning=None):
    return pk.Plan(dims, maps, nb, dtype=dtype, flags=pk.PLAN_HOST_ONLY, tuning=tuning)


def test_status_strings():
    L = pk.lib()
    for s in (0, -1, -2, -3, -4):
        assert L.fftb_status_string(s)
    assert L.fftb_last_error() is not None


@pytest.mark.parametrize("dims,semi,k", [((6, 5, 4), (1.6, 1.3, 1.1), (0.31, -0.22, 0.4)),
                                        ((32, 32, 32), (8, 8, 8), (0, 0, 0)),
                                        ((144, 160, 180), (36, 40, 45), (0.2, -0.1, 0.3))])
def test_column_tables_match_map(dims, semi, k):
    m, lin = synth.sphere_map(dims, semi, k)
    rng = np.random.default_rng(0)
    lin = lin[rng.permutation(lin.shape[0])]
    p = host_plan(dims, [lin])
    nx, ny, nz = dims
    cx, cy, ec, ez = p.sphere_columns(0)
    x = lin % nx
    y = (lin // nx) % ny
    z = lin // (nx * ny)
    # columns = distinct (x, y) ordered by (x, y); entries point at their column and z
    keys = sorted(set(zip(x.tolist(), y.tolist())))
    assert list(zip(cx.tolist(), cy.tolist())) == keys
    np.testing.assert_array_equal(cx[ec], x)
    np.testing.assert_array_equal(cy[ec], y)
    np.testing.assert_array_equal(ez, z)
    ncol, nslab = p.sphere_stats(0)
    assert ncol == len(keys) and nslab == len(set(x.tolist()))
    assert p.info["total_coeffs"] == lin.shape[0]
    assert p.info["grid_elems"] == nx * ny * nz * 2
    assert p.info["sphere_elems"] == lin.shape[0] * 2


def test_128cube_sphere_columns_and_slabs():
    # occupied columns and slabs of the 128^3 |G|<=32 sphere
    w = synth.make_workload("c2", nbands=1)
    p = host_plan(w.dims, [w.spheres[0].lin], nb=256)
    assert p.sphere_stats(0) == (3209, 65)


def test_radix_plans():
    for n, expect in [(128, [16, 8]), (32, [8, 4]), (96, [12, 8]), (144, [12, 12]),
                      (160, [16, 10]), (180, [15, 12]), (4, [4]), (7 * 0 + 1, [1])]:
        lin = np.array([0], np.int32)
        p = host_plan((n, 4, 4), [lin])
        assert p.info["radix_x"] == expect, (n, p.info["radix_x"])


def _expect_status(status, fn):
    with pytest.raises(pk.FftbError) as ei:
        fn()
    assert ei.value.status == status, str(ei.value)


def test_validation_errors():
    ok = np.array([0, 1, 2], np.int32)
    _expect_status(pk.FFTB_ERR_UNSUPPORTED, lambda: host_plan((7, 4, 4), [ok]))
    _expect_status(pk.FFTB_ERR_UNSUPPORTED, lambda: host_plan((4, 11, 4), [ok]))
    _expect_status(pk.FFTB_ERR_INVALID, lambda: host_plan((4, 4, 4), [np.array([0, 0], np.int32)]))
    _expect_status(pk.FFTB_ERR_INVALID, lambda: host_plan((4, 4, 4), [np.array([0, 64], np.int32)]))
    _expect_status(pk.FFTB_ERR_INVALID, lambda: host_plan((4, 4, 4), [np.array([-1], np.int32)]))
    _expect_status(pk.FFTB_ERR_INVALID, lambda: host_plan((4, 4, 4), [np.array([], np.int32)]))
    _expect_status(pk.FFTB_ERR_INVALID, lambda: host_plan((4, 4, 4), [ok], nb=0))
    _expect_status(pk.FFTB_ERR_INVALID, lambda: host_plan((0, 4, 4), [ok]))
    _expect_status(pk.FFTB_ERR_INVALID, lambda: host_plan((4, 4, 4), [ok], tuning=dict(band_chunk=3)))
    _expect_status(pk.FFTB_ERR_INVALID, lambda: host_plan((4, 4, 4), [ok], tuning=dict(y_classes=3)))
    _expect_status(pk.FFTB_ERR_INVALID, lambda: host_plan((4, 4, 4), [ok], tuning=dict(threads=100)))
    _expect_status(pk.FFTB_ERR_INVALID, lambda: host_plan((4, 4, 4), [ok], tuning=dict(fwd_splits=9)))
    _expect_status(pk.FFTB_ERR_INVALID, lambda: host_plan((4, 4, 4), [ok], tuning=dict(acc=5)))
    with pytest.raises(KeyError):
        host_plan((4, 4, 4), [ok], tuning=dict(bogus=1))


def test_null_pointers():
    L = pk.lib()
    h = C.c_void_p()
    d = (C.c_int32 * 3)(4, 4, 4)
    m = np.array([0, 1], np.int32)
    sp = (fb.Sphere_t * 1)()
    sp[0].n_coeffs = 2
    sp[0].map = m.ctypes.data_as(C.POINTER(C.c_int32))
    sp[0].nbands = 1
    assert L.fftb_plan_create(None, d, sp, 1, 0, pk.PLAN_HOST_ONLY, None, None) == pk.FFTB_ERR_INVALID
    assert L.fftb_plan_create(C.byref(h), None, sp, 1, 0, pk.PLAN_HOST_ONLY, None, None) == pk.FFTB_ERR_INVALID
    assert L.fftb_plan_create(C.byref(h), d, None, 1, 0, pk.PLAN_HOST_ONLY, None, None) == pk.FFTB_ERR_INVALID
    assert L.fftb_plan_create(C.byref(h), d, sp, 0, 0, pk.PLAN_HOST_ONLY, None, None) == pk.FFTB_ERR_INVALID
    assert L.fftb_plan_create(C.byref(h), d, sp, 1, 7, pk.PLAN_HOST_ONLY, None, None) == pk.FFTB_ERR_INVALID
    sp[0].map = None
    assert L.fftb_plan_create(C.byref(h), d, sp, 1, 0, pk.PLAN_HOST_ONLY, None, None) == pk.FFTB_ERR_INVALID
    assert b"null map" in L.fftb_last_error()
    sp[0].map = m.ctypes.data_as(C.POINTER(C.c_int32))
    assert L.fftb_plan_create(C.byref(h), d, sp, 1, 0, pk.PLAN_HOST_ONLY, None, None) == 0
    # a host-only plan refuses to execute; null data pointers are rejected
    assert L.fftb_sphere_to_grid(h, C.c_void_p(16), C.c_void_p(16), None) == pk.FFTB_ERR_INVALID
    assert L.fftb_grid_to_sphere(h, None, None, None) == pk.FFTB_ERR_INVALID
    assert L.fftb_sphere_to_grid(None, None, None, None) == pk.FFTB_ERR_INVALID
    info = fb.Info_t()
    assert L.fftb_plan_get_info(None, C.byref(info)) == pk.FFTB_ERR_INVALID
    assert L.fftb_plan_get_info(h, None) == pk.FFTB_ERR_INVALID
    assert L.fftb_plan_sphere_stats(h, 5, None, None) == pk.FFTB_ERR_INVALID
    assert L.fftb_apply_potential(None, None, None, None, None, None) == pk.FFTB_ERR_INVALID
    assert L.fftb_apply_potential(h, C.c_void_p(16), None, C.c_void_p(16), C.c_void_p(16),
                                  None) == pk.FFTB_ERR_INVALID
    assert b"potential" in L.fftb_last_error()
    assert L.fftb_plan_destroy(h) == 0
    assert L.fftb_plan_destroy(None) == 0


def test_tiling_fits_lds():
    # every recipe gets a tiling whose LDS fits (checked inside the library)
    for name in ("c1", "c2", "c3", "c4", "c5"):
        w = synth.make_workload(name, nbands=1, nkpts=1)
        for dt in ("c128", "c64"):
            p = host_plan(w.dims, [w.spheres[0].lin], nb=synth.RECIPES[name]["nb"], dtype=dt)
            for d in ("inv", "fwd"):
                t = p.info["tuning"][d]
                assert w.dims[1] % t["y_classes"] == 0
                assert t["band_chunk"] & (t["band_chunk"] - 1) == 0


def test_default_tiling_c2():
    # the measured default for the 128^3, |G|<=32, 256-band complex128 shape:
    # band-inner lines (path 3: one 128-byte piece of 8 bands per row of
    # lanes); the inverse folds 8 classes of 16 (one workgroup per CU, so 512
    # threads), the forward writes partials of 16 classes of 8 (two
    # workgroups per CU, 256 threads)
    w = synth.make_workload("c2", nbands=1)
    p = host_plan(w.dims, [w.spheres[0].lin], nb=256, dtype="c128")
    inv, fwd = p.info["tuning"]["inv"], p.info["tuning"]["fwd"]
    assert (inv["band_chunk"], inv["y_classes"], inv["threads"], inv["path"]) == (8, 8, 512, 3)
    assert (fwd["band_chunk"], fwd["y_classes"], fwd["threads"], fwd["acc"], fwd["path"]) == \
        (8, 16, 256, 3, 3)
    # the register path of lines over 16 lanes stays selectable
    p = host_plan(w.dims, [w.spheres[0].lin], nb=256, dtype="c128", tuning=dict(path=2))
    assert p.info["tuning"]["inv"]["path"] == 2 and p.info["tuning"]["inv"]["lanes"] == 16
    # an explicit thread count is kept
    p = host_plan(w.dims, [w.spheres[0].lin], nb=256, dtype="c128", tuning=dict(threads=256))
    assert p.info["tuning"]["inv"]["threads"] == 256


def test_half_piece_inverse_tiling():
    # complex64 inverse band chunk of half a 128-byte piece: the band-inner
    # plane kernel on 8 bands per row of lanes, folding classes of 32; the
    # forward and the column kernel keep whole pieces. complex128 has no such
    # form (4 bands per row measured slower): its half chunk takes the
    # register-line path
    w = synth.make_workload("c5", nbands=1)
    lins = [s.lin for s in w.spheres]
    p = host_plan(w.dims, lins, nb=128, dtype="c64", tuning=dict(inv_band_chunk=8))
    inv, fwd = p.info["tuning"]["inv"], p.info["tuning"]["fwd"]
    assert (inv["band_chunk"], inv["y_classes"], inv["path"]) == (8, 5, 3), inv
    assert (fwd["band_chunk"], fwd["path"]) == (16, 3), fwd
    p = host_plan(w.dims, lins, nb=128, dtype="c128", tuning=dict(inv_band_chunk=4))
    assert p.info["tuning"]["inv"]["path"] != 3
    # x lengths without a half-piece line shape fall back to another path
    m2, lin2 = synth.sphere_map((30, 24, 36), (7, 6, 8))
    p = host_plan((30, 24, 36), [lin2], nb=8, dtype="c64", tuning=dict(inv_band_chunk=8))
    assert p.info["tuning"]["inv"]["path"] != 3
    _expect_status(pk.FFTB_ERR_UNSUPPORTED,
                   lambda: host_plan((30, 24, 36), [lin2], nb=8, dtype="c64",
                                     tuning=dict(inv_band_chunk=8, path=3)))


def test_inverse_class_pairs_tiling():
    # the inverse folds two y classes per task (r and r + n1/2) where n1 is
    # even and the classes have 16 rows; one class per task on request
    w = synth.make_workload("c2", nbands=1)
    for dt in ("c128", "c64"):
        p = host_plan(w.dims, [w.spheres[0].lin], nb=256, dtype=dt, tuning=dict(inv_acc=2))
        inv = p.info["tuning"]["inv"]
        assert (inv["y_classes"], inv["acc"], inv["path"]) == (8, 2, 3), inv
        p = host_plan(w.dims, [w.spheres[0].lin], nb=256, dtype=dt, tuning=dict(inv_acc=1))
        assert p.info["tuning"]["inv"]["acc"] == 1
    # classes of 8 cannot pair
    _expect_status(pk.FFTB_ERR_UNSUPPORTED,
                   lambda: host_plan(w.dims, [w.spheres[0].lin], nb=256, dtype="c128",
                                     tuning=dict(inv_acc=2, inv_y_classes=16)))


def test_mfma_flag_validation():
    m, lin = synth.sphere_map((128, 16, 128), (20, 4, 20))
    p = pk.Plan((128, 16, 128), [lin], 16, dtype="c64", flags=pk.PLAN_HOST_ONLY | pk.PLAN_MFMA)
    assert p.info["flags"] & pk.PLAN_MFMA
    # FP64 has no matrix-core DFT_16 stage; a plan without a 16-value lane has none either
    _expect_status(pk.FFTB_ERR_UNSUPPORTED,
                   lambda: pk.Plan((128, 16, 128), [lin], 16, dtype="c128",
                                   flags=pk.PLAN_HOST_ONLY | pk.PLAN_MFMA))
    # classes of 16 give the inverse fold's length-16 transforms to the matrix
    # cores on any x and z (band-inner lines)
    m2, lin2 = synth.sphere_map((96, 16, 96), (20, 4, 20))
    p = pk.Plan((96, 16, 96), [lin2], 16, dtype="c64", flags=pk.PLAN_HOST_ONLY | pk.PLAN_MFMA)
    assert p.info["tuning"]["inv"]["path"] == 3
    # neither classes of 16 nor 128-point lines: no stage for the matrix cores
    m3, lin3 = synth.sphere_map((96, 24, 96), (20, 5, 20))
    _expect_status(pk.FFTB_ERR_UNSUPPORTED,
                   lambda: pk.Plan((96, 24, 96), [lin3], 16, dtype="c64",
                                   flags=pk.PLAN_HOST_ONLY | pk.PLAN_MFMA))


def test_cuboid_plan_tables():
    """The batched cuboid transform: every grid point is a coefficient."""
    dims = (12, 10, 6)
    p = pk.Plan.cuboid(dims, 3, flags=pk.PLAN_HOST_ONLY)
    n = dims[0] * dims[1] * dims[2]
    assert p.info["total_coeffs"] == n
    assert p.info["sphere_elems"] == p.info["grid_elems"] == n * 3
    assert p.info["total_columns"] == dims[0] * dims[1]
    assert p.info["max_slab"] == dims[0]
    _expect_status(pk.FFTB_ERR_INVALID, lambda: pk.Plan.cuboid((12, 0, 6), 3, flags=pk.PLAN_HOST_ONLY))
    _expect_status(pk.FFTB_ERR_INVALID, lambda: pk.Plan.cuboid(dims, 0, flags=pk.PLAN_HOST_ONLY))
    _expect_status(pk.FFTB_ERR_UNSUPPORTED, lambda: pk.Plan.cuboid((14, 10, 6), 3, flags=pk.PLAN_HOST_ONLY))


def test_generic_path_threads_clamped():
    """The LDS-stage kernels are compiled for at most 256 threads: a 512-thread
    request on a grid without register shapes (64^3) is clamped at plan time."""
    m, lin = synth.sphere_map((64, 64, 64), (16, 16, 16))
    p = host_plan((64, 64, 64), [lin], nb=8, tuning=dict(threads=512))
    for d in ("inv", "fwd"):
        t = p.info["tuning"][d]
        assert t["path"] == 1 and t["threads"] == 256, t


def test_device_byte_cap_gives_nomem(monkeypatch):
    """FFTB_MAX_DEVICE_BYTES bounds a plan's device memory; a plan whose
    scratch would exceed it fails with FFTB_ERR_NOMEM before any device call
    (so this runs on a machine without a GPU)."""
    monkeypatch.setenv("FFTB_MAX_DEVICE_BYTES", "4096")
    m, lin = synth.sphere_map((32, 32, 32), (8, 8, 8))
    with pytest.raises(fb.FftbError) as ex:
        pk.Plan((32, 32, 32), [lin], 4, flags=0, stream=0)
    assert ex.value.status == pk.FFTB_ERR_NOMEM
    assert b"FFTB_MAX_DEVICE_BYTES" in pk.lib().fftb_last_error()


def test_plan_log(monkeypatch, capfd):
    """FFTB_LOG prints a plan summary (dims, tiling of both directions) on stderr."""
    monkeypatch.setenv("FFTB_LOG", "1")
    m, lin = synth.sphere_map((32, 32, 32), (8, 8, 8))
    host_plan((32, 32, 32), [lin], nb=4)
    err = capfd.readouterr().err
    assert "fftb plan: grid 32x32x32" in err
    assert "inverse: band chunk" in err and "forward: band chunk" in err
    monkeypatch.setenv("FFTB_LOG", "0")
    host_plan((32, 32, 32), [lin], nb=4)
    assert "fftb plan" not in capfd.readouterr().err


def test_plan_tables_under_sanitizers(tmp_path):
    """plan.cpp (the host table builder) compiled with g++ and the address and
    undefined-behaviour sanitizers, run on spheres, ellipsoids, permuted and
    malformed maps, and every 2,3,5-smooth axis length up to 400."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "plan_check"
    src = os.path.join(ROOT, "tests", "native", "plan_check.cpp")
    plan = os.path.join(ROOT, "paper_2406_05577_amd", "csrc", "plan.cpp")
    subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", src, plan, "-o", str(exe)], check=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    assert "plan_check OK" in res.stdout
