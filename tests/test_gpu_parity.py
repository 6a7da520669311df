"""GPU parity: the HIP path against the FP64 oracle, element by element.

Bars: relative L2 error <= 1e-12 for complex128 and <= 5e-6 for complex64
(E_inv: grid vs oracle inverse; E_fwd: GPU forward of the oracle grid vs the
oracle forward; E_rt: GPU round trip vs the input). Outputs start as NaN so an
element the kernels never write fails the check.
"""
import numpy as np
import pytest

import synth
from gpu_util import TOL, check_workload, rel

pytestmark = pytest.mark.gpu

# dims, semi-axes, k-points, bands, seed -- mixed radix, ellipsoids, k != 0,
# ragged band counts (odd Nb exercises band-chunk tails)
CASES = [
    ((6, 5, 4), (1.6, 1.3, 1.1), [(0.31, -0.22, 0.4)], 3, 1),
    ((12, 10, 15), (3.9, 3.2, 5.1), [(0.2, 0.35, -0.41), (-0.1, 0.0, 0.3)], 7, 2),
    ((8, 9, 10), (2.7, 3.1, 2.2), [(-0.45, 0.12, 0.05)], 1, 3),
    ((4, 4, 4), (1, 1, 1), [(0.0, 0.0, 0.0)], 5, 4),
    ((16, 18, 20), (4.2, 4.4, 4.9), [(0.1, -0.3, 0.2)], 17, 5),
    ((30, 24, 36), (7.1, 5.9, 8.8), [(0.05, 0.4, -0.2), (0.3, 0.3, 0.3), (0, 0, 0)], 9, 6),
]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("path", [0, 1])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_small_default(case, path, dtype):
    dims, semi, kpts, nb, seed = CASES[case]
    w = synth.small_workload(dims, semi, kpts, nb, seed=seed, shuffle=(case % 2 == 1))
    e = check_workload(w, dtype, tuning=dict(path=path) if path else None)
    print(case, path, dtype, e)
    assert max(e) <= TOL[dtype], e


# grids whose x and z lengths have register-line shapes (32, 96, 128, 144, 180)
REG_CASES = [
    ((32, 32, 32), (8, 8, 8), [(0.0, 0.0, 0.0)], 5, 11),
    ((96, 96, 96), (24, 24, 24), [(0.21, -0.33, 0.1), (-0.4, 0.05, 0.45)], 3, 12),
    ((128, 128, 128), (32, 32, 32), [(0.0, 0.0, 0.0)], 2, 13),
    ((144, 160, 180), (36, 40, 45), [(0.12, -0.3, 0.27)], 2, 14),
]
REG_TUNINGS = [None, dict(fwd_acc=2), dict(fwd_acc=1, fwd_band_chunk=2, fwd_splits=3),
               dict(y_classes=16, fwd_y_classes=16), dict(band_chunk=2, col_tile=3, fwd_band_chunk=4),
               dict(fwd_splits=5, threads=512), dict(fwd_acc=3, y_classes=16, threads=512),
               dict(fwd_acc=3, fwd_band_chunk=2, fwd_col_tile=5)]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("ti", range(len(REG_TUNINGS)))
@pytest.mark.parametrize("case", range(len(REG_CASES)))
def test_register_path(case, ti, dtype):
    dims, semi, kpts, nb, seed = REG_CASES[case]
    t = REG_TUNINGS[ti]
    if t and "y_classes" in t and dims[1] % 8:
        pytest.skip("class count does not divide ny")
    w = synth.small_workload(dims, semi, kpts, nb, seed=seed, shuffle=(case % 2 == 0))
    tun = dict(t or {})
    tun["path"] = 2
    try:
        e = check_workload(w, dtype, tuning=tun)
    except Exception as ex:  # a tiling that does not fit is reported, not run
        if "does not fit" in str(ex) or "no register-path" in str(ex):
            pytest.skip(str(ex))
        raise
    print(dims, t, dtype, e)
    assert max(e) <= TOL[dtype], (t, e)


@pytest.mark.parametrize("flags", [0, 5])
@pytest.mark.parametrize("case", range(len(REG_CASES)))
def test_band_inner_half_pieces(case, flags):
    """Band-inner lines with the complex64 inverse plane kernel on half a
    128-byte piece of bands per row of lanes (8 bands; x lines over 8
    positions, the fold over classes of 16 or 32), ragged band counts, plain
    and persistent + graph replays; then the fused potential step."""
    import oracle
    import torch
    from gpu_util import make_plan, to_device, split_sphere
    dtype = "c64"
    dims, semi, kpts, nb, seed = REG_CASES[case]
    w = synth.small_workload(dims, semi, kpts, nb + 5, seed=seed, shuffle=True)
    half = 8
    tun = dict(path=3, inv_band_chunk=half)
    p = make_plan(w, dtype=dtype, flags=flags, tuning=tun)
    inv = p.info["tuning"]["inv"]
    assert inv["path"] == 3 and inv["band_chunk"] == half, inv
    assert p.info["tuning"]["fwd"]["band_chunk"] == 2 * half
    p.close()
    e = check_workload(w, dtype, flags=flags, tuning=tun, reps=2)
    print(dims, dtype, flags, inv, e)
    assert max(e) <= TOL[dtype], e
    # the potential-weighted variant of the same kernel
    npdt, rdt = np.complex64, np.float32
    v = np.random.default_rng(78).standard_normal(dims[::-1]).astype(rdt)
    coeffs = [c.astype(npdt) for c in w.coeffs]
    p = make_plan(w, dtype=dtype, flags=flags, tuning=tun)
    sph = to_device(np.concatenate([c.reshape(-1) for c in coeffs]), dtype)
    out = p.apply_potential(sph, torch.from_numpy(v.reshape(-1)).to("cuda"))
    torch.cuda.synchronize()
    for s, c, o in zip(w.spheres, coeffs, split_sphere(w, out.cpu().numpy())):
        ref = oracle.apply_potential(dims, s.lin, c.astype(np.complex128), v.astype(np.float64))
        assert rel(o, ref) <= TOL[dtype], (rel(o, ref), dtype, flags)
    p.close()


PAIR_VARIANTS = [
    # (tuning, flags): class pairs (the default where they apply), pairs at 256
    # threads (lines past the register lines take the overflow scratch),
    # pairs persistent + graph replayed, one class per task
    (dict(path=3, inv_acc=2), 0),
    (dict(path=3, inv_acc=2, inv_threads=256), 0),
    (dict(path=3, inv_acc=2), 5),
    (dict(path=3, inv_acc=1), 0),
]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("vi", range(len(PAIR_VARIANTS)))
@pytest.mark.parametrize("case", range(len(REG_CASES)))
def test_band_inner_class_pairs(case, vi, dtype):
    """Inverse plane tasks folding two y classes r and r + n1/2 from the same
    column reads (the second class's lines waiting in registers or in the
    overflow scratch), against the oracle; then the fused potential step."""
    import oracle
    import torch
    from gpu_util import make_plan, to_device, split_sphere
    dims, semi, kpts, nb, seed = REG_CASES[case]
    tun, flags = PAIR_VARIANTS[vi]
    w = synth.small_workload(dims, semi, kpts, nb + 9, seed=seed + 40, shuffle=True)
    p = make_plan(w, dtype=dtype, flags=flags, tuning=tun)
    inv = p.info["tuning"]["inv"]
    assert inv["path"] == 3 and inv["acc"] == tun["inv_acc"], inv
    p.close()
    e = check_workload(w, dtype, flags=flags, tuning=tun, reps=2)
    print(dims, dtype, tun, flags, e)
    assert max(e) <= TOL[dtype], e
    npdt = np.complex128 if dtype == "c128" else np.complex64
    rdt = np.float64 if dtype == "c128" else np.float32
    v = np.random.default_rng(79).standard_normal(dims[::-1]).astype(rdt)
    coeffs = [c.astype(npdt) for c in w.coeffs]
    p = make_plan(w, dtype=dtype, flags=flags, tuning=tun)
    sph = to_device(np.concatenate([c.reshape(-1) for c in coeffs]), dtype)
    out = p.apply_potential(sph, torch.from_numpy(v.reshape(-1)).to("cuda"))
    torch.cuda.synchronize()
    for s, c, o in zip(w.spheres, coeffs, split_sphere(w, out.cpu().numpy())):
        ref = oracle.apply_potential(dims, s.lin, c.astype(np.complex128), v.astype(np.float64))
        assert rel(o, ref) <= TOL[dtype], (rel(o, ref), dtype, tun)
    p.close()


TUNINGS = [
    dict(band_chunk=1), dict(band_chunk=2, threads=64), dict(band_chunk=4, col_tile=3),
    dict(band_chunk=16, threads=128), dict(y_classes=2, x_rows=1), dict(y_classes=5, x_rows=2),
    dict(y_classes=10), dict(band_chunk=8, y_classes=1, x_rows=1, col_tile=1),
]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("ti", range(len(TUNINGS)))
def test_tunings(ti, dtype):
    dims, semi, kpts, nb, seed = CASES[1]
    w = synth.small_workload(dims, semi, kpts, nb, seed=seed, shuffle=True)
    e = check_workload(w, dtype, tuning=TUNINGS[ti])
    assert max(e) <= TOL[dtype], (TUNINGS[ti], e)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("flags", [1, 4, 5])
@pytest.mark.parametrize("which", [0, 1])
def test_batched_and_graph(which, flags, dtype):
    if which == 0:
        dims, semi, kpts, nb, seed = CASES[5]
    else:
        dims, semi, kpts, nb, seed = REG_CASES[1]
    w = synth.small_workload(dims, semi, kpts, nb, seed=seed)
    e = check_workload(w, dtype, flags=flags, reps=3)
    assert max(e) <= TOL[dtype], (flags, e)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("case", ["small"] + [f"reg{i}" for i in range(4)])
def test_forward_not_band_limited(case, dtype):
    """The forward of a dense random grid (not band-limited) is the exact
    gather of its full 3D DFT: a small mixed-radix grid, and the register
    line shapes of the benchmark grids (32^3, 96^3, 128^3, 144x160x180)."""
    if case == "small":
        dims, semi, kpts, nb, seed = CASES[4]
    else:
        dims, semi, kpts, nb, seed = REG_CASES[int(case[3:])]
        kpts = kpts[:1]
    w = synth.small_workload(dims, semi, kpts, nb, seed=seed)
    g = [synth.random_grid(np.random.default_rng(99), dims, nb)]
    e = check_workload(w, dtype, grid_in=g)
    print(case, dtype, e)
    assert e[1] <= TOL[dtype], e


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("holes", ["columns", "coeffs"])
def test_map_with_holes(dtype, holes):
    """Maps that are not a convex cutoff sphere: whole columns removed (slabs
    whose y values form more than two runs, which takes the generic fold), or
    single coefficients removed at random (columns with gaps along z)."""
    dims, semi = (64, 32, 48), (20, 10, 15)
    m, lin = synth.sphere_map(dims, semi, (0.2, -0.3, 0.1))
    nx, ny, _ = dims
    x, y = lin % nx, (lin // nx) % ny
    if holes == "columns":
        keep = ((x * 7 + y * 3) % 5) != 0
    else:
        keep = np.random.default_rng(5).random(lin.shape[0]) > 0.3
    lin = np.ascontiguousarray(lin[keep])
    rng = np.random.default_rng(11)
    nb = 12
    c = synth.draw_coefficients(rng, lin.shape[0], nb)
    dt = np.complex128 if dtype == "c128" else np.complex64
    w = synth.Workload(name="holes", dims=dims, spheres=[synth.Sphere(m=m[keep], lin=lin, kpt=(0, 0, 0), nbands=nb)],
                       coeffs=[c.astype(dt)], dtype=np.dtype(dt), seed=11)
    for tun in (None, dict(y_classes=4, fwd_y_classes=2), dict(y_classes=2, band_chunk=4)):
        e = check_workload(w, dtype, tuning=tun)
        assert max(e) <= TOL[dtype], (tun, e)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_directions_keep_their_scratch(dtype):
    """Forward calls with another band chunk than the inverse must leave the
    inverse's results unchanged: inverse, forward, inverse again, bit for bit."""
    import torch
    from gpu_util import make_plan, to_device
    dims, semi, kpts, nb, seed = REG_CASES[0]
    w = synth.small_workload(dims, semi, kpts, 6, seed=seed)
    p = make_plan(w, dtype=dtype, tuning=dict(band_chunk=8, fwd_band_chunk=2))
    npdt = np.complex128 if dtype == "c128" else np.complex64
    sph = to_device(np.concatenate([c.astype(npdt).reshape(-1) for c in w.coeffs]), dtype)
    g1 = p.sphere_to_grid(sph)
    back = p.grid_to_sphere(g1)
    g2 = p.sphere_to_grid(back)
    g3 = p.sphere_to_grid(sph)
    torch.cuda.synchronize()
    assert torch.equal(g1, g3)
    assert torch.isfinite(g2).all()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_full_cube_map(dtype):
    """A map holding every grid point (the padded-cube comparator: no pruning
    left, every column and slab occupied) against the oracle."""
    dims = (16, 12, 10)
    lin = np.arange(dims[0] * dims[1] * dims[2], dtype=np.int32)
    lin = lin[np.random.default_rng(3).permutation(lin.shape[0])]
    nx, ny = dims[0], dims[1]
    m = np.stack([lin % nx, (lin // nx) % ny, lin // (nx * ny)], axis=1).astype(np.int64)
    nb = 6
    c = synth.draw_coefficients(np.random.default_rng(4), lin.shape[0], nb)
    dt = np.complex128 if dtype == "c128" else np.complex64
    w = synth.Workload(name="cube", dims=dims, spheres=[synth.Sphere(m=m, lin=lin, kpt=(0, 0, 0), nbands=nb)],
                       coeffs=[c.astype(dt)], dtype=np.dtype(dt), seed=4)
    e = check_workload(w, dtype)
    assert max(e) <= TOL[dtype], e


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("flags", [0, 1, 5])
@pytest.mark.parametrize("case", [0, 1])
def test_apply_potential(case, flags, dtype):
    """Fused real-space step c' = grid_to_sphere(V * sphere_to_grid(c)) against
    the oracle, twice in a row (graph / persistent replays), for several
    spheres sharing one potential; the work grid holds V * psi."""
    import oracle
    import torch
    from gpu_util import make_plan, to_device, split_grid, split_sphere
    dims, semi, kpts, nb, seed = (CASES[5] if case == 0 else REG_CASES[1])
    w = synth.small_workload(dims, semi, kpts, nb, seed=seed, shuffle=True)
    nx, ny, nz = dims
    npdt = np.complex128 if dtype == "c128" else np.complex64
    rdt = np.float64 if dtype == "c128" else np.float32
    v = np.random.default_rng(77).standard_normal((nz, ny, nx)).astype(rdt)
    coeffs = [c.astype(npdt) for c in w.coeffs]
    p = make_plan(w, dtype=dtype, flags=flags)
    sph = to_device(np.concatenate([c.reshape(-1) for c in coeffs]), dtype)
    vt = torch.from_numpy(v.reshape(-1)).to("cuda")
    grid = torch.empty(p.info["grid_elems"], dtype=sph.dtype, device="cuda")
    for _ in range(2):
        out = p.apply_potential(sph, vt, grid=grid)
        torch.cuda.synchronize()
        got = split_sphere(w, out.cpu().numpy())
        gg = split_grid(w, grid.cpu().numpy())
        for s, c, o, g in zip(w.spheres, coeffs, got, gg):
            c64 = c.astype(np.complex128)
            ref = oracle.apply_potential(dims, s.lin, c64, v.astype(np.float64))
            assert rel(o, ref) <= TOL[dtype], (rel(o, ref), dtype, flags)
            gref = oracle.sphere_to_grid(dims, s.lin, c64) * v.astype(np.float64)[..., None]
            assert rel(g, gref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_cuboid_plan(dtype):
    """fftb_plan_create_cuboid: the batched 3D FFT of cuboid grids, against
    the oracle with the whole grid as the map (and both directions)."""
    import oracle
    import torch
    from gpu_util import to_device
    from paper_2406_05577_amd import Plan
    dims, nb = (24, 20, 18), 5
    nx, ny, nz = dims
    n = nx * ny * nz
    rng = np.random.default_rng(21)
    npdt = np.complex128 if dtype == "c128" else np.complex64
    a = (rng.standard_normal((n, nb)) + 1j * rng.standard_normal((n, nb))).astype(npdt)
    p = Plan.cuboid(dims, nb, dtype=dtype)
    g = p.sphere_to_grid(to_device(a, dtype))
    back = p.grid_to_sphere(g)
    torch.cuda.synchronize()
    lin = np.arange(n)
    ref = oracle.sphere_to_grid(dims, lin, a.astype(np.complex128))
    assert rel(g.cpu().numpy().reshape(nz, ny, nx, nb), ref) <= TOL[dtype]
    assert rel(back.cpu().numpy().reshape(n, nb), a.astype(np.complex128)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("dims", [(1, 6, 10), (8, 1, 9), (10, 6, 1), (1, 1, 12)])
def test_degenerate_dims(dims, dtype):
    """Grids with an axis of length 1 (a plane, a line): the transforms along
    that axis are the identity."""
    semi = tuple(max(d / 3.0, 0.5) for d in dims)
    w = synth.small_workload(dims, semi, [(0.0, 0.0, 0.0)], 3, seed=31)
    e = check_workload(w, dtype)
    assert max(e) <= TOL[dtype], e


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_single_coefficient_sphere(dtype):
    """Ns = 1 (only G = 0): the grid is constant, the round trip exact."""
    lin = np.array([0], np.int32)
    dims = (12, 10, 8)
    c = synth.draw_coefficients(np.random.default_rng(8), 1, 4)
    dt = np.complex128 if dtype == "c128" else np.complex64
    w = synth.Workload(name="one", dims=dims, spheres=[synth.Sphere(m=np.zeros((1, 3), np.int64), lin=lin,
                       kpt=(0, 0, 0), nbands=4)], coeffs=[c.astype(dt)], dtype=np.dtype(dt), seed=8)
    e = check_workload(w, dtype)
    assert max(e) <= TOL[dtype], e


def test_c1_full():
    w = synth.make_workload("c1")
    e = check_workload(w, "c128")
    print("c1", e)
    assert max(e) <= 1e-12, e


def test_c3alt_full():
    w = synth.make_workload("c3alt")
    e = check_workload(w, "c64")
    print("c3alt", e)
    assert max(e) <= 5e-6, e


def test_autotune_and_cache(tmp_path, monkeypatch):
    """FFTB_PLAN_AUTOTUNE times candidate tilings, keeps the fastest per
    direction (parity must hold for the pick) and caches it: a second plan on
    the same inputs reads the cache."""
    from gpu_util import make_plan
    monkeypatch.setenv("FFTB_TUNE_CACHE", str(tmp_path / "tune.txt"))
    dims, semi, kpts, nb, seed = REG_CASES[1]
    w = synth.small_workload(dims, semi, kpts, nb, seed=seed)
    for dtype in ("c128", "c64"):
        p = make_plan(w, dtype=dtype, flags=2)
        assert p.info["autotuned"] == 1
        tun = p.info["tuning"]
        p.close()
        p2 = make_plan(w, dtype=dtype, flags=2)
        assert p2.info["autotuned"] == 2 and p2.info["tuning"] == tun
        p2.close()
        e = check_workload(w, dtype, flags=2)
        assert max(e) <= TOL[dtype], e
    assert (tmp_path / "tune.txt").read_text().count("fftb-tune-v2") == 2


def test_autotune_budget(tmp_path, monkeypatch, capfd):
    """A tiny time budget stops the autotuner after its first trial; the plan
    keeps the best tiling found so far and stays correct; every trial prints
    a progress line."""
    from gpu_util import make_plan
    monkeypatch.setenv("FFTB_TUNE_CACHE", str(tmp_path / "tune.txt"))
    monkeypatch.setenv("FFTB_TUNE_SECONDS", "0.000001")
    dims, semi, kpts, nb, seed = REG_CASES[1]
    w = synth.small_workload(dims, semi, kpts, nb, seed=seed)
    p = make_plan(w, dtype="c64", flags=2)
    assert p.info["autotuned"] == 1
    p.close()
    err = capfd.readouterr().err
    assert err.count("fftb autotune 1/") == 1 and "fftb autotune 2/" not in err
    assert "1 of" in err
    e = check_workload(w, "c64", flags=2)
    assert max(e) <= TOL["c64"], e


@pytest.mark.parametrize("flags", [16, 16 | 1 | 4])
def test_mfma_radix16(flags):
    """complex64 with the in-lane DFT_16 stages on the matrix cores (FP32
    v_mfma_f32_32x32x2f32), against the FP64 oracle: 128-point register lines
    and the inverse fold of classes of 16 (128^3)."""
    dims, semi, kpts, nb, seed = REG_CASES[2]
    w = synth.small_workload(dims, semi, kpts, 5, seed=seed, shuffle=True)
    e = check_workload(w, "c64", flags=flags, reps=2)
    print("mfma", flags, e)
    assert max(e) <= TOL["c64"], e


MFMA_FOLD_CASES = [
    # the inverse fold's length-16 transforms on the matrix cores on the y axes
    # of 96 and 160 (classes of 16), one class and class pairs per task,
    # ragged bands, with the potential; 32^3 has a single class
    (REG_CASES[1], dict(inv_acc=2)),
    (REG_CASES[1], dict(inv_acc=1)),
    (REG_CASES[3], dict()),
    (REG_CASES[3], dict(inv_acc=2, inv_threads=256)),
    (REG_CASES[0], dict()),
]


@pytest.mark.parametrize("flags", [16, 16 | 1 | 4])
@pytest.mark.parametrize("ci", range(len(MFMA_FOLD_CASES)))
def test_mfma_fold(ci, flags):
    import oracle
    import torch
    from gpu_util import make_plan, to_device, split_sphere
    (dims, semi, kpts, nb, seed), tun = MFMA_FOLD_CASES[ci]
    w = synth.small_workload(dims, semi, kpts, nb + 11, seed=seed + 70, shuffle=True)
    p = make_plan(w, dtype="c64", flags=flags, tuning=tun or None)
    assert p.info["flags"] & 16 and p.info["tuning"]["inv"]["path"] == 3, p.info["tuning"]
    p.close()
    e = check_workload(w, "c64", flags=flags, tuning=tun or None, reps=2)
    print("mfma fold", dims, tun, flags, e)
    assert max(e) <= TOL["c64"], e
    v = np.random.default_rng(80).standard_normal(dims[::-1]).astype(np.float32)
    coeffs = [c.astype(np.complex64) for c in w.coeffs]
    p = make_plan(w, dtype="c64", flags=flags, tuning=tun or None)
    sph = to_device(np.concatenate([c.reshape(-1) for c in coeffs]), "c64")
    out = p.apply_potential(sph, torch.from_numpy(v.reshape(-1)).to("cuda"))
    torch.cuda.synchronize()
    for s, c, o in zip(w.spheres, coeffs, split_sphere(w, out.cpu().numpy())):
        ref = oracle.apply_potential(dims, s.lin, c.astype(np.complex128), v.astype(np.float64))
        assert rel(o, ref) <= TOL["c64"], (rel(o, ref), tun, flags)
    p.close()
