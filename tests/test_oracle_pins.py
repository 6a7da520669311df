"""Pins for the FP64 oracle: checks that do not reuse the oracle's own formula.

P1 brute-force triple sums (Section 2.1, 3D DFT as one dense matrix)
P2 single coefficient -> plane wave (closed form)
P3 grid delta -> pure phases (closed form)
P4 constant grid -> only G = 0 survives (closed form)
P5 Parseval
P6 round trip is the identity
P7 numpy.fft (pocketfft) special case
P8 shift theorem; real psi <=> conjugate-symmetric c at Gamma
P9 axis order does not matter (Section 2.1: the 1D stages may be permuted)
plus hand-derived DFT_n entries (tests/golden/dft_small.txt) and checks that
plausible mistakes planted in the oracle are caught by these pins.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import pwfft
from synth import sphere_map, small_workload, random_grid

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

TINY = [
    # dims, semi-axes, k-point
    ((4, 4, 4), (1, 1, 1), (0.0, 0.0, 0.0)),
    ((6, 5, 4), (1.6, 1.3, 1.1), (0.31, -0.22, 0.4)),
    ((8, 9, 10), (2.7, 3.1, 2.2), (-0.45, 0.12, 0.05)),
    ((12, 10, 15), (3.9, 3.2, 5.1), (0.2, 0.35, -0.41)),
]


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _case(i, nb=3, shuffle=False):
    dims, semi, k = TINY[i]
    w = small_workload(dims, semi, [k], nb, seed=100 + i, shuffle=shuffle)
    return w.dims, w.spheres[0], w.coeffs[0]


# --- DFT matrix: hand-derived entries --------------------------------------

def test_dft_matrix_golden_entries():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "dft_small.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) > 20
    for n, l, k, re, im in rows:
        f = oracle.dft_matrix(int(n), -1)
        got = f[int(l), int(k)]
        assert abs(got - complex(float(re), float(im))) < 1e-15, (n, l, k, got)


def test_dft_matrix_unitary_and_inverse_sign():
    for n in (1, 2, 3, 5, 7, 12, 30):
        f = oracle.dft_matrix(n, -1)
        g = oracle.dft_matrix(n, +1)
        np.testing.assert_allclose(f @ g, n * np.eye(n), atol=1e-12 * n)
        np.testing.assert_allclose(g, np.conj(f), atol=0)


# --- P1: brute force --------------------------------------------------------

@pytest.mark.parametrize("i", range(len(TINY)))
def test_p1_brute_force_inverse(i):
    dims, s, c = _case(i)
    got = oracle.sphere_to_grid(dims, s.lin, c)
    ref = oracle.brute_sphere_to_grid(dims, s.m, c)
    assert rel(got, ref) < 1e-13


@pytest.mark.parametrize("i", range(len(TINY)))
def test_p1_brute_force_forward(i):
    dims, s, c = _case(i)
    g = random_grid(np.random.default_rng(7 + i), dims, 2)
    got = oracle.grid_to_sphere(dims, s.lin, g)
    ref = oracle.brute_grid_to_sphere(dims, s.m, g)
    assert rel(got, ref) < 1e-13


# --- P2..P4: closed forms ----------------------------------------------------

@pytest.mark.parametrize("i", range(len(TINY)))
def test_p2_single_coefficient_is_plane_wave(i):
    dims, s, _ = _case(i)
    nx, ny, nz = dims
    gi = s.ns // 3
    c = np.zeros((s.ns, 1), complex)
    c[gi, 0] = 1.0
    psi = oracle.sphere_to_grid(dims, s.lin, c)[..., 0]
    np.testing.assert_allclose(np.abs(psi), 1.0, atol=1e-14)
    mx, my, mz = s.m[gi]
    # ratio between neighbouring grid points along each axis is exp(+2 pi j m/n)
    np.testing.assert_allclose(psi[:, :, 1:] / psi[:, :, :-1], np.exp(2j * np.pi * mx / nx), atol=1e-13)
    np.testing.assert_allclose(psi[:, 1:, :] / psi[:, :-1, :], np.exp(2j * np.pi * my / ny), atol=1e-13)
    np.testing.assert_allclose(psi[1:, :, :] / psi[:-1, :, :], np.exp(2j * np.pi * mz / nz), atol=1e-13)
    assert abs(psi[0, 0, 0] - 1.0) < 1e-15
    back = oracle.grid_to_sphere(dims, s.lin, psi[..., None])
    np.testing.assert_allclose(back, c, atol=1e-14)


@pytest.mark.parametrize("i", range(len(TINY)))
def test_p3_grid_delta(i):
    dims, s, _ = _case(i)
    nx, ny, nz = dims
    r0 = (nx - 1, 1 % ny, nz // 2)
    g = np.zeros((nz, ny, nx, 1), complex)
    g[r0[2], r0[1], r0[0], 0] = 1.0
    c = oracle.grid_to_sphere(dims, s.lin, g)[:, 0]
    n = nx * ny * nz
    expect = np.array([np.exp(-2j * np.pi * (mx * r0[0] / nx + my * r0[1] / ny + mz * r0[2] / nz))
                       for mx, my, mz in s.m]) / n
    np.testing.assert_allclose(c, expect, atol=1e-15)


@pytest.mark.parametrize("i", range(len(TINY)))
def test_p4_constant_grid(i):
    dims, s, _ = _case(i)
    g = np.full(tuple(reversed(dims)) + (1,), 2.5 - 1.0j)
    c = oracle.grid_to_sphere(dims, s.lin, g)[:, 0]
    zero = np.where((s.m == 0).all(axis=1))[0]
    expect = np.zeros(s.ns, complex)
    if zero.size:
        expect[zero[0]] = 2.5 - 1.0j
    np.testing.assert_allclose(c, expect, atol=1e-14)


# --- P5, P6: Parseval and round trip -----------------------------------------

@pytest.mark.parametrize("i", range(len(TINY)))
def test_p5_parseval(i):
    dims, s, c = _case(i)
    n = dims[0] * dims[1] * dims[2]
    psi = oracle.sphere_to_grid(dims, s.lin, c)
    np.testing.assert_allclose((np.abs(psi) ** 2).sum(axis=(0, 1, 2)),
                               n * (np.abs(c) ** 2).sum(axis=0), rtol=1e-13)
    g = random_grid(np.random.default_rng(3), dims, 2)
    cf = oracle.grid_to_sphere(dims, s.lin, g)
    lhs = (np.abs(cf) ** 2).sum(axis=0)
    rhs = (np.abs(g) ** 2).sum(axis=(0, 1, 2)) / n
    assert np.all(lhs <= rhs * (1 + 1e-13))


@pytest.mark.parametrize("i", range(len(TINY)))
@pytest.mark.parametrize("shuffle", [False, True])
def test_p6_round_trip(i, shuffle):
    dims, s, c = _case(i, shuffle=shuffle)
    back = oracle.grid_to_sphere(dims, s.lin, oracle.sphere_to_grid(dims, s.lin, c))
    assert rel(back, c) < 1e-14


# --- P7: library special case ---------------------------------------------------

@pytest.mark.parametrize("i", range(len(TINY)))
def test_p7_numpy_fft(i):
    dims, s, c = _case(i)
    nx, ny, nz = dims
    n = nx * ny * nz
    a = np.zeros((nz * ny * nx, c.shape[1]), complex)
    a[s.lin.astype(np.int64)] = c
    a = a.reshape(nz, ny, nx, -1)
    ref = n * np.fft.ifftn(a, axes=(0, 1, 2))
    assert rel(oracle.sphere_to_grid(dims, s.lin, c), ref) < 1e-13
    g = random_grid(np.random.default_rng(11), dims, 2)
    ref_f = np.fft.fftn(g, axes=(0, 1, 2)).reshape(n, -1)[s.lin.astype(np.int64)] / n
    assert rel(oracle.grid_to_sphere(dims, s.lin, g), ref_f) < 1e-13


# --- P8: shift theorem and conjugate symmetry --------------------------------------

@pytest.mark.parametrize("i", range(len(TINY)))
def test_p8_shift_theorem(i):
    dims, s, _ = _case(i)
    nx, ny, nz = dims
    g = random_grid(np.random.default_rng(21), dims, 1)
    r0 = (1, 2 % ny, 3 % nz)
    shifted = np.roll(g, shift=(r0[2], r0[1], r0[0]), axis=(0, 1, 2))
    c0 = oracle.grid_to_sphere(dims, s.lin, g)[:, 0]
    c1 = oracle.grid_to_sphere(dims, s.lin, shifted)[:, 0]
    ph = np.exp(-2j * np.pi * (s.m[:, 0] * r0[0] / nx + s.m[:, 1] * r0[1] / ny + s.m[:, 2] * r0[2] / nz))
    np.testing.assert_allclose(c1, c0 * ph, atol=1e-14)


def test_p8_real_wave_at_gamma():
    dims = (8, 6, 10)
    m, lin = sphere_map(dims, (2.5, 2.0, 3.5))
    rng = np.random.default_rng(5)
    c = (rng.standard_normal((m.shape[0], 2)) + 1j * rng.standard_normal((m.shape[0], 2)))
    idx = {tuple(v): i for i, v in enumerate(m)}
    # make c(-G) = conj c(G)
    for i, v in enumerate(m):
        j = idx[tuple(-v)]
        if j < i:
            c[i] = np.conj(c[j])
        elif j == i:
            c[i] = c[i].real
    psi = oracle.sphere_to_grid(dims, lin, c)
    assert np.abs(psi.imag).max() < 1e-12 * np.abs(psi).max()


# --- P9: axis order ----------------------------------------------------------------

@pytest.mark.parametrize("i", range(len(TINY)))
def test_p9_axis_order(i):
    dims, s, c = _case(i)
    a = oracle.sphere_to_grid(dims, s.lin, c, order="zyx")
    b = oracle.sphere_to_grid(dims, s.lin, c, order="xyz")
    d = oracle.sphere_to_grid(dims, s.lin, c, order="yxz")
    assert rel(a, b) < 1e-14 and rel(a, d) < 1e-14


# --- sphere maps (inputs) ------------------------------------------------------------

def _ball_count_by_columns(r):
    # independent count: sum over (mx, my) of the z-column length 2*floor(sqrt(r^2-mx^2-my^2))+1
    tot = 0
    for mx in range(-r, r + 1):
        for my in range(-r, r + 1):
            rem = r * r - mx * mx - my * my
            if rem >= 0:
                tot += 2 * math.isqrt(rem) + 1
    return tot


@pytest.mark.parametrize("r", [0, 1, 2, 3, 8, 17])
def test_sphere_counts(r):
    dims = (2 * r + 2,) * 3
    m, lin = sphere_map(dims, (r, r, r))
    assert m.shape[0] == _ball_count_by_columns(r)
    if r == 1:
        assert m.shape[0] == 7
    if r == 2:
        assert m.shape[0] == 33   # 1 + 6 + 12 + 8 + 6 by hand
    # canonical order: lexicographic (mx, my, mz), z fastest
    keys = m[:, 0] * 10 ** 6 + m[:, 1] * 10 ** 3 + m[:, 2]
    assert np.all(np.diff(keys) > 0)
    assert np.unique(lin).shape[0] == lin.shape[0]


def test_sphere_map_kpoint_shift_and_wrap():
    dims = (6, 5, 4)
    k = (0.31, -0.22, 0.4)
    m, lin = sphere_map(dims, (1.6, 1.3, 1.1), k)
    t = (((m + np.array(k)) / np.array([1.6, 1.3, 1.1])) ** 2).sum(axis=1)
    assert np.all(t <= 1.0)
    x, y, z = m[:, 0] % 6, m[:, 1] % 5, m[:, 2] % 4
    np.testing.assert_array_equal(lin, x + 6 * (y + 5 * z))
    with pytest.raises(ValueError):
        sphere_map((4, 4, 4), (2, 2, 2))


# --- planted mistakes are caught ---------------------------------------------------------

def _run_pins(s2g, g2s):
    """Run a subset of the pins on (possibly mutated) oracle functions; return
    True if all pass."""
    dims, s, c = _case(1)
    nx, ny, nz = dims
    n = nx * ny * nz
    try:
        ref = oracle.brute_sphere_to_grid(dims, s.m, c)
        if rel(s2g(dims, s.lin, c), ref) > 1e-13:
            return False
        g = random_grid(np.random.default_rng(1), dims, 2)
        if rel(g2s(dims, s.lin, g), oracle.brute_grid_to_sphere(dims, s.m, g)) > 1e-13:
            return False
        if rel(g2s(dims, s.lin, s2g(dims, s.lin, c)), c) > 1e-14:
            return False
        a = np.zeros((n, c.shape[1]), complex)
        a[s.lin.astype(np.int64)] = c
        if rel(s2g(dims, s.lin, c), n * np.fft.ifftn(a.reshape(nz, ny, nx, -1), axes=(0, 1, 2))) > 1e-13:
            return False
    except Exception:
        return False
    return True


# --- real-space potential step (Section 1) ----------------------------------

@pytest.mark.parametrize("i", range(len(TINY)))
def test_potential_constant_scales(i):
    """V = v0 everywhere multiplies every coefficient by v0 (closed form)."""
    dims, s, c = _case(i)
    nx, ny, nz = dims
    got = oracle.apply_potential(dims, s.lin, c, np.full((nz, ny, nx), 2.5))
    np.testing.assert_allclose(got, 2.5 * c, atol=1e-13 * np.abs(c).max())


@pytest.mark.parametrize("i", range(len(TINY)))
def test_potential_cosine_couples_neighbours(i):
    """V(x) = cos(2 pi x / nx) = (e^{+} + e^{-})/2 couples G to G -+ e_x
    (convolution theorem): c'(G) = (c(G - e_x) + c(G + e_x)) / 2, with
    coefficients outside the sphere counted as zero."""
    dims, s, c = _case(i)
    nx, ny, nz = dims
    x = np.arange(nx)
    v = np.broadcast_to(np.cos(2 * np.pi * x / nx), (nz, ny, nx))
    got = oracle.apply_potential(dims, s.lin, c, v)
    index = {tuple(int(q) for q in mm): g for g, mm in enumerate(s.m)}
    exp = np.zeros_like(c)
    for g, (mx, my, mz) in enumerate(s.m):
        for d in (-1, 1):
            h = index.get((int(mx) + d, int(my), int(mz)))
            if h is not None:
                exp[g] += 0.5 * c[h]
    np.testing.assert_allclose(got, exp, atol=1e-13 * np.abs(c).max())


@pytest.mark.parametrize("i", range(len(TINY)))
def test_potential_brute_force(i):
    """A random real V against the brute-force triple sums on both sides."""
    dims, s, c = _case(i)
    nx, ny, nz = dims
    v = np.random.default_rng(30 + i).standard_normal((nz, ny, nx))
    got = oracle.apply_potential(dims, s.lin, c, v)
    g = oracle.brute_sphere_to_grid(dims, s.m, c) * v[..., None]
    ref = oracle.brute_grid_to_sphere(dims, s.m, g)
    assert rel(got, ref) < 1e-13


def test_pins_pass_on_oracle():
    assert _run_pins(oracle.sphere_to_grid, oracle.grid_to_sphere)


def test_pins_catch_planted_mistakes(monkeypatch):
    mutants = []

    def wrong_sign(dims, lin, c):
        a = pwfft.scatter_sphere(dims, lin, c)
        for ax in "zyx":
            a = pwfft.axis_dft(a, ax, -1)
        return a
    mutants.append((wrong_sign, oracle.grid_to_sphere))

    def one_axis_wrong_sign(dims, lin, c):
        a = pwfft.scatter_sphere(dims, lin, c)
        for ax, sg in zip("zyx", (+1, -1, +1)):
            a = pwfft.axis_dft(a, ax, sg)
        return a
    mutants.append((one_axis_wrong_sign, oracle.grid_to_sphere))

    def dropped_axis(dims, lin, c):
        a = pwfft.scatter_sphere(dims, lin, c)
        for ax in "zx":
            a = pwfft.axis_dft(a, ax, +1)
        return a
    mutants.append((dropped_axis, oracle.grid_to_sphere))

    def no_norm(dims, lin, g):
        return oracle.grid_to_sphere(dims, lin, g) * np.prod(dims)
    mutants.append((oracle.sphere_to_grid, no_norm))

    def norm_by_ns(dims, lin, g):
        return oracle.grid_to_sphere(dims, lin, g) * np.prod(dims) / len(lin)
    mutants.append((oracle.sphere_to_grid, norm_by_ns))

    def transposed_layout(dims, lin, c):
        # x and y swapped in the linear index (x must be fastest)
        nx, ny, nz = dims
        lin = np.asarray(lin, np.int64)
        x, y, z = lin % nx, (lin // nx) % ny, lin // (nx * ny)
        lin2 = y + ny * (x + nx * z)
        a = np.zeros((nx * ny * nz, c.shape[1]), complex)
        a[lin2] = c
        a = a.reshape(nz, ny, nx, -1)
        for ax in "zyx":
            a = pwfft.axis_dft(a, ax, +1)
        return a
    mutants.append((transposed_layout, oracle.grid_to_sphere))

    def transposed_dft(dims, lin, c):
        # l*k replaced by l*(n-k): DFT matrix of the opposite sign on one axis via index flip
        a = pwfft.scatter_sphere(dims, lin, c)
        for ax in "zyx":
            f = pwfft.dft_matrix(a.shape[pwfft._AXIS[ax]], +1)[:, ::-1]
            a = np.moveaxis(np.tensordot(f, a, axes=([1], [pwfft._AXIS[ax]])), 0, pwfft._AXIS[ax])
        return a
    mutants.append((transposed_dft, oracle.grid_to_sphere))

    for s2g, g2s in mutants:
        assert not _run_pins(s2g, g2s), (s2g.__name__, g2s.__name__)
