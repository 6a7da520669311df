"""Seeded synthetic workloads for the plane-wave sphere<->grid transform.

This module only *generates inputs*: the sphere index maps (which plane-wave
vectors G lie inside the cutoff) and the seeded band coefficients. It holds no
part of the transform's arithmetic. Both the FP64 oracle tests and the GPU
path consume what it returns, so the two sides see byte-identical inputs.

Conventions (paper, Section 2.2 and Section 3.3):
  * A sphere keeps every integer G = (mx, my, mz) whose shifted, scaled norm
    sum(((m_i + k_i) / a_i)^2) is at most 1 (the cutoff test is inclusive,
    Section 2.2). At the Gamma point with equal integer semi-axes R the test is
    the exact integer test mx^2 + my^2 + mz^2 <= R^2.
  * Negative frequencies wrap around: the grid coordinate of m_i is m_i mod n_i.
    The wrapped linear index is x + nx * (y + ny * z) (x fastest, Section 2.1).
  * Canonical coefficient order is signed (mx, my, mz) lexicographic with z
    fastest, so each (x, y) column of the offset array is contiguous
    (Section 3.3 describes the xy-projection offset array).
  * Coefficients are complex Gaussians (re + i*im)/sqrt(2); the band index is
    the fastest-varying one in memory (Section 3.3).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED_BASE = 240605577


@dataclasses.dataclass
class Sphere:
    """One k-point's coefficient sphere."""
    m: np.ndarray          # (Ns, 3) int64 signed (mx, my, mz)
    lin: np.ndarray        # (Ns,) int32 wrapped linear index x + nx*(y + ny*z)
    kpt: Tuple[float, float, float]
    nbands: int

    @property
    def ns(self) -> int:
        return int(self.lin.shape[0])


def sphere_map(dims: Sequence[int], semi_axes: Sequence[float],
               kpt: Sequence[float] = (0.0, 0.0, 0.0)) -> Tuple[np.ndarray, np.ndarray]:
    """Integer G inside the (possibly shifted) ellipsoid, in canonical order.

    Returns (m, lin): m is (Ns, 3) int64 signed, lin is (Ns,) int32.
    Raises ValueError if the wrapped indices would collide (the sphere is wider
    than the grid along some axis).
    """
    nx, ny, nz = (int(d) for d in dims)
    ax, ay, az = (float(a) for a in semi_axes)
    kx, ky, kz = (float(k) for k in kpt)
    exact = (kx == 0.0 and ky == 0.0 and kz == 0.0 and ax == ay == az
             and float(ax).is_integer())
    rng_x = range(-int(math.ceil(ax + abs(kx))) - 1, int(math.ceil(ax + abs(kx))) + 2)
    rng_y = range(-int(math.ceil(ay + abs(ky))) - 1, int(math.ceil(ay + abs(ky))) + 2)
    rng_z = np.arange(-int(math.ceil(az + abs(kz))) - 1, int(math.ceil(az + abs(kz))) + 2,
                      dtype=np.int64)
    out = []
    if exact:
        r2 = int(ax) * int(ax)
        for mx in rng_x:
            for my in rng_y:
                rem = r2 - mx * mx - my * my
                if rem < 0:
                    continue
                sel = rng_z[rng_z * rng_z <= rem]
                for mz in sel:
                    out.append((mx, my, int(mz)))
    else:
        tz = ((rng_z.astype(np.float64) + kz) / az) ** 2
        for mx in rng_x:
            tx = ((mx + kx) / ax) ** 2
            for my in rng_y:
                ty = ((my + ky) / ay) ** 2
                sel = rng_z[(tx + ty) + tz <= 1.0]
                for mz in sel:
                    out.append((mx, my, int(mz)))
    m = np.asarray(out, dtype=np.int64).reshape(-1, 3)
    for i, n in enumerate((nx, ny, nz)):
        if m.shape[0] and (m[:, i].max() - m[:, i].min()) >= n:
            raise ValueError(f"sphere wider than grid along axis {i}")
    x = np.mod(m[:, 0], nx)
    y = np.mod(m[:, 1], ny)
    z = np.mod(m[:, 2], nz)
    lin = (x + nx * (y + ny * z)).astype(np.int64)
    if np.unique(lin).shape[0] != lin.shape[0]:
        raise ValueError("wrapped indices collide")
    return m, lin.astype(np.int32)


def draw_coefficients(rng: np.random.Generator, ns: int, nb: int) -> np.ndarray:
    """(Ns, Nb) complex128, re and im i.i.d. N(0, 1/2)."""
    v = rng.standard_normal((ns, nb, 2))
    return (v[..., 0] + 1j * v[..., 1]) / math.sqrt(2.0)


@dataclasses.dataclass
class Workload:
    name: str
    dims: Tuple[int, int, int]
    spheres: List[Sphere]
    coeffs: List[np.ndarray]   # per sphere, (Ns, Nb) in `dtype`
    dtype: np.dtype            # complex128 or complex64
    seed: int

    @property
    def ngrid(self) -> int:
        return self.dims[0] * self.dims[1] * self.dims[2]

    @property
    def nbands_total(self) -> int:
        return sum(s.nbands for s in self.spheres)

    def sphere_concat(self) -> np.ndarray:
        """All spheres' S[g][b] blocks concatenated, flat, in `dtype`."""
        return np.concatenate([c.reshape(-1) for c in self.coeffs])


# Workload recipes (grid dims, cutoff semi-axes, k-points, bands, dtype).
#   c1     32^3, |G|<=8, Gamma, 4 bands, complex128
#   c2     128^3, |G|<=32, Gamma, 256 bands, complex128, scaled by 1/(1+|G|^2)
#   c3     c2 shapes in complex64 (scaled like c2)
#   c3alt  c1 shapes with 256 bands in complex64
#   c4     96^3, 8 k-points in [-0.5,0.5)^3, |G+k|<=24, 64 bands each, complex64
#   c5     144x160x180, ellipsoid semi-axes (36,40,45), 4 k-points, 128 bands each
#   x1     256^3, |G|<=64 (the paper's experiment shape), Gamma, 256 bands, complex128
RECIPES = {
    "c1":    dict(dims=(32, 32, 32), semi=(8, 8, 8), nk=0, nb=4, dtype="c128", cidx=1, scale=False),
    "c2":    dict(dims=(128, 128, 128), semi=(32, 32, 32), nk=0, nb=256, dtype="c128", cidx=2, scale=True),
    "c3":    dict(dims=(128, 128, 128), semi=(32, 32, 32), nk=0, nb=256, dtype="c64", cidx=3, scale=True),
    "c3alt": dict(dims=(32, 32, 32), semi=(8, 8, 8), nk=0, nb=256, dtype="c64", cidx=3, scale=False),
    "c4":    dict(dims=(96, 96, 96), semi=(24, 24, 24), nk=8, nb=64, dtype="c64", cidx=4, scale=False),
    "c5":    dict(dims=(144, 160, 180), semi=(36, 40, 45), nk=4, nb=128, dtype="c64", cidx=5, scale=False),
    # the paper's experiment shape (Section 4.1): 256^3 grid, sphere diameter 128, 256 bands
    "x1":    dict(dims=(256, 256, 256), semi=(64, 64, 64), nk=0, nb=256, dtype="c128", cidx=6, scale=True),
}


def make_workload(name: str, dtype: Optional[str] = None, nbands: Optional[int] = None,
                  nkpts: Optional[int] = None) -> Workload:
    """Build a seeded workload. `dtype` overrides the recipe's precision (the
    values are drawn in FP64 and then rounded, so the draw does not depend on
    it). `nbands` / `nkpts` shrink the workload for quick tests (this changes
    the draw)."""
    r = RECIPES[name]
    seed = SEED_BASE + r["cidx"]
    rng = np.random.default_rng(seed)
    nk = r["nk"] if nkpts is None else min(nkpts, max(r["nk"], 1))
    if r["nk"] > 0:
        kpts = rng.uniform(-0.5, 0.5, (r["nk"], 3))[: max(nk, 1)]
    else:
        kpts = np.zeros((1, 3))
    nb = r["nb"] if nbands is None else int(nbands)
    dt = np.complex128 if (dtype or r["dtype"]) == "c128" else np.complex64
    spheres, coeffs = [], []
    for k in kpts:
        m, lin = sphere_map(r["dims"], r["semi"], tuple(k))
        c = draw_coefficients(rng, m.shape[0], nb)
        if r["scale"]:
            c = c / (1.0 + (m * m).sum(axis=1))[:, None]
        spheres.append(Sphere(m=m, lin=lin, kpt=tuple(float(v) for v in k), nbands=nb))
        coeffs.append(np.ascontiguousarray(c.astype(dt)))
    return Workload(name=name, dims=tuple(r["dims"]), spheres=spheres, coeffs=coeffs,
                    dtype=np.dtype(dt), seed=seed)


def small_workload(dims, semi, kpts, nb, seed, dtype="c128", shuffle=False) -> Workload:
    """A small seeded workload on arbitrary dims (tests of ragged / mixed-radix
    shapes). With shuffle=True each sphere's coefficient order is a seeded
    permutation of the canonical order."""
    rng = np.random.default_rng(seed)
    dt = np.complex128 if dtype == "c128" else np.complex64
    spheres, coeffs = [], []
    for k in kpts:
        m, lin = sphere_map(dims, semi, tuple(k))
        if shuffle:
            p = rng.permutation(m.shape[0])
            m, lin = m[p], lin[p]
        c = draw_coefficients(rng, m.shape[0], nb)
        spheres.append(Sphere(m=m, lin=lin, kpt=tuple(float(v) for v in k), nbands=nb))
        coeffs.append(np.ascontiguousarray(c.astype(dt)))
    return Workload(name="small", dims=tuple(int(d) for d in dims), spheres=spheres,
                    coeffs=coeffs, dtype=np.dtype(dt), seed=seed)


def random_grid(rng: np.random.Generator, dims, nb, dtype=np.complex128) -> np.ndarray:
    """A seeded dense grid G[z][y][x][b] that is not band-limited."""
    nx, ny, nz = dims
    v = rng.standard_normal((nz, ny, nx, nb, 2))
    return ((v[..., 0] + 1j * v[..., 1]) / math.sqrt(2.0)).astype(dtype)
