"""Plain, slow FP64 definition of the batched sphere<->grid transform.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

What is computed, and where the paper defines it:

* DFT_n is the dense n x n matrix [w_n^(l*k)] with w_n = exp(-2*pi*j/n)
  (Section 2.1, 1D DFT equation). A negative exponent is the forward
  direction.
* A 3D DFT is three batches of 1D DFTs, one per dimension, applied in any
  order (Section 2.1, pencil-pencil-pencil algorithm and the remark that the
  order may be permuted). The oracle uses the dense matrices, not an FFT.
* A wavefunction is the plane-wave sum psi_i(r) = sum_g c_i(g) exp(+j g r)
  over the coefficients kept inside the cutoff sphere (Section 2.2). On the FFT
  grid g.r reduces to sum_i m_i * x_i / n_i, so sphere->grid is the inverse
  (positive exponent) DFT of the zero-padded sphere, unnormalised.
* grid->sphere is the forward DFT followed by a gather of the sphere's
  entries, scaled by 1/N with N = nx*ny*nz, so that grid->sphere undoes
  sphere->grid exactly.
* All bands share one index map (Section 2.2, offset array) and the band
  index is fastest in memory (Section 3.3, batch dimension first).

Layouts: sphere S[g][b] = array (Ns, Nb); grid G[z][y][x][b] = array
(nz, ny, nx, Nb); the wrapped linear index of a coefficient is
x + nx*(y + ny*z) with x = m_x mod nx etc.
"""
from __future__ import annotations

import numpy as np


def dft_matrix(n: int, sign: int) -> np.ndarray:
    """F[l, k] = exp(sign * 2*pi*j * l*k / n), with l*k reduced modulo n in
    integers before the angle is formed (Section 2.1; sign=-1 is DFT_n)."""
    if sign not in (-1, 1):
        raise ValueError("sign must be +1 or -1")
    l = np.arange(n, dtype=np.int64)
    r = np.outer(l, l) % n
    ang = (2.0 * np.pi / n) * r.astype(np.float64)
    return np.cos(ang) + 1j * sign * np.sin(ang)


def scatter_sphere(dims, lin: np.ndarray, coeffs: np.ndarray) -> np.ndarray:
    """Zero-pad the sphere into the full cuboid (the padding of Section 2.2):
    A[z][y][x][b] = c[g][b] where lin[g] = x + nx*(y + ny*z), else 0."""
    nx, ny, nz = (int(d) for d in dims)
    lin = np.asarray(lin, dtype=np.int64)
    if np.unique(lin).shape[0] != lin.shape[0]:
        raise ValueError("duplicate index in sphere map")
    nb = coeffs.shape[1]
    a = np.zeros((nz * ny * nx, nb), dtype=np.complex128)
    a[lin] = coeffs
    return a.reshape(nz, ny, nx, nb)


def gather_sphere(lin: np.ndarray, grid: np.ndarray) -> np.ndarray:
    """c[g][b] = A[lin[g]][b] (the inverse of the padding)."""
    nb = grid.shape[-1]
    return grid.reshape(-1, nb)[np.asarray(lin, dtype=np.int64)]


_AXIS = {"x": 2, "y": 1, "z": 0}   # positions in the (nz, ny, nx, Nb) array


def axis_dft(a: np.ndarray, axis: str, sign: int) -> np.ndarray:
    """One batch of 1D DFTs along `axis`: out[..l..] = sum_k F[l,k] a[..k..]."""
    ax = _AXIS[axis]
    f = dft_matrix(a.shape[ax], sign)
    return np.moveaxis(np.tensordot(f, a, axes=([1], [ax])), 0, ax)


def sphere_to_grid(dims, lin, coeffs, order: str = "zyx") -> np.ndarray:
    """Inverse transform: psi_b(x,y,z) = sum_g c_b(g) exp(+2*pi*j*(mx*x/nx +
    my*y/ny + mz*z/nz)), unnormalised (Section 2.2 expansion, Section 2.1
    per-axis decomposition). Returns G (nz, ny, nx, Nb) complex128."""
    a = scatter_sphere(dims, lin, np.asarray(coeffs, dtype=np.complex128))
    for axis in order:
        a = axis_dft(a, axis, +1)
    return a


def grid_to_sphere(dims, lin, grid, order: str = "xyz") -> np.ndarray:
    """Forward transform: c_b(g) = (1/N) sum_r psi_b(r) exp(-2*pi*j*G.r) at the
    sphere's entries (Section 2.1 DFT, then the gather). Returns (Ns, Nb)."""
    nx, ny, nz = (int(d) for d in dims)
    a = np.asarray(grid, dtype=np.complex128).reshape(nz, ny, nx, -1)
    for axis in order:
        a = axis_dft(a, axis, -1)
    return gather_sphere(lin, a) / float(nx * ny * nz)


def apply_potential(dims, lin, coeffs, potential) -> np.ndarray:
    """The real-space step the transforms exist for (Section 1: the Kohn-Sham
    wavefunctions, and operations that are cheaper in real space): go to the
    grid, multiply every band pointwise by a real local potential V(x,y,z)
    (shape (nz, ny, nx), shared by all bands), come back to the sphere:
    c' = grid_to_sphere(V * sphere_to_grid(c))."""
    v = np.asarray(potential, dtype=np.float64)
    nx, ny, nz = (int(d) for d in dims)
    if v.shape != (nz, ny, nx):
        raise ValueError("potential must have shape (nz, ny, nx)")
    g = sphere_to_grid(dims, lin, coeffs)
    return grid_to_sphere(dims, lin, g * v[..., None])


def _phase_table(dims, m: np.ndarray, sign: int) -> np.ndarray:
    """E[g, r] = exp(sign*2*pi*j*(mx*x/nx + my*y/ny + mz*z/nz)) for every grid
    point r (x fastest), evaluated directly from the triple of fractions."""
    nx, ny, nz = (int(d) for d in dims)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    frac = (np.outer(m[:, 0], x.reshape(-1)) / nx
            + np.outer(m[:, 1], y.reshape(-1)) / ny
            + np.outer(m[:, 2], z.reshape(-1)) / nz)
    return np.exp(sign * 2j * np.pi * frac)


def brute_sphere_to_grid(dims, m: np.ndarray, coeffs: np.ndarray) -> np.ndarray:
    """The 3D DFT as one dense matrix (Section 2.1, 3D DFT equation) applied to
    the sphere with signed m: a triple sum at every grid point. Tiny grids only."""
    nx, ny, nz = (int(d) for d in dims)
    e = _phase_table(dims, np.asarray(m, dtype=np.int64), +1)     # (Ns, N)
    out = e.T @ np.asarray(coeffs, dtype=np.complex128)           # (N, Nb)
    return out.reshape(nz, ny, nx, -1)


def brute_grid_to_sphere(dims, m: np.ndarray, grid: np.ndarray) -> np.ndarray:
    """Forward triple sum at each sphere point, scaled by 1/N. Tiny grids only."""
    nx, ny, nz = (int(d) for d in dims)
    e = _phase_table(dims, np.asarray(m, dtype=np.int64), -1)     # (Ns, N)
    g = np.asarray(grid, dtype=np.complex128).reshape(nx * ny * nz, -1)
    return (e @ g) / float(nx * ny * nz)
