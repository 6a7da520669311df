"""Helpers shared by the GPU tests: run the library on a seeded workload and
compare with the FP64 oracle. Only the input generator (synth) and the oracle
are used for expected values; nothing here computes the transform itself."""
from __future__ import annotations

import numpy as np

import oracle
import synth

TOL = {"c128": 1e-12, "c64": 5e-6}


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def to_device(arr, dtype):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(arr.reshape(-1)))
    return t.to("cuda").to(torch.complex128 if dtype == "c128" else torch.complex64)


def make_plan(w: synth.Workload, dtype=None, flags=0, tuning=None):
    from paper_2406_05577_amd import Plan
    return Plan(w.dims, [s.lin for s in w.spheres], [s.nbands for s in w.spheres],
                kpts=[s.kpt for s in w.spheres], dtype=dtype or ("c128" if w.dtype == np.complex128 else "c64"),
                flags=flags, tuning=tuning)


def split_grid(w: synth.Workload, flat: np.ndarray):
    """Split the concatenated grid buffer into per-sphere (nz, ny, nx, Nb) arrays."""
    nx, ny, nz = w.dims
    out, off = [], 0
    for s in w.spheres:
        n = nx * ny * nz * s.nbands
        out.append(flat[off:off + n].reshape(nz, ny, nx, s.nbands))
        off += n
    return out


def split_sphere(w: synth.Workload, flat: np.ndarray):
    out, off = [], 0
    for s in w.spheres:
        n = s.ns * s.nbands
        out.append(flat[off:off + n].reshape(s.ns, s.nbands))
        off += n
    return out


def check_workload(w: synth.Workload, dtype: str, flags=0, tuning=None, grid_in=None, reps=1):
    """Run inverse, forward of the oracle grid, and the round trip on the GPU;
    return (E_inv, E_fwd, E_rt) relative L2 errors against the oracle."""
    import torch
    p = make_plan(w, dtype=dtype, flags=flags, tuning=tuning)
    npdt = np.complex128 if dtype == "c128" else np.complex64
    coeffs = [c.astype(npdt) for c in w.coeffs]   # the values both sides consume
    sph = to_device(np.concatenate([c.reshape(-1) for c in coeffs]), dtype)
    ref_grids = [oracle.sphere_to_grid(w.dims, s.lin, c.astype(np.complex128))
                 for s, c in zip(w.spheres, coeffs)]
    # outputs start as NaN so that any element the kernels fail to write shows up
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    g = torch.full((p.info["grid_elems"],), complex(float("nan"), float("nan")), dtype=tdt, device="cuda")
    for _ in range(reps):
        p.sphere_to_grid(sph, g)
    torch.cuda.synchronize()
    gpu_grids = split_grid(w, g.cpu().numpy())
    e_inv = rel(np.concatenate([x.ravel() for x in gpu_grids]),
                np.concatenate([x.ravel() for x in ref_grids]))
    # forward of the oracle grid (rounded to the plan precision)
    if grid_in is None:
        gin = [x.astype(npdt) for x in ref_grids]
    else:
        gin = [x.astype(npdt) for x in grid_in]
    gdev = to_device(np.concatenate([x.ravel() for x in gin]), dtype)
    s_out = torch.full((p.info["sphere_elems"],), complex(float("nan"), float("nan")), dtype=tdt, device="cuda")
    for _ in range(reps):
        p.grid_to_sphere(gdev, s_out)
    torch.cuda.synchronize()
    gpu_sph = split_sphere(w, s_out.cpu().numpy())
    ref_sph = [oracle.grid_to_sphere(w.dims, s.lin, x.astype(np.complex128))
               for s, x in zip(w.spheres, gin)]
    e_fwd = rel(np.concatenate([x.ravel() for x in gpu_sph]),
                np.concatenate([x.ravel() for x in ref_sph]))
    # round trip on the GPU
    rt = p.grid_to_sphere(p.sphere_to_grid(sph))
    torch.cuda.synchronize()
    e_rt = rel(rt.cpu().numpy(), np.concatenate([c.reshape(-1) for c in coeffs]))
    p.close()
    return e_inv, e_fwd, e_rt
