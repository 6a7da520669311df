"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (the same plan flags and the same tiling, from
paper_2406_05577_amd.tuned). The GPU transforms every band of every sphere;
on 16 seeded bands of every sphere (4 on the 256^3 grid, whose oracle is the
most expensive) the grid (E_inv) and the forward output (E_fwd) are compared
with the FP64 oracle element by element, and the round trip (E_rt) is
checked on every band, a property that holds at any size."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import TOL, rel

pytestmark = pytest.mark.gpu

CONFIGS = [
    # recipe, dtype, flags (1 = persistent work list, 4 = hipGraph replay):
    # the forms bench.py times
    ("c2", "c128", 0),
    ("c3", "c64", 0),
    ("c4", "c64", 5),
    ("c5", "c64", 5),
    ("c4", "c128", 0),
    ("c5", "c128", 0),
    ("x1", "c128", 0),   # the paper's experiment shape
    # the precision form with its radix-16 stages on the matrix cores (16):
    # the inverse fold's length-16 transforms on the y axes of 96 and 160
    ("c4", "c64", 5 | 16),
    ("c5", "c64", 5 | 16),
    ("x1", "c64", 0),    # the 256^3 shape in complex64 (its own frozen tiling)
]


def sampled_bands(nb: int, k: int, seed: int):
    """k seeded bands of nb, always including the first and the last."""
    if nb <= k:
        return list(range(nb))
    rng = np.random.default_rng(seed)
    mid = rng.choice(np.arange(1, nb - 1), size=k - 2, replace=False)
    return sorted({0, nb - 1, *mid.tolist()})


@pytest.mark.parametrize("cfg", range(len(CONFIGS)))
def test_full_config(cfg):
    from paper_2406_05577_amd import Plan
    from paper_2406_05577_amd.tuned import tuning_for
    recipe, dtype, flags = CONFIGS[cfg]
    tuning = tuning_for(recipe, dtype, flags)
    print(f"config {recipe} {dtype} flags={flags} tuning={tuning}", flush=True)
    w = synth.make_workload(recipe, dtype=dtype)
    p = Plan(w.dims, [s.lin for s in w.spheres], [s.nbands for s in w.spheres],
             kpts=[s.kpt for s in w.spheres], dtype=dtype, flags=flags, tuning=tuning)
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    sph = torch.from_numpy(w.sphere_concat()).to("cuda").to(tdt)
    grid = torch.full((p.info["grid_elems"],), complex(float("nan"), 0.0), dtype=tdt, device="cuda")
    back = torch.full_like(sph, complex(float("nan"), 0.0))
    for _ in range(2):   # twice: graph / persistent replays must reproduce
        p.sphere_to_grid(sph, grid)
        p.grid_to_sphere(grid, back)
    torch.cuda.synchronize()
    # round trip on every band
    e_rt = rel(back.cpu().numpy(), sph.cpu().numpy())
    assert not torch.isnan(grid).any().item()
    nx, ny, nz = w.dims
    goff = soff = 0
    worst = [0.0, 0.0]
    nsamp = 4 if recipe == "x1" else 16
    for si, (s, c) in enumerate(zip(w.spheres, w.coeffs)):
        nb = s.nbands
        bands = sampled_bands(nb, nsamp, 1000 + si)
        idx = torch.tensor(bands, device="cuda")
        gv = grid[goff:goff + nx * ny * nz * nb].view(nz, ny, nx, nb)
        got = gv.index_select(3, idx).cpu().numpy()
        ref = oracle.sphere_to_grid(w.dims, s.lin, c[:, bands].astype(np.complex128))
        e_inv = rel(got, ref)
        # the GPU's forward of its grid against the oracle's forward of the same grid
        fwd_gpu = back[soff:soff + s.ns * nb].view(s.ns, nb).index_select(1, idx).cpu().numpy()
        fwd_ref = oracle.grid_to_sphere(w.dims, s.lin, got.astype(np.complex128))
        e_fwd = rel(fwd_gpu, fwd_ref)
        worst = [max(worst[0], e_inv), max(worst[1], e_fwd)]
        print(f"  sphere {si}: {len(bands)} bands, E_inv={e_inv:.3e} E_fwd={e_fwd:.3e}", flush=True)
        del got, ref, fwd_ref
        goff += nx * ny * nz * nb
        soff += s.ns * nb
    print(f"{recipe} {dtype}: E_inv(sampled)={worst[0]:.3e} E_fwd(sampled)={worst[1]:.3e} "
          f"E_rt(all)={e_rt:.3e}", flush=True)
    assert worst[0] <= TOL[dtype] and worst[1] <= TOL[dtype] and e_rt <= TOL[dtype]
    p.close()
