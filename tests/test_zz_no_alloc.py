"""fftb_sphere_to_grid_static, the entry point that allocates nothing: its
column scratch is the library's static device array instead of the plan's.
Two calls in a row, the second on a smaller problem (the array keeps the
first call's contents, so the zero padding the fold reads must be restored),
each checked bit for bit against fftb_sphere_to_grid on the same plan and
inputs, and against the FP64 oracle; a plan whose scratch exceeds the array
is refused."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, make_plan, rel, split_grid, to_device

pytestmark = pytest.mark.gpu


def _run(w, dtype, flags):
    import torch
    p = make_plan(w, dtype=dtype, flags=flags)
    npdt = np.complex128 if dtype == "c128" else np.complex64
    coeffs = [c.astype(npdt) for c in w.coeffs]
    sph = to_device(np.concatenate([c.reshape(-1) for c in coeffs]), dtype)
    tdt = sph.dtype
    g_static = torch.full((p.info["grid_elems"],), complex(float("nan"), 0.0), dtype=tdt, device="cuda")
    p.sphere_to_grid_static(sph, g_static)
    g_ref = torch.full_like(g_static, complex(float("nan"), 0.0))
    p.sphere_to_grid(sph, g_ref)
    torch.cuda.synchronize()
    assert torch.equal(g_static, g_ref)
    got = split_grid(w, g_static.cpu().numpy())
    for s, c, g in zip(w.spheres, coeffs, got):
        ref = oracle.sphere_to_grid(w.dims, s.lin, c.astype(np.complex128))
        assert rel(g, ref) <= TOL[dtype]
    p.close()


@pytest.mark.parametrize("flags", [0, 5])
def test_static_scratch_two_calls(flags):
    big = synth.small_workload((96, 96, 96), (24, 24, 24), [(0.21, -0.33, 0.1), (-0.4, 0.05, 0.45)],
                               8, seed=12)
    small = synth.small_workload((32, 32, 32), (8, 8, 8), [(0.0, 0.0, 0.0)], 5, seed=11)
    _run(big, "c128", flags)
    _run(small, "c64", flags)


def test_static_scratch_too_small():
    from paper_2406_05577_amd import FFTB_ERR_UNSUPPORTED
    from paper_2406_05577_amd.fftb import FftbError
    import torch
    w = synth.make_workload("c2", nbands=64)
    p = make_plan(w, dtype="c128")
    sph = torch.zeros(p.info["sphere_elems"], dtype=torch.complex128, device="cuda")
    grid = torch.empty(p.info["grid_elems"], dtype=torch.complex128, device="cuda")
    with pytest.raises(FftbError) as ex:
        p.sphere_to_grid_static(sph, grid)
    assert ex.value.status == FFTB_ERR_UNSUPPORTED
    p.close()
