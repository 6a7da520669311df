"""FP64 CPU oracle for the plane-wave sphere<->grid 3D FFT.

TEST INFRASTRUCTURE ONLY. Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this package. The library's transform
path never calls it, and it shares no code with the HIP kernels.

Every function is pinned by checks that do not reuse its own formula: brute
force triple sums, numpy.fft (pocketfft), closed forms, Parseval, round trip,
shift theorem, axis-order independence (tests/test_oracle_pins.py).
"""
from .pwfft import (  # noqa: F401
    dft_matrix,
    scatter_sphere,
    gather_sphere,
    axis_dft,
    sphere_to_grid,
    grid_to_sphere,
    brute_sphere_to_grid,
    brute_grid_to_sphere,
    apply_potential,
)
