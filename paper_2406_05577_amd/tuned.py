"""Measured tilings of the benchmark workloads on MI355X (gfx950).

Each entry maps (recipe, dtype, plan flags) to the tiling dict passed to
Plan(..., tuning=...): the pick of the library's autotuner
(FFTB_PLAN_AUTOTUNE, run once on an MI355X) frozen here, so that the
benchmark and the full-size parity tests run the very same tiling. A
workload without an entry uses the library defaults.
"""
from __future__ import annotations

from typing import Optional


def _both(inv: dict, fwd: dict) -> dict:
    out = {f"inv_{k}": v for k, v in inv.items()}
    out.update({f"fwd_{k}": v for k, v in fwd.items()})
    return out


# The autotuner's picks where they differ from the defaults. 144x160x180 and
# 128^3, complex128: the forward plane kernel with half the classes (classes
# of 16) and 512 threads, one workgroup per CU (11.10 -> 11.02 ms and 2.85 ->
# 2.79 ms). 256^3 (register lines): the inverse with 16 classes of 16 (a
# smaller band chunk in complex128, smaller column tiles in complex64): 8.58
# -> 8.76 and 13.04 -> 13.67 round trips/s. Every other benchmark workload's
# pick is its default tiling.
TUNED = {
    ("c5", "c128", 0): _both(
        dict(band_chunk=8, y_classes=10, x_rows=1, col_tile=16, threads=512, path=3, acc=2),
        dict(band_chunk=8, y_classes=10, x_rows=1, col_tile=16, threads=512, path=3, acc=3)),
    ("c2", "c128", 0): _both(
        dict(band_chunk=8, y_classes=8, x_rows=1, col_tile=8, threads=512, path=3, acc=2),
        dict(band_chunk=8, y_classes=8, x_rows=1, col_tile=8, threads=512, path=3, acc=3)),
    ("x1", "c128", 0): _both(
        dict(band_chunk=4, y_classes=16, x_rows=1, col_tile=8, threads=512, path=2, acc=0, lanes=16),
        dict(band_chunk=4, y_classes=16, x_rows=1, col_tile=8, threads=512, path=2, acc=3, lanes=16)),
    ("x1", "c64", 0): _both(
        dict(band_chunk=8, y_classes=16, x_rows=1, col_tile=4, threads=512, path=2, acc=0, lanes=16),
        dict(band_chunk=8, y_classes=16, x_rows=1, col_tile=4, threads=512, path=2, acc=3, lanes=16)),
}


def tuning_for(recipe: str, dtype: str, flags: int) -> Optional[dict]:
    t = TUNED.get((recipe, dtype, flags & ~2))
    return dict(t) if t else None
