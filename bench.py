"""Benchmark: sphere<->grid round trips per second on one MI355X.

One step = one round trip over every band of the workload: sphere_to_grid
(inverse, all bands) followed by grid_to_sphere (forward, all bands), inputs
resident in HBM. The default workload is the 128^3 grid, |G| <= 32 sphere at
Gamma (137,065 coefficients), 256 bands, complex128.

Timing follows the paper's protocol (Section 4.1: warm-up iterations, then the
mean over timed hot iterations). Per-kernel durations come from HIP events
that the library records around each launch on the execute stream.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak, GB/s
WORKLOADS = {
    # name: (recipe, dtype, flags)
    "c2": ("c2", "c128", 0),
    "c3": ("c3", "c64", 0),
    "c1": ("c1", "c128", 0),
    "c3alt": ("c3alt", "c64", 0),
    "c4": ("c4", "c64", 1 | 2 | 4),
    "c4_fp64": ("c4", "c128", 0),
    "c5": ("c5", "c64", 1 | 2 | 4),
    "c5_fp64": ("c5", "c128", 0),
    "x1": ("x1", "c128", 0),
    "x1_fp32": ("x1", "c64", 0),
    # padded-cube comparator: the same bands scattered into the whole grid and
    # transformed without pruning (every column, every slab)
    "c2_full": ("c2", "c128", 0),
    "c3_full": ("c3", "c64", 0),
}
DESCR = {
    "c1": "sphere<->grid 32^3, |G|<=8 (2109 coeffs), Gamma, 4 bands",
    "c2": "sphere<->grid 128^3, |G|<=32 (137065 coeffs), Gamma, 256 bands",
    "c3": "sphere<->grid 128^3, |G|<=32 (137065 coeffs), Gamma, 256 bands",
    "c3alt": "sphere<->grid 32^3, |G|<=8 (2109 coeffs), Gamma, 256 bands",
    "c4": "sphere<->grid 96^3, 8 k-points, |G+k|<=24, 64 bands each (512 spheres)",
    "c5": "sphere<->grid 144x160x180, ellipsoid (36,40,45), 4 k-points, 128 bands each",
    "x1": "sphere<->grid 256^3, |G|<=64 (diameter 128, the paper's experiment shape), Gamma, 256 bands",
    "c2_full": "padded-cube comparator: the 128^3, |G|<=32, 256-band sphere scattered into the "
               "full grid, transformed with every column and slab (no pruning)",
    "c3_full": "padded-cube comparator of c3 (complex64)",
}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2406_05577_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload: str, src_hash: str):
    """HBM traffic of the plane kernel per launch from the committed rocprofv3
    counter summary, only if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
        e = d.get(workload)
        if e and e.get("source_hash") == src_hash:
            return e.get("plane_bytes_per_launch")
    except (OSError, ValueError):
        pass
    return None


def _counter_rows(d: str):
    """Rows of a rocprofv3 --pmc CSV (the *_counter_collection.csv under d)."""
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def _per_kernel_kib(d: str, counter: str):
    """Mean counter value (KiB) per dispatch for each kernel name."""
    acc = {}
    for r in _counter_rows(d):
        if r["Counter_Name"] != counter:
            continue
        name = r["Kernel_Name"].split("(")[0].replace("void ", "")
        acc.setdefault(name, []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def summarize_counters(args):
    """Turn FETCH_SIZE / WRITE_SIZE passes (rocprofv3 --pmc CSV) of the bench
    and of a plain 1 GiB copy into per-launch HBM bytes of the plane kernels:
    each counter is scaled by (bytes the copy moves) / (what it reads for the
    copy). Writes profiles/traffic.json[workload] and prints a summary."""
    fetch_dir, write_dir, copy_fetch_dir, copy_write_dir = args.summarize_counters
    gib_kib = float(1 << 20)
    cf = _per_kernel_kib(copy_fetch_dir, "FETCH_SIZE")
    cw = _per_kernel_kib(copy_write_dir, "WRITE_SIZE")
    copy_name = max(cf, key=lambda k: cf[k])
    f_fetch = gib_kib / cf[copy_name]
    f_write = gib_kib / cw[max(cw, key=lambda k: cw[k])]
    fe = _per_kernel_kib(fetch_dir, "FETCH_SIZE")
    wr = _per_kernel_kib(write_dir, "WRITE_SIZE")
    rows = []
    plane = []
    for k in sorted(set(fe) | set(wr)):
        if "fftb" not in k:
            continue
        byts = (fe.get(k, 0.0) * f_fetch + wr.get(k, 0.0) * f_write) * 1024.0
        rows.append((k, fe.get(k, 0.0), wr.get(k, 0.0), byts))
        if "k2" in k:
            plane.append(byts)
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        d = {}
    d[args.workload] = {"plane_bytes_per_launch": sum(plane) / len(plane) if plane else None,
                        "fetch_factor": f_fetch, "write_factor": f_write,
                        "source_hash": kernel_source_hash()}
    with open(path, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    print(f"calibration: {copy_name} 1 GiB copy, FETCH_SIZE x{f_fetch:.3f}, WRITE_SIZE x{f_write:.3f}")
    print("| kernel | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | HBM bytes/dispatch (calibrated) |")
    print("|---|---|---|---|")
    for k, a, w, byts in rows:
        print(f"| `{k}` | {a:.0f} | {w:.0f} | {byts / 1e9:.3f} GB |")


def cpu_baseline(w_name: str, sample_bands: int):
    """The FP64 oracle, as it stands, timed on the host cores on a band sample
    of the same workload; scaled to round trips of the whole workload."""
    import numpy as np
    import oracle
    import synth
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    rec = synth.RECIPES[w_name]
    w = synth.make_workload(w_name, nbands=sample_bands, nkpts=1)
    s = w.spheres[0]
    c = w.coeffs[0].astype(np.complex128)
    t0 = time.perf_counter()
    g = oracle.sphere_to_grid(w.dims, s.lin, c)
    oracle.grid_to_sphere(w.dims, s.lin, g)
    t = time.perf_counter() - t0
    total_bands = rec["nb"] * max(rec["nk"], 1)
    rt_per_s = 1.0 / (t * total_bands / sample_bands)
    return {"value": rt_per_s, "unit": "round_trips/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{sample_bands} of {total_bands} bands (one k-point), one FP64 round trip "
                      f"in {t:.2f} s, scaled linearly to all bands"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--flags", type=int, default=None, help="override plan flags")
    ap.add_argument("--tuning", default=None, help="JSON dict of tiling knobs")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library time candidate tilings at plan creation (not timed)")
    ap.add_argument("--potential", action="store_true",
                    help="time the fused real-space step (sphere -> V*psi -> sphere) instead of "
                         "the plain round trip")
    ap.add_argument("--cpu-sample-bands", type=int, default=256,
                    help="bands of the first sphere the oracle transforms (capped at the workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip per-kernel event timing (graph replays never record it)")
    ap.add_argument("--summarize-counters", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="rocprofv3 --pmc output folders: write profiles/traffic.json for --workload")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(args)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(bands would shard across GPUs without any exchange). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2406_05577_amd import Plan

    recipe, dtype, flags = WORKLOADS[args.workload]
    if args.flags is not None:
        flags = args.flags
    if args.autotune:
        flags |= 2
    tuning = json.loads(args.tuning) if args.tuning else None
    torch.cuda.set_device(0)
    w = synth.make_workload(recipe, dtype=dtype)
    full = args.workload.endswith("_full")
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    t_plan = time.perf_counter()
    if full:
        # one "sphere" holding every grid point; the coefficients of the
        # (single) sphere are scattered into it on the device
        assert len(w.spheres) == 1
        s0 = w.spheres[0]
        all_pts = np.arange(w.ngrid, dtype=np.int32)
        plan = Plan(w.dims, [all_pts], [s0.nbands], kpts=[s0.kpt], dtype=dtype, flags=flags,
                    tuning=tuning)
    else:
        plan = Plan(w.dims, [s.lin for s in w.spheres], [s.nbands for s in w.spheres],
                    kpts=[s.kpt for s in w.spheres], dtype=dtype, flags=flags, tuning=tuning)
    t_plan = time.perf_counter() - t_plan
    if full:
        sph = torch.zeros((w.ngrid, w.spheres[0].nbands), dtype=tdt, device="cuda")
        sph[torch.from_numpy(w.spheres[0].lin.astype(np.int64)).to("cuda")] = \
            torch.from_numpy(w.coeffs[0]).to("cuda").to(tdt)
        sph = sph.reshape(-1)
    else:
        sph = torch.from_numpy(w.sphere_concat()).to("cuda").to(tdt)
    back = torch.empty_like(sph)
    grid = torch.empty(plan.info["grid_elems"], dtype=tdt, device="cuda")
    es = 16 if dtype == "c128" else 8
    N = w.ngrid
    nb_total = w.nbands_total
    grid_bytes = plan.info["grid_elems"] * es
    # algorithmic bytes per round trip of the pruned problem (for the padded
    # cube too, so that the two figures compare)
    sphere_bytes = sum(s.ns * s.nbands for s in w.spheres) * es
    b_min = 2 * (grid_bytes + sphere_bytes)

    if args.potential:
        rdt = torch.float64 if dtype == "c128" else torch.float32
        vpot = torch.from_numpy(np.random.default_rng(7).uniform(0.5, 1.5, w.ngrid)).to("cuda").to(rdt)

        def step():
            plan.apply_potential(sph, vpot, grid=grid, out=back)
    else:
        def step():
            plan.sphere_to_grid(sph, grid)
            plan.grid_to_sphere(grid, back)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    profile = not args.no_profile and not (flags & 4)
    plan.set_profiling(profile)
    plan.get_profile()   # clear
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    prof = plan.get_profile()
    plan.set_profiling(False)
    ms = ms_total / args.steps
    rt_s = 1000.0 / ms

    # round-trip check on the timed output (every band); the potential step
    # is checked against the oracle by the tests instead
    e_rt = None
    if not args.potential:
        ref = sph.cpu().numpy()
        got = back.cpu().numpy()
        e_rt = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))

    src_hash = kernel_source_hash()
    roofline = None
    kern = {}
    if profile:
        for k, (n, t) in prof.items():
            if n:
                kern[k] = {"launches": n, "avg_ms": t / n}
        n_inv, t_inv = prof["plane_inverse"]
        n_fwd, t_fwd = prof["plane_forward"]
        if n_inv and n_fwd:
            avg_s = (t_inv + t_fwd) / (n_inv + n_fwd) / 1000.0
            ach = grid_bytes / avg_s / 1e9
            traffic = traffic_from_profiles(args.workload, src_hash)
            roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                        "traffic": traffic, "kernel": "plane (y then x transforms), both directions",
                        "algorithmic_bytes_per_launch": grid_bytes,
                        "avg_launch_ms": round(avg_s * 1000.0, 4)}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(recipe, min(args.cpu_sample_bands, synth.RECIPES[recipe]["nb"]))
    out = {
        "metric": ("fused real-space steps/sec (sphere -> V*psi -> sphere)" if args.potential else
                   "sphere<->grid 3D FFT round trips/sec and % HBM roofline, FP32 vs FP64"),
        "value": round(rt_s, 3),
        "unit": "round_trips/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if dtype == "c128" else "f32",
        "data": "synthetic (seeded complex Gaussian bands on the cutoff sphere)",
        "config": {"workload": DESCR.get(args.workload, DESCR.get(recipe, recipe)), "recipe": recipe,
                   "complex_dtype": "complex128" if dtype == "c128" else "complex64",
                   "dims": list(w.dims), "bands": nb_total, "spheres": len(w.spheres),
                   "coeffs": int(plan.info["total_coeffs"]), "plan_flags": flags,
                   "tuning": plan.info["tuning"], "autotuned": plan.info["autotuned"],
                   "plan_seconds": round(t_plan, 3), "radix": {"x": plan.info["radix_x"],
                   "y": plan.info["radix_y"], "z": plan.info["radix_z"]}},
        "step_roofline": {"algorithmic_bytes": b_min, "achieved_GBs": round(b_min / (ms / 1000) / 1e9, 1),
                          "frac": round(b_min / (ms / 1000) / 1e9 / HBM_PEAK_GBS, 4)},
        "roofline": roofline,
        "kernels": kern,
        "band_round_trips_per_s": round(rt_s * nb_total, 1),
        "round_trip_rel_err": e_rt,
        "source_hash": src_hash,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
