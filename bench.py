"""Benchmark: sphere<->grid round trips per second on one MI355X.

One step = one round trip over every band of every sphere of the workload:
sphere_to_grid (inverse) followed by grid_to_sphere (forward), inputs resident
in HBM. The default workload is the largest configuration: the 144x160x180
grid of an orthorhombic cell, ellipsoid cutoff with semi-axes (36, 40, 45)
around 4 seeded k-points, 128 bands each (512 spheres' worth of bands). Its
`value` is the plain FP64 (complex128) form; the complex64 batched form
(persistent work list replayed as a hipGraph) runs on the same inputs and is
reported beside it with its speedup.

Timing follows the paper's protocol (Section 4.1: warm-up iterations, then the
mean over timed hot iterations), repeated over several hot blocks (median and
minimum reported). Per-kernel durations come from HIP events that the library
records around each launch on the execute stream (for a graph replay: from the
same launch sequence run un-captured). Working sets below twice the 256 MB
last-level cache rotate through buffer sets of at least 1 GB.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak, GB/s
MALL_BYTES = 256 << 20  # MI355X last-level (Infinity) cache
WORKLOADS = {
    # name: (recipe, dtype, flags); flags 1 = persistent work list, 4 = hipGraph replay
    "c5_fp64": ("c5", "c128", 0),
    "c5": ("c5", "c64", 1 | 4),
    "c4_fp64": ("c4", "c128", 0),
    "c4": ("c4", "c64", 1 | 4),
    "c2": ("c2", "c128", 0),
    "c2_c64": ("c2", "c64", 0),
    "c3": ("c3", "c64", 0),
    "c1": ("c1", "c128", 0),
    "c3alt": ("c3alt", "c64", 0),
    "x1": ("x1", "c128", 0),
    "x1_fp32": ("x1", "c64", 0),
    # padded-cube comparator: the same bands scattered into the whole grid and
    # transformed without pruning (every column, every slab)
    "c2_full": ("c2", "c128", 0),
    "c3_full": ("c3", "c64", 0),
}
# the second (complex64 batched) form timed on the same inputs
PAIRED = {"c5_fp64": "c5", "c4_fp64": "c4", "c2": "c2_c64"}
DESCR = {
    "c1": "sphere<->grid 32^3, |G|<=8 (2109 coeffs), Gamma, 4 bands",
    "c2": "sphere<->grid 128^3, |G|<=32 (137065 coeffs), Gamma, 256 bands",
    "c3": "sphere<->grid 128^3, |G|<=32 (137065 coeffs), Gamma, 256 bands",
    "c2_c64": "sphere<->grid 128^3, |G|<=32 (137065 coeffs), Gamma, 256 bands (the c2 inputs in complex64)",
    "c3alt": "sphere<->grid 32^3, |G|<=8 (2109 coeffs), Gamma, 256 bands",
    "c4": "sphere<->grid 96^3, 8 k-points, |G+k|<=24, 64 bands each (512 bands)",
    "c5": "sphere<->grid 144x160x180, ellipsoid (36,40,45), 4 k-points, 128 bands each (512 bands)",
    "x1": "sphere<->grid 256^3, |G|<=64 (diameter 128, the paper's experiment shape), Gamma, 256 bands",
    "c2_full": "padded-cube comparator: the 128^3, |G|<=32, 256-band sphere scattered into the "
               "full grid, transformed with every column and slab (no pruning)",
    "c3_full": "padded-cube comparator of c3 (complex64)",
}
KERNEL_UNITS = {
    # algorithmic bytes per launch of each kernel, per band of a sphere:
    # the plane kernels write (inverse) or read (forward) the grid, the column
    # kernels read (inverse) or write (forward) the sphere
    "plane_inverse": "grid", "plane_forward": "grid",
    "column_inverse": "sphere", "column_forward": "sphere", "combine_forward": None,
}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2406_05577_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload: str, src_hash: str, kernel: str):
    """HBM bytes per launch of one kernel from the committed rocprofv3 counter
    summary (profiles/traffic.json), only if it was taken on the current
    kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
        e = d.get(workload)
        if e and e.get("source_hash") == src_hash:
            return e.get("bytes_per_launch", {}).get(kernel)
    except (OSError, ValueError):
        pass
    return None


def kernel_id(name: str):
    """Library kernel id of a rocprofv3 kernel name (template arguments give
    the direction: 1 = inverse, -1 = forward)."""
    n = name.replace(" ", "")
    for tag, inv, fwd in (("k1r_kernel<", "column_inverse", "column_forward"),
                          ("k1b_kernel<", "column_inverse", "column_forward"),
                          ("k1_kernel<", "column_inverse", "column_forward"),
                          ("k2r_kernel<", "plane_inverse", "plane_forward"),
                          ("k2_kernel<", "plane_inverse", "plane_forward")):
        i = n.find(tag)
        if i >= 0:
            return fwd if n[i + len(tag):].startswith("-1") else inv
    if "k3r_kernel" in n:
        return "combine_forward"
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


def _per_kernel_kib(d: str, counter: str, by_id: bool):
    """Mean counter value (KiB) per dispatch for each kernel."""
    acc = {}
    for r in _counter_rows(d):
        if r["Counter_Name"] != counter:
            continue
        name = r["Kernel_Name"]
        key = kernel_id(name) if by_id else name
        if key is None:
            continue
        acc.setdefault(key, []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def summarize_counters(args):
    """Turn FETCH_SIZE / WRITE_SIZE passes (rocprofv3 --pmc CSV) of the bench
    and of a plain 1 GiB copy into HBM bytes per launch of every library
    kernel: each counter is scaled by (bytes the copy moves) / (what the
    counter reads for the copy). Writes profiles/traffic.json[workload] and
    prints a table."""
    fetch_dir, write_dir, copy_fetch_dir, copy_write_dir = args.summarize_counters
    gib_kib = float(1 << 20)
    cf = _per_kernel_kib(copy_fetch_dir, "FETCH_SIZE", False)
    cw = _per_kernel_kib(copy_write_dir, "WRITE_SIZE", False)
    copy_name = max(cf, key=lambda k: cf[k])
    f_fetch = gib_kib / cf[copy_name]
    f_write = gib_kib / cw[max(cw, key=lambda k: cw[k])]
    fe = _per_kernel_kib(fetch_dir, "FETCH_SIZE", True)
    wr = _per_kernel_kib(write_dir, "WRITE_SIZE", True)
    per = {}
    print(f"calibration: {copy_name[:60]} 1 GiB copy, FETCH_SIZE x{f_fetch:.3f}, WRITE_SIZE x{f_write:.3f}")
    print("| kernel | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | HBM bytes/dispatch (calibrated) |")
    print("|---|---|---|---|")
    for k in sorted(set(fe) | set(wr)):
        byts = (fe.get(k, 0.0) * f_fetch + wr.get(k, 0.0) * f_write) * 1024.0
        per[k] = byts
        print(f"| {k} | {fe.get(k, 0.0):.0f} | {wr.get(k, 0.0):.0f} | {byts / 1e9:.3f} GB |")
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        d = {}
    d[args.workload] = {"bytes_per_launch": per, "fetch_factor": f_fetch, "write_factor": f_write,
                        "source_hash": kernel_source_hash()}
    with open(path, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)


def summarize_pmc(dirs):
    """Per-kernel means of the counters in rocprofv3 --pmc passes (one folder
    per pass), with the ratios read from them: instructions per wave, the
    share of resident wave time spent waiting or issuing VALU / LDS work, LDS
    bank-conflict cycles per LDS-active cycle, the L2 hit rate and the mean
    latency of L1-to-L2 reads. With GRBM_GUI_ACTIVE (busy cycles summed over
    the 8 XCDs) it also gives the engine clock during the dispatch and the
    mean resident waves per CU (SQ_WAVE_CYCLES counts in units of 4 cycles,
    over the 256 CUs). Prints markdown tables."""
    acc = {}
    dur = {}
    for d in dirs:
        for r in _counter_rows(d):
            key = kernel_id(r["Kernel_Name"])
            if key is None:
                continue
            acc.setdefault(key, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
            dur.setdefault(key, {})[(d, r["Dispatch_Id"])] = (
                int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    mean = {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in acc.items()}
    names = sorted({c for cs in mean.values() for c in cs})
    print("| kernel | " + " | ".join(names) + " |")
    print("|---|" + "---|" * len(names))
    for k in sorted(mean):
        print(f"| {k} | " + " | ".join(f"{mean[k][c]:.4g}" if c in mean[k] else "" for c in names) + " |")

    def ratio(m, a, b):
        return m[a] / m[b] if a in m and b in m and m[b] else None

    cols = [("VALU insts / wave", "SQ_INSTS_VALU", "SQ_WAVES"),
            ("LDS insts / wave", "SQ_INSTS_LDS", "SQ_WAVES"),
            ("VMEM reads / wave", "SQ_INSTS_VMEM_RD", "SQ_WAVES"),
            ("VMEM writes / wave", "SQ_INSTS_VMEM_WR", "SQ_WAVES"),
            ("waiting / resident", "SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES"),
            ("VALU issuing / resident", "SQ_ACTIVE_INST_VALU", "SQ_WAVE_CYCLES"),
            ("LDS issuing / resident", "SQ_ACTIVE_INST_LDS", "SQ_WAVE_CYCLES"),
            ("bank-conflict cycles / LDS-active cycle", "SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_LDS")]
    print()
    extra = ["L2 hit rate", "L2 read latency (cycles)", "clock (GHz)", "resident waves / CU"]
    print("| kernel | mean dispatch ms | " + " | ".join(c[0] for c in cols + [(e,) for e in extra]) + " |")
    print("|---|---|" + "---|" * (len(cols) + len(extra)))
    for k in sorted(mean):
        m = mean[k]
        ms = sum(dur[k].values()) / len(dur[k]) / 1e6
        cells = [ratio(m, a, b) for _, a, b in cols]
        hit = lat = ghz = waves = None
        if "TCC_HIT_sum" in m and "TCC_MISS_sum" in m:
            hit = m["TCC_HIT_sum"] / max(m["TCC_HIT_sum"] + m["TCC_MISS_sum"], 1.0)
        lat = ratio(m, "TCP_TCC_READ_REQ_LATENCY_sum", "TCP_TCC_READ_REQ_sum")
        if m.get("GRBM_GUI_ACTIVE"):
            ghz = m["GRBM_GUI_ACTIVE"] / 8.0 / (ms * 1e6)
            if "SQ_WAVE_CYCLES" in m:
                waves = 4.0 * m["SQ_WAVE_CYCLES"] / (m["GRBM_GUI_ACTIVE"] / 8.0 * 256.0)
        cells += [hit, lat, ghz, waves]
        print(f"| {k} | {ms:.3f} | " + " | ".join("" if c is None else f"{c:.3g}" for c in cells) + " |")


def host_description():
    """nproc, CPU model and the BLAS thread count of the host."""
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        blas = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        blas = None
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        avail = os.cpu_count()
    return {"nproc": avail, "cpu_model": model, "blas_threads": blas}


def cpu_baseline(w_name: str, sample_bands: int):
    """The FP64 oracle, as it stands, timed on the host cores on a band sample
    of the same workload (its first k-point); scaled to round trips of the
    whole workload."""
    import numpy as np
    import oracle
    import synth
    host = host_description()
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
    return {"value": rt_per_s, "unit": "round_trips/s", "cores": host["blas_threads"] or host["nproc"],
            "kind": "oracle", "host": host,
            "sample": f"{sample_bands} of {total_bands} bands (the first k-point's sphere), one FP64 "
                      f"round trip (dense per-axis DFT through BLAS) in {t:.2f} s, scaled linearly "
                      f"to all bands"}


class Form:
    """One plan on one workload, with its device buffers (rotated sets when
    the working set is small enough to stay in the last-level cache)."""

    def __init__(self, name, w, flags=None, tuning=None, autotune=False, rotate=True):
        import numpy as np
        import torch
        from paper_2406_05577_amd import Plan
        from paper_2406_05577_amd.tuned import tuning_for
        self.name = name
        recipe, dtype, fl = WORKLOADS[name]
        if flags is not None:
            fl = flags
        if autotune:
            fl |= 2
        self.full = name.endswith("_full")
        if tuning is None and not self.full:
            # (the padded-cube comparator's map occupies every slab: its plans
            # take the defaults)
            tuning = tuning_for(recipe, dtype, fl)
        self.recipe, self.dtype, self.flags, self.tuning_req = recipe, dtype, fl, tuning
        tdt = torch.complex128 if dtype == "c128" else torch.complex64
        self.es = 16 if dtype == "c128" else 8
        t0 = time.perf_counter()
        if self.full:
            # one "sphere" holding every grid point; the (single) sphere's
            # coefficients are scattered into it on the device
            assert len(w.spheres) == 1
            s0 = w.spheres[0]
            all_pts = np.arange(w.ngrid, dtype=np.int32)
            self.plan = Plan(w.dims, [all_pts], [s0.nbands], kpts=[s0.kpt], dtype=dtype, flags=fl,
                             tuning=tuning)
        else:
            self.plan = Plan(w.dims, [s.lin for s in w.spheres], [s.nbands for s in w.spheres],
                             kpts=[s.kpt for s in w.spheres], dtype=dtype, flags=fl, tuning=tuning)
        self.plan_seconds = time.perf_counter() - t0
        if self.full:
            sph = torch.zeros((w.ngrid, w.spheres[0].nbands), dtype=tdt, device="cuda")
            sph[torch.from_numpy(w.spheres[0].lin.astype(np.int64)).to("cuda")] = \
                torch.from_numpy(w.coeffs[0]).to("cuda").to(tdt)
            sph = sph.reshape(-1)
        else:
            sph = torch.from_numpy(w.sphere_concat()).to("cuda").to(tdt)
        info = self.plan.info
        self.grid_bytes = info["grid_elems"] * self.es
        # algorithmic bytes of the pruned problem (for the padded cube too, so
        # that the two figures compare): read the sphere and write the grid,
        # then read the grid and write the sphere
        self.sphere_bytes = sum(s.ns * s.nbands for s in w.spheres) * self.es
        self.b_min = 2 * (self.grid_bytes + self.sphere_bytes)
        set_bytes = 2 * info["sphere_elems"] * self.es + self.grid_bytes
        nsets = 1
        if rotate and set_bytes + info["workspace_bytes"] < 2 * MALL_BYTES:
            nsets = max(2, -(-(1 << 30) // set_bytes))
        self.sets = []
        for i in range(nsets):
            src = sph if i == 0 else sph.clone()
            self.sets.append((src, torch.empty(info["grid_elems"], dtype=tdt, device="cuda"),
                              torch.empty_like(sph)))
        self.nsets = nsets
        self.i = 0
        self.used = set()   # buffer sets a step has run on

    def step(self):
        sph, grid, back = self.sets[self.i]
        self.used.add(self.i)
        self.i = (self.i + 1) % self.nsets
        self.plan.sphere_to_grid(sph, grid)
        self.plan.grid_to_sphere(grid, back)

    def step_potential(self, vpot):
        sph, grid, back = self.sets[self.i]
        self.used.add(self.i)
        self.i = (self.i + 1) % self.nsets
        self.plan.apply_potential(sph, vpot, grid=grid, out=back)

    def rt_error(self):
        """Relative round-trip error, worst over the buffer sets that ran."""
        import numpy as np
        errs = []
        for i in sorted(self.used):
            sph, _, back = self.sets[i]
            ref = sph.cpu().numpy()
            errs.append(float(np.linalg.norm(back.cpu().numpy() - ref) / np.linalg.norm(ref)))
        return max(errs)


def time_blocks(step, steps, warmup, repeats, after_warmup=None):
    """W untimed warm-up steps, then `repeats` hot blocks of exactly `steps`
    steps, each bracketed by device synchronisations and timed with events on
    the execute stream; returns the per-step milliseconds of every block."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    if after_warmup is not None:
        after_warmup()
    stream = torch.cuda.current_stream()
    out = []
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1) / steps)
    return out


def kernel_table(prof):
    kern = {}
    for k, (n, t) in prof.items():
        if n:
            kern[k] = {"launches": n, "avg_ms": round(t / n, 4), "total_ms": round(t, 3)}
    return kern


def dominant_roofline(form, kern, src_hash, workload):
    """HBM roofline of the kernel with the largest share of the step: its
    algorithmic bytes per launch over its average launch duration."""
    cands = [(v["total_ms"], k) for k, v in kern.items() if KERNEL_UNITS.get(k)]
    if not cands:
        return None
    _, k = max(cands)
    unit = KERNEL_UNITS[k]
    alg = form.grid_bytes if unit == "grid" else form.sphere_bytes
    avg_s = kern[k]["avg_ms"] / 1000.0
    ach = alg / avg_s / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profiles(workload, src_hash, k),
            "kernel": k, "algorithmic_bytes_per_launch": alg, "avg_launch_ms": kern[k]["avg_ms"],
            "share_of_step": round(kern[k]["total_ms"] / sum(v["total_ms"] for v in kern.values()), 3)}


def measure(form, args, step, profile_form=None):
    """Time a form; per-kernel durations from the library's events over the
    timed blocks, or (graph replays) from the same launch sequence run
    un-captured on `profile_form`."""
    import torch
    graph = bool(form.flags & 4)

    def start_profile():
        form.plan.set_profiling(not graph)
        form.plan.get_profile()   # clear what the warm-up recorded
    blocks = time_blocks(step, args.steps, args.warmup, args.repeats, start_profile)
    prof = form.plan.get_profile()
    form.plan.set_profiling(False)
    if graph and profile_form is not None:
        pf = profile_form
        pf.plan.set_profiling(False)
        for _ in range(2):
            pf.step()
        torch.cuda.synchronize()
        pf.plan.set_profiling(True)
        pf.plan.get_profile()
        for _ in range(args.steps):
            pf.step()
        torch.cuda.synchronize()
        prof = pf.plan.get_profile()
        pf.plan.set_profiling(False)
    return blocks, kernel_table(prof)


def step_roofline(form, ms):
    ach = form.b_min / (ms / 1000.0) / 1e9
    return {"algorithmic_bytes": form.b_min, "achieved_GBs": round(ach, 1),
            "frac": round(ach / HBM_PEAK_GBS, 4)}


def form_record(name, form, blocks, kern, src_hash, nb_total, e_rt):
    med = statistics.median(blocks)
    info = form.plan.info
    return {
        "workload": name, "complex_dtype": "complex128" if form.dtype == "c128" else "complex64",
        "plan_flags": form.flags, "tuning": info["tuning"], "autotuned": info["autotuned"],
        "plan_seconds": round(form.plan_seconds, 3),
        "value": round(1000.0 / med, 3), "unit": "round_trips/s", "ms_per_step": round(med, 4),
        "hot_blocks_ms_per_step": [round(b, 4) for b in blocks],
        "min_ms_per_step": round(min(blocks), 4), "buffer_sets": form.nsets,
        "band_round_trips_per_s": round(1000.0 / med * nb_total, 1),
        "step_roofline": step_roofline(form, med),
        "roofline": dominant_roofline(form, kern, src_hash, name) if kern else None,
        "kernels": kern, "round_trip_rel_err": e_rt,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--repeats", type=int, default=5, help="hot blocks of --steps steps each")
    ap.add_argument("--workload", default="c5_fp64", choices=sorted(WORKLOADS))
    ap.add_argument("--pair", default=None,
                    help="second form timed on the same inputs (default: the complex64 batched "
                         "form of the FP64 workloads; 'none' to skip)")
    ap.add_argument("--flags", type=int, default=None, help="override plan flags")
    ap.add_argument("--tuning", default=None, help="JSON dict of tiling knobs")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library time candidate tilings at plan creation (not timed)")
    ap.add_argument("--potential", action="store_true",
                    help="time the fused real-space step (sphere -> V*psi -> sphere) instead of "
                         "the plain round trip")
    ap.add_argument("--no-rotate", action="store_true",
                    help="keep one buffer set even when the working set fits the last-level cache")
    ap.add_argument("--cpu-sample-bands", type=int, default=128,
                    help="bands of the first sphere the oracle transforms (capped at the workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--summarize-counters", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="rocprofv3 --pmc output folders: write profiles/traffic.json for --workload")
    ap.add_argument("--summarize-pmc", nargs="+", metavar="DIR",
                    help="rocprofv3 --pmc output folders: print per-kernel counter means and ratios")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 1 GiB device-to-device copy three times (the reference "
                         "kernel whose FETCH_SIZE / WRITE_SIZE calibrate the HBM counters)")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc)
        return
    if args.summarize_counters:
        summarize_counters(args)
        return
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4, "launches": 3}))
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(bands would shard across GPUs without any exchange). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth

    torch.cuda.set_device(0)
    recipe, dtype, _ = WORKLOADS[args.workload]
    src_hash = kernel_source_hash()
    w = synth.make_workload(recipe, dtype=dtype)
    nb_total = w.nbands_total
    tuning = json.loads(args.tuning) if args.tuning else None
    form = Form(args.workload, w, flags=args.flags, tuning=tuning, autotune=args.autotune,
                rotate=not args.no_rotate)
    print(f"bench: {args.workload} plan ready in {form.plan_seconds:.2f} s, "
          f"{form.nsets} buffer set(s)", file=sys.stderr, flush=True)

    if args.potential:
        rdt = torch.float64 if dtype == "c128" else torch.float32
        vpot = torch.from_numpy(np.random.default_rng(7).uniform(0.5, 1.5, w.ngrid)).to("cuda").to(rdt)
        step = lambda: form.step_potential(vpot)  # noqa: E731
    else:
        step = form.step
    blocks, kern = measure(form, args, step)
    e_rt = None if args.potential else form.rt_error()
    rec = form_record(args.workload, form, blocks, kern, src_hash, nb_total, e_rt)
    print(f"bench: {args.workload} {rec['value']} rt/s", file=sys.stderr, flush=True)
    resident = None
    if form.nsets > 1 and not args.potential:
        # the same plan on one buffer set (cache-resident working set), for context
        form.nsets = 1
        form.i = 0
        rb = time_blocks(form.step, args.steps, args.warmup, args.repeats)
        resident = {"value": round(1000.0 / statistics.median(rb), 3), "unit": "round_trips/s",
                    "ms_per_step": round(statistics.median(rb), 4),
                    "note": "one buffer set: the working set stays in the last-level cache"}

    pair_name = args.pair if args.pair is not None else PAIRED.get(args.workload)
    pair = None
    if pair_name and pair_name != "none" and not args.potential:
        form.plan.close()
        del form.sets
        torch.cuda.empty_cache()
        pr, pdt, pfl = WORKLOADS[pair_name]
        assert pr == recipe, "the paired form must run on the same inputs"
        w2 = synth.make_workload(recipe, dtype=pdt)   # same draw, rounded to the pair's precision
        f2 = Form(pair_name, w2, rotate=not args.no_rotate)
        print(f"bench: {pair_name} plan ready in {f2.plan_seconds:.2f} s", file=sys.stderr, flush=True)
        prof_form = None
        if f2.flags & 4:
            # per-kernel durations of the graph's launch sequence, run un-captured
            prof_form = Form(pair_name, w2, flags=f2.flags & ~4, tuning=f2.tuning_req, rotate=False)
        b2, k2 = measure(f2, args, f2.step, prof_form)
        if prof_form is not None:
            prof_form.plan.close()
        pair = form_record(pair_name, f2, b2, k2, src_hash, nb_total, f2.rt_error())
        pair["speedup_vs_value"] = round(pair["value"] / rec["value"], 3)
        print(f"bench: {pair_name} {pair['value']} rt/s", file=sys.stderr, flush=True)
        f2.plan.close()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(recipe, min(args.cpu_sample_bands, synth.RECIPES[recipe]["nb"]))
    med = statistics.median(blocks)
    out = {
        "metric": ("fused real-space steps/sec (sphere -> V*psi -> sphere)" if args.potential else
                   "sphere<->grid 3D FFT round trips/sec and % HBM roofline, FP32 vs FP64"),
        "value": rec["value"],
        "unit": "round_trips/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if dtype == "c128" else "f32",
        "data": "synthetic (seeded complex Gaussian bands on the cutoff spheres)",
        "config": {"workload": DESCR.get(args.workload, DESCR.get(recipe, recipe)), "recipe": recipe,
                   "complex_dtype": rec["complex_dtype"], "dims": list(w.dims), "bands": nb_total,
                   "spheres": len(w.spheres), "coeffs": int(form.plan.info["total_coeffs"]),
                   "plan_flags": form.flags, "tuning": rec["tuning"], "autotuned": rec["autotuned"],
                   "plan_seconds": rec["plan_seconds"],
                   "radix": {"x": form.plan.info["radix_x"], "y": form.plan.info["radix_y"],
                             "z": form.plan.info["radix_z"]}},
        "repeats": {"blocks": args.repeats, "ms_per_step": rec["hot_blocks_ms_per_step"],
                    "median": round(med, 4), "min": rec["min_ms_per_step"],
                    "buffer_sets": form.nsets},
        "roofline": rec["roofline"],
        "step_roofline": rec["step_roofline"],
        "kernels": kern,
        "band_round_trips_per_s": rec["band_round_trips_per_s"],
        "round_trip_rel_err": e_rt,
        "resident": resident,
        "fp32_batched": pair,
        "source_hash": src_hash,
        "cpu_baseline": cpu,
        "env": {"torch": torch.__version__, "hip": getattr(torch.version, "hip", None),
                "gpu": torch.cuda.get_device_name(0)},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
