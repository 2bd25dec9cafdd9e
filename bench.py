#!/usr/bin/env python
"""Benchmark of the hybrid sphere convolution on one MI355X.

Workload: HEALPix nside 2048 (50,331,648 pixels), FP32, Gaussian beam of
5' FWHM truncated at 20' (Planck-HFI-like channel); input 1e-4 N(0,1) white
noise plus 2000 point sources with log-uniform amplitudes in [1e-3, 1]
(synthetic, seeded).  A step is one full forward convolution (ring R2C,
ring-pair accumulation streaming precomputed K_ij(m) tables, fold + C2R,
pole-ring fix) of the map already resident in HBM.  The plan (geometry,
kernel samples, bands) is built once before timing and reported separately.

Prints one JSON line: output pixels/s of the plain forward form, the
roofline of the dominant kernel (HIP events on the library's stream), the
adjoint form's throughput, the same forward without the artifact
suppression (the paper's Sect. 4.1 algorithm alone), the spline-kernel and
batched forms, and the FP64 oracle timed on the host cores on a bounded
sample of output pixels.
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

METRIC = "output pixels/sec (nside 2048, 5' beam) & % HBM roofline, plain vs batched/adjoint"
HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz, packed FP32 off
STAGES = ["ring_r2c", "accumulate", "fold_c2r", "pole_fix"]
KERNEL_NAMES = {"ring_r2c": "r2c_kernel", "accumulate": "accumulate_kernel", "fold_c2r": "c2r_kernel",
                "pole_fix": "pole_forward_kernel"}
# the accumulation stage runs one of these (the plan's tuned shape: one unit
# per wavefront, or two or three)
STAGE_KERNELS = {"accumulate": ("accumulate_kernel", "accumulate_u_kernel")}


def stage_of(kernel: str):
    """The forward stage a kernel (short name) belongs to, or None."""
    for stage, name in KERNEL_NAMES.items():
        if kernel == name or kernel in STAGE_KERNELS.get(stage, ()):
            return stage
    return None
KERNEL_SOURCES = {"ring_r2c": ["fft.hip", "device_common.h"], "accumulate": ["accum.hip", "device_common.h"],
                  "fold_c2r": ["fft.hip", "device_common.h"], "pole_fix": ["pole.hip"]}
# the batched form's kernels per stage (their sources: the stage's and the
# batch planner's)
BATCH_KERNELS = {"ring_r2c": ("r2c_batch_kernel",), "accumulate": ("accumulate_batch_kernel", "accumulate_batch_u_kernel"),
                 "fold_c2r": ("c2r_batch_kernel",), "pole_fix": ("pole_batch_kernel",)}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash(stage: str, batched: bool = False) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[stage] + (["batch.hip"] if batched else []):
        with open(os.path.join(ROOT, "paper_1104_0672_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def batch_stage_of(kernel: str):
    for stage, names in BATCH_KERNELS.items():
        if kernel in names:
            return stage
    return None


COUNTERS_JSON = os.path.join(ROOT, "profiles", "counters_valu.json")


def batched_valu_issue():
    """VALU issue fraction of each stage of the batched form, from the
    committed SQ counter summary (a 64-map batch; VALU wave instructions x 4
    cycles over 1024 SIMDs x 2.4 GHz x the stage's profiled time, summed over
    its launch shapes), if it was taken on the current kernel sources."""
    if not os.path.exists(COUNTERS_JSON):
        return None
    with open(COUNTERS_JSON) as fh:
        data = json.load(fh)
    out = {}
    for stage in BATCH_KERNELS:
        valu = us = 0.0
        for ent in data.get("kernels", []):
            if batch_stage_of(ent["kernel"]) != stage:
                continue
            if ent.get("source_sha") != kernel_source_hash(stage, batched=True):
                return None
            valu += ent["valu_wave_insts"] * ent["dispatches"]
            us += ent["us"] * ent["dispatches"]
        if us > 0:
            out[stage] = round(valu * 4 / (1024 * 2.4e9 * us * 1e-6), 3)
    return {"stages": out, "source": "profiles/counters_valu.json"} if out else None


def algorithmic_bytes(stage: str, plan, elem: int) -> int:
    """Compulsory HBM bytes per launch of each staged kernel: the map in and
    its half spectrum out (R2C), the input spectra in and the output-ring
    coefficients out (accumulation), the output coefficients in and the map
    out (C2R): elem bytes per pixel each way, i.e. 2*elem per pixel per stage
    (3 stages: 24 B/px in FP32).  The pole fix reads and writes 8 pixels."""
    npix = plan.npix
    if stage == "pole_fix":
        return 16 * elem
    return 2 * elem * npix


def measured_traffic(stage: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_healpix2048_5arcmin.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    ent = data.get("kernels", {}).get(KERNEL_NAMES[stage])
    if not ent or ent.get("source_sha") != kernel_source_hash(stage):
        return None
    return ent.get("hbm_bytes_per_launch")


def copy_calibration(mib: int, dev):
    """A plain device-to-device copy of known size (mib MiB read, mib MiB
    written), run before the workload so that a counter run can scale the
    kernels' FETCH_SIZE / WRITE_SIZE by what the counters read for it."""
    import torch
    n = mib * 2**20 // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()


def _counter_rows(path):
    import csv
    with open(path) as fh:
        return list(csv.DictReader(fh))


def _short(name: str) -> str:
    name = name.split("(")[0].replace("void ", "")
    return name.split("::")[-1].split("<")[0]


def summarize_traffic(fetch_csv: str, write_csv: str, calib_mib: int, out_path: str, cmd: str):
    """Per-stage HBM bytes per forward step from two rocprofv3 --pmc runs
    (FETCH_SIZE, WRITE_SIZE, KiB per dispatch), each scaled by the ratio of
    the known size of the copy-calibration dispatches to what the same counter
    reads for them.  Only dispatches from the first ring transform on count:
    the plan's shape tuner launches the accumulation before it."""
    import collections
    calib_bytes = calib_mib * 2**20
    res = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        per = collections.defaultdict(float)
        steps = 0
        cal = []
        rows = sorted((r for r in _counter_rows(path) if r["Counter_Name"] == counter),
                      key=lambda r: int(r["Dispatch_Id"]))
        started = False
        for r in rows:
            name = _short(r["Kernel_Name"])
            kib = float(r["Counter_Value"])
            if name == "__amd_rocclr_copyBuffer" and kib * 1024 > 0.5 * calib_bytes:
                cal.append(kib * 1024)
                continue
            started = started or name == KERNEL_NAMES["ring_r2c"]
            if not started:
                continue
            st = stage_of(name)
            per[KERNEL_NAMES[st] if st else name] += kib * 1024
            if st == "accumulate":
                steps += 1
        if not cal or not steps:
            raise SystemExit(f"{path}: no calibration copy or no accumulate dispatch found")
        factor = calib_bytes / (sum(cal) / len(cal))
        res[counter] = (per, steps, factor, sum(cal) / len(cal))
    kernels = {}
    for stage, kname in KERNEL_NAMES.items():
        fper, fsteps, ffac, _ = res["FETCH_SIZE"]
        wper, wsteps, wfac, _ = res["WRITE_SIZE"]
        fb = fper.get(kname, 0.0) / fsteps * ffac
        wb = wper.get(kname, 0.0) / wsteps * wfac
        kernels[kname] = {"stage": stage, "source_sha": kernel_source_hash(stage),
                          "fetch_bytes_per_launch": round(fb), "write_bytes_per_launch": round(wb),
                          "hbm_bytes_per_launch": round(fb + wb)}
    out = {"workload": "healpix2048_5arcmin (forward step)", "command": cmd,
           "calibration": {"copy_bytes": calib_bytes,
                           "fetch_counter_bytes": res["FETCH_SIZE"][3], "fetch_factor": res["FETCH_SIZE"][2],
                           "write_counter_bytes": res["WRITE_SIZE"][3], "write_factor": res["WRITE_SIZE"][2]},
           "steps_counted": {"fetch": res["FETCH_SIZE"][1], "write": res["WRITE_SIZE"][1]},
           "kernels": kernels}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out, indent=1))


def summarize_kernels(trace_dir: str, cmd: str, title: str, only: str = "", top: int = 0):
    """Markdown summary of a rocprofv3 --kernel-trace --stats run: the stats
    table (its first `top` rows if top > 0) plus per-launch-shape averages of
    the convolution kernels (those whose name holds `only`, if given)."""
    import collections
    stats = _counter_rows(os.path.join(trace_dir, "run_kernel_stats.csv"))
    trace = _counter_rows(os.path.join(trace_dir, "run_kernel_trace.csv"))
    lines = [f"# {title}", "", "Command (from the repository root, one MI355X):", "", "```", cmd, "```", "",
             "All dispatches of the run (plan build, warmup and timed steps), from `run_kernel_stats.csv`:", "",
             "| kernel | calls | total us | average us | % |", "|---|---:|---:|---:|---:|"]
    for s in (stats[:top] if top > 0 else stats):
        lines.append(f"| `{_short(s['Name'])}` | {s['Calls']} | {float(s['TotalDurationNs']) / 1e3:.1f} | "
                     f"{float(s['AverageNs']) / 1e3:.1f} | {float(s['Percentage']):.1f} |")
    agg = collections.defaultdict(list)
    for r in trace:
        n = _short(r["Kernel_Name"])
        if (stage_of(n) or "batch" in n or "grad" in n or "adjoint" in n) and only in n:
            key = (n, int(r["Grid_Size_X"]) // max(1, int(r["Workgroup_Size_X"])), int(r["Workgroup_Size_X"]),
                   int(r["LDS_Block_Size"]))
            agg[key].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    lines += ["", "Per launch shape, from `run_kernel_trace.csv`:", "",
              "| kernel | workgroups | threads | LDS bytes | launches | average us | average us after the first launch |",
              "|---|---:|---:|---:|---:|---:|---:|"]
    for k, v in sorted(agg.items()):
        warm = f"{sum(v[1:]) / (len(v) - 1) / 1e3:.1f}" if len(v) > 1 else "-"
        lines.append(f"| `{k[0]}` | {k[1]} | {k[2]} | {k[3]} | {len(v)} | {sum(v) / len(v) / 1e3:.1f} | {warm} |")
    print("\n".join(lines))


def summarize_counters(csv_path: str, cmd: str, title: str):
    """Markdown summary of one rocprofv3 --pmc run of SQ instruction counters
    (summed over the device, per dispatch): per kernel and launch shape the
    wave instructions by kind, and the VALU issue fraction = VALU wave
    instructions x 4 cycles / (1024 SIMDs x 2.4 GHz x dispatch duration under
    the profiler)."""
    import collections
    rows = sorted(_counter_rows(csv_path), key=lambda r: int(r["Dispatch_Id"]))
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    durs = collections.defaultdict(dict)
    # accumulation dispatches of the shape tuners (plan and batch creation)
    # are left out: a counted one follows a ring transform
    name_of = {}
    for r in rows:
        n = _short(r["Kernel_Name"])
        if stage_of(n) or "grad" in n or "batch" in n:
            name_of.setdefault(int(r["Dispatch_Id"]), n)
    skip, prev = set(), ""
    for d in sorted(name_of):
        if name_of[d].startswith("accumulate") and not prev.startswith("r2c"):
            skip.add(d)
        prev = name_of[d]
    for r in rows:
        n = _short(r["Kernel_Name"])
        if not (stage_of(n) or "grad" in n or "batch" in n) or int(r["Dispatch_Id"]) in skip:
            continue
        key = (n, int(r["Grid_Size"]) // max(1, int(r["Workgroup_Size"])), int(r["Workgroup_Size"]))
        per[key][r["Counter_Name"]] += float(r["Counter_Value"])
        durs[key][r["Dispatch_Id"]] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    names = ["SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR"]
    lines = [f"# {title}", "", "Command (from the repository root, one MI355X):", "", "```", cmd, "```", "",
             "Per dispatch (averages over the run's dispatches of each launch shape; wave instructions "
             "summed over the device); VALU issue = VALU x 4 cycles / (1024 SIMDs x 2.4 GHz x duration):", "",
             "| kernel | workgroups | threads | dispatches | us (profiled) | VALU | SALU | LDS | VMEM rd | VMEM wr | VALU issue |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    ents = []
    for key in sorted(per):
        nd = len(durs[key])
        us = sum(durs[key].values()) / nd / 1e3
        c = {k: v / nd for k, v in per[key].items()}
        valu = c.get("SQ_INSTS_VALU", 0.0)
        frac = valu * 4 / (1024 * 2.4e9 * us * 1e-6) if us > 0 else 0.0
        cells = " | ".join(f"{c.get(k, 0.0) / 1e6:.2f} M" for k in names)
        lines.append(f"| `{key[0]}` | {key[1]} | {key[2]} | {nd} | {us:.1f} | {cells} | {frac:.2f} |")
        st, bst = stage_of(key[0]), batch_stage_of(key[0])
        sha = kernel_source_hash(bst, batched=True) if bst else (kernel_source_hash(st) if st else None)
        ents.append({"kernel": key[0], "workgroups": key[1], "threads": key[2], "dispatches": nd,
                     "us": round(us, 2), "valu_wave_insts": round(valu), "valu_issue": round(frac, 3),
                     "source_sha": sha})
    print("\n".join(lines))
    with open(COUNTERS_JSON, "w") as fh:
        json.dump({"title": title, "command": cmd, "kernels": ents}, fh, indent=1)
        fh.write("\n")


def cpu_baseline(w, x, budget_s: float):
    import numpy as np

    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
    n = 512
    while True:
        idx = np.sort(np.random.default_rng(99).choice(w.grid.npix, size=n, replace=False))
        t0 = time.perf_counter()
        oracle.direct(w.grid, w.profile, w.radius, x, idx=idx, nthreads=threads)
        dt = time.perf_counter() - t0
        if dt >= budget_s / 4 or n >= w.grid.npix:
            break
        n = min(w.grid.npix, int(n * max(2.0, min(16.0, budget_s / 4 / max(dt, 1e-3)))))
    # the same oracle on one core, beside the paper's one-core figures
    n1 = max(64, n // max(threads, 1))
    idx1 = np.sort(np.random.default_rng(98).choice(w.grid.npix, size=n1, replace=False))
    t0 = time.perf_counter()
    oracle.direct(w.grid, w.profile, w.radius, x, idx=idx1, nthreads=1)
    dt1 = time.perf_counter() - t0
    return {"value": n / dt, "unit": "pixels/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} random output pixels of the nside-2048 map (FP64 direct sum, "
                      f"{dt:.1f} s wall), throughput extrapolated per pixel",
            "single_core": {"value": n1 / dt1, "unit": "pixels/s", "cores": 1,
                            "sample": f"{n1} random output pixels, {dt1:.1f} s wall"}}


def time_form(plan, fn, x, y, steps, warmup):
    import torch
    for _ in range(warmup):
        fn(x, out=y)
    torch.cuda.synchronize()
    plan.start_timing(steps)
    t0 = time.perf_counter()
    for _ in range(steps):
        fn(x, out=y)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms, calls = plan.stage_times()
    plan.start_timing(0)
    return wall, [t / max(calls, 1) for t in stage_ms]


def bench_batch(n_maps: int, steps: int, dev):
    """Batched form: n_maps HEALPix maps, nside drawn from {512, 1024, 2048}
    (weights 0.5/0.3/0.2), each with its own Gaussian beam of FWHM U[4', 30']
    truncated at 3 FWHM; N(0,1) white noise generated on the GPU from the
    map's seed; forward and transpose, each one batched call."""
    import torch

    import workloads as W
    from paper_1104_0672_amd import Batch, Plan

    wl = W.batch256(n_maps)
    log(f"bench: batch of {n_maps} maps, building plans")
    t0 = time.perf_counter()
    plans = [Plan.from_workload(w) for w in wl]
    batch = Batch(plans)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    info = batch.info
    npix = int(info.npix_total)
    log(f"bench: batch plans {plan_s:.1f} s, {info.n_items} items, {info.seg_units} units per band "
        f"({info.units_per_wave} per wave), "
        f"grid {info.grid}, {npix / 1e9:.2f} Gpix, workspace {info.workspace_bytes / 2**30:.1f} GiB")
    xs = []
    for w in wl:
        g = torch.Generator(device=dev)
        g.manual_seed(w.seed)
        xs.append(torch.randn(w.grid.npix, generator=g, device=dev, dtype=torch.float32))
    ys = [torch.empty_like(x) for x in xs]
    ws = batch.workspace()
    out = {"n_maps": n_maps, "npix_total": npix, "plan_seconds": round(plan_s, 2),
           "seg_units": int(info.seg_units), "group": int(info.group), "units_per_wave": int(info.units_per_wave),
           "grid": int(info.grid), "items": int(info.n_items)}
    total_alg = 3 * 2 * 4 * npix
    for name, adj in (("forward", False), ("adjoint", True)):
        batch.convolve(xs, outs=ys, adjoint=adj, ws=ws)
        torch.cuda.synchronize()
        batch.start_timing(steps)
        t0 = time.perf_counter()
        for _ in range(steps):
            batch.convolve(xs, outs=ys, adjoint=adj, ws=ws)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st, calls = batch.stage_times()
        batch.start_timing(0)
        ms = 1e3 * wall / steps
        out[name] = {"pixels_per_s": npix * steps / wall, "ms": ms,
                     "hbm_roofline_frac_24B_per_px": round(total_alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "stages_ms": dict(zip(STAGES, [round(t / max(calls, 1), 3) for t in st]))}
        log(f"bench: batch {name} {ms:.2f} ms, {npix * steps / wall:.3e} px/s")
    # the forward call captured once in a hipGraph (through torch.cuda.CUDAGraph) and replayed
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        batch.convolve(xs, outs=ys, ws=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.convolve(xs, outs=ys, ws=ws)
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = 1e3 * wall / steps
    out["graph_forward"] = {"pixels_per_s": npix * steps / wall, "ms": ms,
                            "hbm_roofline_frac_24B_per_px": round(total_alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    log(f"bench: batch forward as a replayed hipGraph {ms:.2f} ms, {npix * steps / wall:.3e} px/s")
    out["valu_issue"] = batched_valu_issue()
    if out["valu_issue"]:
        log("bench: batch VALU issue per stage (committed SQ counters, 64-map batch): "
            + ", ".join(f"{k}={v}" for k, v in out["valu_issue"]["stages"].items()))
    del graph, xs, ys, ws, batch, plans
    torch.cuda.empty_cache()
    return out


def bench_spline(steps: int, dev):
    """The spline-kernel workload (HEALPix nside 1024, 64 knots on [0, 40']):
    forward convolution and the knot gradient of 1/2 |C x - t|^2 given the
    residual, each timed over `steps` calls (wall clock, maps resident)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1104_0672_amd import Plan

    w = W.healpix1024_spline()
    t0 = time.perf_counter()
    plan = Plan.from_workload(w)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    rng = np.random.default_rng(w.seed)
    x = torch.tensor(rng.standard_normal(w.grid.npix), dtype=torch.float32, device=dev)
    r = torch.tensor(rng.standard_normal(w.grid.npix), dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    ws = plan.workspace()
    out = {"workload": w.name, "npix": plan.npix, "oversample": int(plan.info.oversample),
           "plan_seconds": round(plan_s, 2), "table_fft_rows": int(plan.info.table_fft_rows),
           "grad_fft_rows": int(plan.info.grad_fft_rows)}
    log(f"bench: spline plan {plan_s:.2f} s, rows by FFT: tables {plan.info.table_fft_rows}, "
        f"gradient {plan.info.grad_fft_rows}")
    for name, fn in (("forward", lambda: plan.convolve(x, out=y, ws=ws)),
                     ("knot_gradient", lambda: plan.kernel_grad(x, r, ws=ws))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        out[name] = {"ms": round(ms, 3), "pixels_per_s": plan.npix / (ms * 1e-3)}
        log(f"bench: spline {name} {ms:.3f} ms")
    # a knot update on the stream (new samples and K_ij(m) tables), and one
    # training step through the autograd function: forward, loss 1/2 |y - t|^2,
    # backward (transpose for d/dx and the knot gradient), a plain gradient
    # step on the knots (so every step applies new knots)
    from paper_1104_0672_amd import convolve
    knots = torch.tensor(w.profile.knots, dtype=torch.float64, device=dev)
    plan.set_knots_async(knots)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.set_knots_async(knots)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    out["set_knots"] = {"ms": round(ms, 3)}
    log(f"bench: spline set_knots {ms:.3f} ms")
    kp = knots.clone().requires_grad_(True)
    xg = x.clone().requires_grad_(True)
    tgt = r

    def train_step():
        y_ = convolve(xg, plan, kp)
        loss = 0.5 * ((y_ - tgt) ** 2).sum()
        gx, gk = torch.autograd.grad(loss, (xg, kp))
        with torch.no_grad():
            kp.sub_(1e-9 * gk)
        return gx

    train_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        train_step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    out["training_step"] = {"ms": round(ms, 3), "pixels_per_s": plan.npix / (ms * 1e-3),
                            "what": "forward + backward (d/dx and d/dknots) + knot update, autograd"}
    log(f"bench: spline training step {ms:.3f} ms")
    del plan, ws
    torch.cuda.empty_cache()
    return out


def bench_shared(n_kernels: int, steps: int, dev):
    """Shared-input form (an asymmetric beam split into symmetric kernels):
    the nside-2048 input map convolved with n_kernels Gaussian kernels of
    FWHM 4' .. 13' (each cut at 3 FWHM) through one set of input spectra,
    against the same n_kernels convolutions run one plan at a time."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1104_0672_amd import Batch, Plan

    w = W.healpix2048()
    fwhms = np.linspace(4.0, 13.0, n_kernels)
    t0 = time.perf_counter()
    plans = [Plan("healpix", 3.0 * f * W.ARCMIN, nside=2048, fwhm=f * W.ARCMIN) for f in fwhms]
    batch = Batch(plans, shared_input=True)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    x = torch.tensor(W.make_input(w), dtype=torch.float32, device=dev)
    ys = [torch.empty_like(x) for _ in plans]
    ws = batch.workspace()
    out = {"workload": f"healpix2048, {n_kernels} Gaussian kernels FWHM {fwhms[0]:g}'..{fwhms[-1]:g}', R = 3 FWHM",
           "n_kernels": n_kernels, "plan_seconds": round(plan_s, 2),
           "workspace_bytes": int(batch.workspace_bytes)}

    def run_shared():
        batch.convolve_shared(x, outs=ys, ws=ws)

    def run_separate():
        for p, y in zip(plans, ys):
            p.convolve(x, out=y)

    for name, fn in (("shared_input", run_shared), ("one_plan_at_a_time", run_separate)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        out[name] = {"ms": round(ms, 3), "output_pixels_per_s": n_kernels * x.numel() / (ms * 1e-3)}
        log(f"bench: {n_kernels} kernels, {name}: {ms:.3f} ms")
    del batch, plans, ws, ys
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle budget (0: skip)")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--batch-maps", type=int, default=256, help="maps in the batched form (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--spline-steps", type=int, default=5, help="spline-kernel forward and gradient (0: skip)")
    ap.add_argument("--shared-kernels", type=int, default=10,
                    help="kernels of the shared-input form (an asymmetric beam's components; 0: skip)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run a device copy of this size first (for counter calibration)")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="offline: write the per-kernel HBM traffic summary from two counter runs")
    ap.add_argument("--summarize-kernels", metavar="TRACE_DIR",
                    help="offline: print a markdown summary of a kernel-trace run")
    ap.add_argument("--summarize-counters", metavar="COUNTER_CSV",
                    help="offline: print a markdown summary of an SQ instruction-counter run")
    ap.add_argument("--summary-command", default="", help="command line recorded in a summary")
    ap.add_argument("--summary-title", default="")
    ap.add_argument("--summary-only", default="", help="kernel summary: launch shapes of these kernels only")
    ap.add_argument("--summary-top", type=int, default=0, help="kernel summary: first rows of the stats table")
    args = ap.parse_args()
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic, args.copy_calibration_mib,
                          os.path.join(ROOT, "profiles", "traffic_healpix2048_5arcmin.json"), args.summary_command)
        return
    if args.summarize_kernels:
        summarize_kernels(args.summarize_kernels, args.summary_command, args.summary_title,
                          args.summary_only, args.summary_top)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters, args.summary_command, args.summary_title)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the single-map path "
              "would shard by latitude band across GPUs, which is a design only: nothing here runs on more "
              "than one GPU.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_1104_0672_amd import Plan

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration_mib > 0:
        log(f"bench: copy calibration, {args.copy_calibration_mib} MiB")
        copy_calibration(args.copy_calibration_mib, dev)
    w = W.healpix2048()
    log(f"bench: building plan for {w.name}")
    t0 = time.perf_counter()
    plan = Plan.from_workload(w)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    info = plan.info
    log(f"bench: plan {plan_s:.2f} s, oversample {info.oversample}, pairs {info.n_pairs}, "
        f"pair modes {info.pair_modes}, workspace {info.workspace_bytes / 2**20:.0f} MiB")
    xh = W.make_input(w)
    x = torch.tensor(xh, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    plan.workspace()

    log(f"bench: forward, {args.warmup} warmup + {args.steps} timed steps")
    wall, stage_ms = time_form(plan, plan.convolve, x, y, args.steps, args.warmup)
    ms_per_step = 1e3 * wall / args.steps
    value = plan.npix * args.steps / wall
    log(f"bench: forward {ms_per_step:.3f} ms/step, stages (ms) "
        + ", ".join(f"{n}={t:.3f}" for n, t in zip(STAGES, stage_ms)))

    elem = 4
    dom = int(np.argmax(stage_ms))
    stage = STAGES[dom]
    dur_s = stage_ms[dom] * 1e-3
    bytes_per_launch = algorithmic_bytes(stage, plan, elem)
    achieved = bytes_per_launch / dur_s / 1e9
    traffic = measured_traffic(stage)
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": ("accumulate_u_kernel" if stage == "accumulate" and plan.info.acc_units_per_wave > 1
                           else KERNEL_NAMES[stage]),
                "kernel_ms": round(stage_ms[dom], 4), "algorithmic_bytes_per_launch": bytes_per_launch}
    total_alg = 3 * 2 * elem * plan.npix
    forms = {"plain": {"pixels_per_s": value, "ms": ms_per_step,
                       "hbm_roofline_frac_24B_per_px": round(total_alg / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "stages_ms": dict(zip(STAGES, [round(t, 4) for t in stage_ms]))}}

    if not args.no_adjoint:
        steps_a = max(3, args.steps // 2)
        log(f"bench: adjoint, {steps_a} timed steps")
        wall_a, stage_a = time_form(plan, plan.adjoint, x, y, steps_a, 1)
        ms_a = 1e3 * wall_a / steps_a
        forms["adjoint"] = {"pixels_per_s": plan.npix * steps_a / wall_a, "ms": ms_a,
                            "hbm_roofline_frac_24B_per_px": round(total_alg / (ms_a * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                            "stages_ms": dict(zip(STAGES, [round(t, 4) for t in stage_a]))}
        # the paper's plain algorithm of Sect. 4.1 on the same map (plan
        # option mode = 1), for the A/B comparison with the suppressed mode
        log("bench: plain mode of Sect. 4.1 (no artifact suppression)")
        plan_d = Plan.from_workload(w, mode="default")
        plan_d.workspace()
        wall_d, stage_d = time_form(plan_d, plan_d.convolve, x, y, steps_a, 1)
        ms_d = 1e3 * wall_d / steps_a
        log(f"bench: plain mode forward {ms_d:.3f} ms/step")
        forms["forward_sect4_1_without_suppression"] = {"pixels_per_s": plan.npix * steps_a / wall_d, "ms": ms_d,
                                       "pair_modes": int(plan_d.info.pair_modes),
                                       "stages_ms": dict(zip(STAGES, [round(t, 4) for t in stage_d]))}
        del plan_d
    forms["spline"] = None
    if args.spline_steps > 0:
        log("bench: spline kernel, nside 1024")
        forms["spline"] = bench_spline(args.spline_steps, dev)
    forms["shared_input"] = None
    if args.shared_kernels > 0:
        log(f"bench: shared-input form, {args.shared_kernels} kernels")
        forms["shared_input"] = bench_shared(args.shared_kernels, max(3, args.steps // 4), dev)
    forms["batched"] = None
    if args.batch_maps > 0:
        forms["batched"] = bench_batch(args.batch_maps, args.batch_steps, dev)

    cpu = None
    if args.cpu_seconds > 0:
        log("bench: oracle CPU baseline")
        cpu = cpu_baseline(w, xh, args.cpu_seconds)

    out = {"metric": METRIC, "value": value, "unit": "pixels/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": w.name, "nside": 2048, "npix": plan.npix, "fwhm_arcmin": 5.0,
                      "radius_arcmin": 20.0, "oversample": int(info.oversample), "kgen": "auto",
                      "plan_seconds": round(plan_s, 3)},
           "roofline": roofline, "cpu_baseline": cpu, "forms": forms}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
