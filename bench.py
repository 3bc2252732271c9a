"""Benchmark of the per-frame detection path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload disks1024|grf4096|channel2048]
python bench.py --workload mixed64 [--fields 64] [--frames 5] [--steps 20]
python bench.py --workload serve32 [--fields 32] [--gap-ms 2] [--steps 10000]

A step is one frame through the whole path (threshold, labelling, centres,
digital Voronoi, Delaunay couples, matching, flips) on synthetic input of the
workload's shape, its record and flips delivered to the host.  The default
workload is the 4096^2 AR(1) Gaussian random field.  All frames of the ring
are resident in HBM before the timed region (at least 768 MB of distinct
frames, larger than the 256 MB Infinity Cache); steps cycle through the ring.
The timed region ends when every frame's results are on the host.  Prints one
JSON line.

Reported beside the throughput:
  roofline      one stage timed with HIP events on the context's stream over the
                timed region; algorithmic bytes per launch / mean duration
  latency_ms    p50 / p99 of push -> flips returned (host-synchronous loop)
  flips_only    the same frames without label / owner maps (4 B/site compulsory)
  unbatched     the same frames with one frame per launch
  copy ceiling  a plain device copy timed with HIP events (roofline.copy_ceiling_gbs)
  cpu_baseline  the CPU oracle on a bounded sample of the same frames, with the
                host's CPU model and core counts

HBM traffic of the roofline stage comes from two rocprofv3 counter runs
(FETCH_SIZE, then WRITE_SIZE) of this script with --copy-probe-mib, which first
runs a plain elementwise copy of known size in the same process; the counters
of that copy give the scale from counter KiB to bytes.  --counters-from turns
the two CSV outputs into profiles/counters.json, keyed by the stage's source
hash so that a changed kernel reports traffic null until counted again.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
# compulsory HBM bytes per site of each per-site stage (maps kept / flips only)
STAGE_BYTES = {
    "tile_ccl": (4, 4),        # field read
    "relabel": (4, 0),         # label map write
    "owner_edges": (4, 0),     # owner map write
}
# with an obstacle mask, both of these also read its byte per site
OBSTACLE_BYTES = {"tile_ccl": 1, "owner_edges": 1}
STAGE_SOURCES = {
    "tile_ccl": "k_label.hip", "relabel": "k_label.hip", "owner_edges": "k_voronoi.hip",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(stage: str) -> str:
    p = os.path.join(ROOT, "paper_1607_00908_amd", "csrc", STAGE_SOURCES[stage])
    h = hashlib.sha256()
    for f in sorted({p, os.path.join(ROOT, "paper_1607_00908_amd", "csrc", "dv_internal.h"),
                     os.path.join(ROOT, "paper_1607_00908_amd", "csrc", "dv_device.h")}):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def _default_batch() -> int:
    from paper_1607_00908_amd import dv
    return dv.DEFAULT_BATCH


def counter_key(stage: str, workload: str, maps: bool, frames: int) -> str:
    """Key of a counter entry: stage, workload, mode and the frames per launch."""
    return f"{stage}:{workload}:{'maps' if maps else 'flips'}:frames{frames}"


def counter_traffic(stage: str, workload: str, maps: bool, frames: int):
    """HBM bytes per launch of `frames` frames from the committed rocprofv3
    counter summary, when it was taken on the current source of the stage and
    at that launch size; else None."""
    p = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except ValueError:
        return None
    e = d.get(counter_key(stage, workload, maps, frames))
    if not e or e.get("source_sha") != source_hash(stage):
        return None
    return int(round(e["bytes_per_dispatch"]))


COPY_PROBE_REPS = 8


def copy_probe(mib: int):
    """A plain elementwise copy (read 4 B, write 4 B per element) of known size,
    the calibration kernel for the HBM counters."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, device="cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(COPY_PROBE_REPS):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    del a, b


def _read_counter_csv(path: str):
    """(kernel name, grid size, counter value) per dispatch from a rocprofv3
    counter CSV."""
    import csv
    out = {}
    with open(path, newline="") as fh:
        for row in csv.DictReader(fh):
            key = (row.get("Dispatch_Id") or row.get("Correlation_Id"), row["Counter_Name"])
            out[key] = (row["Kernel_Name"], int(row.get("Grid_Size") or 0),
                        float(row["Counter_Value"]))
    return list(out.values())


def counters_from(fetch_csv: str, write_csv: str, stage: str, workload: str, maps: bool,
                  copy_mib: int, frames: int):
    """Scaled HBM bytes per dispatch of `stage` from FETCH_SIZE / WRITE_SIZE runs."""
    import statistics
    kname = "k_" + stage
    res = {}
    for tag, path in (("fetch", fetch_csv), ("write", write_csv)):
        rows = _read_counter_csv(path)
        # dispatches of the full batch only (the largest grid of the kernel)
        kr = [(g, v) for k, g, v in rows if re.search(r"\b%s\b" % kname, k)]
        gmax = max((g for g, _ in kr), default=0)
        ker = [v for g, v in kr if g == gmax]
        cpy = [v for k, g, v in rows if "neg" in k.lower()]
        if not ker or not cpy:
            raise SystemExit(f"{path}: no dispatches of {kname} or of the copy probe")
        expect_kib = copy_mib * 1024.0
        scale = expect_kib / statistics.median(cpy)
        res[tag] = {"kib_per_dispatch": statistics.mean(ker), "dispatches": len(ker),
                    "copy_kib_median": statistics.median(cpy), "copy_expected_kib": expect_kib,
                    "scale": scale}
    bytes_per = sum(r["kib_per_dispatch"] * r["scale"] * 1024.0 for r in res.values())
    p = os.path.join(ROOT, "profiles", "counters.json")
    d = json.load(open(p)) if os.path.exists(p) else {}
    d[counter_key(stage, workload, maps, frames)] = {
        "source_sha": source_hash(stage), "bytes_per_dispatch": bytes_per, **res}
    with open(p, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
    print(json.dumps({"stage": stage, "bytes_per_dispatch": round(bytes_per), **res}))


def trace_from(csv_path: str, title: str, command: str):
    """Markdown summary of a rocprofv3 kernel-trace CSV: dispatches grouped by
    kernel and launch grid, mean and total duration, largest grids first."""
    import collections
    import csv
    groups = collections.defaultdict(list)
    with open(csv_path, newline="") as fh:
        for row in csv.DictReader(fh):
            name = row.get("Kernel_Name", "")
            if not re.search(r"\bk_[a-z_]+", name):
                continue
            grid = ",".join(row.get(k, "?") for k in ("Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"))
            if grid == "?,?,?":
                grid = row.get("Grid_Size", "?")
            dur = (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1e3
            short = re.sub(r"\(.*", "", name.replace("(anonymous namespace)::", "")).strip()
            groups[(short, grid)].append(dur)
    rows = sorted(groups.items(), key=lambda kv: (-max(int(x) if x.isdigit() else 0
                                                       for x in kv[0][1].split(",")),
                                                  -sum(kv[1])))
    out = [f"# {title}", "", "Command (from the repository root, on one MI355X):", "",
           "    cd /tmp && export TMPDIR=/tmp && cd -", f"    {command}",
           f"    python bench.py --trace-from <kernel_trace.csv> --title '...' --command '...'", "",
           "| kernel | grid (x,y,z) | launches | mean us | total us |", "|---|---|---|---|---|"]
    for (k, g), d in rows:
        out.append(f"| {k} | {g} | {len(d)} | {sum(d) / len(d):.2f} | {sum(d):.0f} |")
    print("\n".join(out))


def unbatched_rate(dv, args, spec, lx, ly, kmax, maps, stream, ptrs, F, N, geom):
    """The same pushes with one frame per launch of each stage, every frame's
    results delivered as in the batched run."""
    det1 = dv.Detector(lx, ly, spec["threshold"], spec["phase"], 8, max_components=kmax,
                       keep_maps=maps, max_batch=1, stream=stream, keep_results=True, **geom)
    n1 = min(args.steps, 500)
    el1, got, _, _ = timed_run(dv, det1, ptrs, n1, args.warmup, None, 1)
    det1.close()
    log(f"max_batch 1: {1e6 * el1 / n1:.1f} us/frame")
    return {"max_batch": 1, "value": round(N * n1 / el1 / 1e6, 2), "unit": "Msites/s",
            "ms_per_step": round(1e3 * el1 / n1, 5), "steps": n1}


def _mixed_frames(args):
    """Frames of field i of the mixed batch (runs in a worker process)."""
    i, n, nf = args
    from paper_1607_00908_amd import synth
    sim, spec = synth.mixed_fields(n)[i]
    return list(sim.frames(nf)), spec


def bench_mixed(args):
    """Batching of many independent fields: one group launch per stage for all
    fields against the same frames pushed field by field with one launch per
    stage each.  Prints one JSON line."""
    import concurrent.futures as cf
    import torch
    from paper_1607_00908_amd import dv
    n, nf = args.fields, args.frames or 5
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        res = list(ex.map(_mixed_frames, [(i, n, nf) for i in range(n)]))
    log(f"generated {n} fields x {nf} frames in {time.perf_counter() - t0:.1f} s")
    specs = [sp for _, sp in res]
    sites = sum(sp["lx"] * sp["ly"] for sp in specs)
    rings = [torch.from_numpy(np.stack(fr)).cuda() for fr, _ in res]
    torch.cuda.synchronize()
    ptrs = [[r[k].data_ptr() for k in range(nf)] for r in rings]
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)

    def make():
        return [dv.Detector(sp["lx"], sp["ly"], sp["threshold"], sp["phase"], 8,
                            max_components=4 * sp["k_expect"] + 256, keep_maps=True,
                            max_batch=1, stream=stream, keep_results=True) for sp in specs]

    def collect(dets, wait):
        n = 0
        for d in dets:
            res = d.results(wait=wait)
            assert all(fi.status == 0 for fi, _ in res)
            n += len(res)
        return n

    # one launch per stage for all fields; every frame's results are read
    # (without waiting) every 4 steps and at the end
    dets = make()
    grp = dv.Group(dets)
    for w in range(args.warmup):
        grp.push([p[w % nf] for p in ptrs])
    collect(dets, True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    delivered = 0
    for k in range(args.steps):
        grp.push([p[(args.warmup + k) % nf] for p in ptrs])
        if k % 4 == 3:
            delivered += collect(dets, False)
    delivered += collect(dets, True)
    el_g = time.perf_counter() - t1
    assert delivered == n * args.steps, (delivered, n * args.steps)
    infos = [d.info() for d in dets]
    assert all(fi.status == 0 for fi in infos), [fi.status for fi in infos]
    grp.close()
    for d in dets:
        d.close()
    # the same frames, field by field (one launch per stage per field)
    dets = make()
    for w in range(args.warmup):
        for d, p in zip(dets, ptrs):
            d.push(p[w % nf])
    collect(dets, True)
    t1 = time.perf_counter()
    delivered = 0
    for k in range(args.steps):
        for d, p in zip(dets, ptrs):
            d.push(p[(args.warmup + k) % nf])
        if k % 4 == 3:
            delivered += collect(dets, False)
    delivered += collect(dets, True)
    el_s = time.perf_counter() - t1
    assert delivered == n * args.steps
    for d in dets:
        d.close()
    v_g = sites * args.steps / el_g / 1e6
    v_s = sites * args.steps / el_s / 1e6
    print(json.dumps({
        "metric": f"Msites/s, {n} independent fields of uneven sizes, one launch per stage for all",
        "value": round(v_g, 2), "unit": "Msites/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * el_g / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32->int64",
        "data": "synthetic",
        "config": {"workload": f"mixed{n}", "fields": n, "frames_in_ring": nf,
                   "sites_per_step": sites, "side_min": min(sp["lx"] for sp in specs),
                   "side_max": max(sp["lx"] for sp in specs),
                   "disk_fields": sum(1 for sp in specs if sp["kind"] == "disks"),
                   "components": sum(fi.n_components for fi in infos),
                   "parallelism": "single-gpu"},
        "delivered": "every frame's record and flips read inside the timed region",
        "field_by_field": {"value": round(v_s, 2), "unit": "Msites/s",
                           "ms_per_step": round(1e3 * el_s / args.steps, 4)},
        "speedup": round(v_g / v_s, 3)}))


def _serve_frames(args):
    i, n, nf, seed, lmin, lmax = args
    from paper_1607_00908_amd import synth
    sim, spec = synth.mixed_fields(n, seed=seed, l_min=lmin, l_max=lmax)[i]
    return list(sim.frames(nf)), spec


def bench_serve(args):
    """Continuous batching under Poisson arrivals: `fields` streams, sides
    log-uniform in [512, 4096], frames arriving with exponential gaps of mean
    `gap_ms` per stream until `steps` frames in all.  Throughput and latency
    (arrival to results ready) of the served frames.  Prints one JSON line."""
    import concurrent.futures as cf
    import torch
    from paper_1607_00908_amd import serve
    n, nf = args.fields, args.frames or 3
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        res = list(ex.map(_serve_frames, [(i, n, nf, 5, 512, 4096) for i in range(n)]))
    log(f"generated {n} streams x {nf} frames in {time.perf_counter() - t0:.1f} s")
    specs = [sp for _, sp in res]
    rings = [torch.from_numpy(np.stack(fr)).cuda() for fr, _ in res]
    torch.cuda.synchronize()
    srv = serve.Server(reserve_bytes=8 << 30)
    sids = [srv.open(sp["lx"], sp["ly"], sp["threshold"], sp["phase"],
                     max_components=4 * sp["k_expect"] + 256) for sp in specs]
    admitted = [i for i, s in enumerate(sids) if srv.admitted(s)]
    # warm-up: every stream's first frames
    for w in range(2):
        for i in admitted:
            srv.submit(sids[i], rings[i][w % nf])
        srv.drain()
    # arrival times (seconds from the start), per stream a Poisson process
    rng = np.random.default_rng(17)
    arrivals = []
    per = -(-args.steps // len(admitted))
    for i in admitted:
        t = np.cumsum(rng.exponential(args.gap_ms * 1e-3, per))
        arrivals += [(float(tt), i, k) for k, tt in enumerate(t)]
    arrivals.sort()
    arrivals = arrivals[:args.steps]
    lat, sites, batches, served, flips, ok = [], 0, 0, 0, 0, True
    j = 0
    start = time.perf_counter()
    while served < len(arrivals):
        now = time.perf_counter() - start
        while j < len(arrivals) and arrivals[j][0] <= now:
            ta, i, k = arrivals[j]
            srv.submit(sids[i], rings[i][(k + 2) % nf], tag=i, t_arrival=start + ta)
            j += 1
        if not srv.pending():
            time.sleep(max(0.0, min(arrivals[j][0] - now, 1e-3)))
            continue
        out = srv.step()
        if out:
            batches += 1
        for sid, i, ta, td, info, fl in out:
            lat.append(td - ta)
            sites += specs[i]["lx"] * specs[i]["ly"]
            served += 1
            flips += len(fl)
            ok = ok and info.status == 0
    elapsed = time.perf_counter() - start
    srv.shutdown()
    lat = np.array(lat) * 1e3
    offered = sum(specs[i]["lx"] * specs[i]["ly"] for i in admitted) / (args.gap_ms * 1e-3) / 1e6
    print(json.dumps({
        "metric": "Msites/s served, continuous batching of Poisson frame arrivals; p50/p99 latency",
        "value": round(sites / elapsed / 1e6, 2), "unit": "Msites/s", "n_gpus": 1,
        "steps": len(arrivals), "warmup": 2, "ms_per_step": round(1e3 * elapsed / len(arrivals), 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32->int64",
        "data": "synthetic",
        "config": {"workload": f"serve{n}", "streams": n, "admitted": len(admitted),
                   "gap_ms": args.gap_ms, "offered_msites_s": round(offered, 1),
                   "side_min": min(sp["lx"] for sp in specs), "side_max": max(sp["lx"] for sp in specs),
                   "mean_sites_per_frame": round(float(np.mean([sp["lx"] * sp["ly"] for sp in specs]))),
                   "parallelism": "single-gpu"},
        "frames_per_s": round(len(arrivals) / elapsed, 1), "batches": batches,
        "mean_batch": round(len(arrivals) / max(batches, 1), 2), "all_accepted": ok,
        "delivered_flips": flips,
        "latency": "arrival to the frame's record and flips on the host",
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                       "p99": round(float(np.percentile(lat, 99)), 3), "samples": len(lat)}}))


def make_frames(workload: str, frames: int | None):
    """(frames, spec, geometry keywords: walls and the obstacle mask)."""
    from paper_1607_00908_amd import synth
    sim, spec = synth.workload(workload)
    if frames is None:
        # a ring larger than the 256 MB Infinity Cache, so field reads come from HBM
        per = spec["lx"] * spec["ly"] * 4
        frames = min(spec["frames"], max(8, -(-(768 << 20) // per)))
    out = list(sim.frames(frames))
    geom = {"open_x": bool(spec.get("open_x", False)), "open_y": bool(spec.get("open_y", False)),
            "obstacles": sim.obstacles() if hasattr(sim, "obstacles") else None}
    return out, spec, geom


def host_cpu():
    """CPU model and the cores this process may use (the oracle's host)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def cpu_baseline(frames, spec, seconds: float, geom, threads: int):
    """The oracle (as it stands) on the first frames of the workload, whole
    path, until about `seconds` of work have passed (at least two frames, so
    that one comparison is included)."""
    import oracle
    ly, lx = frames[0].shape
    seq = oracle.Sequence(spec["threshold"], spec["phase"], 8, nthreads=threads, **geom)
    t0 = time.perf_counter()
    n = 0
    for f in frames:
        seq.push(f)
        n += 1
        if n >= 2 and time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    model, ncpu, usable = host_cpu()
    return {"value": round(n * lx * ly / dt / 1e6, 4), "unit": "Msites/s", "cores": threads,
            "kind": "oracle",
            "sample": f"frames 0-{n - 1} of {spec.get('name', '')} ({n} frames, {n - 1} "
                      f"comparisons), whole path, {threads} thread(s) (OpenMP over sites in the "
                      f"colouring, the rest sequential), {dt:.1f} s",
            "cpu_model": model, "nproc": ncpu, "usable_cpus": usable}


def measure_copy_ceiling(gib: float = 2.0, reps: int = 10):
    """Bandwidth of a plain device copy (read + write) of `gib` GiB, timed with
    HIP events: the measured ceiling beside the 8 TB/s peak."""
    import torch
    n = int(gib * (1 << 30)) // 4
    a = torch.ones(n, device="cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return round(2 * n * 4 / (ms * 1e-3) / 1e9, 1)


def timed_run(dv, det, ptrs, steps: int, warmup: int, stage: str | None, batch: int):
    """Push `steps` frames (after `warmup`) and return every frame's results;
    the timed region ends when all of them are on the host.  Results are read
    without waiting after each full batch, so the host copies one batch's
    flips while the next one runs.  The flips land in one pinned host buffer
    allocated before the timed region (sized from the warm-up frames; frames
    that do not fit are read into a fresh array at the end)."""
    import torch
    F = len(ptrs)
    for i in range(warmup):
        det.push(ptrs[i % F])
    warm = det.results(wait=True)
    per = max([fi.n_flips for fi, _ in warm] + [0])
    cap = steps * (2 * per + 256)
    buf = torch.empty((cap, 6), dtype=torch.int32, pin_memory=True).numpy()
    if stage:
        det.set_profile(stage, capacity=steps)
    torch.cuda.synchronize()
    got = []
    used = 0

    def take(wait):
        nonlocal used
        res = det.results(wait=wait, out=buf[used:])
        used += sum(fi.n_flips for fi, _ in res)
        return res

    t0 = time.perf_counter()
    for i in range(steps):
        det.push(ptrs[(warmup + i) % F])
        if (i + 1) % batch == 0:
            got += take(False)
    got += take(True)
    if len(got) < steps:
        got += det.results(wait=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stage_ms, launches = det.get_profile() if stage else (0.0, 0)
    if stage:
        det.set_profile(None)
    assert len(got) == steps, (len(got), steps)
    assert all(fi.status == 0 for fi, _ in got), [fi.status for fi, _ in got]
    return elapsed, got, stage_ms, launches


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--workload", default="grf4096")
    ap.add_argument("--frames", type=int, default=None, help="frames in the ring (default: >= 768 MB)")
    ap.add_argument("--fields", type=int, default=64,
                    help="fields of the mixed workload (streams of the serving one: 32)")
    ap.add_argument("--gap-ms", type=float, default=2.0,
                    help="mean gap between frame arrivals of one stream (serving)")
    ap.add_argument("--flips-only", action="store_true", help="do not write label / owner maps")
    ap.add_argument("--stage", default="owner_edges", help="stage timed for the roofline")
    ap.add_argument("--max-batch", type=int, default=0,
                    help="frames per launch of each stage (0: the library default)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick max_batch with the autotuner (timed over the candidates first)")
    ap.add_argument("--latency-frames", type=int, default=1000)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="oracle threads for the CPU baseline (0: 1 below 4096^2, else up to 16)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--weighted", action="store_true",
                    help="density-weighted centres (the centroid of Sec. 2 with the field as density)")
    ap.add_argument("--no-unbatched", action="store_true",
                    help="skip the one-frame-per-launch comparison run")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the timed run (no flips-only run, copy ceiling, latency)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run the counter calibration copy of this size first")
    ap.add_argument("--counters-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/counters.json from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--trace-from", metavar="KERNEL_TRACE_CSV",
                    help="print a markdown summary of a rocprofv3 kernel trace and exit")
    ap.add_argument("--title", default="Kernel trace")
    ap.add_argument("--command", default="")
    args = ap.parse_args()

    if args.trace_from:
        trace_from(args.trace_from, args.title, args.command)
        return

    if args.counters_from:
        counters_from(*args.counters_from, args.stage, args.workload, not args.flips_only,
                      args.copy_probe_mib, launch_frames(args))
        return

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        log("bench.py measures one GPU only (no multi-GPU path in this build)")
        sys.exit(2)
    if args.workload.startswith("mixed"):
        if args.steps == 64:
            args.steps = 20
        bench_mixed(args)
        return
    if args.workload.startswith("serve"):
        if args.steps == 64:
            args.steps = 10000
        if args.fields == 64:
            args.fields = 32
        bench_serve(args)
        return

    import torch
    from paper_1607_00908_amd import dv

    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
    t0 = time.perf_counter()
    frames, spec, geom = make_frames(args.workload, args.frames)
    geom["weighted"] = bool(args.weighted)
    spec["name"] = args.workload
    ly, lx = frames[0].shape
    N = lx * ly
    log(f"generated {len(frames)} frames {lx}x{ly} in {time.perf_counter() - t0:.1f} s")

    dev = torch.device("cuda", 0)
    ring = torch.from_numpy(np.stack(frames)).to(dev)
    torch.cuda.synchronize()
    maps = not args.flips_only
    kmax = 32768 if N > (1 << 22) else 4096
    autotune = None
    if args.autotune:
        from paper_1607_00908_amd import tune
        cands = tuple(b for b in tune.CANDIDATES if b >= (8 if N >= (1 << 22) else 1))
        t_us = tune.tune_batch(
            lambda b: dv.Detector(lx, ly, spec["threshold"], spec["phase"], 8, max_components=kmax,
                                  keep_maps=maps, max_batch=b, keep_results=True, **geom),
            [ring[i] for i in range(ring.shape[0])], candidates=cands, frames=64)
        args.max_batch = tune.choose(t_us)
        autotune = {"us_per_frame": {str(k): round(v, 2) for k, v in t_us.items()},
                    "chosen": args.max_batch, "size_class": tune.size_class(N)}
        log(f"autotune: {autotune}")
    batch = args.max_batch or dv.DEFAULT_BATCH
    det = dv.Detector(lx, ly, spec["threshold"], spec["phase"], 8, max_components=kmax,
                      keep_maps=maps, max_batch=args.max_batch, keep_results=True, **geom)
    F = ring.shape[0]
    # the ring is complete on the device (synchronised above): frames are
    # pushed as raw device pointers, no per-push stream bookkeeping
    torch.cuda.set_stream(det.stream)
    ptrs = [ring[i].data_ptr() for i in range(F)]

    elapsed, got, stage_ms, launches = timed_run(dv, det, ptrs, args.steps, args.warmup,
                                                 args.stage, batch)
    n_flips = sum(fi.n_flips for fi, _ in got)
    info = got[-1][0]
    ms_per_step = 1e3 * elapsed / args.steps
    msites = N * args.steps / elapsed / 1e6
    log(f"timed {args.steps} steps: {ms_per_step * 1e3:.1f} us/frame, {msites:.0f} Msites/s, "
        f"{n_flips} flips delivered; K={info.n_components} E={info.n_edges}")

    extras = {}
    if not args.no_extras:
        # flips-only mode (no label / owner maps): compulsory traffic 4 B/site
        if maps:
            det_f = dv.Detector(lx, ly, spec["threshold"], spec["phase"], 8, max_components=kmax,
                                keep_maps=False, max_batch=args.max_batch, keep_results=True,
                                stream=det.stream, **geom)
            el_f, got_f, _, _ = timed_run(dv, det_f, ptrs, args.steps, args.warmup, None, batch)
            det_f.close()
            for (a, fa), (b, fb) in zip(got, got_f):
                assert a == b and np.array_equal(fa, fb), "flips-only results differ"
            v_f = N * args.steps / el_f / 1e6
            log(f"flips-only: {1e6 * el_f / args.steps:.1f} us/frame")
            extras["flips_only"] = {"value": round(v_f, 2), "unit": "Msites/s",
                                    "ms_per_step": round(1e3 * el_f / args.steps, 5),
                                    "hbm_frac_4B": round(v_f * 1e6 * 4 / (HBM_PEAK_GBS * 1e9), 5)}
        # latency: push -> flips returned, host-synchronous
        lat = []
        for i in range(args.latency_frames):
            a = time.perf_counter()
            det.push(ptrs[i % F])
            det.flips()
            lat.append(time.perf_counter() - a)
        det.results(wait=True)    # the latency frames' records, not counted
        lat = np.array(lat) * 1e3
        extras["latency_ms"] = {"p50": round(float(np.percentile(lat, 50)), 4),
                                "p99": round(float(np.percentile(lat, 99)), 4),
                                "samples": len(lat)}

    # the same pushes with one frame per launch (no batching), for comparison
    unbatched = None
    if not args.no_unbatched:
        unbatched = unbatched_rate(dv, args, spec, lx, ly, kmax, maps, det.stream, ptrs, F, N, geom)
    copy_gbs = None if args.no_extras else measure_copy_ceiling()

    # one launch of a stage covers every frame of a batch
    stage_avg_ms = stage_ms / max(launches, 1)
    frames_per_launch = args.steps / max(launches, 1)
    has_obst = geom["obstacles"] is not None
    per_site = STAGE_BYTES.get(args.stage, (0, 0))[0 if maps else 1]
    per_site += OBSTACLE_BYTES.get(args.stage, 0) if has_obst else 0
    alg_bytes = per_site * N * frames_per_launch
    achieved = alg_bytes / (stage_avg_ms * 1e-3) / 1e9 if stage_avg_ms > 0 else 0.0
    fpl = int(round(frames_per_launch)) if abs(frames_per_launch - round(frames_per_launch)) < 1e-9 else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": (counter_traffic(args.stage, args.workload, maps, fpl)
                            if fpl is not None else None),
                "kernel": args.stage, "launch_us": round(stage_avg_ms * 1e3, 2),
                "launches": launches, "frames_per_launch": round(frames_per_launch, 3),
                "algorithmic_bytes_per_launch": int(round(alg_bytes)),
                "copy_ceiling_gbs": copy_gbs}

    out = {
        "metric": "Msites/s through label+Voronoi+flip pipeline (%HBM peak); p50/p99 frame latency",
        "value": round(msites, 2),
        "unit": "Msites/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32->int64",
        "data": "synthetic",
        "config": {"workload": args.workload, "lx": lx, "ly": ly, "frames_in_ring": F,
                   "components": info.n_components, "edges": info.n_edges,
                   "mode": "maps+flips" if maps else "flips-only",
                   "walls": "".join(a for a in ("x", "y") if geom[f"open_{a}"]) or "none",
                   "obstacle_sites": int(geom["obstacles"].sum()) if has_obst else 0,
                   "max_batch": batch, "centres": "weighted" if args.weighted else "unit weight",
                   "parallelism": "single-gpu"},
        "delivered": {"frames": len(got), "flips": n_flips,
                      "note": "every frame's record and flips copied to the host inside the "
                              "timed region"},
        "frames_per_s": round(args.steps / elapsed, 1),
        "hbm_frac_pipeline": round(msites * 1e6 * ((12 if maps else 4) + (2 if has_obst else 0))
                                   / (HBM_PEAK_GBS * 1e9), 5),
        **extras,
        "roofline": roofline,
        "unbatched": unbatched,
    }
    if autotune:
        out["autotune"] = autotune
    if not args.no_cpu_baseline:
        threads = args.cpu_threads or (1 if N < (1 << 24) else min(16, host_cpu()[2]))
        log(f"cpu baseline (oracle, {threads} thread(s)) ...")
        out["cpu_baseline"] = cpu_baseline(frames, spec, args.cpu_seconds, geom, threads)
    det.close()
    print(json.dumps(out))


def launch_frames(args) -> int:
    """Frames per launch of the timed region: full batches, or the one partial
    launch when the steps are fewer than a batch."""
    b = args.max_batch or _default_batch()
    return b if args.steps >= b else args.steps


if __name__ == "__main__":
    main()
