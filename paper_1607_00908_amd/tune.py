"""Autotuning of the batch size (frames per launch) per lattice-size class.

What varies between workloads is how many frames one launch of each stage
should carry: small lattices need many frames per launch to fill the chip,
large ones fill it with few, and every slot of a batch holds its own per-site
buffers (memory and latency grow with the batch).  The tile shape is not
tuned: the 32x32 tile is fixed by the row-per-wave layout of every per-site
kernel.

tune_batch() times the whole path (every frame's results delivered) for each
candidate batch on frames the caller provides, and choose() picks the batch
with the lowest time per frame, preferring the smaller batch when two are
within `tolerance`.  Results are cached per device name and size class in a
JSON file.
"""
from __future__ import annotations

import json
import os
import time

# size classes by sites per frame: upper bounds (the last class is open)
CLASS_BOUNDS = (1 << 18, 1 << 20, 1 << 22)
CANDIDATES = (1, 2, 4, 8, 16, 32, 64)


def size_class(n_sites: int) -> int:
    """Index of the size class of a lattice with n_sites sites."""
    for k, hi in enumerate(CLASS_BOUNDS):
        if n_sites <= hi:
            return k
    return len(CLASS_BOUNDS)


def choose(us_per_frame: dict, tolerance: float = 0.02) -> int:
    """The batch with the lowest time per frame; a smaller batch wins when its
    time is within `tolerance` (relative) of the best."""
    if not us_per_frame:
        raise ValueError("no timings")
    best = min(us_per_frame.values())
    ok = [b for b, t in us_per_frame.items() if t <= best * (1.0 + tolerance)]
    return min(ok)


def tune_batch(make_detector, fields, candidates=CANDIDATES, frames: int = 64, warmup: int = 8):
    """Time `frames` pushes (after `warmup`) of the device fields (cycled) for
    each candidate batch, every frame's results read back; returns {batch: us
    per frame}.  make_detector(batch) builds a detector with keep_results."""
    import torch
    out = {}
    for b in candidates:
        det = make_detector(b)
        try:
            for i in range(warmup):
                det.push(fields[i % len(fields)])
            det.results(wait=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            got = 0
            for i in range(frames):
                det.push(fields[(warmup + i) % len(fields)])
                if (i + 1) % b == 0:
                    got += len(det.results(wait=False))
            got += len(det.results(wait=True))
            el = time.perf_counter() - t0
        finally:
            det.close()
        if got != frames:
            raise RuntimeError(f"batch {b}: {got} results for {frames} frames")
        out[b] = 1e6 * el / frames
    return out


class TuneCache:
    """Chosen batch per (device name, size class), kept in a JSON file."""

    def __init__(self, path: str):
        self.path = path
        self.data = {}
        if os.path.exists(path):
            with open(path) as fh:
                self.data = json.load(fh)

    def get(self, device: str, n_sites: int):
        return self.data.get(device, {}).get(str(size_class(n_sites)))

    def put(self, device: str, n_sites: int, batch: int, timings: dict) -> None:
        self.data.setdefault(device, {})[str(size_class(n_sites))] = batch
        self.data.setdefault("_timings", {}).setdefault(device, {})[str(size_class(n_sites))] = {
            str(k): round(v, 2) for k, v in timings.items()}
        tmp = self.path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(self.data, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)
