"""Serving many simulation streams on one device with continuous batching.

Each admitted stream owns a detection context (its past centres and couples
stay resident in device memory between frames).  Frames arrive at any time and
wait in the stream's queue; every step sends the oldest waiting frame of each
stream that has one to the device in one launch per stage (a group push over
the subset of streams with work), waits for it and returns the results.  Frames
that arrive while a step runs join the next step.  A stream is admitted only
when the device memory its context needs fits in the free memory left above a
reserve.
"""
from __future__ import annotations

import collections
import time

from . import dv

MAX_STREAMS = 64          # members of one group


def context_bytes(lx: int, ly: int, max_components: int, max_degree: int = 48) -> int:
    """Device memory of a context with one slot (maps kept): per site the
    parent, tile roots, piece lists, label and owner maps and segment words;
    per component the frame and two past component sets with their rows, the
    sums, the grid, the matching and the staged and placed flips."""
    n = lx * ly
    per_site = 4 + 2 + 2 + 4 + 4 + 1
    per_comp = 3 * (36 + 4 * max_degree) + 28 + 20 + 24 + 16 + 72 * max_degree
    return n * per_site + max_components * per_comp + (1 << 20)


class Server:
    """Continuous batching of frames from many streams (one device, one HIP
    stream shared by all contexts)."""

    def __init__(self, device: int = 0, reserve_bytes: int = 4 << 30):
        import torch
        self._torch = torch
        self.device = device
        self.reserve = reserve_bytes
        self.stream = torch.cuda.Stream(device=device)
        self.dets: list[dv.Detector] = []
        self.queues: list[collections.deque] = []
        self.group = None

    def admit(self, lx: int, ly: int, threshold: float, phase: int = dv.PHASE_ABOVE,
              connectivity: int = 8, max_components: int = 4096):
        """Open a stream; returns its id, or None when the device memory it
        needs is not free (above the reserve) or the server is full."""
        if len(self.dets) >= MAX_STREAMS:
            return None
        free, _ = self._torch.cuda.mem_get_info(self.device)
        if free - context_bytes(lx, ly, max_components) < self.reserve:
            return None
        det = dv.Detector(lx, ly, threshold, phase, connectivity, max_components=max_components,
                          keep_maps=True, device=self.device, stream=self.stream, max_batch=1)
        self.dets.append(det)
        self.queues.append(collections.deque())
        if self.group is not None:
            self.group.close()
            self.group = None
        return len(self.dets) - 1

    def submit(self, sid: int, field, tag=None, t_arrival: float | None = None) -> None:
        """Queue a frame of stream sid (float32 device tensor [ly, lx], kept
        alive by the server until its result is returned)."""
        self.queues[sid].append((field, tag, time.perf_counter() if t_arrival is None else t_arrival))

    def pending(self) -> int:
        return sum(len(q) for q in self.queues)

    def step(self, collect: bool = True):
        """Send the oldest waiting frame of every stream that has one, wait for
        them and return [(sid, tag, t_arrival, t_done, info, flips)] (info and
        flips None when collect is False)."""
        members = [i for i, q in enumerate(self.queues) if q]
        if not members:
            return []
        if self.group is None:
            self.group = dv.Group(self.dets)
        items = [self.queues[i].popleft() for i in members]
        self.group.push_some(members, [it[0] for it in items])
        self.dets[members[0]].sync()
        t_done = time.perf_counter()
        out = []
        for i, (f, tag, ta) in zip(members, items):
            info = fl = None
            if collect:
                d = self.dets[i]
                info = d.info()
                fl = d.flips() if info.status == 0 else None
            out.append((i, tag, ta, t_done, info, fl))
        return out

    def close(self):
        if self.group is not None:
            self.group.close()
            self.group = None
        for d in self.dets:
            d.close()
        self.dets = []
