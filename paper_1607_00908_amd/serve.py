"""Serving many simulation streams on one device with continuous batching.

Each admitted stream owns a detection context: its past centres and couples
stay resident in device memory between frames (the sequence state of the
paper's Sec. 3.2.3), and every frame's record and flips are kept until they are
returned (Sec. 3.2.4).  Frames arrive at any time and wait in their stream's
queue.  A step sends the oldest waiting frame of every admitted stream that
has one to the device in one launch per stage (a group push over that subset,
any lattice sizes); up to `depth` steps are in flight, so the next step is
enqueued before the host waits for the previous one and frames that arrive
meanwhile join it.

Streams are admitted when the device memory their context needs is free:
`open` returns a stream id at once, and the stream waits in the admission
queue until free device memory (above a reserve, and within an optional byte
budget) covers its context; `close` retires a stream once its frames are
served, which frees its context and lets waiting streams in.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

from . import dv

MAX_STREAMS = 64          # members of one group


def context_bytes(lx: int, ly: int, max_components: int, max_degree: int = 0, max_batch: int = 1,
                  open_x: bool = False, open_y: bool = False, obstacles=None) -> int:
    """Device memory of a serving context (results kept, no maps), as the
    library lays it out."""
    return dv.device_bytes(lx, ly, max_components=max_components, max_degree=max_degree,
                           keep_maps=False, max_batch=max_batch, keep_results=True,
                           open_x=open_x, open_y=open_y, with_obstacles=obstacles is not None)


@dataclass
class _Stream:
    sid: int
    params: dict
    need: int                          # estimated device bytes of the context
    det: dv.Detector | None = None     # None until admitted
    queue: collections.deque = field(default_factory=collections.deque)
    inflight: collections.deque = field(default_factory=collections.deque)  # (tag, t_arrival, field)
    closing: bool = False


class Server:
    """Continuous batching of frames from many streams (one device, one HIP
    stream shared by all contexts).

    reserve_bytes: device memory left free when admitting a stream.
    budget_bytes: optional cap on the summed context memory of the admitted
    streams.  depth: steps in flight (1: every step waits for its own frames).
    """

    def __init__(self, device: int = 0, reserve_bytes: int = 4 << 30,
                 budget_bytes: int | None = None, depth: int = 2):
        import torch
        self._torch = torch
        self.device = device
        self.reserve = reserve_bytes
        self.budget = budget_bytes
        self.depth = max(1, int(depth))
        self.stream = torch.cuda.Stream(device=device)
        self.streams: dict[int, _Stream] = {}
        self.admission: collections.deque[int] = collections.deque()
        self.members: list[int] = []      # sids of the current group, in member order
        self.group = None
        self.steps: collections.deque = collections.deque()   # (event, [sid, ...])
        self._next_sid = 0

    # -- stream lifecycle ----------------------------------------------------
    def open(self, lx: int, ly: int, threshold: float, phase: int = dv.PHASE_ABOVE,
             connectivity: int = 8, max_components: int = 4096, **geometry) -> int:
        """Request a stream; returns its id.  It is admitted now if its context
        fits, else when enough memory is freed (frames may be submitted
        meanwhile and wait)."""
        sid = self._next_sid
        self._next_sid += 1
        params = dict(lx=lx, ly=ly, threshold=threshold, phase=phase,
                      connectivity=connectivity, max_components=max_components, **geometry)
        self.streams[sid] = _Stream(sid, params, context_bytes(lx, ly, max_components, **geometry))
        self.admission.append(sid)
        self._admit()
        return sid

    def admit(self, lx: int, ly: int, threshold: float, phase: int = dv.PHASE_ABOVE,
              connectivity: int = 8, max_components: int = 4096, **geometry):
        """Open a stream only if it is admitted at once; else None."""
        sid = self.open(lx, ly, threshold, phase, connectivity, max_components, **geometry)
        if self.streams[sid].det is None:
            self.admission.remove(sid)
            del self.streams[sid]
            return None
        return sid

    def admitted(self, sid: int) -> bool:
        return self.streams[sid].det is not None

    def close(self, sid: int) -> None:
        """No more frames for this stream: it retires (its context is freed)
        once its waiting and in-flight frames have been served."""
        self.streams[sid].closing = True
        self._retire()

    def _used(self) -> int:
        return sum(s.need for s in self.streams.values() if s.det is not None)

    def _admit(self) -> None:
        while self.admission:
            s = self.streams[self.admission[0]]
            if sum(1 for x in self.streams.values() if x.det is not None) >= MAX_STREAMS:
                return
            if self.budget is not None and self._used() + s.need > self.budget:
                return
            free, _ = self._torch.cuda.mem_get_info(self.device)
            if free - s.need < self.reserve:
                return
            p = s.params
            geo = {k: v for k, v in p.items()
                   if k not in ("lx", "ly", "threshold", "phase", "connectivity", "max_components")}
            s.det = dv.Detector(p["lx"], p["ly"], p["threshold"], p["phase"], p["connectivity"],
                                max_components=p["max_components"], keep_maps=False,
                                device=self.device, stream=self.stream, max_batch=1,
                                keep_results=True, **geo)
            self.admission.popleft()
            self._drop_group()

    def _retire(self) -> None:
        # closed before admission with nothing queued: never admitted
        for s in [s for s in self.streams.values() if s.closing and s.det is None and not s.queue]:
            self.admission.remove(s.sid)
            del self.streams[s.sid]
        gone = [s for s in self.streams.values()
                if s.closing and s.det is not None and not s.queue and not s.inflight]
        if not gone:
            return
        self._drop_group()
        for s in gone:
            s.det.close()
            del self.streams[s.sid]
        self._admit()

    def _drop_group(self) -> None:
        if self.group is not None:
            self.group.close()      # waits for the shared stream
            self.group = None

    # -- frames ----------------------------------------------------------------
    def submit(self, sid: int, field, tag=None, t_arrival: float | None = None) -> None:
        """Queue a frame of stream sid (float32 device tensor [ly, lx], kept
        alive by the server until its result is returned)."""
        s = self.streams[sid]
        if s.closing:
            raise ValueError(f"stream {sid} is closed")
        s.queue.append((field, tag, time.perf_counter() if t_arrival is None else t_arrival))

    def pending(self) -> int:
        """Frames waiting or in flight."""
        return sum(len(s.queue) + len(s.inflight) for s in self.streams.values())

    def _launch(self) -> bool:
        ready = [s for s in self.streams.values() if s.det is not None and s.queue]
        if not ready:
            return False
        if self.group is None:
            live = [s for s in self.streams.values() if s.det is not None]
            self.members = [s.sid for s in live]
            self.group = dv.Group([s.det for s in live])
        pos = {sid: k for k, sid in enumerate(self.members)}
        items = [s.queue.popleft() for s in ready]
        self.group.push_some([pos[s.sid] for s in ready], [it[0] for it in items])
        ev = self._torch.cuda.Event()
        ev.record(self.stream)
        for s, (f, tag, ta) in zip(ready, items):
            s.inflight.append((tag, ta, f))
        self.steps.append((ev, [s.sid for s in ready]))
        return True

    def step(self):
        """Send the oldest waiting frame of every admitted stream that has one
        (when fewer than `depth` steps are in flight), then wait for the oldest
        step in flight once `depth` are, or when there is nothing new to send,
        and return its frames' results:
        [(sid, tag, t_arrival, t_done, FrameInfo, flips int32 [F, 6])],
        t_done being when the results reached the host."""
        self._admit()
        launched = False
        if len(self.steps) < self.depth:
            launched = self._launch()
        if not self.steps or (launched and len(self.steps) < self.depth):
            return []
        ev, sids = self.steps.popleft()
        ev.synchronize()
        out = []
        for sid in sids:
            s = self.streams[sid]
            for info, fl in s.det.results(wait=False):
                tag, ta, _ = s.inflight.popleft()
                out.append((sid, tag, ta, time.perf_counter(), info, fl))
        self._retire()
        return out

    def drain(self):
        """Serve every frame of the admitted streams, waiting or in flight;
        returns the results (frames of streams still waiting for admission stay
        queued)."""
        out = []
        while self.steps or any(s.det is not None and s.queue for s in self.streams.values()):
            out += self.step()
        return out

    def shutdown(self):
        self._drop_group()
        for s in self.streams.values():
            if s.det is not None:
                s.det.close()
        self.streams = {}
        self.admission.clear()

    # compatibility name
    def close_all(self):
        self.shutdown()
