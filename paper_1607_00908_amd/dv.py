"""Python binding of libdv (the C ABI in include/dv.h).

Argument marshalling only: every step of the detection path runs in the HIP
kernels of libdv.so.  PyTorch supplies device memory (the field tensor) and
the stream.  The library must have been built (``__graft_entry__.build()``);
loading fails loudly otherwise -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdv.so")

MAXLINK = 0x77777777
NO_LABEL = -1
PHASE_ABOVE = 0
PHASE_BELOW = 1
KEEP_MAPS = 1
CLASSIFY = 2
OBSTACLES = 4
OPEN_X = 8
OPEN_Y = 16
KEEP_RESULTS = 32
WEIGHTED = 64        # centres weighted by the quantised field (Sec. 2 centroid)
FLIP_BULK, FLIP_BOUNDARY = 1, 2

OK, ERR_ARG, ERR_CAPACITY, ERR_NOMEM, ERR_DEVICE, ERR_STATE, ERR_INTERNAL = range(7)

# every entry point declared in include/dv.h
EXPORTS = ("dv_create", "dv_push_frame", "dv_get_flips", "dv_get_info", "dv_sync", "dv_destroy",
           "dv_get_labels", "dv_get_owner", "dv_get_components", "dv_get_edges",
           "dv_get_matching", "dv_set_obstacles", "dv_group_create", "dv_group_push", "dv_group_push_some",
           "dv_group_destroy", "dv_results_ready", "dv_get_results", "dv_compare_static", "dv_device_bytes",
           "dv_set_profile", "dv_get_profile", "dv_stage_name", "dv_status_str", "dv_last_error")

DEFAULT_BATCH = 32   # what max_batch = 0 selects

STAGES = ("tile_ccl", "merge", "resolve", "relabel", "finalize", "owner_edges", "rows",
          "match", "diff", "events", "place")


class DVConfig(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("lx", ctypes.c_int32), ("ly", ctypes.c_int32),
                ("threshold", ctypes.c_float), ("phase", ctypes.c_int32),
                ("connectivity", ctypes.c_int32), ("max_components", ctypes.c_int32),
                ("max_degree", ctypes.c_int32), ("device", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("max_batch", ctypes.c_int32)]


class DVFlip(ctypes.Structure):
    _fields_ = [("a", ctypes.c_int32), ("b", ctypes.c_int32), ("pa", ctypes.c_int32),
                ("pb", ctypes.c_int32), ("kind", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class DVFrameInfo(ctypes.Structure):
    _fields_ = [("frame", ctypes.c_int64), ("status", ctypes.c_int32),
                ("n_components", ctypes.c_int32), ("n_edges", ctypes.c_int32),
                ("n_flips", ctypes.c_int32), ("n_breaking", ctypes.c_int32),
                ("n_excluded_past", ctypes.c_int32), ("n_excluded_now", ctypes.c_int32),
                ("n_ambiguous_centroids", ctypes.c_int32), ("global_trigger", ctypes.c_uint32)]


class DVError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libdv.so and declare the C signatures.  Raises when it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.dv_create.restype = i32
    lib.dv_create.argtypes = [ctypes.POINTER(DVConfig), vp, ctypes.POINTER(vp)]
    lib.dv_push_frame.restype = i32
    lib.dv_push_frame.argtypes = [vp, vp]
    lib.dv_get_flips.restype = i32
    lib.dv_get_flips.argtypes = [vp, vp, i32, i32p]
    lib.dv_get_info.restype = i32
    lib.dv_get_info.argtypes = [vp, ctypes.POINTER(DVFrameInfo)]
    lib.dv_results_ready.restype = i32
    lib.dv_results_ready.argtypes = [vp, i32, i32p, i32p]
    lib.dv_get_results.restype = i32
    lib.dv_get_results.argtypes = [vp, i32, vp, i32, i32p, vp, i32, i32p]
    lib.dv_compare_static.restype = i32
    lib.dv_compare_static.argtypes = [ctypes.POINTER(DVConfig), vp, vp, vp, vp, i32, vp]
    lib.dv_device_bytes.restype = i32
    lib.dv_device_bytes.argtypes = [ctypes.POINTER(DVConfig), ctypes.POINTER(ctypes.c_uint64)]
    lib.dv_sync.restype = i32
    lib.dv_sync.argtypes = [vp]
    lib.dv_destroy.restype = None
    lib.dv_destroy.argtypes = [vp]
    lib.dv_get_labels.restype = i32
    lib.dv_get_labels.argtypes = [vp, vp]
    lib.dv_get_owner.restype = i32
    lib.dv_get_owner.argtypes = [vp, vp]
    lib.dv_get_components.restype = i32
    lib.dv_get_components.argtypes = [vp, vp, vp, vp, i32, i32p]
    lib.dv_get_edges.restype = i32
    lib.dv_get_edges.argtypes = [vp, vp, i32, i32p]
    lib.dv_get_matching.restype = i32
    lib.dv_get_matching.argtypes = [vp, vp, i32, i32p]
    lib.dv_set_obstacles.restype = i32
    lib.dv_set_obstacles.argtypes = [vp, vp, i32]
    lib.dv_group_create.restype = i32
    lib.dv_group_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp)]
    lib.dv_group_push.restype = i32
    lib.dv_group_push.argtypes = [vp, ctypes.POINTER(vp)]
    lib.dv_group_push_some.restype = i32
    lib.dv_group_push_some.argtypes = [vp, i32p, ctypes.POINTER(vp), i32]
    lib.dv_group_destroy.restype = None
    lib.dv_group_destroy.argtypes = [vp]
    lib.dv_set_profile.restype = i32
    lib.dv_set_profile.argtypes = [vp, i32, i32]
    lib.dv_get_profile.restype = i32
    lib.dv_get_profile.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32p]
    lib.dv_stage_name.restype = ctypes.c_char_p
    lib.dv_stage_name.argtypes = [i32]
    lib.dv_status_str.restype = ctypes.c_char_p
    lib.dv_status_str.argtypes = [i32]
    lib.dv_last_error.restype = ctypes.c_char_p
    lib.dv_last_error.argtypes = [vp]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class FrameInfo:
    frame: int
    status: int
    n_components: int
    n_edges: int
    n_flips: int
    n_breaking: int
    n_excluded_past: int
    n_excluded_now: int
    n_ambiguous_centroids: int
    global_trigger: int


def _frame_info(fi: DVFrameInfo) -> FrameInfo:
    return FrameInfo(fi.frame, fi.status, fi.n_components, fi.n_edges, fi.n_flips,
                     fi.n_breaking, fi.n_excluded_past, fi.n_excluded_now,
                     fi.n_ambiguous_centroids, fi.global_trigger)


def _config(lx, ly, threshold, phase, connectivity, max_components, max_degree, device, keep_maps,
            max_batch, classify, open_x, open_y, with_obstacles, keep_results,
            weighted=False) -> DVConfig:
    flags = ((KEEP_MAPS if keep_maps else 0) | (CLASSIFY if classify else 0)
             | (OPEN_X if open_x else 0) | (OPEN_Y if open_y else 0)
             | (KEEP_RESULTS if keep_results else 0) | (OBSTACLES if with_obstacles else 0)
             | (WEIGHTED if weighted else 0))
    return DVConfig(ctypes.sizeof(DVConfig), int(lx), int(ly), float(threshold), int(phase),
                    int(connectivity), int(max_components), int(max_degree), int(device),
                    flags, int(max_batch))


def device_bytes(lx: int, ly: int, threshold: float = 0.5, phase: int = PHASE_ABOVE,
                 connectivity: int = 8, max_components: int = 4096, max_degree: int = 0,
                 keep_maps: bool = True, max_batch: int = 0, classify: bool = False,
                 open_x: bool = False, open_y: bool = False, with_obstacles: bool = False,
                 keep_results: bool = False, weighted: bool = False) -> int:
    """Device memory a Detector of this configuration allocates (the library's
    own layout; no device is touched)."""
    lib = load()
    cfg = _config(lx, ly, threshold, phase, connectivity, max_components, max_degree, 0, keep_maps,
                  max_batch, classify, open_x, open_y, with_obstacles, keep_results, weighted)
    out = ctypes.c_uint64(0)
    st = lib.dv_device_bytes(ctypes.byref(cfg), ctypes.byref(out))
    if st != OK:
        raise DVError(st, lib.dv_last_error(None).decode())
    return int(out.value)


class Detector:
    """One detection context (one sequence of frames) on one device.

    ``stream``: the torch.cuda.Stream that orders the context's input; None
    creates one.  Before each push that stream waits (on the device, without
    a host synchronisation) for the caller's current stream, and the frame's
    kernels start after it, so a field produced there is complete when they
    read it.  ``max_batch``: frames queued and sent to the device together
    (0: the library's default).  ``classify``: fill the flips' event flags
    (FLIP_BULK, FLIP_BOUNDARY).  ``keep_results``: every frame's record and
    flips are kept until ``results`` returns them (no frame of a batch is lost
    unread).  ``open_x`` / ``open_y``: walls across that
    axis instead of the periodic wrap.  ``obstacles``: a [ly, lx] mask
    (nonzero = obstacle; numpy array or device tensor) set at creation; it can
    be replaced later with ``set_obstacles`` (the context then holds a mask
    even when this is None, with ``with_obstacles=True``).  ``weighted``: the
    centres are the centroids of Sec. 2 with the field as density (site weight
    floor(256 rho + 1/2) clamped to [1, 65535]) instead of the unit-weight
    centres of mass.
    """

    def __init__(self, lx: int, ly: int, threshold: float, phase: int = PHASE_ABOVE,
                 connectivity: int = 8, max_components: int = 4096, max_degree: int = 0,
                 device: int = 0, keep_maps: bool = True, stream=None, max_batch: int = 0,
                 classify: bool = False, open_x: bool = False, open_y: bool = False,
                 obstacles=None, with_obstacles: bool = False, keep_results: bool = False,
                 weighted: bool = False):
        self.lib = load()
        self.lx, self.ly = int(lx), int(ly)
        cfg = _config(self.lx, self.ly, threshold, phase, connectivity, max_components, max_degree,
                      device, keep_maps, max_batch, classify, open_x, open_y,
                      with_obstacles or obstacles is not None, keep_results, weighted)
        import torch
        self._torch = torch
        self.device = torch.device("cuda", int(device))
        if stream is None:
            stream = torch.cuda.Stream(device=self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        st = self.lib.dv_create(ctypes.byref(cfg), ctypes.c_void_p(stream.cuda_stream),
                                ctypes.byref(h))
        if st != OK:
            raise DVError(st, self.lib.dv_last_error(None).decode())
        self.h = h
        self.cfg = cfg
        self._field_refs = []
        if obstacles is not None:
            self.set_obstacles(obstacles)

    # -- lifecycle -----------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self.lib.dv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st: int, allow=()):
        if st != OK and st not in allow:
            raise DVError(st, self.lib.dv_last_error(self.h).decode())
        return st

    # -- frames --------------------------------------------------------------
    def push(self, field) -> None:
        """Enqueue one frame.  ``field``: float32 device tensor [ly, lx]
        (contiguous), or a raw device pointer (int)."""
        if isinstance(field, int):
            ptr = field
        else:
            if not (field.is_cuda and field.dtype == self._torch.float32):
                raise TypeError("field must be a float32 device tensor")
            if tuple(field.shape) != (self.ly, self.lx) or not field.is_contiguous():
                raise ValueError(f"field must be contiguous with shape ({self.ly}, {self.lx})")
            if field.device != self.device:
                raise ValueError(f"field is on {field.device}, the context on {self.device}")
            ptr = field.data_ptr()
            cur = self._torch.cuda.current_stream(self.device)
            if cur.cuda_stream != self.stream.cuda_stream:
                self.stream.wait_stream(cur)
                field.record_stream(self.stream)
            # frames overlap on the device: every field pushed since the last
            # synchronising call may still be read
            self._field_refs.append(field)
        self._check(self.lib.dv_push_frame(self.h, ctypes.c_void_p(ptr)))

    def sync(self):
        self._check(self.lib.dv_sync(self.h))
        self._field_refs.clear()

    def set_obstacles(self, mask) -> None:
        """Replace the obstacle mask ([ly, lx], nonzero = obstacle; numpy array,
        device tensor, or None to clear).  Frames pushed before keep the old one."""
        if mask is None:
            self._check(self.lib.dv_set_obstacles(self.h, None, 0))
            return
        if hasattr(mask, "is_cuda") and mask.is_cuda:
            if tuple(mask.shape) != (self.ly, self.lx):
                raise ValueError(f"mask must have shape ({self.ly}, {self.lx})")
            m = (mask != 0).to(self._torch.uint8).contiguous()
            if m.device != self.device:
                raise ValueError(f"mask is on {m.device}, the context on {self.device}")
            # the copy runs on the context's stream after the caller's work
            self.stream.wait_stream(self._torch.cuda.current_stream(self.device))
            self._check(self.lib.dv_set_obstacles(self.h, ctypes.c_void_p(m.data_ptr()), 1))
            return
        m = np.ascontiguousarray(np.asarray(mask) != 0, dtype=np.uint8)
        if m.shape != (self.ly, self.lx):
            raise ValueError(f"mask must have shape ({self.ly}, {self.lx})")
        self._check(self.lib.dv_set_obstacles(self.h, _ptr(m), 0))

    def flips(self) -> np.ndarray:
        """Flips of the most recent frame: int32 [F, 6] = (a, b, pa, pb, kind, flags)."""
        n = ctypes.c_int32(0)
        self._check(self.lib.dv_get_flips(self.h, None, 0, ctypes.byref(n)), allow=(ERR_CAPACITY,))
        out = np.zeros((max(n.value, 1), 6), dtype=np.int32)
        self._check(self.lib.dv_get_flips(self.h, _ptr(out), n.value, ctypes.byref(n)))
        self._field_refs.clear()
        return out[:n.value]

    def info(self) -> FrameInfo:
        fi = DVFrameInfo()
        self._check(self.lib.dv_get_info(self.h, ctypes.byref(fi)), allow=(ERR_CAPACITY,))
        self._field_refs.clear()
        return _frame_info(fi)

    def results(self, wait: bool = True, out: np.ndarray | None = None):
        """Every unread frame, oldest first: a list of (FrameInfo, flips int32
        [F, 6]).  ``wait``: send the queued frames and wait for all of them;
        else only frames already complete on the device.  Needs
        ``keep_results``.

        ``out``: a C-contiguous int32 [cap, 6] host array of the caller's
        (pinned memory makes the copy a direct DMA); the flips are views into
        it.  Whole frames are returned while they fit; the others stay unread
        for the next call."""
        if out is not None and (out.dtype != np.int32 or out.ndim != 2 or out.shape[1] != 6
                                or not out.flags["C_CONTIGUOUS"] or not out.flags["WRITEABLE"]):
            raise ValueError("out must be a writeable C-contiguous int32 array of shape [cap, 6]")
        nf, nfl = ctypes.c_int32(0), ctypes.c_int32(0)
        self._check(self.lib.dv_results_ready(self.h, int(bool(wait)), ctypes.byref(nf),
                                              ctypes.byref(nfl)))
        if wait:
            self._field_refs.clear()
        if nf.value == 0:
            return []
        infos = (DVFrameInfo * nf.value)()
        if out is None:
            flips = np.empty((max(nfl.value, 1), 6), dtype=np.int32)
            cap = nfl.value
        else:
            flips = out
            cap = min(out.shape[0], nfl.value)
        got_f, got_fl = ctypes.c_int32(0), ctypes.c_int32(0)
        self._check(self.lib.dv_get_results(self.h, 0, infos, nf.value, ctypes.byref(got_f),
                                            _ptr(flips), cap, ctypes.byref(got_fl)),
                    allow=(ERR_CAPACITY,))
        out, o = [], 0
        for k in range(got_f.value):
            fi = _frame_info(infos[k])
            out.append((fi, flips[o:o + fi.n_flips]))
            o += fi.n_flips
        assert o == got_fl.value
        return out

    # -- measurement -----------------------------------------------------------
    def set_profile(self, stage, capacity: int = 4096):
        """Time every launch of one stage (name or index) with HIP events;
        None stops."""
        if stage is None:
            idx = -1
        elif isinstance(stage, str):
            idx = STAGES.index(stage)
        else:
            idx = int(stage)
        self._check(self.lib.dv_set_profile(self.h, idx, int(capacity)))

    def get_profile(self):
        """(total milliseconds, launches) recorded since the last call."""
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int32(0)
        self._check(self.lib.dv_get_profile(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    # -- inspection ------------------------------------------------------------
    def labels(self) -> np.ndarray:
        out = np.empty((self.ly, self.lx), dtype=np.int32)
        self._check(self.lib.dv_get_labels(self.h, _ptr(out)))
        return out

    def owner(self) -> np.ndarray:
        out = np.empty((self.ly, self.lx), dtype=np.int32)
        self._check(self.lib.dv_get_owner(self.h, _ptr(out)))
        return out

    def components(self) -> dict:
        n = ctypes.c_int32(0)
        self._check(self.lib.dv_get_components(self.h, None, None, None, 0, ctypes.byref(n)),
                    allow=(ERR_CAPACITY,))
        K = n.value
        q = np.zeros((max(K, 1), 2), dtype=np.int32)
        f = np.zeros((max(K, 1), 2), dtype=np.float64)
        s = np.zeros(max(K, 1), dtype=np.int32)
        self._check(self.lib.dv_get_components(self.h, _ptr(q), _ptr(f), _ptr(s), K, ctypes.byref(n)))
        return {"qx": q[:K, 0].copy(), "qy": q[:K, 1].copy(), "fx": f[:K, 0].copy(),
                "fy": f[:K, 1].copy(), "n": s[:K].copy()}

    def edges(self) -> np.ndarray:
        n = ctypes.c_int32(0)
        self._check(self.lib.dv_get_edges(self.h, None, 0, ctypes.byref(n)), allow=(ERR_CAPACITY,))
        out = np.zeros((max(n.value, 1), 2), dtype=np.int32)
        self._check(self.lib.dv_get_edges(self.h, _ptr(out), n.value, ctypes.byref(n)))
        return out[:n.value]

    def matching(self) -> np.ndarray:
        n = ctypes.c_int32(0)
        self._check(self.lib.dv_get_matching(self.h, None, 0, ctypes.byref(n)), allow=(ERR_CAPACITY,))
        out = np.zeros(max(n.value, 1), dtype=np.int32)
        self._check(self.lib.dv_get_matching(self.h, _ptr(out), n.value, ctypes.byref(n)))
        return out[:n.value]


class Group:
    """Frames of several detectors sent to the device together: one launch per
    stage for all of them, whatever their lattice sizes.  The detectors must be
    on one device and share one stream (pass the same ``stream`` to each);
    each keeps its own past and getters."""

    def __init__(self, detectors):
        self.lib = load()
        self.members = list(detectors)
        n = len(self.members)
        arr = (ctypes.c_void_p * n)(*[d.h.value for d in self.members])
        h = ctypes.c_void_p()
        st = self.lib.dv_group_create(arr, n, ctypes.byref(h))
        if st != OK:
            raise DVError(st, self.lib.dv_last_error(None).decode())
        self.h = h

    def _ptr(self, d, f) -> int:
        if isinstance(f, int):
            return f
        if not (f.is_cuda and f.dtype == d._torch.float32):
            raise TypeError("fields must be float32 device tensors")
        if tuple(f.shape) != (d.ly, d.lx) or not f.is_contiguous():
            raise ValueError(f"field must be contiguous with shape ({d.ly}, {d.lx})")
        cur = d._torch.cuda.current_stream(d.device)
        if cur.cuda_stream != d.stream.cuda_stream:
            d.stream.wait_stream(cur)
            f.record_stream(d.stream)
        d._field_refs.append(f)
        return f.data_ptr()

    def push(self, fields) -> None:
        """One float32 device tensor [ly, lx] (contiguous) per member, or raw
        device pointers (int)."""
        if len(fields) != len(self.members):
            raise ValueError("one field per member")
        self.push_some(range(len(self.members)), fields)

    def push_some(self, members, fields) -> None:
        """Frames for the listed members only (distinct indices), in one launch
        per stage; the other members are untouched."""
        members = [int(k) for k in members]
        if len(fields) != len(members) or not members:
            raise ValueError("one field per listed member")
        ptrs = [self._ptr(self.members[k], f) for k, f in zip(members, fields)]
        idx = (ctypes.c_int32 * len(members))(*members)
        arr = (ctypes.c_void_p * len(ptrs))(*ptrs)
        st = self.lib.dv_group_push_some(self.h, idx, arr, len(members))
        if st != OK:
            raise DVError(st, self.lib.dv_last_error(self.members[members[0]].h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.dv_group_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
