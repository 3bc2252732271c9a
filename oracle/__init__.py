"""CPU oracle for the detection path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never does, and it
shares no code with the HIP library.

Thin ctypes wrapper over ``oracle.cpp`` (plain C++17), plus two helpers that
chain the steps in the paper's order:

* ``frame(field, ...)``  -- Sec. 3.1 and 3.2.1-3.2.2 on one field
* ``Sequence``           -- keeps the past frame and applies Sec. 3.2.3-3.2.4
* ``classify``           -- event flags of the flips (Sec. 3.2.4, optional)
* ``centroids(..., field=)`` -- the density-weighted centroids of Sec. 2
  (optional variant of the centres)

Geometry: every function takes ``open_x`` / ``open_y`` (that axis has walls
instead of wrapping; default periodic) and, where sites are coloured or
labelled, ``obstacles`` (one byte per site, nonzero = obstacle; Sec. 3.2.1).

Each function's docstring names the section it follows; the readings of the
paper that the oracle fixes are stated in ``oracle.cpp``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

MAXLINK = 0x77777777

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
# (DV_ORACLE_LIB: another build of the oracle, for the mutation probe of the pins)
_LIB = os.environ.get("DV_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = ctypes.POINTER(ctypes.c_int32)
_f32p = ctypes.POINTER(ctypes.c_float)
_f64p = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build(verbose: bool = False) -> str:
    """Compile oracle.cpp into liboracle.so beside it (g++, C++17, OpenMP)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-Wall",
           _SRC, "-o", _LIB + ".tmp"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    i32, f32, i64 = ctypes.c_int32, ctypes.c_float, ctypes.c_int64
    lib.or_label.restype = i32
    lib.or_label.argtypes = [_f32p, i32, i32, f32, i32, i32, _u8p, i32, _i32p]
    lib.or_centroids.restype = None
    lib.or_centroids.argtypes = [_i32p, i32, i32, i32, i32, i32, _i32p, _i32p, _i32p, _i32p,
                                 _f64p, _f64p, _i32p]
    lib.or_centroids_weighted.restype = None
    lib.or_centroids_weighted.argtypes = [_i32p, _f32p, i32, i32, i32, i32, _i32p, _i32p, _i32p,
                                          _f64p, _f64p, ctypes.POINTER(ctypes.c_int64)]
    lib.or_owner.restype = None
    lib.or_owner.argtypes = [i32, i32, i32, _u8p, i32, _i32p, _i32p, _i32p, i32]
    lib.or_colour_at.restype = i32
    lib.or_colour_at.argtypes = [i64, i64, i32, i32, i32, i32, _i32p, _i32p]
    lib.or_edges.restype = i32
    lib.or_edges.argtypes = [i32, i32, i32, i32, _i32p, _i32p, _i32p, _i32p, i32]
    lib.or_edges_window.restype = i32
    lib.or_edges_window.argtypes = [i32, i32, i32, _u8p, i32, _i32p, _i32p, i32, i32, i32, i32,
                                    _i32p, i32, i32]
    lib.or_match.restype = None
    lib.or_match.argtypes = [i32, i32, i32, i32, _i32p, _i32p, i32, _i32p, _i32p, _i32p, _i32p]
    lib.or_diff.restype = i32
    lib.or_diff.argtypes = [i32, i32, _i32p, _i32p, i32, i32, _i32p, _i32p, _i32p, i32,
                            _i32p, _i32p]
    _lib = lib
    return lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def _c32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _open(open_x: bool, open_y: bool) -> int:
    return (1 if open_x else 0) | (2 if open_y else 0)


def _obst(obstacles, lx: int, ly: int):
    """(array kept alive, pointer) of the obstacle mask, or (None, None)."""
    if obstacles is None:
        return None, None
    m = np.ascontiguousarray(np.asarray(obstacles) != 0, dtype=np.uint8)
    if m.shape != (ly, lx):
        raise ValueError(f"obstacle mask of shape {m.shape}, lattice is {(ly, lx)}")
    return m, _p(m, _u8p)


# --------------------------------------------------------------------- Sec. 3.1
def label(field: np.ndarray, threshold: float, phase: int = 0, conn: int = 8,
          obstacles=None, open_x: bool = False, open_y: bool = False):
    """Threshold + cluster labelling (Sec. 3.1).  Returns (labels int32 [ly,lx], K)."""
    f = np.ascontiguousarray(field, dtype=np.float32)
    ly, lx = f.shape
    keep, om = _obst(obstacles, lx, ly)
    lab = np.empty((ly, lx), dtype=np.int32)
    K = _load().or_label(_p(f, _f32p), lx, ly, float(threshold), int(phase), int(conn),
                         om, _open(open_x, open_y), _p(lab, _i32p))
    return lab, int(K)


def centroids(labels: np.ndarray, K: int, conn: int = 8, open_x: bool = False,
              open_y: bool = False, field: np.ndarray | None = None) -> dict:
    """Sizes and centres of mass (Sec. 3.1), exact Q.8 and float64.  With
    ``field``: the centres are the weighted centroids of Sec. 2 with the field
    as density (quantised weights, ``weights``); sizes and the ambiguity flag
    are those of the unweighted step, and ``w`` holds each component's total
    weight."""
    lab = _c32(labels)
    ly, lx = lab.shape
    out = {k: np.zeros(K, dtype=np.int32) for k in ("n", "root", "qx", "qy", "amb")}
    out["fx"] = np.zeros(K, dtype=np.float64)
    out["fy"] = np.zeros(K, dtype=np.float64)
    if K:
        _load().or_centroids(_p(lab, _i32p), lx, ly, int(conn), _open(open_x, open_y), int(K),
                             _p(out["n"], _i32p), _p(out["root"], _i32p),
                             _p(out["qx"], _i32p), _p(out["qy"], _i32p),
                             _p(out["fx"], _f64p), _p(out["fy"], _f64p),
                             _p(out["amb"], _i32p))
    if field is not None:
        f = np.ascontiguousarray(field, dtype=np.float32)
        if f.shape != lab.shape:
            raise ValueError("field and labels differ in shape")
        out["w"] = np.zeros(K, dtype=np.int64)
        if K:
            _load().or_centroids_weighted(_p(lab, _i32p), _p(f, _f32p), lx, ly,
                                          _open(open_x, open_y), int(K), _p(out["root"], _i32p),
                                          _p(out["qx"], _i32p), _p(out["qy"], _i32p),
                                          _p(out["fx"], _f64p), _p(out["fy"], _f64p),
                                          _p(out["w"], ctypes.POINTER(ctypes.c_int64)))
    return out


def weights(field: np.ndarray) -> np.ndarray:
    """Quantised site weights of the weighted centroid (Sec. 2 density):
    floor(256 rho + 1/2) clamped to [1, 65535], int64."""
    v = np.floor(256.0 * np.asarray(field, dtype=np.float32).astype(np.float64) + 0.5)
    return np.clip(np.nan_to_num(v, nan=1.0), 1, 65535).astype(np.int64)


# ------------------------------------------------------------------- Sec. 3.2.1
def owner(lx: int, ly: int, qx, qy, nthreads: int = 0, obstacles=None, open_x: bool = False,
          open_y: bool = False) -> np.ndarray:
    """Digital Voronoi colouring by brute force over all centres (Sec. 3.2.1);
    obstacle sites get MAXLINK."""
    qx, qy = _c32(qx), _c32(qy)
    keep, om = _obst(obstacles, lx, ly)
    out = np.empty((ly, lx), dtype=np.int32)
    _load().or_owner(lx, ly, _open(open_x, open_y), om, len(qx), _p(qx, _i32p), _p(qy, _i32p),
                     _p(out, _i32p), int(nthreads))
    return out


def colour_at(X: int, Y: int, lx: int, ly: int, qx, qy, open_x: bool = False,
              open_y: bool = False) -> int:
    """Colour of one Q.8 point (Sec. 3.2.1 rule at an arbitrary point)."""
    qx, qy = _c32(qx), _c32(qy)
    return int(_load().or_colour_at(int(X), int(Y), lx, ly, _open(open_x, open_y), len(qx),
                                    _p(qx, _i32p), _p(qy, _i32p)))


# ------------------------------------------------------------------- Sec. 3.2.2
def edges(lx: int, ly: int, qx, qy, owner_map: np.ndarray, open_x: bool = False,
          open_y: bool = False) -> np.ndarray:
    """Delaunay couples from Voronoi-vertex sites (Sec. 3.2.2); int32 [E,2], sorted.
    Obstacles enter through the owner map (MAXLINK sites)."""
    qx, qy = _c32(qx), _c32(qy)
    om = _c32(owner_map)
    lib = _load()
    cap = 1 << 12
    while True:
        ab = np.empty((cap, 2), dtype=np.int32)
        E = lib.or_edges(lx, ly, _open(open_x, open_y), len(qx), _p(qx, _i32p), _p(qy, _i32p),
                         _p(om, _i32p), _p(ab, _i32p), cap)
        if E <= cap:
            return ab[:E].copy()
        cap = E


def edges_window(lx: int, ly: int, qx, qy, x0: int, y0: int, w: int, h: int,
                 nthreads: int = 0, obstacles=None, open_x: bool = False,
                 open_y: bool = False) -> np.ndarray:
    """Couples emitted by the sites of one window, colours by brute force."""
    qx, qy = _c32(qx), _c32(qy)
    keep, om = _obst(obstacles, lx, ly)
    lib = _load()
    cap = 1 << 12
    while True:
        ab = np.empty((cap, 2), dtype=np.int32)
        E = lib.or_edges_window(lx, ly, _open(open_x, open_y), om, len(qx), _p(qx, _i32p),
                                _p(qy, _i32p), x0, y0, w, h, _p(ab, _i32p), cap, int(nthreads))
        if E <= cap:
            return ab[:E].copy()
        cap = E


# ------------------------------------------------------------------- Sec. 3.2.3
def match(lx: int, ly: int, pqx, pqy, nqx, nqy, open_x: bool = False, open_y: bool = False):
    """Kinematic isomorphism Phi_{P->N} and preimage counts (Sec. 3.2.3)."""
    pqx, pqy, nqx, nqy = _c32(pqx), _c32(pqy), _c32(nqx), _c32(nqy)
    phi = np.empty(len(pqx), dtype=np.int32)
    cnt = np.empty(len(nqx), dtype=np.int32)
    _load().or_match(lx, ly, _open(open_x, open_y), len(pqx), _p(pqx, _i32p), _p(pqy, _i32p), len(nqx),
                     _p(nqx, _i32p), _p(nqy, _i32p), _p(phi, _i32p), _p(cnt, _i32p))
    return phi, cnt


def diff(KP: int, past_edges, phi, KN: int, now_edges, cnt):
    """Translation, exclusion and breaking / arising couples (Sec. 3.2.3-3.2.4).

    Returns (flips int32 [F,6] = (a, b, pa, pb, kind, flags), local_trigger [KP],
    (excluded_past, excluded_now, global_trigger)).
    """
    pe = _c32(np.asarray(past_edges).reshape(-1, 2))
    ne = _c32(np.asarray(now_edges).reshape(-1, 2))
    phi, cnt = _c32(phi), _c32(cnt)
    lt = np.zeros(max(KP, 1), dtype=np.int32)
    counts = np.zeros(3, dtype=np.int32)
    lib = _load()
    cap = 256
    while True:
        fl = np.empty((cap, 6), dtype=np.int32)
        F = lib.or_diff(KP, len(pe), _p(pe, _i32p), _p(phi, _i32p), KN, len(ne),
                        _p(ne, _i32p), _p(cnt, _i32p), _p(fl, _i32p), cap, _p(lt, _i32p),
                        _p(counts, _i32p))
        if F <= cap:
            return fl[:F].copy(), lt[:KP].copy(), tuple(int(c) for c in counts)
        cap = F


def classify(past_edges, phi, now_edges, cnt, flips) -> np.ndarray:
    """Event flags of the flips (Sec. 3.2.4, extraction of topology change
    events), written out with plain sets; returns int32 [F].

    Both graphs keep only points with exactly one preimage (the exclusion of
    Sec. 3.2.3), the past one translated through Phi.  The active points are
    the endpoints of the flips (the points whose rows changed, the local
    trigger).  For each active point count the other active points it is
    connected to in either graph.  A couple of a graph is a boundary couple
    when its two ends share fewer than two neighbours in that graph, and a
    point with a boundary couple is a boundary point.  Flag bit 0 (bulk): both
    ends have at least three active neighbours.  Flag bit 1 (boundary): both
    ends are boundary points of the graph that holds the couple (past graph
    for a breaking couple, now graph for an arising one).
    """
    phi = np.asarray(phi)
    cnt = np.asarray(cnt)

    def kept_now(n):
        return 0 <= n < len(cnt) and cnt[n] == 1

    adjP, adjN = {}, {}
    for a, b in np.asarray(past_edges).reshape(-1, 2):
        ta, tb = int(phi[a]), int(phi[b])
        if kept_now(ta) and kept_now(tb) and ta != tb:
            adjP.setdefault(ta, set()).add(tb)
            adjP.setdefault(tb, set()).add(ta)
    for a, b in np.asarray(now_edges).reshape(-1, 2):
        a, b = int(a), int(b)
        if kept_now(a) and kept_now(b):
            adjN.setdefault(a, set()).add(b)
            adjN.setdefault(b, set()).add(a)
    flips = np.asarray(flips).reshape(-1, 6)
    active = set(int(v) for v in flips[:, :2].ravel())
    count = {}
    for p in active:
        nb = adjP.get(p, set()) | adjN.get(p, set())
        count[p] = len(nb & active)

    def boundary_point(adj, p):
        return any(len(adj.get(p, set()) & adj.get(q, set())) < 2 for q in adj.get(p, set()))

    out = np.zeros(len(flips), dtype=np.int32)
    for i, (a, b, _, _, kind, _) in enumerate(flips):
        a, b = int(a), int(b)
        f = 1 if (count[a] >= 3 and count[b] >= 3) else 0
        g = adjP if kind == -1 else adjN
        if boundary_point(g, a) and boundary_point(g, b):
            f |= 2
        out[i] = f
    return out


# -------------------------------------------------------------- whole frames
@dataclass
class FrameResult:
    labels: np.ndarray
    K: int
    comps: dict
    owner: np.ndarray
    edges: np.ndarray
    open_x: bool = False
    open_y: bool = False


def frame(field: np.ndarray, threshold: float, phase: int = 0, conn: int = 8,
          nthreads: int = 0, obstacles=None, open_x: bool = False,
          open_y: bool = False, weighted: bool = False) -> FrameResult:
    """Sec. 3.1 then Sec. 3.2.1-3.2.2 on one field (``weighted``: the centres
    are the density-weighted centroids of Sec. 2)."""
    g = dict(open_x=open_x, open_y=open_y)
    lab, K = label(field, threshold, phase, conn, obstacles, **g)
    comps = centroids(lab, K, conn, **g, field=field if weighted else None)
    ly, lx = lab.shape
    om = owner(lx, ly, comps["qx"], comps["qy"], nthreads, obstacles, **g)
    ab = edges(lx, ly, comps["qx"], comps["qy"], om, **g)
    return FrameResult(lab, K, comps, om, ab, bool(open_x), bool(open_y))


@dataclass
class DiffResult:
    flips: np.ndarray
    phi: np.ndarray
    cnt: np.ndarray
    local_trigger: np.ndarray
    excluded_past: int
    excluded_now: int
    global_trigger: int


class Sequence:
    """Frame-to-frame driver: the past triangulation is kept between calls."""

    def __init__(self, threshold: float, phase: int = 0, conn: int = 8, nthreads: int = 0,
                 classify_events: bool = False, obstacles=None, open_x: bool = False,
                 open_y: bool = False, weighted: bool = False):
        self.threshold, self.phase, self.conn, self.nthreads = threshold, phase, conn, nthreads
        self.classify_events = classify_events
        self.obstacles, self.open_x, self.open_y = obstacles, open_x, open_y
        self.weighted = weighted
        self.past: FrameResult | None = None

    def push(self, field: np.ndarray):
        now = frame(field, self.threshold, self.phase, self.conn, self.nthreads,
                    self.obstacles, self.open_x, self.open_y, self.weighted)
        res = compare(self.past, now, self.classify_events)
        self.past = now
        return now, res


def compare(past: FrameResult | None, now: FrameResult, classify_events: bool = False) -> DiffResult:
    """Diff of two frames; with no past frame there is nothing to compare.
    classify_events: fill the flags column of the flips (``classify``)."""
    if past is None:
        z = np.zeros(0, dtype=np.int32)
        return DiffResult(np.zeros((0, 6), np.int32), z, np.zeros(now.K, np.int32), z, 0, 0, 0)
    ly, lx = now.labels.shape
    phi, cnt = match(lx, ly, past.comps["qx"], past.comps["qy"], now.comps["qx"],
                     now.comps["qy"], now.open_x, now.open_y)
    fl, lt, (exP, exN, g) = diff(past.K, past.edges, phi, now.K, now.edges, cnt)
    if classify_events and len(fl):
        fl = fl.copy()
        fl[:, 5] = classify(past.edges, phi, now.edges, cnt, fl)
    return DiffResult(fl, phi, cnt, lt, exP, exN, g)
