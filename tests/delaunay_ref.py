"""Exact periodic Delaunay triangulation of Q.8 points, used to pin the oracle.

Independent of the oracle: the triangulation comes from Qhull
(scipy.spatial.Delaunay) on the 3x3 periodic images, and every triangle that
touches the central copy is then certified with an exact integer in-circle
test (Python integers) against every image point.  The Delaunay graph is the
dual of the continuous Voronoi diagram that the paper's digital tessellation
approximates (Sec. 1 and Sec. 3.2).
"""
from __future__ import annotations

import numpy as np


def _incircle(a, b, c, d) -> int:
    """> 0 when d lies strictly inside the circle through a, b, c (ccw)."""
    adx, ady = a[0] - d[0], a[1] - d[1]
    bdx, bdy = b[0] - d[0], b[1] - d[1]
    cdx, cdy = c[0] - d[0], c[1] - d[1]
    ad = adx * adx + ady * ady
    bd = bdx * bdx + bdy * bdy
    cd = cdx * cdx + cdy * cdy
    return (adx * (bdy * cd - bd * cdy) - ady * (bdx * cd - bd * cdx)
            + ad * (bdx * cdy - bdy * cdx))


def _orient(a, b, c) -> int:
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])


def _circumcenter(a, b, c):
    ax, ay = float(a[0]), float(a[1])
    bx, by = float(b[0]), float(b[1])
    cx, cy = float(c[0]), float(c[1])
    d = 2.0 * (ax * (by - cy) + bx * (cy - ay) + cx * (ay - by))
    ux = ((ax * ax + ay * ay) * (by - cy) + (bx * bx + by * by) * (cy - ay)
          + (cx * cx + cy * cy) * (ay - by)) / d
    uy = ((ax * ax + ay * ay) * (cx - bx) + (bx * bx + by * by) * (ax - cx)
          + (cx * cx + cy * cy) * (bx - ax)) / d
    return ux, uy


def periodic_delaunay(qx, qy, lx: int, ly: int, return_lengths: bool = False):
    """Return (edges set of (a<b), min Voronoi edge length in lattice units, ok).

    With ``return_lengths`` a fourth item maps each couple to the length (in
    lattice units) of its dual Voronoi edge.

    ``ok`` is False when the triangulation is not certified (a co-circular
    quadruple, or a pair of points joined through two different images so the
    label graph would not be simple).
    """
    from scipy.spatial import Delaunay

    qx = [int(v) for v in qx]
    qy = [int(v) for v in qy]
    V = len(qx)
    W, H = 256 * lx, 256 * ly
    pts, orig, central = [], [], []
    for iy in (-1, 0, 1):
        for ix in (-1, 0, 1):
            for i in range(V):
                pts.append((qx[i] + ix * W, qy[i] + iy * H))
                orig.append(i)
                central.append(ix == 0 and iy == 0)
    P = np.array(pts, dtype=np.float64)
    P_index = {p: i for i, p in enumerate(pts)}
    tri = Delaunay(P)
    simp = tri.simplices
    touch = np.array([any(central[v] for v in s) for s in simp])
    simp = simp[touch]
    ok = True
    # exact certificate: each triangle's circumcircle holds no image point
    pf = P
    for s in simp:
        a, b, c = (pts[s[0]], pts[s[1]], pts[s[2]])
        if _orient(a, b, c) < 0:
            b, c = c, b
        # float pre-filter, then exact test for anything near the circle
        ux, uy = _circumcenter(a, b, c)
        r2 = (a[0] - ux) ** 2 + (a[1] - uy) ** 2
        d2 = (pf[:, 0] - ux) ** 2 + (pf[:, 1] - uy) ** 2
        near = np.nonzero(d2 <= r2 * (1 + 1e-9) + 4.0)[0]
        for q in near:
            if q in (s[0], s[1], s[2]):
                continue
            v = _incircle(a, b, c, pts[q])
            if v >= 0:
                ok = False
    edges = set()
    pair_image = {}
    for s in simp:
        for u, v in ((s[0], s[1]), (s[1], s[2]), (s[2], s[0])):
            a, b = orig[u], orig[v]
            if a == b:
                ok = False
                continue
            key = (min(a, b), max(a, b))
            # displacement between the two endpoints identifies the image used
            if orig[u] == key[0]:
                disp = (pts[v][0] - pts[u][0], pts[v][1] - pts[u][1])
            else:
                disp = (pts[u][0] - pts[v][0], pts[u][1] - pts[v][1])
            prev = pair_image.setdefault(key, disp)
            if prev != disp:
                ok = False
            edges.add(key)
    # shortest Voronoi edge: distance between circumcentres of the two
    # triangles sharing each Delaunay edge (edges keyed by image coordinates)
    cc = {}
    for s in simp:
        a, b, c = (pts[s[0]], pts[s[1]], pts[s[2]])
        cen = _circumcenter(a, b, c)
        for u, v in ((s[0], s[1]), (s[1], s[2]), (s[2], s[0])):
            pu, pv = pts[u], pts[v]
            k = (min(pu, pv), max(pu, pv))
            cc.setdefault(k, []).append(cen)
    lmin = float("inf")
    vlen = {}
    for k, cs in cc.items():
        if len(cs) == 2:
            d = ((cs[0][0] - cs[1][0]) ** 2 + (cs[0][1] - cs[1][1]) ** 2) ** 0.5 / 256.0
            lmin = min(lmin, d)
            a, b = orig[P_index[k[0]]], orig[P_index[k[1]]]
            key = (min(a, b), max(a, b))
            vlen[key] = min(vlen.get(key, d), d)
    if return_lengths:
        return edges, lmin, ok, vlen
    return edges, lmin, ok


def spread_points(rng, V: int, lx: int, ly: int, min_sep: float):
    """Random points (Q.8 ints) with pairwise periodic separation >= min_sep sites."""
    pts = []
    tries = 0
    while len(pts) < V and tries < 100000:
        tries += 1
        x = rng.uniform(0, lx)
        y = rng.uniform(0, ly)
        good = True
        for (px, py) in pts:
            dx = (x - px + lx / 2) % lx - lx / 2
            dy = (y - py + ly / 2) % ly - ly / 2
            if dx * dx + dy * dy < min_sep * min_sep:
                good = False
                break
        if good:
            pts.append((x, y))
    qx = np.array([int(np.floor(256 * p[0])) % (256 * lx) for p in pts], dtype=np.int32)
    qy = np.array([int(np.floor(256 * p[1])) % (256 * ly) for p in pts], dtype=np.int32)
    return qx, qy
