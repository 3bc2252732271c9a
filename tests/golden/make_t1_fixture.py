"""Writes t1_fixture.json: an embedded T1 rearrangement on a periodic lattice.

A T1 event is the simplest plastic rearrangement: four bubbles A, B, C, D in
a rhombus exchange the short diagonal, so exactly one Delaunay link breaks
(A-C) and one arises (B-D) while the total coordination is conserved
(Sec. 2.1 and Sec. 3.2.4, bulk event of the T1 figure).

The quartet sits inside a static background of disks.  The background is
drawn from a seed and accepted only when, in both frames, the exact periodic
Delaunay triangulation (``tests/delaunay_ref.py``, independent of the oracle)
is certified, every dual Voronoi edge is at least 2 lattice units long, and
the only difference between the frames is A-C -> B-D.  The file stores the
inputs only; the expected couples are recomputed by the tests.

Run:  python tests/golden/make_t1_fixture.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
from delaunay_ref import periodic_delaunay  # noqa: E402

LX, LY = 128, 112
R = 3                      # disk radius (sites); centres are integer sites
O = (64, 56)
QUARTET = {                # frame 0: A-C short; frame 1: B-D short
    0: {"A": (O[0] - 7, O[1]), "C": (O[0] + 7, O[1]), "B": (O[0], O[1] + 11), "D": (O[0], O[1] - 11)},
    1: {"A": (O[0] - 11, O[1]), "C": (O[0] + 11, O[1]), "B": (O[0], O[1] + 7), "D": (O[0], O[1] - 7)},
}


def _pdist(a, b):
    dx = (a[0] - b[0] + LX / 2) % LX - LX / 2
    dy = (a[1] - b[1] + LY / 2) % LY - LY / 2
    return (dx * dx + dy * dy) ** 0.5


def candidate(seed):
    """Jittered triangular background (8 rows of 8, spacing 16 x 14) with the
    points near the quartet removed."""
    rng = np.random.default_rng(seed)
    fixed = list(QUARTET[0].values()) + list(QUARTET[1].values())
    bg = []
    for j in range(8):
        for i in range(8):
            x = int(round((i + 0.5 * (j % 2)) * 16 + rng.normal(0, 1.5))) % LX
            y = int(round(j * 14 + rng.normal(0, 1.5))) % LY
            p = (x, y)
            if all(_pdist(p, q) >= 12 for q in fixed):
                bg.append(p)
    return bg


def check(bg):
    names = ["A", "B", "C", "D"]
    sets = []
    for fr in (0, 1):
        pts = [QUARTET[fr][n] for n in names] + bg
        qx = [256 * p[0] for p in pts]
        qy = [256 * p[1] for p in pts]
        E, lmin, ok = periodic_delaunay(qx, qy, LX, LY)
        if not ok or lmin < 2.0:
            return False
        sets.append(E)
    brk, ari = sets[0] - sets[1], sets[1] - sets[0]
    return brk == {(0, 2)} and ari == {(1, 3)}


def main():
    for seed in range(1000):
        bg = candidate(seed)
        if check(bg):
            out = {
                "citation": "T1 rearrangement: Sec. 2.1 and Sec. 3.2.4 (bulk event: one "
                            "breaking and one arising link, coordination conserved)",
                "lx": LX, "ly": LY, "radius": R, "threshold": 0.5, "phase": 0,
                "quartet": {str(k): {n: list(v) for n, v in q.items()} for k, q in QUARTET.items()},
                "background": [list(p) for p in bg],
                "seed": seed,
                "expected": {"breaking": [["A", "C"]], "arising": [["B", "D"]]},
            }
            with open(os.path.join(HERE, "t1_fixture.json"), "w") as f:
                json.dump(out, f, indent=1)
            print("seed", seed, "background", len(bg))
            return
    raise SystemExit("no acceptable background found")


if __name__ == "__main__":
    main()
