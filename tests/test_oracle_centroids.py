"""Pins for the oracle's sizes and centres of mass (Sec. 3.1).

References used: digital disks whose centre is known by symmetry, exact
rational means of components unwrapped by a flood fill written here, and
integer roll covariance of the Q.8 centres.
"""
from collections import deque
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1607_00908_amd import synth


def _disk_mask(lx, ly, cx2, cy2, r2x4):
    """Sites with |2s - c2|^2 < r2x4 (all in doubled coordinates, periodic)."""
    yy, xx = np.mgrid[0:ly, 0:lx]
    dx = (2 * xx - cx2 + lx) % (2 * lx) - lx
    dy = (2 * yy - cy2 + ly) % (2 * ly) - ly
    return (dx * dx + dy * dy) < r2x4


@pytest.mark.parametrize("cx2,cy2,r", [(40, 50, 5), (41, 50, 4), (41, 61, 6), (0, 0, 3), (1, 127, 7)])
def test_symmetric_disk_centre_is_exact(cx2, cy2, r):
    lx, ly = 64, 64
    m = _disk_mask(lx, ly, cx2, cy2, 4 * r * r)
    lab, K = oracle.label(m.astype(np.float32), 0.5, 0, 8)
    assert K == 1
    c = oracle.centroids(lab, K, 8)
    assert c["n"][0] == m.sum()
    assert c["qx"][0] == (128 * cx2) % (256 * lx)
    assert c["qy"][0] == (128 * cy2) % (256 * ly)
    assert c["fx"][0] == (cx2 / 2) % lx and c["fy"][0] == (cy2 / 2) % ly
    assert c["amb"][0] == 0


def _unwrap_by_flood(lab, l, conn):
    """Unwrapped coordinates of component l by walking neighbour steps from its
    first raster site (no modular offset formula involved)."""
    ly, lx = lab.shape
    ys, xs = np.nonzero(lab == l)
    start = (int(xs[0]), int(ys[0]))
    if conn == 8:
        nb = [(dx, dy) for dx in (-1, 0, 1) for dy in (-1, 0, 1) if (dx, dy) != (0, 0)]
    else:
        nb = [(1, 0), (-1, 0), (0, 1), (0, -1)]
    pos = {start: start}
    q = deque([start])
    while q:
        (x, y) = q.popleft()
        ux, uy = pos[(x, y)]
        for dx, dy in nb:
            nx, ny = (x + dx) % lx, (y + dy) % ly
            if lab[ny, nx] == l and (nx, ny) not in pos:
                pos[(nx, ny)] = (ux + dx, uy + dy)
                q.append((nx, ny))
    return list(pos.values())


@pytest.mark.parametrize("seed", range(12))
def test_centroids_equal_exact_rational_means(seed):
    rng = np.random.default_rng(300 + seed)
    lx, ly = int(rng.integers(24, 64)), int(rng.integers(24, 64))
    centers = np.stack([rng.uniform(0, lx, 6), rng.uniform(0, ly, 6)], 1)
    f = synth.disk_field(lx, ly, centers, rng.uniform(2.0, 5.0, 6))
    lab, K = oracle.label(f, 0.5, 0, 8)
    c = oracle.centroids(lab, K, 8)
    for l in range(K):
        if c["amb"][l]:
            continue
        pts = _unwrap_by_flood(lab, l, 8)
        n = len(pts)
        mx = Fraction(sum(p[0] for p in pts), n)
        my = Fraction(sum(p[1] for p in pts), n)
        # round half up of 256*mean, then wrap
        qx = int((256 * mx + Fraction(1, 2)) // 1) % (256 * lx)
        qy = int((256 * my + Fraction(1, 2)) // 1) % (256 * ly)
        assert c["n"][l] == n
        assert c["qx"][l] == qx and c["qy"][l] == qy
        assert abs(c["fx"][l] - float(mx % lx)) < 1e-9 * lx
        assert abs(c["fy"][l] - float(my % ly)) < 1e-9 * ly


@pytest.mark.parametrize("seed", range(8))
def test_integer_roll_shifts_q8_exactly(seed):
    rng = np.random.default_rng(400 + seed)
    lx, ly = 48, 40
    centers = np.stack([rng.uniform(0, lx, 5), rng.uniform(0, ly, 5)], 1)
    f = synth.disk_field(lx, ly, centers, rng.uniform(2.0, 4.5, 5))
    dx, dy = int(rng.integers(-lx, lx)), int(rng.integers(-ly, ly))
    lab, K = oracle.label(f, 0.5, 0, 8)
    lab2, K2 = oracle.label(np.roll(f, (dy, dx), (0, 1)), 0.5, 0, 8)
    c, c2 = oracle.centroids(lab, K, 8), oracle.centroids(lab2, K2, 8)
    assert K == K2
    rolled = np.roll(lab, (dy, dx), (0, 1))
    for l in range(K):
        if c["amb"][l]:
            continue
        ys, xs = np.nonzero(rolled == l)
        l2 = lab2[ys[0], xs[0]]
        assert c2["qx"][l2] == (c["qx"][l] + 256 * dx) % (256 * lx)
        assert c2["qy"][l2] == (c["qy"][l] + 256 * dy) % (256 * ly)
        assert c2["n"][l2] == c["n"][l]


def test_seam_straddling_shape_equals_unwrapped_copy():
    lx, ly = 40, 30
    shape = np.zeros((ly, lx), np.float32)
    shape[10:16, 12:21] = 1.0
    shape[16:19, 14:16] = 1.0
    lab, K = oracle.label(shape, 0.5, 0, 8)
    c = oracle.centroids(lab, K, 8)
    for dx, dy in ((-15, 0), (0, -12), (-16, -14), (25, 20)):
        lab2, K2 = oracle.label(np.roll(shape, (dy, dx), (0, 1)), 0.5, 0, 8)
        c2 = oracle.centroids(lab2, K2, 8)
        assert K2 == 1
        assert c2["qx"][0] == (c["qx"][0] + 256 * dx) % (256 * lx)
        assert c2["qy"][0] == (c["qy"][0] + 256 * dy) % (256 * ly)
        assert abs(((c2["fx"][0] - c["fx"][0] - dx) + lx / 2) % lx - lx / 2) < 1e-12
        assert c2["amb"][0] == 0


def test_half_up_rounding_of_q8():
    """Hand-computed Q.8 centres of three tiny shapes (offsets from the
    smallest-index site, mean rounded half up in units of 1/256)."""
    f = np.zeros((8, 8), np.float32)
    f[3, 3] = 1
    f[3, 4] = 1                       # x offsets 0, 1: mean 1/2 -> 128
    lab, K = oracle.label(f, 0.5, 0, 8)
    c = oracle.centroids(lab, K, 8)
    assert c["qx"][0] == 256 * 3 + 128
    f = np.zeros((8, 8), np.float32)
    f[3, 3:6] = 1
    f[4, 3] = 1                       # x offsets 0,1,2,0: 3/4 -> 192; y: 1/4 -> 64
    lab, K = oracle.label(f, 0.5, 0, 8)
    c = oracle.centroids(lab, K, 8)
    assert c["qx"][0] == 256 * 3 + 192
    assert c["qy"][0] == 256 * 3 + 64
    f = np.zeros((8, 8), np.float32)
    f[3, 3:6] = 1
    f[2, 5] = 1                       # root (5,2): x offsets -2,-1,0,0 -> -3/4
    lab, K = oracle.label(f, 0.5, 0, 8)
    c = oracle.centroids(lab, K, 8)
    assert c["qx"][0] == 256 * 5 - 192
    assert c["qy"][0] == 256 * 2 + 192  # y offsets 1,1,1,0 -> 3/4
    f = np.zeros((8, 8), np.float32)
    f[3, 3:6] = 1                     # x offsets 0,1,2 -> 1: exact
    f[2, 2] = 1                       # root (2,2): x offsets 1,2,3,0 -> 6/4 = 1.5 -> 384
    lab, K = oracle.label(f, 0.5, 0, 8)
    c = oracle.centroids(lab, K, 8)
    assert c["qx"][0] == 256 * 2 + 384
    f = np.zeros((8, 8), np.float32)
    f[4, 4] = 1
    f[3, 5] = 1
    f[3, 6] = 1                       # root (5,3): x offsets 0,1,-1 -> 0; y 0,0,1 -> 1/3 -> 85.33 -> 85
    lab, K = oracle.label(f, 0.5, 0, 8)
    c = oracle.centroids(lab, K, 8)
    assert c["qx"][0] == 256 * 5 and c["qy"][0] == 256 * 3 + 85


@pytest.mark.parametrize("L", [12, 13])
def test_full_width_strip_centre_follows_the_stated_wrap(L):
    """A strip that wraps the torus has no well-defined centre; the oracle's
    reading takes offsets from the root in [-floor(L/2), L-1-floor(L/2)], so a
    strip of even width L averages to -1/2 (x = L - 1/2) and of odd width to 0."""
    f = np.zeros((7, L), np.float32)
    f[3, :] = 1.0
    lab, K = oracle.label(f, 0.5, 0, 8)
    c = oracle.centroids(lab, K, 8)
    assert K == 1 and c["amb"][0] == 1 and c["n"][0] == L
    want = (256 * L - 128) if L % 2 == 0 else 0
    assert c["qx"][0] == want and c["qy"][0] == 3 * 256
    assert c["fx"][0] == (L - 0.5 if L % 2 == 0 else 0.0)
