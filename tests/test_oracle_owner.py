"""Pins for the oracle's digital Voronoi colouring (Sec. 3.2.1).

References: scipy's periodic k-d tree (a different nearest-neighbour
algorithm), hand-built equidistant ties, translation covariance, and the
areas of the exact Voronoi polygons from scipy.spatial.Voronoi.
"""
import numpy as np
import pytest

import oracle
from delaunay_ref import spread_points

MAXLINK = 0x77777777


@pytest.mark.parametrize("seed", range(8))
def test_owner_distance_equals_periodic_kdtree(seed):
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(500 + seed)
    lx, ly = int(rng.integers(20, 90)), int(rng.integers(20, 90))
    K = int(rng.integers(1, 40))
    qx = rng.integers(0, 256 * lx, K).astype(np.int32)
    qy = rng.integers(0, 256 * ly, K).astype(np.int32)
    om = oracle.owner(lx, ly, qx, qy)
    tree = cKDTree(np.stack([qx, qy], 1).astype(np.float64),
                   boxsize=[256.0 * lx, 256.0 * ly])
    yy, xx = np.mgrid[0:ly, 0:lx]
    sites = np.stack([256.0 * xx.ravel(), 256.0 * yy.ravel()], 1)
    d, _ = tree.query(sites, k=1)
    # squared distances are integers below 2^53: exact in float64
    d2_kd = np.rint(d * d).astype(np.int64)
    o = om.ravel()
    ddx = (256 * xx.ravel() - qx[o] + 128 * lx) % (256 * lx) - 128 * lx
    ddy = (256 * yy.ravel() - qy[o] + 128 * ly) % (256 * ly) - 128 * ly
    d2_or = ddx.astype(np.int64) ** 2 + ddy.astype(np.int64) ** 2
    assert np.array_equal(d2_or, d2_kd)


def test_equidistant_ties_go_to_lowest_label():
    lx, ly = 32, 16
    # label 0 at x=20, label 1 at x=10, same row: sites with x=15 are tied
    qx = np.array([20 * 256, 10 * 256], np.int32)
    qy = np.array([8 * 256, 8 * 256], np.int32)
    om = oracle.owner(lx, ly, qx, qy)
    assert np.all(om[:, 15] == 0)
    assert np.all(om[:, 14] == 1)
    assert np.all(om[:, 16] == 0)
    # the other bisector (x = 31 | 0 wraps: 20+16 = 36 = 4, 10-16 = -6 = 26... )
    # x = 31 is at distance 11 from 20 and 11 from 10 (through the seam): tie -> 0
    assert np.all(om[:, 31] == 0)
    # swapping the labels moves the tied column to the other centre
    om2 = oracle.owner(lx, ly, qx[::-1].copy(), qy[::-1].copy())
    assert np.all(om2[:, 15] == 0) and np.all(om2[:, 16] == 1)


def test_no_centres_gives_maxlink():
    om = oracle.owner(7, 5, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert np.all(om == MAXLINK)


@pytest.mark.parametrize("seed", range(5))
def test_translation_covariance(seed):
    rng = np.random.default_rng(600 + seed)
    lx, ly = 40, 36
    K = 12
    qx = rng.integers(0, 256 * lx, K).astype(np.int32)
    qy = rng.integers(0, 256 * ly, K).astype(np.int32)
    dx, dy = int(rng.integers(0, lx)), int(rng.integers(0, ly))
    om = oracle.owner(lx, ly, qx, qy)
    om2 = oracle.owner(lx, ly, (qx + 256 * dx) % (256 * lx), (qy + 256 * dy) % (256 * ly))
    assert np.array_equal(np.roll(om, (dy, dx), (0, 1)), om2)


@pytest.mark.parametrize("seed", range(6))
def test_cell_areas_track_exact_voronoi_polygons(seed):
    from scipy.spatial import Voronoi
    rng = np.random.default_rng(700 + seed)
    L = 80
    qx, qy = spread_points(rng, 25, L, L, 10.0)
    om = oracle.owner(L, L, qx, qy)
    counts = np.bincount(om.ravel(), minlength=len(qx))
    assert counts.sum() == L * L
    pts = []
    for iy in (-1, 0, 1):
        for ix in (-1, 0, 1):
            pts.append(np.stack([qx / 256.0 + ix * L, qy / 256.0 + iy * L], 1))
    P = np.concatenate(pts)
    vor = Voronoi(P)
    V = len(qx)
    for i in range(V):
        reg = vor.regions[vor.point_region[4 * V + i]]   # central copy
        assert -1 not in reg
        poly = vor.vertices[reg]
        x, y = poly[:, 0], poly[:, 1]
        area = 0.5 * abs(np.dot(x, np.roll(y, -1)) - np.dot(y, np.roll(x, -1)))
        perim = np.sum(np.hypot(np.diff(np.r_[x, x[0]]), np.diff(np.r_[y, y[0]])))
        assert abs(counts[i] - area) <= 0.75 * perim + 4, (i, counts[i], area, perim)
