"""Pins for the oracle's threshold and cluster labelling (Sec. 3.1).

Each check compares the oracle with something other than itself: numpy's
comparison operators, a breadth-first flood fill written here, scipy's
ndimage.label, closed forms (checkerboards, strips) and roll covariance.
"""
from collections import deque

import numpy as np
import pytest

import oracle


def bfs_labels(mask: np.ndarray, conn: int) -> np.ndarray:
    """Flood fill on the torus; labels numbered by each component's first site
    in raster order (independent of the oracle's union-find)."""
    ly, lx = mask.shape
    lab = -np.ones((ly, lx), dtype=np.int64)
    if conn == 8:
        nb = [(dx, dy) for dx in (-1, 0, 1) for dy in (-1, 0, 1) if (dx, dy) != (0, 0)]
    else:
        nb = [(1, 0), (-1, 0), (0, 1), (0, -1)]
    k = 0
    for y in range(ly):
        for x in range(lx):
            if not mask[y, x] or lab[y, x] >= 0:
                continue
            lab[y, x] = k
            q = deque([(x, y)])
            while q:
                cx, cy = q.popleft()
                for dx, dy in nb:
                    nx, ny = (cx + dx) % lx, (cy + dy) % ly
                    if mask[ny, nx] and lab[ny, nx] < 0:
                        lab[ny, nx] = k
                        q.append((nx, ny))
            k += 1
    return lab


def test_threshold_strict_and_nan():
    f = np.array([[0.5, 0.49, 0.51, np.nan],
                  [np.inf, -np.inf, 0.5000001, 0.4999999],
                  [1.0, 0.0, 0.5, 0.7]], dtype=np.float32)
    for phase in (0, 1):
        lab, K = oracle.label(f, 0.5, phase, 8)
        with np.errstate(invalid="ignore"):
            want = (f > np.float32(0.5)) if phase == 0 else (f < np.float32(0.5))
        assert np.array_equal(lab >= 0, want)


@pytest.mark.parametrize("seed", range(40))
def test_labels_match_bfs(seed):
    rng = np.random.default_rng(seed)
    lx, ly = int(rng.integers(3, 14)), int(rng.integers(3, 14))
    p = rng.uniform(0.2, 0.7)
    field = rng.random((ly, lx)).astype(np.float32)
    for conn in (4, 8):
        lab, K = oracle.label(field, p, 1, conn)
        want = bfs_labels(field < np.float32(p), conn)
        assert K == want.max() + 1
        assert np.array_equal(lab, want)


@pytest.mark.parametrize("seed", range(20))
def test_labels_match_scipy_away_from_seams(seed):
    from scipy import ndimage
    rng = np.random.default_rng(100 + seed)
    lx, ly = int(rng.integers(6, 40)), int(rng.integers(6, 40))
    field = rng.random((ly, lx)).astype(np.float32)
    field[0, :] = 1.0
    field[-1, :] = 1.0
    field[:, 0] = 1.0
    field[:, -1] = 1.0
    for conn, st in ((8, np.ones((3, 3), int)), (4, ndimage.generate_binary_structure(2, 1))):
        lab, K = oracle.label(field, 0.45, 1, conn)
        ref, n = ndimage.label(field < np.float32(0.45), structure=st)
        assert K == n
        assert np.array_equal(lab, ref.astype(np.int64) - 1)


@pytest.mark.parametrize("L", [4, 6, 10, 32])
def test_checkerboard_closed_forms(L):
    yy, xx = np.mgrid[0:L, 0:L]
    f = ((xx + yy) % 2).astype(np.float32)
    lab4, K4 = oracle.label(f, 0.5, 0, 4)
    lab8, K8 = oracle.label(f, 0.5, 0, 8)
    assert K4 == L * L // 2          # every black site is its own component
    assert K8 == 1                   # diagonals join them all (even L)
    # raster order of the first site of each singleton
    ys, xs = np.nonzero(f > 0.5)
    assert np.array_equal(lab4[ys, xs], np.arange(L * L // 2))


def test_strip_wraps_into_one_component():
    f = np.zeros((9, 12), np.float32)
    f[4, :] = 1.0
    f[0, 3] = 1.0
    f[8, 3] = 1.0   # touches row 0 through the y seam
    lab, K = oracle.label(f, 0.5, 0, 8)
    assert K == 2
    assert lab[0, 3] == 0 and lab[8, 3] == 0
    assert np.all(lab[4, :] == 1)
    c = oracle.centroids(lab, K, 8)
    assert c["amb"].tolist() == [0, 1]   # the strip crosses its own antipodal line


@pytest.mark.parametrize("seed", range(10))
def test_roll_covariance_of_partition(seed):
    rng = np.random.default_rng(200 + seed)
    lx, ly = 17, 13
    f = rng.random((ly, lx)).astype(np.float32)
    dx, dy = int(rng.integers(0, lx)), int(rng.integers(0, ly))
    lab, K = oracle.label(f, 0.55, 1, 8)
    lab2, K2 = oracle.label(np.roll(f, (dy, dx), (0, 1)), 0.55, 1, 8)
    assert K == K2
    rolled = np.roll(lab, (dy, dx), (0, 1))
    # same partition: a bijection between the two labellings
    pairs = set(zip(rolled[rolled >= 0].tolist(), lab2[lab2 >= 0].tolist()))
    assert len(pairs) == K
    assert np.array_equal(rolled < 0, lab2 < 0)
