"""Pins of the oracle's density-weighted centroids (the centroid equation of
Sec. 2 with the field as density; the procedure of Sec. 3.1 is its unit-
weight case).  Each pin checks the oracle against something other than
itself: closed forms of weighted sums, symmetry, roll covariance, the unit-
weight centres, and exact rational arithmetic over positions unwrapped by a
flood fill."""
from fractions import Fraction

import numpy as np
import pytest

import oracle


def _q8(v: Fraction) -> int:
    """floor(256 v + 1/2) of an exact rational."""
    t = 256 * v + Fraction(1, 2)
    return t.numerator // t.denominator


def test_quantised_weights():
    rho = np.array([0.0, -3.0, 1.0 / 512, 1.0 / 256, 0.5, 1.0, 255.99, 1e6, np.nan], np.float32)
    w = oracle.weights(rho)
    # 1/512 * 256 + 1/2 = 1 exactly; below one weight unit the clamp gives 1
    assert w.tolist() == [1, 1, 1, 1, 128, 256, 65533, 65535, 1]


def test_constant_density_gives_the_unweighted_centres():
    rng = np.random.default_rng(3)
    for seed in range(6):
        f = (rng.random((40, 56)) > 0.55).astype(np.float32)
        lab, K = oracle.label(f, 0.5)
        a = oracle.centroids(lab, K)
        b = oracle.centroids(lab, K, field=np.where(lab >= 0, 0.75, 0.0).astype(np.float32))
        assert K > 3
        assert np.array_equal(a["qx"], b["qx"]) and np.array_equal(a["qy"], b["qy"])
        assert np.allclose(a["fx"], b["fx"], rtol=0, atol=1e-9)
        assert np.allclose(a["fy"], b["fy"], rtol=0, atol=1e-9)
        assert np.array_equal(b["w"], 192 * a["n"])


@pytest.mark.parametrize("L,H,a,b,x0,y0", [(7, 3, 5, 2, 4, 6), (12, 1, 1, 9, 0, 0),
                                          (9, 4, 300, 17, 10, 2), (31, 2, 2, 0, 1, 1)])
def test_linear_ramp_closed_form(L, H, a, b, x0, y0):
    """Density a + b i (i = 0..L-1 along x, in 1/256 units) on an L x H
    rectangle: the x centre is x0 + (a S1 + b S2) / (a L + b S1) with S1 =
    L(L-1)/2 and S2 = (L-1)L(2L-1)/6; the y centre is the middle row."""
    lx, ly = 64, 32
    f = np.zeros((ly, lx), np.float32)
    for i in range(L):
        f[y0:y0 + H, x0 + i] = (a + b * i) / 256.0
    lab, K = oracle.label(f, 0.0)
    assert K == 1
    c = oracle.centroids(lab, K, field=f)
    S1, S2 = Fraction(L * (L - 1), 2), Fraction((L - 1) * L * (2 * L - 1), 6)
    cx = x0 + (a * S1 + b * S2) / (a * L + b * S1)
    cy = y0 + Fraction(H - 1, 2)
    assert c["qx"][0] == _q8(cx) and c["qy"][0] == _q8(cy)
    assert c["w"][0] == H * (a * L + b * S1)
    assert abs(c["fx"][0] - float(cx)) < 1e-9 and abs(c["fy"][0] - float(cy)) < 1e-9


def test_symmetric_density_centre():
    """A disk whose density depends only on the distance to a lattice site
    (or to a half-integer point) has its weighted centre exactly there."""
    lx = ly = 48
    for cx2, cy2 in ((40, 38), (41, 38), (41, 39)):        # twice the centre
        yy, xx = np.mgrid[0:ly, 0:lx]
        d2 = (2 * xx - cx2) ** 2 + (2 * yy - cy2) ** 2       # 4 x squared distance
        f = np.where(d2 <= 4 * 9 ** 2, 1.0 + d2 / 1000.0, 0.0).astype(np.float32)
        lab, K = oracle.label(f, 0.5)
        c = oracle.centroids(lab, K, field=f)
        assert K == 1
        assert c["qx"][0] == 128 * cx2 and c["qy"][0] == 128 * cy2


@pytest.mark.parametrize("conn", [4, 8])
def test_roll_covariance_across_the_seams(conn):
    """Rolling the field moves every weighted centre by the roll (mod the
    lattice), also for components split by the periodic seams."""
    rng = np.random.default_rng(11)
    lx, ly = 40, 36
    base = np.zeros((ly, lx), np.float32)
    yy, xx = np.mgrid[0:ly, 0:lx]
    ox, oy = rng.integers(0, lx), rng.integers(0, ly)
    # nine blobs of radius 2-4 on a jittered 3 x 3 grid (13 / 12 apart, so no
    # two merge and none reaches half the lattice); the grid offset puts some
    # of them across the seams
    for i in range(3):
        for j in range(3):
            x = (ox + 13 * i + rng.integers(-1, 2)) % lx
            y = (oy + 12 * j + rng.integers(-1, 2)) % ly
            r = rng.integers(2, 5)
            dx = (xx - x + lx // 2) % lx - lx // 2
            dy = (yy - y + ly // 2) % ly - ly // 2
            d = dx ** 2 + dy ** 2
            base = np.maximum(base, np.where(d <= r * r, 1.0 + (r * r - d + 3 * dx) / 7.0,
                                             0.0).astype(np.float32))
    lab0, K0 = oracle.label(base, 0.5, conn=conn)
    c0 = oracle.centroids(lab0, K0, field=base)
    assert K0 == 9
    for sx, sy in ((0, 0), (17, 0), (0, 29), (33, 5)):
        f = np.roll(np.roll(base, sy, axis=0), sx, axis=1)
        lab, K = oracle.label(f, 0.5, conn=conn)
        c = oracle.centroids(lab, K, field=f)
        assert K == K0
        got = sorted(zip(c["qx"].tolist(), c["qy"].tolist(), c["w"].tolist()))
        exp = sorted(zip(((c0["qx"] + 256 * sx) % (256 * lx)).tolist(),
                         ((c0["qy"] + 256 * sy) % (256 * ly)).tolist(), c0["w"].tolist()))
        assert got == exp


def _flood_centres(f, lab, K, lx, ly, conn):
    """Exact weighted centres from positions unwrapped by a flood fill from
    each component's raster-first site (components smaller than half the
    lattice, so the unwrapping is unique)."""
    w = oracle.weights(f)
    nb = [(1, 0), (-1, 0), (0, 1), (0, -1)] + ([(1, 1), (1, -1), (-1, 1), (-1, -1)] if conn == 8 else [])
    out = {}
    for k in range(K):
        ys, xs = np.nonzero(lab == k)
        i0 = np.argmin(ys * lx + xs)
        start = (int(xs[i0]), int(ys[i0]))
        pos = {start: start}
        stack = [start]
        while stack:
            (x, y) = stack.pop()
            ux, uy = pos[(x, y)]
            for dx, dy in nb:
                xx, yy = (x + dx) % lx, (y + dy) % ly
                if lab[yy, xx] == k and (xx, yy) not in pos:
                    pos[(xx, yy)] = (ux + dx, uy + dy)
                    stack.append((xx, yy))
        W = sum(int(w[y, x]) for (x, y) in pos)
        Sx = sum(int(w[y, x]) * ux for (x, y), (ux, uy) in pos.items())
        Sy = sum(int(w[y, x]) * uy for (x, y), (ux, uy) in pos.items())
        us = np.array(list(pos.values()))
        ext = (int(np.ptp(us[:, 0])), int(np.ptp(us[:, 1])))
        out[k] = ((_q8(Fraction(Sx, W)) % (256 * lx), _q8(Fraction(Sy, W)) % (256 * ly), W), ext)
    return out


@pytest.mark.parametrize("seed", range(8))
def test_brute_force_exact_rationals(seed):
    rng = np.random.default_rng(100 + seed)
    lx, ly = int(rng.integers(12, 30)), int(rng.integers(12, 30))
    conn = 8 if seed % 2 else 4
    f = (rng.random((ly, lx)) * 3.0).astype(np.float32)
    f[rng.random((ly, lx)) < (0.84 if conn == 8 else 0.76)] = 0.0
    lab, K = oracle.label(f, 0.2, conn=conn)
    c = oracle.centroids(lab, K, conn=conn, field=f)
    exp = _flood_centres(f, lab, K, lx, ly, conn)
    # components whose unwrapped extent stays below half the lattice have a
    # unique unwrapping; the others are left out
    checked = 0
    for k in range(K):
        centre, (ex, ey) = exp[k]
        if 2 * (ex + 1) >= lx or 2 * (ey + 1) >= ly:
            continue
        assert (int(c["qx"][k]), int(c["qy"][k]), int(c["w"][k])) == centre, k
        checked += 1
    assert checked >= 5


def test_clamped_weights_in_the_centres():
    """Bubbles (inside below the threshold): sites with a density of zero or
    below weigh one unit, so a bubble of such sites has the unweighted
    centre; a bubble with one column at density 1/4 (64 units) beside zero
    columns has the closed-form centre."""
    lx, ly = 32, 24
    f = np.ones((ly, lx), np.float32)
    f[3:8, 4:10] = -2.0                      # all clamped: unit weights
    f[12:15, 20:24] = 0.0                    # columns 20..23 at weight 1 ...
    f[12:15, 23] = 0.25                      # ... except column 23 at 64
    lab, K = oracle.label(f, 0.5, phase=1)
    assert K == 2
    c = oracle.centroids(lab, K, field=f)
    u = oracle.centroids(lab, K)
    assert c["qx"][0] == u["qx"][0] == 256 * 4 + 640 and c["qy"][0] == u["qy"][0] == 256 * 5
    assert c["w"][0] == 30
    cx = 20 + Fraction(0 + 1 + 2 + 64 * 3, 3 + 64)
    assert c["qx"][1] == _q8(cx) and c["qy"][1] == 256 * 13 and c["w"][1] == 3 * 67


def test_scaling_the_density_keeps_the_centres():
    rng = np.random.default_rng(7)
    f = np.where(rng.random((30, 30)) > 0.5, rng.integers(1, 40, (30, 30)) / 8.0, 0).astype(np.float32)
    lab, K = oracle.label(f, 0.01)
    a = oracle.centroids(lab, K, field=f)
    b = oracle.centroids(lab, K, field=4 * f)            # exact: weights times four
    assert np.array_equal(a["qx"], b["qx"]) and np.array_equal(a["qy"], b["qy"])
    assert np.array_equal(4 * a["w"], b["w"])


def test_weighted_sequence_runs_and_moves_centres():
    """The weighted variant changes centres where the density is uneven and
    the rest of the path runs on them (a two-frame sequence)."""
    lx = ly = 64
    yy, xx = np.mgrid[0:ly, 0:lx]
    f = np.zeros((ly, lx), np.float32)
    for (x, y) in ((16, 16), (48, 16), (16, 48), (48, 48), (32, 32)):
        d = (xx - x) ** 2 + (yy - y) ** 2
        f = np.maximum(f, np.where(d <= 36, 1.0 + 0.2 * (xx - x), 0.0).astype(np.float32))
    s_w = oracle.Sequence(0.5, weighted=True)
    s_u = oracle.Sequence(0.5)
    now_w, _ = s_w.push(f)
    now_u, _ = s_u.push(f)
    assert now_w.K == now_u.K == 5
    # density grows with x inside every disk: weighted centres sit right of the unweighted
    assert np.all(now_w.comps["qx"] > now_u.comps["qx"])
    assert np.array_equal(now_w.comps["qy"], now_u.comps["qy"])
    _, d = s_w.push(np.roll(f, 3, axis=1))
    assert d.flips.shape == (0, 6)
