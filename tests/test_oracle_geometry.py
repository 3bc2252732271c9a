"""Pins for the oracle's obstacles and open (walled) axes.

Obstacles (Sec. 3.2.1): sites of a binary field take the colour MAXLINK and,
since gaps involving MAXLINK are not counted (Sec. 3.2.2), cells separated by
an obstacle are not neighbours.  Open axes (Sec. 3.2.2, frame on the domain
boundary): no wrap, and the frame keeps only in-domain neighbours.

References independent of the oracle's code: scipy.ndimage.label (bounded
connected components), numpy means and argmins, and Qhull's Delaunay
triangulation of the centres (scipy.spatial.Delaunay), whose dual Voronoi
vertices decide which couples a walled domain can show.  The equality
"open axis == periodic axis of twice the length whose extra half is obstacle"
then ties the two features together on whole sequences.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_1607_00908_amd.synth import GRFSim, tiny_random_field

M = oracle.MAXLINK


def canon(lab):
    """Relabel components 0..K-1 by their smallest raster index (-1 stays)."""
    out = np.full(lab.shape, -1, dtype=np.int64)
    flat = lab.ravel()
    order = {}
    for v in flat:
        if v >= 0 and v not in order:
            order[v] = len(order)
    for v, k in order.items():
        out[lab == v] = k
    return out


# ----------------------------------------------------------- labelling (Sec. 3.1)
@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("seed", range(6))
def test_walled_labels_equal_scipy(conn, seed):
    lx, ly = 53 + seed, 41
    f = tiny_random_field(lx, ly, 300 + seed)
    rng = np.random.default_rng(seed)
    obst = rng.random((ly, lx)) < 0.12
    lab, K = oracle.label(f, 0.45, 0, conn, obstacles=obst, open_x=True, open_y=True)
    inside = (f > np.float32(0.45)) & ~obst
    st = np.ones((3, 3), int) if conn == 8 else None
    ref, n = ndimage.label(inside, structure=st)
    assert K == n
    assert np.array_equal(lab, canon(ref - 1))
    assert np.all(lab[obst] == -1)


def test_open_axis_cuts_components_at_the_edge():
    lx, ly = 24, 16
    f = np.zeros((ly, lx), np.float32)
    f[5:9, 0:3] = 1.0          # touches the left edge
    f[6:8, lx - 2:lx] = 1.0    # touches the right edge, same rows
    f[0:2, 10:12] = 1.0        # touches the bottom edge
    f[ly - 1, 10:12] = 1.0     # and the top edge above it
    assert oracle.label(f, 0.5)[1] == 2
    assert oracle.label(f, 0.5, open_x=True)[1] == 3
    assert oracle.label(f, 0.5, open_y=True)[1] == 3
    assert oracle.label(f, 0.5, open_x=True, open_y=True)[1] == 4


def test_obstacle_sites_are_never_inside():
    f = np.ones((8, 8), np.float32)
    obst = np.zeros((8, 8), bool)
    obst[:, 3] = True
    obst[:, 6] = True
    # periodic: three strips 0-2, 4-5, 7 where 7 joins 0-2 across the seam
    assert oracle.label(f, 0.5, obstacles=obst)[1] == 2
    assert oracle.label(f, 0.5, obstacles=obst, open_x=True)[1] == 3


# ----------------------------------------------------------- centres (Sec. 3.1)
@pytest.mark.parametrize("seed", range(5))
def test_walled_centres_are_exact_means(seed):
    lx, ly = 64, 48
    f = GRFSim(lx, ly, 2.5, 0.9, 700 + seed).field()
    lab, K = oracle.label(f, 0.8, open_x=True, open_y=True)
    c = oracle.centroids(lab, K, open_x=True, open_y=True)
    ys, xs = np.nonzero(lab >= 0)
    ids = lab[ys, xs]
    for k in range(K):
        sel = ids == k
        n = int(sel.sum())
        sx, sy = int(xs[sel].sum()), int(ys[sel].sum())
        # round half up of 256 * mean, from absolute coordinates
        assert c["n"][k] == n
        assert c["qx"][k] == (512 * sx + n) // (2 * n)
        assert c["qy"][k] == (512 * sy + n) // (2 * n)
        assert c["fx"][k] == pytest.approx(sx / n, abs=1e-12)
        assert c["fy"][k] == pytest.approx(sy / n, abs=1e-12)
        assert c["amb"][k] == 0


@pytest.mark.parametrize("conn", [4, 8])
def test_walled_centre_of_a_component_longer_than_half_the_lattice(conn):
    """On a walled axis offsets are plain differences however far apart the
    sites are (a minimum image would fold the far end back)."""
    lx, ly = 40, 30
    f = np.zeros((ly, lx), np.float32)
    f[3, 1:35] = 1.0          # x = 1..34, mean 17.5
    f[10:27, 20] = 1.0        # y = 10..26 in one column, mean 18
    f[2, 37] = 1.0
    lab, K = oracle.label(f, 0.5, conn=conn, open_x=True, open_y=True)
    c = oracle.centroids(lab, K, conn=conn, open_x=True, open_y=True)
    assert K == 3
    assert c["qx"][1] == 256 * 17 + 128 and c["qy"][1] == 256 * 3
    assert c["qx"][2] == 256 * 20 and c["qy"][2] == 256 * 18
    assert list(c["amb"]) == [0, 0, 0]


def test_centre_of_a_component_on_the_seam_depends_on_the_axis():
    lx, ly = 20, 10
    f = np.zeros((ly, lx), np.float32)
    f[4, 0:2] = 1.0
    f[4, lx - 2:lx] = 1.0
    lab, K = oracle.label(f, 0.5)
    assert K == 1
    c = oracle.centroids(lab, K)
    # offsets -2, -1, 0, 1 from the root at x = 0: mean -0.5 -> 19.5
    assert c["qx"][0] == 256 * 19 + 128
    lab, K = oracle.label(f, 0.5, open_x=True)
    c = oracle.centroids(lab, K, open_x=True)
    assert K == 2 and list(c["qx"]) == [128, 256 * 18 + 128]


# ----------------------------------------------------------- colouring (Sec. 3.2.1)
def brute_owner(lx, ly, qx, qy, ox, oy):
    Y, X = np.mgrid[0:ly, 0:lx]
    X = 256 * X[..., None].astype(np.int64)
    Y = 256 * Y[..., None].astype(np.int64)
    dx = X - np.asarray(qx, np.int64)
    dy = Y - np.asarray(qy, np.int64)
    if not ox:
        dx = np.minimum(np.abs(dx), 256 * lx - np.abs(dx))
    if not oy:
        dy = np.minimum(np.abs(dy), 256 * ly - np.abs(dy))
    return np.argmin(dx * dx + dy * dy, axis=2)   # first minimum = lowest label


@pytest.mark.parametrize("ox,oy", [(True, True), (True, False), (False, True)])
@pytest.mark.parametrize("seed", range(4))
def test_walled_owner_brute_force(ox, oy, seed):
    rng = np.random.default_rng(40 + seed)
    lx, ly = 70, 52
    K = 25
    qx = rng.integers(0, 256 * lx, K)
    qy = rng.integers(0, 256 * ly, K)
    # exact ties on purpose: a few centres on the same point
    qx[3], qy[3] = qx[7], qy[7]
    obst = rng.random((ly, lx)) < 0.05
    om = oracle.owner(lx, ly, qx, qy, obstacles=obst, open_x=ox, open_y=oy)
    ref = brute_owner(lx, ly, qx, qy, ox, oy)
    ref[obst] = M
    assert np.array_equal(om, ref)
    # obstacles change only their own sites
    om0 = oracle.owner(lx, ly, qx, qy, open_x=ox, open_y=oy)
    assert np.array_equal(om0[~obst], om[~obst])


# ----------------------------------------------------------- couples (Sec. 3.2.2)
def _plain_points(rng, V, lx, ly, min_sep, free):
    pts = []
    tries = 0
    while len(pts) < V and tries < 20000:
        tries += 1
        x, y = rng.uniform(0, lx - 1), rng.uniform(0, ly - 1)
        if not free[int(round(y)), int(round(x))]:
            continue
        if all((x - a) ** 2 + (y - b) ** 2 >= min_sep ** 2 for a, b in pts):
            pts.append((x, y))
    qx = np.array([int(np.floor(256 * p[0])) for p in pts], np.int32)
    qy = np.array([int(np.floor(256 * p[1])) for p in pts], np.int32)
    return qx, qy


def _tri_points(rng, lx, ly, a, jit, free):
    """Jittered triangular arrangement inside the domain (long Voronoi edges)."""
    pts = []
    h = a * np.sqrt(3) / 2
    x0, y0 = rng.uniform(0, a), rng.uniform(0, h)
    j = 0
    y = y0
    while y < ly - 1:
        x = x0 + 0.5 * a * (j % 2)
        while x < lx - 1:
            px, py = x + rng.normal(0, jit), y + rng.normal(0, jit)
            if 0 <= px <= lx - 1 and 0 <= py <= ly - 1 and free[int(round(py)), int(round(px))]:
                pts.append((px, py))
            x += a
        y += h
        j += 1
    qx = np.array([int(np.floor(256 * p[0])) for p in pts], np.int32)
    qy = np.array([int(np.floor(256 * p[1])) for p in pts], np.int32)
    return qx, qy


def _circumcentre(a, b, c):
    ax, ay = a
    bx, by = b
    cx, cy = c
    d = 2.0 * (ax * (by - cy) + bx * (cy - ay) + cx * (ay - by))
    ux = ((ax * ax + ay * ay) * (by - cy) + (bx * bx + by * by) * (cy - ay)
          + (cx * cx + cy * cy) * (ay - by)) / d
    uy = ((ax * ax + ay * ay) * (cx - bx) + (bx * bx + by * by) * (ax - cx)
          + (cx * cx + cy * cy) * (bx - ax)) / d
    return ux, uy


def bounded_expectation(qx, qy, fluid):
    """Couples a walled, obstructed digital diagram must and must not show.

    Each Delaunay couple (Qhull) is dual to a Voronoi edge whose ends are the
    circumcentres of its triangles.  The digital rules see a couple at a
    Voronoi vertex whose neighbourhood is fluid; a vertex with no fluid site
    near it shows nothing.  Near degeneracy (a Voronoi edge shorter than 1.5
    sites) the lattice may swap the diagonal of the two triangles: both
    diagonals are then left open.  Returns (must, must_not, delaunay,
    allowed extra couples)."""
    from scipy.spatial import Delaunay
    ly, lx = fluid.shape
    P = np.stack([qx / 256.0, qy / 256.0], axis=1)
    tri = Delaunay(P)
    cen, opp = {}, {}
    for s in tri.simplices:
        c = _circumcentre(P[s[0]], P[s[1]], P[s[2]])
        for u, v, w in ((s[0], s[1], s[2]), (s[1], s[2], s[0]), (s[2], s[0], s[1])):
            e = (min(u, v), max(u, v))
            cen.setdefault(e, []).append(c)
            opp.setdefault(e, []).append(int(w))

    def window(c, r):
        x, y = int(round(c[0])), int(round(c[1]))
        xs = np.arange(x - r, x + r + 1)
        ys = np.arange(y - r, y + r + 1)
        inx = (xs >= 0) & (xs < lx)
        iny = (ys >= 0) & (ys < ly)
        return xs, ys, inx, iny

    def clearly_in(c):
        xs, ys, inx, iny = window(c, 3)
        return inx.all() and iny.all() and fluid[np.ix_(ys, xs)].all()

    def clearly_out(c):
        xs, ys, inx, iny = window(c, 5)
        if not inx.any() or not iny.any():
            return True
        return not fluid[np.ix_(ys[iny], xs[inx])].any()

    open_ = set()
    extra = set()
    for e, cs in cen.items():
        if len(cs) == 2 and np.hypot(cs[0][0] - cs[1][0], cs[0][1] - cs[1][1]) < 1.5:
            o = opp[e]
            open_.add(e)
            extra.add((min(o), max(o)))
    must, must_not = set(), set()
    for e, cs in cen.items():
        if e in open_:
            continue
        if any(clearly_in(c) for c in cs):
            must.add(e)
        elif all(clearly_out(c) for c in cs):
            must_not.add(e)
    return must, must_not, set(cen), extra


def _check_bounded(lx, ly, qx, qy, obst, ox, oy):
    fluid = ~obst if obst is not None else np.ones((ly, lx), bool)
    must, must_not, dela, extra = bounded_expectation(qx, qy, fluid)
    om = oracle.owner(lx, ly, qx, qy, obstacles=obst, open_x=ox, open_y=oy)
    got = set(map(tuple, oracle.edges(lx, ly, qx, qy, om, open_x=ox, open_y=oy).tolist()))
    assert must <= got, sorted(must - got)
    assert not (must_not & got), sorted(must_not & got)
    assert got - dela <= extra, sorted(got - dela)
    return len(must), len(must_not)


@pytest.mark.parametrize("seed", range(12))
def test_walled_couples_follow_bounded_delaunay(seed):
    rng = np.random.default_rng(900 + seed)
    lx, ly = 150, 110
    free = np.ones((ly, lx), bool)
    qx, qy = _tri_points(rng, lx, ly, 16.0, 2.0, free)
    r = _check_bounded(lx, ly, qx, qy, None, True, True)
    assert r[0] >= 60 and r[1] >= 1


@pytest.mark.parametrize("seed", range(12))
def test_channel_with_posts_follows_bounded_delaunay(seed):
    """The paper's geometry in small: walls across x, posts on the left wall."""
    rng = np.random.default_rng(950 + seed)
    lx, ly = 120, 160
    obst = np.zeros((ly, lx), bool)
    for y0 in range(0, ly, 40):
        obst[y0:y0 + 16, 0:18] = True
    qx, qy = _tri_points(rng, lx, ly, 16.0, 2.0, ~obst)
    r = _check_bounded(lx, ly, qx, qy, obst, True, True)
    assert r[0] >= 60 and r[1] >= 1


@pytest.mark.parametrize("walls", ["open", "obstacles"])
def test_corridor_of_collinear_centres_shows_no_couple(walls):
    """Centres in one line along a corridor: every Voronoi edge runs from
    wall to wall and there is no Voronoi vertex, so no site has three gaps
    that do not involve MAXLINK, and there is no couple at all.  (Counting
    the gaps next to a wall would join every consecutive pair.)"""
    ly = 128
    if walls == "open":
        lx, ox, obst = 12, True, None
    else:
        lx, ox = 20, False
        obst = np.zeros((ly, lx), bool)
        obst[:, :4] = True
        obst[:, 16:] = True
    qx = np.full(8, 256 * (lx // 2) + 128, np.int32)
    qy = (256 * (8 + 16 * np.arange(8)) + 77).astype(np.int32)
    om = oracle.owner(lx, ly, qx, qy, obstacles=obst, open_x=ox)
    assert len(set(om[:, lx // 2].tolist())) == 8
    assert len(oracle.edges(lx, ly, qx, qy, om, open_x=ox)) == 0


def test_thick_wall_separates_the_two_sides():
    """A wall across a periodic lattice, thicker than any cell: no couple
    joins centres on opposite sides (through the wall or around it)."""
    rng = np.random.default_rng(5)
    lx, ly = 128, 128
    obst = np.zeros((ly, lx), bool)
    obst[56:72, :] = True
    free = ~obst
    free[46:82, :] = False   # keep centres away from the wall
    qx, qy = _plain_points(rng, 60, lx, ly, 11.0, free)
    om = oracle.owner(lx, ly, qx, qy, obstacles=obst)
    ab = oracle.edges(lx, ly, qx, qy, om)
    below = (qy // 256) < 56
    across = [(a, b) for a, b in ab.tolist() if below[a] != below[b]]
    # the periodic seam at y = 0 / 127 is open fluid: couples cross it, but
    # only between centres that the wall does not separate
    for a, b in across:
        ya, yb = qy[a] / 256.0, qy[b] / 256.0
        assert min(ya, yb) < 40 and max(ya, yb) > 88, (a, b, ya, yb)
    # without the wall the same centres do get couples through y = 64
    om0 = oracle.owner(lx, ly, qx, qy)
    ab0 = oracle.edges(lx, ly, qx, qy, om0)
    mid = [(a, b) for a, b in ab0.tolist()
           if below[a] != below[b] and max(qy[a], qy[b]) / 256 < 100 and min(qy[a], qy[b]) / 256 > 20]
    assert mid


def test_posts_away_from_voronoi_vertices_change_no_couple():
    rng = np.random.default_rng(11)
    lx, ly = 128, 96
    free = np.ones((ly, lx), bool)
    qx, qy = _plain_points(rng, 40, lx, ly, 14.0, free)
    om0 = oracle.owner(lx, ly, qx, qy)
    ab0 = oracle.edges(lx, ly, qx, qy, om0)
    # vertex sites of the unobstructed diagram: three colours in the 3x3 block
    pad = np.pad(om0, 1, mode="wrap")
    ncol = np.zeros_like(om0)
    stack = np.stack([pad[1 + dy:1 + dy + ly, 1 + dx:1 + dx + lx]
                      for dy in (-1, 0, 1) for dx in (-1, 0, 1)], axis=0)
    for y in range(ly):
        for x in range(lx):
            ncol[y, x] = len(set(stack[:, y, x].tolist()))
    near_vertex = ndimage.maximum_filter(ncol >= 3, size=11, mode="wrap")
    obst = np.zeros((ly, lx), bool)
    placed = 0
    for _ in range(400):
        x, y = rng.integers(0, lx - 3), rng.integers(0, ly - 3)
        if not near_vertex[y:y + 3, x:x + 3].any():
            obst[y:y + 3, x:x + 3] = True
            placed += 1
    assert placed >= 30
    om = oracle.owner(lx, ly, qx, qy, obstacles=obst)
    assert np.array_equal(om[~obst], om0[~obst]) and np.all(om[obst] == M)
    assert np.array_equal(oracle.edges(lx, ly, qx, qy, om), ab0)
    # posts straddle cell borders too (not only cell interiors)
    assert len(set(om0[obst].tolist())) > 1 and any(
        len(set(om0[y:y + 3, x:x + 3].ravel().tolist())) > 1
        for y, x in zip(*np.nonzero(obst)))


def test_edges_window_matches_full_map_on_a_walled_lattice():
    rng = np.random.default_rng(3)
    lx, ly = 90, 70
    obst = np.zeros((ly, lx), bool)
    obst[10:20, 0:12] = True
    obst[40:50, 0:12] = True
    qx, qy = _plain_points(rng, 30, lx, ly, 10.0, ~obst)
    om = oracle.owner(lx, ly, qx, qy, obstacles=obst, open_x=True)
    full = set(map(tuple, oracle.edges(lx, ly, qx, qy, om, open_x=True).tolist()))
    parts = set()
    for x0 in range(0, lx, 30):
        for y0 in range(0, ly, 35):
            w = oracle.edges_window(lx, ly, qx, qy, x0, y0, 30, 35, obstacles=obst, open_x=True)
            parts |= set(map(tuple, w.tolist()))
    assert parts == full


# ----------------------------------------------------------- matching (Sec. 3.2.3)
@pytest.mark.parametrize("ox,oy", [(True, True), (True, False)])
def test_walled_match_brute_force(ox, oy):
    rng = np.random.default_rng(77)
    lx, ly = 100, 60
    nqx = rng.integers(0, 256 * lx, 30)
    nqy = rng.integers(0, 256 * ly, 30)
    pqx = np.concatenate([rng.integers(0, 256 * lx, 25), nqx[:3], [0, 256 * lx - 1]])
    pqy = np.concatenate([rng.integers(0, 256 * ly, 25), nqy[:3], [0, 256 * ly - 1]])
    phi, cnt = oracle.match(lx, ly, pqx, pqy, nqx, nqy, open_x=ox, open_y=oy)
    for p in range(len(pqx)):
        dx = np.abs(pqx[p] - nqx.astype(np.int64))
        dy = np.abs(pqy[p] - nqy.astype(np.int64))
        if not ox:
            dx = np.minimum(dx, 256 * lx - dx)
        if not oy:
            dy = np.minimum(dy, 256 * ly - dy)
        assert phi[p] == int(np.argmin(dx * dx + dy * dy))
    assert np.array_equal(cnt, np.bincount(phi, minlength=30))
    if ox:
        # a past centre at x = 0 is not near a now centre at x = L - 1
        far = oracle.match(lx, ly, [0], [256 * 30], [256 * (lx - 1), 256 * 50], [256 * 30, 256 * 30],
                           open_x=True)[0]
        assert far[0] == 1


# ------------------------------------------------ open axis == obstacle padding
def _pad(a, lx, ly, px, py, fill):
    out = np.full((ly * (2 if py else 1), lx * (2 if px else 1)), fill, dtype=a.dtype)
    out[:ly, :lx] = a
    return out


@pytest.mark.parametrize("ox,oy", [(True, False), (False, True), (True, True)])
def test_open_axis_equals_periodic_axis_padded_with_obstacles(ox, oy):
    """A walled axis of length L is the periodic axis of length 2L whose far
    half is obstacle: every output agrees, frame after frame, flags included."""
    lx, ly = 72, 56
    sim = GRFSim(lx, ly, 3.0, 0.9, 31)
    posts = np.zeros((ly, lx), bool)
    posts[8:14, 0:9] = True
    posts[30:36, 0:9] = True
    posts[20:24, 40:46] = True
    pad_obst = _pad(posts, lx, ly, ox, oy, True)
    open_seq = oracle.Sequence(0.7, classify_events=True, obstacles=posts, open_x=ox, open_y=oy)
    pad_seq = oracle.Sequence(0.7, classify_events=True, obstacles=pad_obst)
    flips_seen = 0
    for f in sim.frames(4):
        a_now, a_res = open_seq.push(f)
        b_now, b_res = pad_seq.push(_pad(f, lx, ly, ox, oy, np.float32(5.0)))
        assert a_now.K == b_now.K
        assert np.array_equal(b_now.labels[:ly, :lx], a_now.labels)
        assert np.all(b_now.labels[ly:, :] == -1) and np.all(b_now.labels[:, lx:] == -1)
        for k in ("n", "qx", "qy", "amb"):
            assert np.array_equal(a_now.comps[k], b_now.comps[k]), k
        assert np.array_equal(a_now.comps["fx"], b_now.comps["fx"])
        plx = b_now.labels.shape[1]
        assert np.array_equal(a_now.comps["root"] % lx, b_now.comps["root"] % plx)
        assert np.array_equal(a_now.comps["root"] // lx, b_now.comps["root"] // plx)
        assert np.array_equal(b_now.owner[:ly, :lx], a_now.owner)
        assert np.all(b_now.owner[ly:, :] == M) and np.all(b_now.owner[:, lx:] == M)
        assert np.array_equal(a_now.edges, b_now.edges)
        assert np.array_equal(a_res.flips, b_res.flips)
        assert np.array_equal(a_res.phi, b_res.phi)
        assert np.array_equal(a_res.local_trigger, b_res.local_trigger)
        flips_seen += len(a_res.flips)
    assert flips_seen > 0
