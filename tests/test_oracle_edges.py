"""Pins for the oracle's Delaunay couples from the digital Voronoi diagram
(Sec. 3.2.2): vertex detection by frame gaps and the nearest-neighbour rules.

References: the exact periodic Delaunay triangulation (Qhull on 3x3 images,
certified by integer in-circle tests, ``delaunay_ref``), Euler's relation
E = 3V for a triangulation of the torus, and hand-built colour maps.
"""
import numpy as np
import pytest

import oracle
from delaunay_ref import periodic_delaunay, spread_points


def tri_lattice(rng, nx, ny, a, jit):
    """Jittered triangular arrangement: every Voronoi edge stays long."""
    lx = nx * a
    ly = int(round(ny * a * np.sqrt(3) / 2))
    pts = []
    for j in range(ny):
        for i in range(nx):
            x = (i + 0.5 * (j % 2)) * a + rng.normal(0, jit)
            y = j * ly / ny + rng.normal(0, jit)
            pts.append((x % lx, y % ly))
    pts = np.array(pts)
    qx = np.floor(pts[:, 0] * 256).astype(np.int64) % (256 * lx)
    qy = np.floor(pts[:, 1] * 256).astype(np.int64) % (256 * ly)
    return qx.astype(np.int32), qy.astype(np.int32), lx, ly


def _oracle_edges(lx, ly, qx, qy):
    om = oracle.owner(lx, ly, qx, qy)
    return oracle.edges(lx, ly, qx, qy, om)


@pytest.mark.parametrize("seed", range(30))
def test_edges_equal_exact_delaunay_when_well_conditioned(seed):
    rng = np.random.default_rng(800 + seed)
    qx, qy, lx, ly = tri_lattice(rng, 6, 6, 16, 2.0)
    E, lmin, ok = periodic_delaunay(qx, qy, lx, ly)
    if not ok or lmin < 1.0:
        pytest.skip("configuration too close to degeneracy for an exact comparison")
    ab = _oracle_edges(lx, ly, qx, qy)
    assert set(map(tuple, ab.tolist())) == E
    assert len(ab) == 3 * len(qx)


def test_enough_well_conditioned_cases_ran():
    n = 0
    for seed in range(30):
        rng = np.random.default_rng(800 + seed)
        qx, qy, lx, ly = tri_lattice(rng, 6, 6, 16, 2.0)
        E, lmin, ok = periodic_delaunay(qx, qy, lx, ly)
        n += ok and lmin >= 1.0
    assert n >= 12


@pytest.mark.parametrize("seed", range(25))
def test_differences_only_at_the_lattice_cutoff(seed):
    """On arbitrary generic points the digital rules may flip a diagonal only
    when the dual Voronoi edge is shorter than one lattice spacing (the lattice
    cut-off the paper attributes to the digital setting and to the fifth
    second-neighbour condition); every such difference is a swapped diagonal,
    so the count of couples still obeys E = 3V."""
    rng = np.random.default_rng(900 + seed)
    L = int(rng.integers(64, 112))
    qx, qy = spread_points(rng, 40, L, L, 8.0)
    E, lmin, ok, vlen = periodic_delaunay(qx, qy, L, L, return_lengths=True)
    if not ok:
        pytest.skip("degenerate")
    got = set(map(tuple, _oracle_edges(L, L, qx, qy).tolist()))
    missing, extra = E - got, got - E
    assert len(missing) == len(extra)
    for e in missing:
        assert vlen[e] < 1.0, (e, vlen[e])
    assert len(got) == 3 * len(qx)


def test_edge_list_structure():
    rng = np.random.default_rng(5)
    qx, qy = spread_points(rng, 30, 70, 60, 7.0)
    ab = _oracle_edges(70, 60, qx, qy)
    assert np.all(ab[:, 0] < ab[:, 1])
    keys = ab[:, 0].astype(np.int64) * 1000 + ab[:, 1]
    assert np.all(np.diff(keys) > 0)          # sorted and unique


def _map_with_colours(rows):
    return np.array(rows, dtype=np.int32)


def test_gap_counting_bulk_edge_vertex():
    """Hand-built colour maps: uniform (no gaps), a straight two-cell
    boundary (2 gaps per site) and a three-cell corner (a vertex)."""
    # centres are only consulted for inner-frame points; place them so that
    # the diagonal rule is never the deciding one here
    qx = np.array([0, 0, 0], np.int32)
    qy = np.array([0, 0, 0], np.int32)
    one = np.zeros((6, 6), np.int32)
    assert len(oracle.edges(6, 6, qx[:1], qy[:1], one)) == 0
    two = np.zeros((6, 8), np.int32)
    two[:, 4:] = 1        # two straight boundaries on the torus, no vertex
    assert len(oracle.edges(8, 6, qx[:2], qy[:2], two)) == 0
    # three vertical stripes: still only two-gap sites
    three = np.zeros((6, 9), np.int32)
    three[:, 3:6] = 1
    three[:, 6:] = 2
    assert len(oracle.edges(9, 6, qx, qy, three)) == 0


def test_isolated_site_is_not_a_vertex():
    """An island (a site whose eight neighbours share one other colour) has a
    gap-free frame and links nothing."""
    m = np.zeros((7, 7), np.int32)
    m[3, 3] = 1
    qx = np.array([0, 3 * 256], np.int32)
    qy = np.array([0, 3 * 256], np.int32)
    assert len(oracle.edges(7, 7, qx, qy, m)) == 0


def test_t_junction_links_all_three_cells():
    """Cells 0 (left half), 1 (top right), 2 (bottom right) meet in T
    junctions; every pair of the three is linked."""
    lx, ly = 12, 12
    m = np.zeros((ly, lx), np.int32)
    m[:6, 6:] = 1
    m[6:, 6:] = 2
    qx = np.array([3 * 256, 9 * 256, 9 * 256], np.int32)
    qy = np.array([6 * 256, 3 * 256, 9 * 256], np.int32)
    ab = oracle.edges(lx, ly, qx, qy, m)
    assert set(map(tuple, ab.tolist())) == {(0, 1), (0, 2), (1, 2)}


def test_first_neighbour_rule_needs_its_long_diagonal():
    """Worked example of the first-neighbour rule of Sec. 3.2.2 (reading 9):
    a vertex site v of colour A links to its neighbour spx only when the
    long diagonal spy / smypx is split.  Background C; A = v = (5, 5), its
    left neighbour and the site below it; B = the single site right of v.
    v's frame, cyclic from spx: B, C, C, C, A, C, A, C (six gaps, a vertex);
    spx = B, but spy = smypx = C, so v does not link A to B (a rule checking
    spy against smy, or no diagonal at all, would).  The other vertex sites
    of colour A or B cannot link them either: the site below v has B at
    spxpy, but its inner point (5.5, 4.5) is nearest to the centre placed
    there for C, so the second-neighbour rule does not fire; the other A
    site and the B site see two gaps only.  A and C are linked (spy of v)."""
    L = 12
    m = np.full((L, L), 2, np.int32)          # C
    m[5, 5] = m[5, 4] = m[4, 5] = 0          # A: v, its left neighbour, the site below
    m[5, 6] = 1                              # B: right of v
    qx = np.array([256 * 4 + 128, 256 * 6, 256 * 5 + 128], np.int32)
    qy = np.array([256 * 5, 256 * 5, 256 * 4 + 128], np.int32)
    ab = set(map(tuple, oracle.edges(L, L, qx, qy, m).tolist()))
    assert (0, 1) not in ab
    assert (0, 2) in ab


def test_short_diagonal_condition_blocks_link_across_thin_band():
    """Colours by (x + y) mod 24: 0 | one-site diagonal band 1 | 2 | band 3.
    Cells 0 and 2 are diagonal lattice neighbours across band 1; the fourth
    second-neighbour condition (spx and spy of one colour) must keep them
    apart (short-diagonal pathology, Sec. 3.2.2).  All centres coincide, so
    every inner-frame point takes colour 0 and the fifth condition alone
    would let 0-2 through."""
    L = 24
    yy, xx = np.mgrid[0:L, 0:L]
    s = (xx + yy) % L
    m = np.where(s <= 10, 0, np.where(s == 11, 1, np.where(s <= 22, 2, 3))).astype(np.int32)
    q = np.zeros(4, np.int32)
    ab = oracle.edges(L, L, q, q, m)
    assert set(map(tuple, ab.tolist())) == {(0, 1), (1, 2), (2, 3), (0, 3)}


def test_obstacle_sites_do_not_count_as_gaps():
    """Two straight stripes (no Voronoi vertex) with an obstacle block
    (colour MAXLINK) on their boundary: transitions to or from an obstacle are
    not gaps (Sec. 3.2.2), so no site becomes a vertex and nothing is linked."""
    M = 0x77777777
    m = np.zeros((16, 16), np.int32)
    m[:, 8:] = 1
    m[4:8, 6:10] = M
    q = np.zeros(2, np.int32)
    assert len(oracle.edges(16, 16, q, q, m)) == 0
