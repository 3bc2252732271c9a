"""Pins for the oracle's event flags (Sec. 3.2.4, extraction of topology change
events): bulk events (both ends of a flip connected to at least three active
points) and boundary events (both ends on the boundary of the graph holding
the couple), on hand-built graphs whose answer follows from the definitions,
and on the exact periodic Delaunay T1 of ``golden/t1_fixture.json``.
"""
import numpy as np

import oracle
from test_oracle_diff import _t1_fields


def _flip(a, b, kind):
    return [min(a, b), max(a, b), min(a, b), max(a, b), kind, 0]


def test_isolated_quadrangle_flip_is_bulk_and_boundary():
    # four points, one diagonal swapped: every couple is shared by one
    # triangle only, and each point is connected to the three others in the
    # union of the two graphs
    past = np.array([[0, 1], [1, 2], [2, 3], [0, 3], [0, 2]])
    now = np.array([[0, 1], [1, 2], [2, 3], [0, 3], [1, 3]])
    flips = np.array([_flip(0, 2, -1), _flip(1, 3, +1)])
    f = oracle.classify(past, np.arange(4), now, np.ones(4, np.int32), flips)
    assert f.tolist() == [3, 3]


def test_t1_inside_a_periodic_triangulation_is_bulk_only():
    d, fields, names = _t1_fields()
    seq = oracle.Sequence(d["threshold"], d["phase"], 8, classify_events=True)
    seq.push(fields[0])
    _, res = seq.push(fields[1])
    assert len(res.flips) == 2
    assert res.flips[:, 5].tolist() == [1, 1]


def test_lost_couple_without_replacement_is_neither():
    # a closed periodic triangulation loses one couple and gains none: the two
    # ends have one active neighbour each and no boundary couple
    d, fields, names = _t1_fields()
    fr = oracle.frame(fields[0], d["threshold"])
    K = fr.K
    now = fr.edges[1:]
    a, b = fr.edges[0]
    flips = np.array([_flip(int(a), int(b), -1)])
    f = oracle.classify(fr.edges, np.arange(K), now, np.ones(K, np.int32), flips)
    assert f.tolist() == [0]


def test_boundary_couple_lost_on_an_open_fan_is_boundary_only():
    # hexagonal fan: centre 0, ring 1..6; the ring couples are boundary
    # couples (one shared neighbour, the centre)
    spokes = [[0, i] for i in range(1, 7)]
    ring = [[i, i % 6 + 1] for i in range(1, 7)]
    past = np.array(spokes + ring)
    now = np.array(spokes + ring[1:])          # couple (1, 2) is lost
    flips = np.array([_flip(1, 2, -1)])
    f = oracle.classify(past, np.arange(7), now, np.ones(7, np.int32), flips)
    assert f.tolist() == [2]


def test_excluded_points_do_not_count():
    # the quadrangle of the first test, with point 3 matched twice in the now
    # frame: its couples leave both graphs, so the remaining flip's ends are
    # no longer connected to three active points
    past = np.array([[0, 1], [1, 2], [2, 3], [0, 3], [0, 2]])
    now = np.array([[0, 1], [1, 2], [2, 3], [0, 3], [1, 3]])
    cnt = np.array([1, 1, 1, 2], np.int32)
    flips = np.array([_flip(0, 2, -1)])
    f = oracle.classify(past, np.arange(4), now, cnt, flips)
    assert f[0] & 1 == 0


def test_flags_do_not_depend_on_the_labels():
    d, fields, names = _t1_fields()
    fa, fb = oracle.frame(fields[0], d["threshold"]), oracle.frame(fields[1], d["threshold"])
    res = oracle.compare(fa, fb, classify_events=True)
    K = fb.K
    perm = np.random.default_rng(3).permutation(K)
    past_e = perm[fa.edges]
    now_e = perm[fb.edges]
    phi = np.empty(K, np.int64)
    phi[perm] = perm[res.phi]
    fl = res.flips.copy()
    fl[:, :4] = perm[fl[:, :4]]
    f = oracle.classify(past_e, phi, now_e, res.cnt[np.argsort(perm)], fl)
    assert f.tolist() == res.flips[:, 5].tolist()
