"""Pins for the oracle's isomorphism, translation and flip extraction
(Sec. 3.2.3 and 3.2.4).

References: the embedded T1 rearrangement of ``golden/t1_fixture.json``
(expected couples recomputed from the exact periodic Delaunay of both frames),
identity / reversal / integer-roll symmetries, and the paper's row-compare
trigger, which must flag exactly the endpoints of the flips.
"""
import json
import os

import numpy as np
import pytest

import oracle
from delaunay_ref import periodic_delaunay
from paper_1607_00908_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "t1_fixture.json")


def _t1_fields():
    d = json.load(open(GOLDEN))
    lx, ly, r = d["lx"], d["ly"], d["radius"]
    fields, names = [], ["A", "B", "C", "D"]
    for fr in ("0", "1"):
        pts = [d["quartet"][fr][n] for n in names] + d["background"]
        c = np.array(pts, dtype=np.float64)
        fields.append(synth.disk_field(lx, ly, c, np.full(len(pts), float(r))))
    return d, fields, names


def test_t1_fixture_is_an_exact_delaunay_t1():
    d, fields, names = _t1_fields()
    sets = []
    for fr in ("0", "1"):
        pts = [d["quartet"][fr][n] for n in names] + d["background"]
        E, lmin, ok = periodic_delaunay([256 * p[0] for p in pts], [256 * p[1] for p in pts],
                                        d["lx"], d["ly"])
        assert ok and lmin >= 2.0
        sets.append(E)
    assert sets[0] - sets[1] == {(0, 2)} and sets[1] - sets[0] == {(1, 3)}


def test_t1_oracle_reports_one_breaking_one_arising():
    d, fields, names = _t1_fields()
    seq = oracle.Sequence(d["threshold"], d["phase"], 8)
    now0, _ = seq.push(fields[0])
    now1, res = seq.push(fields[1])
    assert now0.K == now1.K == 4 + len(d["background"])
    # centroids of the integer-centred disks are exact
    lab0 = {n: int(now0.labels[d["quartet"]["0"][n][1], d["quartet"]["0"][n][0]]) for n in names}
    lab1 = {n: int(now1.labels[d["quartet"]["1"][n][1], d["quartet"]["1"][n][0]]) for n in names}
    for n in names:
        assert now1.comps["qx"][lab1[n]] == 256 * d["quartet"]["1"][n][0]
        assert now1.comps["qy"][lab1[n]] == 256 * d["quartet"]["1"][n][1]
    fl = res.flips
    assert len(fl) == 2
    a, c = sorted((lab1["A"], lab1["C"]))
    b, dd = sorted((lab1["B"], lab1["D"]))
    assert fl[0].tolist()[:2] == [a, c] and fl[0][4] == -1
    assert fl[1].tolist()[:2] == [b, dd] and fl[1][4] == +1
    # past labels map onto now labels through Phi
    for f in fl:
        assert res.phi[f[2]] == f[0] and res.phi[f[3]] == f[1]
    assert {int(fl[0][2]), int(fl[0][3])} == {lab0["A"], lab0["C"]}
    assert res.global_trigger == 1
    assert set(np.nonzero(res.local_trigger)[0].tolist()) == {lab0[n] for n in names}
    assert len(now0.edges) == len(now1.edges) == 3 * now0.K


def _disk_frames(n, seed=7, L=160, nd=40):
    sim = synth.DiskSim(L, L, nd, 5.0, 8.0, 0.6, 2e-3, seed)
    return list(sim.frames(n))


def test_identical_frames_give_identity_and_no_flips():
    f = _disk_frames(1)[0]
    seq = oracle.Sequence(0.5)
    seq.push(f)
    now, res = seq.push(f)
    assert np.array_equal(res.phi, np.arange(now.K))
    assert np.all(res.cnt == 1)
    assert len(res.flips) == 0 and res.global_trigger == 0
    assert res.excluded_past == 0 and res.excluded_now == 0


def test_reversal_swaps_breaking_and_arising():
    frames = _disk_frames(12)
    a, b = frames[0], frames[11]
    fa = oracle.frame(a, 0.5)
    fb = oracle.frame(b, 0.5)
    ab = oracle.compare(fa, fb)
    ba = oracle.compare(fb, fa)
    assert len(ab.flips) > 0

    def past_pairs(r, kind):
        return {(min(f[2], f[3]), max(f[2], f[3])) for f in r.flips if f[4] == kind}

    def now_pairs(r, kind):
        return {(f[0], f[1]) for f in r.flips if f[4] == kind}
    assert past_pairs(ab, -1) == now_pairs(ba, +1)
    assert past_pairs(ab, +1) == now_pairs(ba, -1)


def test_integer_roll_gives_no_flips():
    f = _disk_frames(1, seed=11)[0]
    seq = oracle.Sequence(0.5)
    seq.push(f)
    now, res = seq.push(np.roll(f, (1, 2), (0, 1)))
    assert len(res.flips) == 0
    assert res.excluded_past == 0 and res.excluded_now == 0


def test_deleted_droplet_is_excluded_with_its_match():
    d, fields, names = _t1_fields()
    lx, ly, r = d["lx"], d["ly"], d["radius"]
    pts = [d["quartet"]["0"][n] for n in names] + d["background"]
    keep = [p for i, p in enumerate(pts) if i != 7]
    f_all = synth.disk_field(lx, ly, np.array(pts, float), np.full(len(pts), float(r)))
    f_del = synth.disk_field(lx, ly, np.array(keep, float), np.full(len(keep), float(r)))
    seq = oracle.Sequence(0.5)
    seq.push(f_all)
    now, res = seq.push(f_del)
    # the vanished bubble and its nearest neighbour share one now label
    assert res.excluded_past == 2 and res.excluded_now == 1
    assert int(np.sum(res.cnt == 2)) == 1 and int(np.sum(res.cnt == 0)) == 0


def test_appearing_droplet_is_excluded():
    d, fields, names = _t1_fields()
    lx, ly, r = d["lx"], d["ly"], d["radius"]
    pts = [d["quartet"]["0"][n] for n in names] + d["background"]
    keep = [p for i, p in enumerate(pts) if i != 9]
    f_all = synth.disk_field(lx, ly, np.array(pts, float), np.full(len(pts), float(r)))
    f_del = synth.disk_field(lx, ly, np.array(keep, float), np.full(len(keep), float(r)))
    seq = oracle.Sequence(0.5)
    seq.push(f_del)
    now, res = seq.push(f_all)
    assert res.excluded_now == 1 and res.excluded_past == 0
    # no flip may touch the new bubble
    new = int(np.nonzero(res.cnt == 0)[0][0])
    assert all(new not in (f[0], f[1]) for f in res.flips)


@pytest.mark.parametrize("seed", range(4))
def test_local_trigger_marks_exactly_flip_endpoints(seed):
    frames = _disk_frames(6, seed=20 + seed)
    seq = oracle.Sequence(0.5)
    for f in frames:
        now, res = seq.push(f)
        ends = set()
        for fl in res.flips:
            ends.update((int(fl[2]), int(fl[3])))
        assert set(np.nonzero(res.local_trigger)[0].tolist()) == ends
        assert res.global_trigger == int(len(res.flips) > 0)
        # canonical order: breaking before arising, each by (a, b)
        kinds = res.flips[:, 4].tolist()
        assert kinds == sorted(kinds)
        for k in (-1, 1):
            sel = res.flips[res.flips[:, 4] == k]
            keys = sel[:, 0].astype(np.int64) * (1 << 32) + sel[:, 1]
            assert np.all(np.diff(keys) > 0)


def test_first_frame_and_empty_frames():
    seq = oracle.Sequence(0.5)
    now, res = seq.push(np.zeros((20, 20), np.float32))
    assert now.K == 0 and len(now.edges) == 0 and len(res.flips) == 0
    now, res = seq.push(_disk_frames(1, L=60, nd=6)[0][:20, :20].copy())
    assert res.excluded_now == now.K and len(res.flips) == 0
