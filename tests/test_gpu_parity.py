"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Labels, Q.8 centres, sizes, colour map, couples, matching and flips must be
bit-identical; float64 centres agree to 1e-6 relative (they are computed by the
same correctly rounded operations, so they are in fact identical).
Sizes span several tiles with ragged tails; the named workloads run at their
full sizes in the launch configuration the benchmark uses.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1607_00908_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1607_00908_amd import dv  # noqa: E402

NTHREADS = min(16, os.cpu_count() or 1)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check_frame(det, now, ref, lx, ly, maps=True):
    info = det.info()
    assert info.status == 0
    assert info.n_components == now.K
    if maps:
        assert np.array_equal(det.labels(), now.labels), "labels"
        assert np.array_equal(det.owner(), now.owner), "owner"
    comps = det.components()
    assert np.array_equal(comps["qx"], now.comps["qx"]), "qx"
    assert np.array_equal(comps["qy"], now.comps["qy"]), "qy"
    assert np.array_equal(comps["n"], now.comps["n"]), "sizes"
    assert np.allclose(comps["fx"], now.comps["fx"], rtol=1e-6, atol=0)
    assert np.allclose(comps["fy"], now.comps["fy"], rtol=1e-6, atol=0)
    assert info.n_ambiguous_centroids == int(now.comps["amb"].sum())
    e = det.edges()
    assert np.array_equal(e, now.edges), "couples"
    assert info.n_edges == len(now.edges)
    fl = det.flips()
    assert np.array_equal(fl, ref.flips), "flips"
    assert info.n_flips == len(ref.flips)
    assert info.n_breaking == int(np.sum(ref.flips[:, 4] == -1)) if len(ref.flips) else info.n_breaking == 0
    assert info.n_excluded_past == ref.excluded_past
    assert info.n_excluded_now == ref.excluded_now
    assert info.global_trigger == ref.global_trigger
    phi = det.matching()
    if len(ref.phi):
        want = ref.phi.copy()
        keep = (want >= 0)
        keep[keep] = ref.cnt[want[keep]] == 1
        want[~keep] = -1
        assert np.array_equal(phi, want), "matching"
    else:
        assert len(phi) == 0


def check_results(res, refs, tag=""):
    """Every frame's record and flips from Detector.results() (push order)
    against the oracle's (now, diff) of the same frame; a None entry in refs
    skips the oracle comparison of that frame, whose record must still say
    accepted.  Frames are numbered by the accepted frames up to them."""
    assert len(res) == len(refs), (tag, len(res), len(refs))
    for k, ((fi, fl), r) in enumerate(zip(res, refs)):
        assert fi.status == 0, (tag, k, fi)
        assert fi.frame == k + 1, (tag, k, fi.frame)
        assert len(fl) == fi.n_flips
        if r is None:
            continue
        now, ref = r
        assert fi.n_components == now.K, (tag, k)
        assert fi.n_edges == len(now.edges), (tag, k)
        assert fi.n_ambiguous_centroids == int(now.comps["amb"].sum()), (tag, k)
        assert np.array_equal(fl, ref.flips), (tag, k, "flips")
        assert fi.n_breaking == int(np.sum(ref.flips[:, 4] == -1)), (tag, k)
        assert fi.n_excluded_past == ref.excluded_past, (tag, k)
        assert fi.n_excluded_now == ref.excluded_now, (tag, k)
        assert fi.global_trigger == ref.global_trigger, (tag, k)


def run_sequence(fields, thr, phase=0, conn=8, kmax=None, maps=True, max_degree=0, tag="",
                 classify=False, open_x=False, open_y=False, obstacles=None, weighted=False,
                 max_batch=0):
    ly, lx = fields[0].shape
    if kmax is None:
        kmax = lx * ly
    det = dv.Detector(lx, ly, thr, phase, conn, max_components=kmax, max_degree=max_degree,
                      keep_maps=maps, classify=classify, open_x=open_x, open_y=open_y,
                      obstacles=obstacles, keep_results=True, weighted=weighted,
                      max_batch=max_batch)
    seq = oracle.Sequence(thr, phase, conn, NTHREADS, classify_events=classify,
                          obstacles=obstacles, open_x=open_x, open_y=open_y, weighted=weighted)
    refs = []
    for i, f in enumerate(fields):
        say(f"  [{tag}] frame {i} {lx}x{ly} conn={conn} phase={phase} open={int(open_x)}{int(open_y)}"
            f" obstacles={obstacles is not None} weighted={weighted}")
        det.push(torch.from_numpy(np.ascontiguousarray(f)).to("cuda"))
        now, ref = seq.push(f)
        refs.append((now, ref))
        check_frame(det, now, ref, lx, ly, maps)
    check_results(det.results(), refs, tag)
    det.close()
    return now


@pytest.mark.parametrize("seed", range(40))
def test_fuzz_small_lattices(seed):
    rng = np.random.default_rng(1000 + seed)
    lx, ly = int(rng.integers(3, 80)), int(rng.integers(3, 80))
    conn = int(rng.choice([4, 8]))
    phase = int(rng.integers(0, 2))
    p = float(rng.uniform(0.15, 0.6))
    thr = p if phase == 1 else 1.0 - p
    fields = [synth.tiny_random_field(lx, ly, 5000 + 7 * seed + k) for k in range(3)]
    run_sequence(fields, thr, phase, conn, tag=f"fuzz{seed}")


@pytest.mark.parametrize("seed", range(12))
def test_moving_disks_small(seed):
    rng = np.random.default_rng(2000 + seed)
    lx, ly = int(rng.integers(40, 200)), int(rng.integers(40, 200))
    nd = int(rng.integers(3, 40))
    sim = synth.DiskSim(lx, ly, nd, 3.0, 6.0, 0.7, 3e-3, seed=3000 + seed)
    run_sequence(list(sim.frames(5)), 0.5, tag=f"disks{seed}")


@pytest.mark.parametrize("lx,ly", [(3, 3), (3, 17), (64, 3), (32, 32), (33, 31), (65, 97), (31, 200)])
def test_shapes_and_ragged_tiles(lx, ly):
    fields = [synth.tiny_random_field(lx, ly, 17 * lx + ly + k) for k in range(3)]
    for conn in (4, 8):
        run_sequence(fields, 0.4, 1, conn, tag=f"shape{lx}x{ly}")


def test_empty_and_single_component():
    lx, ly = 70, 45
    empty = np.zeros((ly, lx), np.float32)
    one = np.zeros((ly, lx), np.float32)
    one[10:20, 30:40] = 1.0
    full = np.ones((ly, lx), np.float32)
    run_sequence([empty, one, empty, full, one], 0.5, tag="empty/one")


def test_wrapping_strip_and_checkerboard():
    lx, ly = 50, 40
    strip = np.zeros((ly, lx), np.float32)
    strip[7, :] = 1.0
    strip[20:23, 5:9] = 1.0
    yy, xx = np.mgrid[0:ly, 0:lx]
    cb = ((xx + yy) % 2).astype(np.float32)
    run_sequence([strip, cb, strip], 0.5, 0, 4, tag="strip/cb4")
    run_sequence([strip, cb, strip], 0.5, 0, 8, tag="strip/cb8")


def test_tiles_with_hundreds_of_pieces():
    """Tiles holding 253, 254, 255 and 256 pieces (isolated sites two apart),
    then a 4-connected checkerboard (512 pieces a tile, the most a tile can
    hold) below them: piece slots and ranks beyond one byte and beyond the
    first 64 slots of a tile."""
    lx, ly = 128, 64
    f = np.zeros((ly, lx), np.float32)
    for tile, n in enumerate((253, 254, 255, 256)):
        idx = np.arange(n)
        f[2 * (idx // 16), 32 * tile + 2 * (idx % 16)] = 1.0
    yy, xx = np.mgrid[0:32, 0:lx]
    cb = f.copy()
    cb[32:, :] = ((xx + yy) % 2).astype(np.float32)
    run_sequence([f, cb, f], 0.5, 0, 4, tag="slots4")
    run_sequence([f, cb, f], 0.5, 0, 8, tag="slots8")


def test_threshold_equality_and_nan_are_outside():
    rng = np.random.default_rng(9)
    f = rng.random((48, 40)).astype(np.float32)
    f[rng.random(f.shape) < 0.2] = np.float32(0.5)
    f[rng.random(f.shape) < 0.05] = np.nan
    run_sequence([f, f[::-1].copy()], 0.5, 0, 8, tag="nan")
    run_sequence([f, f[::-1].copy()], 0.5, 1, 8, tag="nan-below")


def test_t1_fixture_on_gpu():
    import json
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "t1_fixture.json")))
    names = ["A", "B", "C", "D"]
    fields = []
    for fr in ("0", "1"):
        pts = [d["quartet"][fr][n] for n in names] + d["background"]
        fields.append(synth.disk_field(d["lx"], d["ly"], np.array(pts, float),
                                       np.full(len(pts), float(d["radius"]))))
    run_sequence(fields, 0.5, tag="t1")
    det = dv.Detector(d["lx"], d["ly"], 0.5, max_components=128)
    for f in fields:
        det.push(torch.from_numpy(f).cuda())
    fl = det.flips()
    assert len(fl) == 2 and fl[0, 4] == -1 and fl[1, 4] == 1
    det.close()


def test_capacity_rejection_keeps_the_past():
    """K > K_max rejects the frame; the next frame is compared with the last
    accepted one."""
    sim = synth.DiskSim(120, 100, 12, 4.0, 6.0, 0.8, 2e-3, seed=77)
    a, b, c = list(sim.frames(3))
    # 15% of sites inside, below site percolation: hundreds of components
    noise = (synth.tiny_random_field(120, 100, 4) > 0.85).astype(np.float32)
    det = dv.Detector(120, 100, 0.5, max_components=64)
    det.push(torch.from_numpy(a).cuda())
    assert det.info().status == 0
    det.push(torch.from_numpy(noise).cuda())
    with pytest.raises(dv.DVError) as e:
        det.flips()
    assert e.value.status == dv.ERR_CAPACITY
    assert det.info().status == dv.ERR_CAPACITY
    det.push(torch.from_numpy(c).cuda())
    got = det.flips()
    fa, fc = oracle.frame(a, 0.5), oracle.frame(c, 0.5)
    ref = oracle.compare(fa, fc)
    assert np.array_equal(got, ref.flips)
    assert det.info().frame == 2
    # the rejected frame leaves no trace in the next frame's sums
    check_frame(det, fc, ref, 120, 100)
    det.close()


@pytest.mark.parametrize("depth", [1, 2, 3, 4, 8, 16, 32, 64])
def test_batched_bursts_match_the_oracle(depth):
    """Frames pushed back to back with no synchronisation in between go to the
    device in batches (each stage one launch over the batch, the comparisons
    of a batch in parallel); the state after each burst (flips against the
    previous frame, labels, couples, matching) must equal the oracle's."""
    lx, ly = 200, 160
    sim = synth.DiskSim(lx, ly, 30, 4.0, 7.0, 0.6, 3e-3, seed=91 + depth)
    # bursts: a full batch (frames 1 .. depth), then a full and a partial one
    n = max(11, 2 * depth + 3)
    frames = list(sim.frames(n))
    dev = [torch.from_numpy(f).cuda() for f in frames]
    det = dv.Detector(lx, ly, 0.5, max_components=256, max_batch=depth, keep_results=True)
    seq = oracle.Sequence(0.5, 0, 8, NTHREADS)
    refs = []
    for k, f in enumerate(frames):
        now, ref = seq.push(f)
        refs.append((now, ref))
        det.push(dev[k])
        if k in (0, depth, n - 1):
            say(f"  [batch{depth}] burst ends at frame {k}")
            check_frame(det, now, ref, lx, ly)
    assert det.info().frame == len(frames)
    # every frame's flips, also those inside a batch
    check_results(det.results(), refs, f"batch{depth}")
    det.close()


@pytest.mark.parametrize("depth,collect_every", [(4, 3), (8, 5), (32, 7), (2, 1)])
def test_results_collected_while_pushing(depth, collect_every):
    """Results read with and without waiting while frames are still being
    pushed (pages of unread frames reused, frames moved to host memory first):
    together, every frame exactly once, in push order, equal to the oracle."""
    lx, ly = 130, 110
    sim = synth.DiskSim(lx, ly, 20, 4.0, 7.0, 0.6, 3e-3, seed=191 + depth)
    n = 3 * depth + 5
    frames = list(sim.frames(n))
    dev = [torch.from_numpy(f).cuda() for f in frames]
    det = dv.Detector(lx, ly, 0.5, max_components=256, max_batch=depth, keep_results=True)
    seq = oracle.Sequence(0.5, 0, 8, NTHREADS)
    refs = [seq.push(f) for f in frames]
    got = []
    for k in range(n):
        det.push(dev[k])
        if k % collect_every == collect_every - 1:
            got += det.results(wait=(k // collect_every) % 2 == 1)
    got += det.results(wait=True)
    assert det.results(wait=True) == []
    check_results(got, refs, f"collect{depth}/{collect_every}")
    det.close()


def test_results_capacity_returns_whole_frames():
    """Small result buffers: whole frames while they fit, the rest stays
    unread for the next call."""
    import ctypes
    lx, ly = 120, 120
    sim = synth.DiskSim(lx, ly, 24, 4.0, 7.0, 0.8, 4e-3, seed=5)
    frames = list(sim.frames(9))
    det = dv.Detector(lx, ly, 0.5, max_components=256, max_batch=4, keep_results=True)
    for f in frames:
        det.push(torch.from_numpy(f).cuda())
    seq = oracle.Sequence(0.5, 0, 8, NTHREADS)
    refs = [seq.push(f) for f in frames]
    nf, nfl = ctypes.c_int32(0), ctypes.c_int32(0)
    assert det.lib.dv_results_ready(det.h, 1, ctypes.byref(nf), ctypes.byref(nfl)) == dv.OK
    assert nf.value == 9 and nfl.value == sum(len(r.flips) for _, r in refs)
    infos = (dv.DVFrameInfo * 2)()
    fl = np.zeros((max(nfl.value, 1), 6), np.int32)
    gf, gfl = ctypes.c_int32(0), ctypes.c_int32(0)
    st = det.lib.dv_get_results(det.h, 0, infos, 2, ctypes.byref(gf), fl.ctypes.data_as(ctypes.c_void_p),
                                nfl.value, ctypes.byref(gfl))
    assert st == dv.ERR_CAPACITY and gf.value == 2
    assert gfl.value == len(refs[0][1].flips) + len(refs[1][1].flips)
    first = [(dv._frame_info(infos[k]), None) for k in range(2)]
    # a caller-owned pinned buffer that holds the flips of frames 2 and 3
    sizes = [len(r.flips) for _, r in refs]
    cap = sizes[2] + sizes[3]
    fits, acc = 0, 0
    for n in sizes[2:]:
        if acc + n > cap:
            break
        acc += n
        fits += 1
    out = torch.full((cap, 6), -7, dtype=torch.int32, pin_memory=True).numpy()
    mid = det.results(wait=False, out=out)
    assert len(mid) == fits >= 2
    rest = mid + det.results(wait=False)
    assert len(rest) == 7
    assert [fi.frame for fi, _ in first + rest] == list(range(1, 10))
    for (fi, f), (now, ref) in zip(rest, refs[2:]):
        assert fi.n_components == now.K
        assert np.array_equal(f, ref.flips)
    for _, f in mid:
        assert f.size == 0 or np.shares_memory(f, out)
    with pytest.raises(ValueError):
        det.results(out=np.zeros((4, 5), np.int32))
    det.close()


def test_rejection_inside_a_batch():
    """A rejected frame in the middle of a batch: the frame after it is compared
    with the last accepted one, inside the same batch and across batches."""
    sim = synth.DiskSim(120, 100, 12, 4.0, 6.0, 0.8, 2e-3, seed=78)
    a, b, c, d = list(sim.frames(4))
    noise = (synth.tiny_random_field(120, 100, 5) > 0.85).astype(np.float32)
    dev = [torch.from_numpy(x).cuda() for x in (a, b, noise, c)]
    det = dv.Detector(120, 100, 0.5, max_components=64, max_batch=3, keep_results=True)
    for x in dev:
        det.push(x)
    got = det.flips()
    ref = oracle.compare(oracle.frame(b, 0.5), oracle.frame(c, 0.5))
    assert np.array_equal(got, ref.flips)
    assert det.info().frame == 3
    det.push(torch.from_numpy(d).cuda())
    det.push(dev[2])
    with pytest.raises(dv.DVError):
        det.flips()
    det.push(dev[1])
    ref = oracle.compare(oracle.frame(d, 0.5), oracle.frame(b, 0.5))
    assert np.array_equal(det.flips(), ref.flips)
    # every frame's record: the rejections are reported where they happened
    res = det.results()
    assert [fi.status for fi, _ in res] == [0, 0, dv.ERR_CAPACITY, 0, 0, dv.ERR_CAPACITY, 0]
    assert [fi.frame for fi, _ in res] == [1, 2, 2, 3, 4, 4, 5]
    fa, fb, fc, fd = (oracle.frame(x, 0.5) for x in (a, b, c, d))
    want = [oracle.compare(None, fa), oracle.compare(fa, fb), None, oracle.compare(fb, fc),
            oracle.compare(fc, fd), None, oracle.compare(fd, fb)]
    for k, ((fi, fl), w) in enumerate(zip(res, want)):
        if w is None:
            assert len(fl) == 0 and fi.n_flips == 0
        else:
            assert np.array_equal(fl, w.flips), k
    det.close()


def _group(sizes, kmax=512, max_batch=2):
    stream = torch.cuda.Stream()
    dets = [dv.Detector(lx, ly, 0.5, max_components=kmax, max_batch=max_batch, stream=stream,
                        keep_results=True) for lx, ly in sizes]
    return dets, dv.Group(dets)


def test_group_of_uneven_lattices_matches_the_oracle():
    """Five sequences of different lattice sizes go through one launch per
    stage; every member's frame equals the oracle's."""
    sizes = [(64, 64), (100, 70), (200, 160), (33, 97), (256, 256)]
    sims = [synth.DiskSim(lx, ly, max(3, lx * ly // 2500), 3.0, 6.0, 0.6, 3e-3, seed=700 + i)
            for i, (lx, ly) in enumerate(sizes)]
    frames = [list(sm.frames(4)) for sm in sims]
    dets, grp = _group(sizes)
    seqs = [oracle.Sequence(0.5, 0, 8, NTHREADS) for _ in sizes]
    refs = [[] for _ in sizes]
    for k in range(4):
        say(f"  [group] frame {k}")
        grp.push([torch.from_numpy(frames[i][k]).cuda() for i in range(len(sizes))])
        for i, (lx, ly) in enumerate(sizes):
            now, ref = seqs[i].push(frames[i][k])
            refs[i].append((now, ref))
            check_frame(dets[i], now, ref, lx, ly)
    for i in range(len(sizes)):
        check_results(dets[i].results(), refs[i], f"group member {i}")
    grp.close()
    for d in dets:
        d.close()


def test_group_of_mixed_fields_matches_the_oracle():
    """The batching workload's generator at small sides: disk and random-field
    sequences with their own thresholds in one group, three frames."""
    fields = synth.mixed_fields(6, seed=5, l_min=64, l_max=200)
    stream = torch.cuda.Stream()
    dets = [dv.Detector(sp["lx"], sp["ly"], sp["threshold"], sp["phase"], 8,
                        max_components=4 * sp["k_expect"] + 256, max_batch=1, stream=stream)
            for _, sp in fields]
    grp = dv.Group(dets)
    frames = [list(sm.frames(3)) for sm, _ in fields]
    seqs = [oracle.Sequence(sp["threshold"], sp["phase"], 8, NTHREADS) for _, sp in fields]
    for k in range(3):
        say(f"  [mixed group] frame {k}")
        grp.push([torch.from_numpy(frames[i][k]).cuda() for i in range(len(fields))])
        for i, (_, sp) in enumerate(fields):
            now, ref = seqs[i].push(frames[i][k])
            check_frame(dets[i], now, ref, sp["lx"], sp["ly"])
    grp.close()
    for d in dets:
        d.close()


def test_group_bursts_and_single_pushes_mix():
    """Group pushes without synchronisation, interleaved with pushes of single
    members; each member's last comparison equals the oracle's."""
    sizes = [(96, 80), (130, 150), (64, 200)]
    sims = [synth.DiskSim(lx, ly, 10, 3.0, 6.0, 0.6, 3e-3, seed=800 + i)
            for i, (lx, ly) in enumerate(sizes)]
    frames = [list(sm.frames(6)) for sm in sims]
    dev = [[torch.from_numpy(f).cuda() for f in fr] for fr in frames]
    dets, grp = _group(sizes, max_batch=3)
    for k in range(3):
        grp.push([dev[i][k] for i in range(3)])
    dets[1].push(dev[1][3])                 # member 1 alone
    for k in (4, 5):
        grp.push([dev[0][k], dev[1][k], dev[2][k]])
    for i, (lx, ly) in enumerate(sizes):
        order = [0, 1, 2, 3, 4, 5] if i == 1 else [0, 1, 2, 4, 5]
        seq = oracle.Sequence(0.5, 0, 8, NTHREADS)
        refs = [seq.push(frames[i][k]) for k in order]
        now, ref = refs[-1]
        check_frame(dets[i], now, ref, lx, ly)
        assert dets[i].info().frame == len(order)
        # every frame of every member, group pushes and single pushes alike
        check_results(dets[i].results(), refs, f"mix member {i}")
    grp.close()
    for d in dets:
        d.close()


def test_group_subsets_as_frames_arrive():
    """Continuous batching: each push carries the members that have a new
    frame, in any order; every member's results equal the oracle's for its own
    sequence, whatever it was batched with."""
    sizes = [(80, 64), (128, 96), (64, 128), (150, 150)]
    sims = [synth.DiskSim(lx, ly, 8, 3.0, 6.0, 0.6, 3e-3, seed=1100 + i)
            for i, (lx, ly) in enumerate(sizes)]
    frames = [list(sm.frames(5)) for sm in sims]
    dets, grp = _group(sizes, max_batch=1)
    seqs = [oracle.Sequence(0.5, 0, 8, NTHREADS) for _ in sizes]
    refs = [[] for _ in sizes]
    nxt = [0] * len(sizes)
    schedule = [[0, 1, 2, 3], [2, 0], [3], [1, 3, 0], [0], [2, 1], [3, 2, 1], [1, 0]]
    for step, members in enumerate(schedule):
        members = [m for m in members if nxt[m] < 5]
        say(f"  [subsets] step {step} members {members}")
        grp.push_some(members, [torch.from_numpy(frames[m][nxt[m]]).cuda() for m in members])
        for m in members:
            now, ref = seqs[m].push(frames[m][nxt[m]])
            refs[m].append((now, ref))
            nxt[m] += 1
            check_frame(dets[m], now, ref, *sizes[m])
    for m in range(len(sizes)):
        check_results(dets[m].results(), refs[m], f"subset member {m}")
    grp.close()
    for d in dets:
        d.close()


def test_group_member_rejection_is_isolated():
    """A frame over one member's K_max is rejected for that member only."""
    sizes = [(120, 100), (120, 100), (90, 110)]
    sims = [synth.DiskSim(lx, ly, 12, 4.0, 6.0, 0.8, 2e-3, seed=900 + i)
            for i, (lx, ly) in enumerate(sizes)]
    frames = [list(sm.frames(3)) for sm in sims]
    noise = (synth.tiny_random_field(120, 100, 6) > 0.85).astype(np.float32)
    dets, grp = _group(sizes, kmax=64)
    grp.push([torch.from_numpy(frames[i][0]).cuda() for i in range(3)])
    grp.push([torch.from_numpy(frames[0][1]).cuda(), torch.from_numpy(noise).cuda(),
              torch.from_numpy(frames[2][1]).cuda()])
    assert dets[0].info().status == 0 and dets[2].info().status == 0
    assert dets[1].info().status == dv.ERR_CAPACITY
    grp.push([torch.from_numpy(frames[i][2]).cuda() for i in range(3)])
    for i in range(3):
        past = frames[i][0] if i == 1 else frames[i][1]
        ref = oracle.compare(oracle.frame(past, 0.5), oracle.frame(frames[i][2], 0.5))
        assert np.array_equal(dets[i].flips(), ref.flips), i
    assert dets[1].info().frame == 2 and dets[0].info().frame == 3
    grp.close()
    for d in dets:
        d.close()


def test_event_flags_t1_fixture():
    import json
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "t1_fixture.json")))
    names = ["A", "B", "C", "D"]
    fields = []
    for fr in ("0", "1"):
        pts = [d["quartet"][fr][n] for n in names] + d["background"]
        fields.append(synth.disk_field(d["lx"], d["ly"], np.array(pts, float),
                                       np.full(len(pts), float(d["radius"]))))
    run_sequence(fields, 0.5, tag="t1-events", classify=True)
    det = dv.Detector(d["lx"], d["ly"], 0.5, max_components=128, classify=True)
    for f in fields:
        det.push(torch.from_numpy(f).cuda())
    fl = det.flips()
    assert fl[:, 5].tolist() == [dv.FLIP_BULK, dv.FLIP_BULK]
    det.close()


@pytest.mark.parametrize("seed", range(6))
def test_event_flags_moving_disks(seed):
    rng = np.random.default_rng(4000 + seed)
    lx, ly = int(rng.integers(60, 220)), int(rng.integers(60, 220))
    sim = synth.DiskSim(lx, ly, int(rng.integers(8, 60)), 3.0, 6.0, 0.9, 4e-3, seed=5000 + seed)
    run_sequence(list(sim.frames(6)), 0.5, tag=f"events{seed}", classify=True)


def test_event_flags_random_field_with_exclusions():
    sim = synth.GRFSim(256, 256, 4.0, 0.9, seed=41)
    run_sequence(list(sim.frames(5)), 1.0, kmax=4096, tag="events-grf", classify=True)


def test_event_flags_disks1024_batched():
    sim, spec = synth.workload("disks1024")
    frames = list(sim.frames(9))
    dev = torch.from_numpy(np.stack(frames)).cuda()
    det = dv.Detector(1024, 1024, spec["threshold"], spec["phase"], 8, max_components=4096,
                      classify=True, keep_results=True)
    for k in range(len(frames)):
        det.push(dev[k])
    seq = oracle.Sequence(spec["threshold"], spec["phase"], 8, NTHREADS, classify_events=True)
    refs = [seq.push(f) for f in frames]
    now, ref = refs[-1]
    check_frame(det, now, ref, 1024, 1024)
    check_results(det.results(), refs, "events-disks1024")
    det.close()


def test_degree_overflow_is_reported():
    sim = synth.DiskSim(128, 128, 30, 3.0, 5.0, 0.5, 1e-3, seed=8)
    f = next(sim.frames(1))
    det = dv.Detector(128, 128, 0.5, max_components=64, max_degree=4)
    det.push(torch.from_numpy(f).cuda())
    assert det.info().status == dv.ERR_CAPACITY
    det.close()


def test_flip_buffer_too_small_reports_count():
    import ctypes
    sim = synth.DiskSim(160, 160, 40, 5.0, 8.0, 0.6, 2e-3, seed=7)
    frames = list(sim.frames(12))
    det = dv.Detector(160, 160, 0.5, max_components=128)
    det.push(torch.from_numpy(frames[0]).cuda())
    det.push(torch.from_numpy(frames[11]).cuda())
    n = ctypes.c_int32(-1)
    st = det.lib.dv_get_flips(det.h, None, 0, ctypes.byref(n))
    ref = oracle.compare(oracle.frame(frames[0], 0.5), oracle.frame(frames[11], 0.5))
    assert len(ref.flips) > 0
    assert st == dv.ERR_CAPACITY and n.value == len(ref.flips)
    assert np.array_equal(det.flips(), ref.flips)
    det.close()


def test_disks256_all_frames():
    sim, spec = synth.workload("disks256")
    run_sequence(list(sim.frames(spec["frames"])), spec["threshold"], kmax=1024, tag="disks256")


def test_disks1024_frames():
    sim, spec = synth.workload("disks1024")
    run_sequence(list(sim.frames(6)), spec["threshold"], kmax=4096, tag="disks1024")


def test_disks1024_batched_burst():
    """Twenty full-size frames pushed back to back in the benchmark's launch
    configuration (default batch); the last comparison against the oracle."""
    sim, spec = synth.workload("disks1024")
    frames = list(sim.frames(40))
    dev = torch.from_numpy(np.stack(frames)).cuda()
    det = dv.Detector(1024, 1024, spec["threshold"], spec["phase"], 8, max_components=4096,
                      keep_results=True)
    for k in range(len(frames)):
        det.push(dev[k])
    seq = oracle.Sequence(spec["threshold"], spec["phase"], 8, NTHREADS)
    refs = []
    for k, f in enumerate(frames):
        if k % 10 == 0:
            say(f"  [disks1024 burst] oracle frame {k}")
        refs.append(seq.push(f))
    now, ref = refs[-1]
    check_frame(det, now, ref, 1024, 1024)
    assert det.info().frame == len(frames)
    # every frame: a full batch of 32 and a partial one of 8
    check_results(det.results(), refs, "disks1024 burst")
    det.close()


def test_grf1024_frames():
    """The random-field workload's statistics at 1024^2 (same smoothing,
    threshold and AR(1) step): many components appear, vanish and wrap."""
    sim = synth.GRFSim(1024, 1024, 6.0, 0.98, seed=33)
    run_sequence(list(sim.frames(4)), 1.0, kmax=8192, tag="grf1024")


@pytest.mark.timeout(600)
def test_grf4096_full_size():
    """Full-size random-field frames (16.8 M sites, ~9k components), frames
    0-4 (four comparisons): labels, centres, colour map, couples and flips
    against the oracle."""
    sim, spec = synth.workload("grf4096")
    fields = list(sim.frames(5))
    run_sequence(fields, spec["threshold"], kmax=32768, tag="grf4096")


@pytest.mark.timeout(600)
def test_grf4096_batched_burst():
    """The benchmark's launch shape at 4096^2: 34 frames pushed back to back
    with the default batch of 32 (a full launch and a partial one).  Every
    frame's record and flips equal those of the same frames pushed one per
    launch; frames 30-33 (four comparisons, across the batch boundary) equal
    the oracle's."""
    sim, spec = synth.workload("grf4096")
    frames = list(sim.frames(34))
    say("  [grf4096 burst] frames generated")
    dev = torch.from_numpy(np.stack(frames)).cuda()
    det = dv.Detector(4096, 4096, spec["threshold"], spec["phase"], 8, max_components=32768,
                      keep_results=True, keep_maps=False)
    for k in range(len(frames)):
        det.push(dev[k])
    batched = det.results()
    assert len(batched) == 34
    det.close()
    det1 = dv.Detector(4096, 4096, spec["threshold"], spec["phase"], 8, max_components=32768,
                       keep_results=True, keep_maps=False, max_batch=1)
    for k in range(len(frames)):
        det1.push(dev[k])
    alone = det1.results()
    det1.close()
    say("  [grf4096 burst] GPU runs done")
    for k, ((fa, la), (fb, lb)) in enumerate(zip(batched, alone)):
        assert fa == fb, k
        assert np.array_equal(la, lb), k
    seq = oracle.Sequence(spec["threshold"], spec["phase"], 8, NTHREADS)
    refs = [None] * 34
    seq.push(frames[29])
    for k in range(30, 34):
        say(f"  [grf4096 burst] oracle frame {k}")
        refs[k] = seq.push(frames[k])
    check_results(batched, refs, "grf4096 burst")
    assert sum(1 for fi, _ in batched if fi.n_flips > 0) > 20


def test_sparse_cluster_exercises_candidate_overflow():
    """1600 one-site components packed in one corner of an empty lattice:
    far tiles must consider every centre, more than one LDS chunk holds."""
    L = 512
    f = np.zeros((L, L), np.float32)
    f[10:90:2, 20:100:2] = 1.0
    g = f.copy()
    g[10:90:2, 20:100:2] = 0.0
    g[11:91:2, 21:101:2] = 1.0          # the whole cluster moves by (1, 1)
    run_sequence([f, g], 0.5, kmax=2048, tag="cluster")


def test_few_far_centres_mix_integer_and_float_colouring():
    """Five small droplets on a 768^2 lattice: tiles near a droplet have their
    candidates within the 32-bit range, distant tiles do not and take the
    float64 form; both must give the oracle's colours, couples and flips."""
    L = 768
    rng = np.random.default_rng(21)
    frames = []
    c = rng.uniform(0, L, (5, 2))
    for k in range(3):
        f = np.zeros((L, L), np.float32)
        for x, y in c + k * np.array([1.3, -0.7]):
            yy, xx = np.ogrid[0:L, 0:L]
            dx = (xx - x + L / 2) % L - L / 2
            dy = (yy - y + L / 2) % L - L / 2
            f[(dx * dx + dy * dy) < 36.0] = 1.0
        frames.append(f)
    run_sequence(frames, 0.5, kmax=64, tag="far5")


def test_serving_results_equal_alone_and_in_the_mix():
    """Frames of six streams arriving in a random order are served in mixed
    batches with two steps in flight; every served frame's record and flips
    equal the oracle's for its own stream and those of the same stream run
    alone, frame by frame."""
    from paper_1607_00908_amd import serve
    rng = np.random.default_rng(12)
    fields = synth.mixed_fields(6, seed=6, l_min=48, l_max=160)
    nf = 5
    frames = [list(sm.frames(nf)) for sm, _ in fields]
    srv = serve.Server(reserve_bytes=0)
    sids = [srv.open(sp["lx"], sp["ly"], sp["threshold"], sp["phase"],
                     max_components=4 * sp["k_expect"] + 256) for _, sp in fields]
    assert all(srv.admitted(s) for s in sids)
    # arrivals: a random interleaving of the streams' frames, in per-stream order
    order = [i for i in range(len(fields)) for _ in range(nf)]
    rng.shuffle(order)
    nxt = [0] * len(fields)
    mixed = {}
    for step_i, i in enumerate(order):
        srv.submit(sids[i], torch.from_numpy(frames[i][nxt[i]]).cuda(), tag=(i, nxt[i]))
        nxt[i] += 1
        if rng.random() < 0.5:
            for sid, tag, ta, td, info, fl in srv.step():
                mixed[tag] = (info, fl)
    for sid, tag, ta, td, info, fl in srv.drain():
        mixed[tag] = (info, fl)
    srv.shutdown()
    assert len(mixed) == len(order)
    for i, (_, sp) in enumerate(fields):
        seq = oracle.Sequence(sp["threshold"], sp["phase"], 8, NTHREADS)
        refs = [seq.push(f) for f in frames[i]]
        check_results([mixed[(i, k)] for k in range(nf)], refs, f"served stream {i}")
        det = dv.Detector(sp["lx"], sp["ly"], sp["threshold"], sp["phase"], 8,
                          max_components=4 * sp["k_expect"] + 256, max_batch=1, keep_results=True)
        for k in range(nf):
            det.push(torch.from_numpy(frames[i][k]).cuda())
        alone = det.results()
        det.close()
        for k in range(nf):
            assert alone[k][0] == mixed[(i, k)][0], (i, k)
            assert np.array_equal(alone[k][1], mixed[(i, k)][1]), (i, k)


def test_serving_admission_and_retirement():
    """A byte budget admits two streams at a time: the third waits (its frames
    queue) until a stream closes and retires, then it is admitted and served.
    Every frame of every stream equals the oracle's."""
    from paper_1607_00908_amd import serve
    fields = synth.mixed_fields(3, seed=9, l_min=64, l_max=128)
    nf = 4
    frames = [list(sm.frames(nf)) for sm, _ in fields]
    need = [serve.context_bytes(sp["lx"], sp["ly"], 4 * sp["k_expect"] + 256) for _, sp in fields]
    srv = serve.Server(reserve_bytes=0, budget_bytes=max(need[0] + need[1], need[0] + need[2],
                                                         need[1] + need[2]) + 1)
    sids = [srv.open(sp["lx"], sp["ly"], sp["threshold"], sp["phase"],
                     max_components=4 * sp["k_expect"] + 256) for _, sp in fields]
    assert srv.admitted(sids[0]) and srv.admitted(sids[1]) and not srv.admitted(sids[2])
    got = {i: [] for i in range(3)}
    for k in range(nf):
        for i in range(3):
            srv.submit(sids[i], torch.from_numpy(frames[i][k]).cuda(), tag=(i, k))
    for sid, tag, ta, td, info, fl in srv.drain():
        got[tag[0]].append((info, fl))
    # stream 2 is still waiting for memory: none of its frames was served
    assert len(got[0]) == nf and len(got[1]) == nf and got[2] == []
    assert srv.pending() == nf
    srv.close(sids[0])
    assert sids[0] not in srv.streams and srv.admitted(sids[2])
    for sid, tag, ta, td, info, fl in srv.drain():
        got[tag[0]].append((info, fl))
    srv.shutdown()
    for i, (_, sp) in enumerate(fields):
        seq = oracle.Sequence(sp["threshold"], sp["phase"], 8, NTHREADS)
        check_results(got[i], [seq.push(f) for f in frames[i]], f"admission stream {i}")


def test_batch_autotuner_times_every_candidate():
    """The autotuner times each candidate batch on device frames (every
    frame's results read back) and picks one of them."""
    from paper_1607_00908_amd import tune
    sim = synth.DiskSim(256, 256, 40, 4.0, 7.0, 0.4, 2e-3, seed=44)
    fields = [torch.from_numpy(f).cuda() for f in sim.frames(6)]
    t = tune.tune_batch(lambda b: dv.Detector(256, 256, 0.5, max_components=512, max_batch=b,
                                              keep_results=True),
                        fields, candidates=(1, 4, 16), frames=16, warmup=4)
    assert sorted(t) == [1, 4, 16] and all(v > 0 for v in t.values())
    assert tune.choose(t) in (1, 4, 16)


# ------------------------------------------------------------ walls and obstacles
@pytest.mark.parametrize("seed", range(24))
def test_walls_and_obstacles_fuzz_small_lattices(seed):
    rng = np.random.default_rng(7000 + seed)
    lx, ly = int(rng.integers(3, 90)), int(rng.integers(3, 90))
    conn = int(rng.choice([4, 8]))
    phase = int(rng.integers(0, 2))
    ox, oy = [(True, False), (False, True), (True, True), (False, False)][seed % 4]
    obst = rng.random((ly, lx)) < rng.uniform(0.0, 0.2) if seed % 3 else None
    p = float(rng.uniform(0.15, 0.6))
    thr = p if phase == 1 else 1.0 - p
    fields = [synth.tiny_random_field(lx, ly, 8000 + 7 * seed + k) for k in range(3)]
    run_sequence(fields, thr, phase, conn, tag=f"walls{seed}", open_x=ox, open_y=oy,
                 obstacles=obst)


@pytest.mark.parametrize("lx,ly", [(3, 3), (3, 17), (64, 3), (32, 32), (33, 31), (65, 97), (31, 200)])
def test_walled_shapes_and_ragged_tiles(lx, ly):
    fields = [synth.tiny_random_field(lx, ly, 31 * lx + ly + k) for k in range(3)]
    for ox, oy in ((True, False), (False, True), (True, True)):
        run_sequence(fields, 0.4, 1, 8, tag=f"wshape{lx}x{ly}", open_x=ox, open_y=oy)


def test_walls_empty_full_and_edge_components():
    """Components touching the walls, one covering everything, none; the same
    fields on the torus join across the seams instead."""
    lx, ly = 70, 45
    edge = np.zeros((ly, lx), np.float32)
    edge[10:20, 0:4] = 1.0
    edge[12:18, lx - 3:lx] = 1.0
    edge[0:3, 30:40] = 1.0
    edge[ly - 2:ly, 33:37] = 1.0
    full = np.ones((ly, lx), np.float32)
    empty = np.zeros((ly, lx), np.float32)
    for ox, oy in ((True, False), (False, True), (True, True)):
        run_sequence([edge, full, empty, edge], 0.5, tag="walls-edge", open_x=ox, open_y=oy)


@pytest.mark.parametrize("seed", range(6))
def test_channel_with_posts_small(seed):
    """The paper's channel in small: walls across x, posts on the left wall,
    drifting droplets; event flags on."""
    sim = synth.ChannelSim(192, 256, 60, 7.0, 9.0, 24, 32, 64, 1.5, 0.4, seed=60 + seed)
    run_sequence(list(sim.frames(5)), 0.5, kmax=256, tag=f"channel{seed}", classify=True,
                 open_x=True, obstacles=sim.obstacles())


def test_channel2048_batched_burst():
    """Full-size channel frames (2048 x 1024, 2000 droplets, posts) pushed back
    to back in batches of 32 (the default); the first two and the last comparisons against
    the oracle."""
    sim, spec = synth.workload("channel2048")
    obst = sim.obstacles()
    frames = list(sim.frames(18))
    dev = torch.from_numpy(np.stack(frames)).cuda()
    det = dv.Detector(2048, 1024, spec["threshold"], spec["phase"], 8, max_components=8192,
                      open_x=True, obstacles=obst, classify=True, keep_results=True)
    seq = oracle.Sequence(spec["threshold"], spec["phase"], 8, NTHREADS, classify_events=True,
                          obstacles=obst, open_x=True)
    refs = []
    for k in range(2):
        say(f"  [channel2048] frame {k}")
        det.push(dev[k])
        now, ref = seq.push(frames[k])
        refs.append((now, ref))
        check_frame(det, now, ref, 2048, 1024)
    for k in range(2, len(frames)):
        det.push(dev[k])
    say("  [channel2048] burst done")
    for k in range(2, len(frames)):
        refs.append(seq.push(frames[k]))
    now, ref = refs[-1]
    check_frame(det, now, ref, 2048, 1024)
    assert det.info().frame == len(frames)
    check_results(det.results(), refs, "channel2048 burst")
    det.close()


def test_obstacle_mask_replaced_between_pushes():
    """Frames queued before set_obstacles keep the old mask, later ones the
    new one (also when the mask comes from device memory)."""
    lx, ly = 96, 80
    sim = synth.DiskSim(lx, ly, 20, 4.0, 7.0, 0.6, 2e-3, seed=91)
    fr = list(sim.frames(6))
    rng = np.random.default_rng(3)
    m1 = rng.random((ly, lx)) < 0.05
    m2 = np.zeros((ly, lx), bool)
    m2[30:50, 10:70] = True
    masks = [m1, m1, m2, m2, None, None]
    det = dv.Detector(lx, ly, 0.5, max_components=512, with_obstacles=True, max_batch=4)
    det.set_obstacles(m1)
    det.push(torch.from_numpy(fr[0]).cuda())
    det.push(torch.from_numpy(fr[1]).cuda())
    det.set_obstacles(torch.from_numpy(m2.astype(np.uint8)).cuda())
    det.push(torch.from_numpy(fr[2]).cuda())
    det.push(torch.from_numpy(fr[3]).cuda())
    det.set_obstacles(None)
    det.push(torch.from_numpy(fr[4]).cuda())
    det.push(torch.from_numpy(fr[5]).cuda())
    past = oracle.frame(fr[4], 0.5, obstacles=masks[4])
    now = oracle.frame(fr[5], 0.5, obstacles=masks[5])
    check_frame(det, now, oracle.compare(past, now), lx, ly)
    assert det.info().frame == 6
    # the same frames with a mask per frame, compared one at a time
    det2 = dv.Detector(lx, ly, 0.5, max_components=512, with_obstacles=True, max_batch=1)
    past = None
    for k in range(6):
        det2.set_obstacles(masks[k])
        det2.push(torch.from_numpy(fr[k]).cuda())
        now = oracle.frame(fr[k], 0.5, obstacles=masks[k])
        check_frame(det2, now, oracle.compare(past, now), lx, ly)
        past = now
    det.close()
    det2.close()


def test_group_of_mixed_geometries():
    """Periodic, walled and obstructed members in one launch per stage."""
    stream = torch.cuda.Stream()
    specs = [(96, 64, False, False, False), (80, 120, True, False, True),
             (128, 96, False, True, False), (70, 70, True, True, True)]
    sims, dets, seqs = [], [], []
    for i, (lx, ly, ox, oy, ob) in enumerate(specs):
        sim = synth.DiskSim(lx, ly, max(4, lx * ly // 400), 3.0, 6.0, 0.6, 3e-3, seed=820 + i)
        mask = (np.random.default_rng(i).random((ly, lx)) < 0.04) if ob else None
        sims.append(list(sim.frames(4)))
        dets.append(dv.Detector(lx, ly, 0.5, max_components=512, max_batch=2, stream=stream,
                                open_x=ox, open_y=oy, obstacles=mask, classify=True))
        seqs.append(oracle.Sequence(0.5, 0, 8, NTHREADS, classify_events=True, obstacles=mask,
                                    open_x=ox, open_y=oy))
    grp = dv.Group(dets)
    for k in range(4):
        say(f"  [group-geometry] frame {k}")
        grp.push([torch.from_numpy(sims[i][k]).cuda() for i in range(len(specs))])
        for i, (lx, ly, _, _, _) in enumerate(specs):
            now, ref = seqs[i].push(sims[i][k])
            check_frame(dets[i], now, ref, lx, ly)
    grp.close()
    for d in dets:
        d.close()


def test_walled_sparse_cluster_exercises_candidate_overflow():
    """The grid search behind a candidate-list overflow, with walls and an
    obstacle band between the cluster and the far tiles."""
    L = 384
    f = np.zeros((L, L), np.float32)
    f[10:90:2, 20:100:2] = 1.0
    g = f.copy()
    g[10:90:2, 20:100:2] = 0.0
    g[11:91:2, 21:101:2] = 1.0
    obst = np.zeros((L, L), bool)
    obst[150:160, :300] = True
    for ox, oy in ((True, True), (True, False)):
        run_sequence([f, g], 0.5, kmax=2048, tag="wcluster", open_x=ox, open_y=oy,
                     obstacles=obst)


# ------------------------------------------------------- density-weighted centres
@pytest.mark.parametrize("seed", range(8))
def test_weighted_centres_moving_disks(seed):
    """Centres as the centroids of Sec. 2 with the field as density: disks with
    smooth interfaces, so the weights vary inside every component and the
    weighted centres differ from the unit-weight ones."""
    rng = np.random.default_rng(9100 + seed)
    lx, ly = int(rng.integers(40, 200)), int(rng.integers(40, 200))
    sim = synth.DiskSim(lx, ly, int(rng.integers(3, 30)), 3.0, 7.0, 0.7, 3e-3, seed=9200 + seed)
    fields = list(sim.frames(4))
    conn = 8 if seed % 2 else 4
    now = run_sequence(fields, 0.3, conn=conn, tag=f"weighted{seed}", weighted=True)
    plain = oracle.frame(fields[-1], 0.3, conn=conn)
    assert np.any(now.comps["qx"] != plain.comps["qx"]) or np.any(now.comps["qy"] != plain.comps["qy"])


@pytest.mark.parametrize("seed", range(6))
def test_weighted_centres_random_fields_walls_and_obstacles(seed):
    """Uniform-noise fields (weights 1..256 per site, bubbles clamped at one
    unit), walls and obstacles in turn, both phases."""
    rng = np.random.default_rng(9300 + seed)
    lx, ly = int(rng.integers(3, 90)), int(rng.integers(3, 90))
    conn = int(rng.choice([4, 8]))
    phase = seed % 2
    ox, oy = [(False, False), (True, False), (False, True), (True, True)][seed % 4]
    obst = rng.random((ly, lx)) < 0.1 if seed % 3 == 0 else None
    thr = 0.4 if phase == 1 else 0.6
    fields = [synth.tiny_random_field(lx, ly, 9400 + 7 * seed + k) for k in range(3)]
    run_sequence(fields, thr, phase, conn, tag=f"wrand{seed}", open_x=ox, open_y=oy,
                 obstacles=obst, weighted=True)


@pytest.mark.parametrize("depth", [4, 32])
def test_weighted_centres_batched(depth):
    """Batches of weighted frames: every frame's results against the oracle."""
    lx, ly = 256, 192
    sim = synth.DiskSim(lx, ly, 40, 4.0, 8.0, 0.6, 3e-3, seed=9500 + depth)
    frames = list(sim.frames(2 * depth + 3))
    det = dv.Detector(lx, ly, 0.3, max_components=256, max_batch=depth, keep_results=True,
                      weighted=True)
    seq = oracle.Sequence(0.3, 0, 8, NTHREADS, weighted=True)
    refs = []
    for f in frames:
        refs.append(seq.push(f))
        det.push(torch.from_numpy(f).cuda())
    say(f"  [weighted batch{depth}] {len(frames)} frames")
    check_frame(det, refs[-1][0], refs[-1][1], lx, ly)
    check_results(det.results(), refs, f"weighted batch{depth}")
    det.close()


def test_group_of_weighted_and_unweighted_members():
    """One launch per stage over members with and without weighted centres:
    each member's frames equal its own oracle."""
    sizes = [(96, 80), (128, 128), (70, 150), (200, 100)]
    weighted = [True, False, True, False]
    sims = [synth.DiskSim(lx, ly, max(3, lx * ly // 2000), 3.0, 7.0, 0.7, 3e-3, seed=9600 + i)
            for i, (lx, ly) in enumerate(sizes)]
    frames = [list(sm.frames(4)) for sm in sims]
    stream = torch.cuda.Stream()
    dets = [dv.Detector(lx, ly, 0.3, max_components=512, max_batch=2, stream=stream,
                        keep_results=True, weighted=w) for (lx, ly), w in zip(sizes, weighted)]
    grp = dv.Group(dets)
    seqs = [oracle.Sequence(0.3, 0, 8, NTHREADS, weighted=w) for w in weighted]
    refs = [[] for _ in sizes]
    for k in range(4):
        say(f"  [weighted group] frame {k}")
        grp.push([torch.from_numpy(frames[i][k]).cuda() for i in range(len(sizes))])
        for i, (lx, ly) in enumerate(sizes):
            now, ref = seqs[i].push(frames[i][k])
            refs[i].append((now, ref))
            check_frame(dets[i], now, ref, lx, ly)
    for i in range(len(sizes)):
        check_results(dets[i].results(), refs[i], f"weighted group member {i}")
    grp.close()
    for d in dets:
        d.close()


def test_weighted_centres_grf1024():
    """A 1024^2 random field (weights up to a few thousand units, components
    across the seams) with weighted centres, in one batch of four."""
    sim = synth.GRFSim(1024, 1024, 6.0, 0.98, seed=9700)
    run_sequence(list(sim.frames(4)), 1.0, kmax=8192, tag="weighted grf1024", weighted=True,
                 max_batch=4)
