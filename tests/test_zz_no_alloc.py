"""The entry point that allocates nothing (dv_compare_static) against the
context path (dv_create, two pushes, dv_get_info, dv_get_flips), through the C
ABI: two calls in a row, the second on a smaller lattice, outputs bit-equal."""
import ctypes
import os

import numpy as np
import pytest

from paper_1607_00908_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1607_00908_amd import dv  # noqa: E402


def _cfg(lx, ly, kmax, flags=0):
    return dv.DVConfig(ctypes.sizeof(dv.DVConfig), lx, ly, 0.5, 0, 8, kmax, 0, 0, flags, 0)


def _static(lib, cfg, past, now, cap, stream):
    flips = torch.full((max(cap, 1), 6), -7, dtype=torch.int32, device="cuda")
    info = torch.zeros(ctypes.sizeof(dv.DVFrameInfo), dtype=torch.uint8, device="cuda")
    st = lib.dv_compare_static(ctypes.byref(cfg), ctypes.c_void_p(stream.cuda_stream),
                               ctypes.c_void_p(past.data_ptr()), ctypes.c_void_p(now.data_ptr()),
                               ctypes.c_void_p(flips.data_ptr()), cap, ctypes.c_void_p(info.data_ptr()))
    assert st == dv.OK, lib.dv_last_error(None)
    stream.synchronize()
    fi = dv.DVFrameInfo.from_buffer_copy(info.cpu().numpy().tobytes())
    return dv._frame_info(fi), flips.cpu().numpy()


def _context(lx, ly, kmax, past, now, flags=0):
    det = dv.Detector(lx, ly, 0.5, max_components=kmax, keep_maps=False,
                      classify=bool(flags & dv.CLASSIFY), weighted=bool(flags & dv.WEIGHTED))
    det.push(past)
    det.push(now)
    fi, fl = det.info(), det.flips()
    det.close()
    return fi, fl


def test_static_entry_point_equals_the_context_path():
    lib = dv.load()
    stream = torch.cuda.Stream()
    cases = [(300, 260, 60, 1), (150, 120, 18, 2)]   # the second call is smaller
    for lx, ly, nd, seed in cases:
        sim = synth.DiskSim(lx, ly, nd, 4.0, 7.0, 1.2, 4e-3, seed=400 + seed)
        frames = list(sim.frames(6))
        past = torch.from_numpy(frames[0]).cuda()
        now = torch.from_numpy(frames[5]).cuda()
        torch.cuda.synchronize()
        want_fi, want_fl = _context(lx, ly, 512, past, now)
        assert want_fi.n_flips > 0
        got_fi, got_fl = _static(lib, _cfg(lx, ly, 512), past, now, 4096, stream)
        assert got_fi == want_fi, (lx, ly)
        assert np.array_equal(got_fl[:got_fi.n_flips], want_fl), (lx, ly)
        # a capacity below the count: the count is reported, the first flips written
        got_fi2, got_fl2 = _static(lib, _cfg(lx, ly, 512), past, now, 1, stream)
        assert got_fi2.n_flips == want_fi.n_flips
        assert np.array_equal(got_fl2[:1], want_fl[:1])


def test_static_entry_point_weighted_centres():
    """The same with density-weighted centres (two calls, the second smaller)."""
    lib = dv.load()
    stream = torch.cuda.Stream()
    for lx, ly, nd, seed in [(260, 220, 40, 5), (120, 100, 12, 6)]:
        sim = synth.DiskSim(lx, ly, nd, 4.0, 7.0, 1.2, 4e-3, seed=500 + seed)
        frames = list(sim.frames(6))
        past = torch.from_numpy(frames[0]).cuda()
        now = torch.from_numpy(frames[5]).cuda()
        torch.cuda.synchronize()
        want_fi, want_fl = _context(lx, ly, 512, past, now, dv.WEIGHTED)
        got_fi, got_fl = _static(lib, _cfg(lx, ly, 512, dv.WEIGHTED), past, now, 4096, stream)
        assert got_fi == want_fi, (lx, ly)
        assert np.array_equal(got_fl[:got_fi.n_flips], want_fl), (lx, ly)


def test_static_entry_point_rejects_what_does_not_fit():
    lib = dv.load()
    f = torch.zeros((1024, 1024), dtype=torch.float32, device="cuda")
    flips = torch.zeros((4, 6), dtype=torch.int32, device="cuda")
    info = torch.zeros(64, dtype=torch.uint8, device="cuda")
    cfg = _cfg(1024, 1024, 4096)
    st = lib.dv_compare_static(ctypes.byref(cfg), None, ctypes.c_void_p(f.data_ptr()),
                               ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(flips.data_ptr()), 4,
                               ctypes.c_void_p(info.data_ptr()))
    assert st == dv.ERR_CAPACITY
    assert b"static scratch" in lib.dv_last_error(None)
