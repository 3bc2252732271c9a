"""Seeded synthetic lattice fields that stand in for the paper's simulation data.

The paper's emulsion fields (lattice-Boltzmann droplets in a 2048x1024 channel,
Sec. 4) and its random-field sample program (Sec. 1) are not available, so the
workloads here are generated from a seed.  This module holds input generation
only: it contains none of the detection method's arithmetic (no thresholding,
labelling, centroids, tessellation or diffing).  Both the HIP path and the CPU
oracle consume the same float32 bytes produced here.

Generators
----------
* ``DiskSim``   -- polydisperse disks with a tanh interface profile, moved each
  frame by Gaussian jitter plus simple shear and then relaxed so that no two
  disks come within ``gap`` lattice units (so they never touch under 8-neighbour
  connectivity).  Stand-in for the droplet emulsion of Sec. 4.
* ``GRFSim``    -- periodic Gaussian random field (white noise smoothed by a
  Gaussian kernel via FFT, standardised), evolved as AR(1).  Thresholding it
  gives irregular "bubbles" like the random-field sample of Sec. 1.
* ``ChannelSim`` -- disks in a channel with walls across x and rectangular
  posts on the left wall, drifting along y with a parabolic (Poiseuille-like)
  profile plus jitter, kept clear of each other, the walls and the posts.
  Stand-in for the pressure-driven emulsion in a channel with posts of Sec. 4;
  ``obstacles()`` gives the posts as a binary site field.
* ``tiny_random_field`` -- uniform noise for fuzzing small lattices.

All arithmetic is float64; fields are cast to float32 exactly once.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field as dc_field

import numpy as np

__all__ = [
    "DiskSim",
    "GRFSim",
    "ChannelSim",
    "tiny_random_field",
    "disk_field",
    "workload",
    "WORKLOADS",
    "mixed_fields",
]


def _wrap_delta(d: np.ndarray, L: float) -> np.ndarray:
    """Minimum-image displacement on a ring of length L (float64)."""
    return d - L * np.round(d / L)


def disk_field(lx: int, ly: int, centers: np.ndarray, radii: np.ndarray,
               width: float = 2.0, reach: float = 10.0) -> np.ndarray:
    """rho(s) = max_i 0.5*(1 - tanh((|s - c_i|_periodic - r_i)/width)).

    Evaluated only within ``r_i + reach`` of each centre (beyond that the
    profile is below 5e-5 and is taken as 0).  Returns float32 [ly, lx].
    """
    rho = np.zeros((ly, lx), dtype=np.float64)
    if len(radii) == 0:
        return rho.astype(np.float32)
    rmax = float(np.max(radii)) + reach
    span = int(math.ceil(rmax)) + 1
    off = np.arange(-span, span + 1)
    P = off.size
    cx = centers[:, 0]
    cy = centers[:, 1]
    bx = np.floor(cx).astype(np.int64)
    by = np.floor(cy).astype(np.int64)
    dx = (bx[:, None] + off[None, :]) - cx[:, None]          # [K, P]
    dy = (by[:, None] + off[None, :]) - cy[:, None]          # [K, P]
    dist = np.sqrt(dy[:, :, None] ** 2 + dx[:, None, :] ** 2)  # [K, P(y), P(x)]
    val = 0.5 * (1.0 - np.tanh((dist - radii[:, None, None]) / width))
    val[dist > (radii[:, None, None] + reach)] = 0.0
    if P <= lx and P <= ly:
        # each patch touches P distinct rows and columns: max-combine in place
        for i in range(len(radii)):
            x0 = int(bx[i]) - span
            y0 = int(by[i]) - span
            if 0 <= x0 and x0 + P <= lx and 0 <= y0 and y0 + P <= ly:
                sub = rho[y0:y0 + P, x0:x0 + P]
                np.maximum(sub, val[i], out=sub)
            else:
                iy = np.mod(np.arange(y0, y0 + P), ly)
                ix = np.mod(np.arange(x0, x0 + P), lx)
                blk = np.ix_(iy, ix)
                rho[blk] = np.maximum(rho[blk], val[i])
        return rho.astype(np.float32)
    # tiny lattice: a patch wraps onto itself; combine by sorting (site, value)
    sx = np.mod(bx[:, None, None] + off[None, None, :], lx) + 0 * off[None, :, None]
    sy = np.mod(by[:, None, None] + off[None, :, None], ly) + 0 * off[None, None, :]
    flat = (sy * lx + sx).ravel()
    v = val.ravel()
    order = np.lexsort((v, flat))
    fs = flat[order]
    vs = v[order]
    last = np.ones(fs.shape, dtype=bool)
    last[:-1] = fs[1:] != fs[:-1]
    out = rho.ravel()
    out[fs[last]] = vs[last]
    return out.reshape(ly, lx).astype(np.float32)


@dataclass
class DiskSim:
    """Polydisperse disks under jitter + simple shear with overlap relaxation."""

    lx: int
    ly: int
    n_disks: int
    r_min: float
    r_max: float
    sigma: float          # per-axis Gaussian jitter per frame (lattice units)
    shear: float          # dx = shear * (y - ly/2) per frame
    seed: int
    gap: float = 2.0      # minimum surface-to-surface distance kept between disks
    width: float = 2.0    # tanh interface width
    relax_iters: int = 200
    centers: np.ndarray = dc_field(init=False, repr=False)
    radii: np.ndarray = dc_field(init=False, repr=False)
    rng: np.random.Generator = dc_field(init=False, repr=False)

    def __post_init__(self):
        self.rng = np.random.default_rng(self.seed)
        self.radii = self.rng.uniform(self.r_min, self.r_max, self.n_disks)
        self.centers = np.stack([
            self.rng.uniform(0, self.lx, self.n_disks),
            self.rng.uniform(0, self.ly, self.n_disks)], axis=1)
        self._relax()

    def _relax(self):
        """Jacobi relaxation: push every overlapping pair apart symmetrically."""
        from scipy.spatial import cKDTree
        c = self.centers
        r = self.radii
        reach = 2.0 * float(np.max(r)) + self.gap if len(r) else 0.0
        box = np.array([self.lx, self.ly], dtype=np.float64)
        for _ in range(self.relax_iters):
            c[:, 0] %= self.lx
            c[:, 1] %= self.ly
            tree = cKDTree(c, boxsize=box)
            pairs = tree.query_pairs(reach, output_type="ndarray")
            if pairs.size == 0:
                break
            i, j = pairs[:, 0], pairs[:, 1]
            dx = _wrap_delta(c[i, 0] - c[j, 0], self.lx)
            dy = _wrap_delta(c[i, 1] - c[j, 1], self.ly)
            d = np.sqrt(dx * dx + dy * dy)
            over = r[i] + r[j] + self.gap - d
            m = over > 0
            if not np.any(m):
                break
            i, j, dx, dy, d, over = i[m], j[m], dx[m], dy[m], d[m], over[m]
            # small margin so that relaxed pairs do not sit exactly on the limit
            push = 0.5 * (over + 1e-3)
            dsafe = np.where(d > 1e-9, d, 1.0)
            ux = np.where(d > 1e-9, dx / dsafe, 1.0)
            uy = np.where(d > 1e-9, dy / dsafe, 0.0)
            mv = np.zeros_like(c)
            np.add.at(mv[:, 0], i, push * ux)
            np.add.at(mv[:, 1], i, push * uy)
            np.add.at(mv[:, 0], j, -push * ux)
            np.add.at(mv[:, 1], j, -push * uy)
            c += mv
        c[:, 0] %= self.lx
        c[:, 1] %= self.ly
        self.centers = c

    def field(self) -> np.ndarray:
        return disk_field(self.lx, self.ly, self.centers, self.radii, self.width)

    def step(self):
        c = self.centers
        c += self.rng.normal(0.0, self.sigma, c.shape)
        c[:, 0] += self.shear * (c[:, 1] - self.ly / 2.0)
        c[:, 0] %= self.lx
        c[:, 1] %= self.ly
        self.centers = c
        self._relax()

    def frames(self, n: int):
        """Yield n float32 fields; frame 0 is the initial placement."""
        for t in range(n):
            if t:
                self.step()
            yield self.field()


@dataclass
class ChannelSim:
    """Disks in a channel: walls at x = -1/2 and x = lx - 1/2 (no wrap in x),
    periodic in y, posts of post_w x post_h sites on the left wall every
    post_period sites along y.  Each frame moves disk i by
    vmax * 4 u (1 - u) along y (u = x / lx, the parabolic profile of a
    pressure-driven channel flow) plus Gaussian jitter, then relaxes overlaps
    with each other, the walls and the posts (gap sites kept free)."""

    lx: int
    ly: int
    n_disks: int
    r_min: float
    r_max: float
    post_w: int
    post_h: int
    post_period: int
    vmax: float
    sigma: float
    seed: int
    gap: float = 2.0
    width: float = 2.0
    relax_iters: int = 300
    centers: np.ndarray = dc_field(init=False, repr=False)
    radii: np.ndarray = dc_field(init=False, repr=False)
    rng: np.random.Generator = dc_field(init=False, repr=False)

    def __post_init__(self):
        self.rng = np.random.default_rng(self.seed)
        self.radii = self.rng.uniform(self.r_min, self.r_max, self.n_disks)
        self.centers = np.stack([
            self.rng.uniform(self.post_w, self.lx, self.n_disks),
            self.rng.uniform(0, self.ly, self.n_disks)], axis=1)
        self._relax()

    def obstacles(self) -> np.ndarray:
        """bool [ly, lx]: True on post sites."""
        m = np.zeros((self.ly, self.lx), dtype=bool)
        rows = (np.arange(self.ly) % self.post_period) < self.post_h
        m[rows, :self.post_w] = True
        return m

    def _post_push(self, c: np.ndarray, r: np.ndarray) -> np.ndarray:
        """Displacement that takes each disk gap/2 + r clear of the nearest
        post rectangle [-inf, post_w - 1/2] x [y0 - 1/2, y0 + post_h - 1/2]."""
        y0 = np.floor(c[:, 1] / self.post_period) * self.post_period
        mv = np.zeros_like(c)
        for off in (-self.post_period, 0.0, self.post_period):
            lo = y0 + off - 0.5
            hi = lo + self.post_h
            nx = np.minimum(c[:, 0], self.post_w - 0.5)
            ny = np.clip(c[:, 1], lo, hi)
            dx, dy = c[:, 0] - nx, c[:, 1] - ny
            d = np.sqrt(dx * dx + dy * dy)
            need = r + self.gap
            m = d < need
            inside = d < 1e-9
            ux = np.where(inside, 1.0, dx / np.where(inside, 1.0, d))
            uy = np.where(inside, 0.0, dy / np.where(inside, 1.0, d))
            amt = np.where(m, need - d + 1e-3, 0.0)
            mv[:, 0] += amt * ux
            mv[:, 1] += amt * uy
        return mv

    def _relax(self):
        """Jacobi relaxation of disk pairs, walls and posts."""
        from scipy.spatial import cKDTree
        c = self.centers
        r = self.radii
        reach = 2.0 * float(np.max(r)) + self.gap if len(r) else 0.0
        # x lies in [0, lx): a period of 2 lx in the tree never joins the walls
        box = np.array([2.0 * self.lx, self.ly], dtype=np.float64)
        lo_x = r + 0.5 * self.gap
        hi_x = self.lx - 1.0 - r - 0.5 * self.gap
        for _ in range(self.relax_iters):
            c[:, 0] = np.clip(c[:, 0], lo_x, hi_x)
            c[:, 1] %= self.ly
            mv = self._post_push(c, r)
            tree = cKDTree(c, boxsize=box)
            pairs = tree.query_pairs(reach, output_type="ndarray")
            if pairs.size:
                i, j = pairs[:, 0], pairs[:, 1]
                dx = c[i, 0] - c[j, 0]
                dy = _wrap_delta(c[i, 1] - c[j, 1], self.ly)
                d = np.sqrt(dx * dx + dy * dy)
                over = r[i] + r[j] + self.gap - d
                m = over > 0
                i, j, dx, dy, d, over = i[m], j[m], dx[m], dy[m], d[m], over[m]
                push = 0.5 * (over + 1e-3)
                dsafe = np.where(d > 1e-9, d, 1.0)
                ux = np.where(d > 1e-9, dx / dsafe, 1.0)
                uy = np.where(d > 1e-9, dy / dsafe, 0.0)
                np.add.at(mv[:, 0], i, push * ux)
                np.add.at(mv[:, 1], i, push * uy)
                np.add.at(mv[:, 0], j, -push * ux)
                np.add.at(mv[:, 1], j, -push * uy)
            if not np.any(mv):
                break
            c += mv
        c[:, 0] = np.clip(c[:, 0], lo_x, hi_x)
        c[:, 1] %= self.ly
        self.centers = c

    def field(self) -> np.ndarray:
        f = disk_field(self.lx, self.ly, self.centers, self.radii, self.width)
        f[self.obstacles()] = 0.0
        return f

    def step(self):
        c = self.centers
        u = c[:, 0] / self.lx
        c[:, 1] += self.vmax * 4.0 * u * (1.0 - u)
        c += self.rng.normal(0.0, self.sigma, c.shape)
        self.centers = c
        self._relax()

    def frames(self, n: int):
        """Yield n float32 fields; frame 0 is the initial placement."""
        for t in range(n):
            if t:
                self.step()
            yield self.field()


def _smooth_noise(rng: np.random.Generator, lx: int, ly: int, sigma: float,
                  workers: int) -> np.ndarray:
    import scipy.fft as sfft
    g = rng.standard_normal((ly, lx))
    fy = np.fft.fftfreq(ly)[:, None]
    fx = np.fft.rfftfreq(lx)[None, :]
    kern = np.exp(-2.0 * (math.pi ** 2) * sigma * sigma * (fx * fx + fy * fy))
    s = sfft.irfft2(sfft.rfft2(g, workers=workers) * kern, s=(ly, lx), workers=workers)
    s -= s.mean()
    s /= s.std()
    return s


@dataclass
class GRFSim:
    """Periodic Gaussian random field evolved as AR(1): f' = rho f + sqrt(1-rho^2) g."""

    lx: int
    ly: int
    sigma: float
    rho: float
    seed: int
    workers: int = -1
    f: np.ndarray = dc_field(init=False, repr=False)
    rng: np.random.Generator = dc_field(init=False, repr=False)

    def __post_init__(self):
        self.rng = np.random.default_rng(self.seed)
        self.f = _smooth_noise(self.rng, self.lx, self.ly, self.sigma, self.workers)

    def field(self) -> np.ndarray:
        return self.f.astype(np.float32)

    def step(self):
        g = _smooth_noise(self.rng, self.lx, self.ly, self.sigma, self.workers)
        self.f = self.rho * self.f + math.sqrt(1.0 - self.rho * self.rho) * g

    def frames(self, n: int):
        for t in range(n):
            if t:
                self.step()
            yield self.field()


def tiny_random_field(lx: int, ly: int, seed: int) -> np.ndarray:
    """Uniform [0,1) float32 noise; thresholding it at p gives site percolation."""
    return np.random.default_rng(seed).random((ly, lx)).astype(np.float32)


# ---------------------------------------------------------------------------
# Named workloads.  Each entry: constructor, frame count, threshold, phase
# (0: inside means rho > threshold, droplets; 1: rho < threshold, bubbles).
# ---------------------------------------------------------------------------
WORKLOADS = {
    # 256^2, 64 disks r~U(8,12), jitter 0.3, shear 1e-3, 10 frames
    "disks256": dict(kind="disks", lx=256, ly=256, n_disks=64, r_min=8.0, r_max=12.0,
                     sigma=0.3, shear=1e-3, seed=1, frames=10, threshold=0.5, phase=0),
    # 1024^2, 1000 disks r~U(10,16), jitter 0.2, shear 5e-4, 100 frames
    "disks1024": dict(kind="disks", lx=1024, ly=1024, n_disks=1000, r_min=10.0, r_max=16.0,
                      sigma=0.2, shear=5e-4, seed=2, frames=100, threshold=0.5, phase=0),
    # 4096^2 Gaussian random field, smoothing sigma 6, AR(1) rho 0.98, 50 frames,
    # thresholded at +1 std
    "grf4096": dict(kind="grf", lx=4096, ly=4096, sigma=6.0, rho=0.98, seed=3,
                    frames=50, threshold=1.0, phase=0),
    # 2048 (wall to wall, x) x 1024 (periodic, y) channel, posts 48 x 64 every
    # 128 on the left wall, 2000 disks r~U(12.5,15), parabolic drift 1.0 at the
    # centre line, jitter 0.2, 20 frames
    "channel2048": dict(kind="channel", lx=2048, ly=1024, n_disks=2000, r_min=12.5,
                        r_max=15.0, post_w=48, post_h=64, post_period=128, vmax=1.0,
                        sigma=0.2, seed=5, frames=20, threshold=0.5, phase=0, open_x=True),
}


def workload(name: str, **override):
    """Return (simulator, spec) for a named workload; ``override`` edits the spec."""
    spec = dict(WORKLOADS[name])
    spec.update(override)
    if spec["kind"] == "disks":
        sim = DiskSim(spec["lx"], spec["ly"], spec["n_disks"], spec["r_min"], spec["r_max"],
                      spec["sigma"], spec["shear"], spec["seed"])
    elif spec["kind"] == "grf":
        sim = GRFSim(spec["lx"], spec["ly"], spec["sigma"], spec["rho"], spec["seed"])
    elif spec["kind"] == "channel":
        sim = ChannelSim(spec["lx"], spec["ly"], spec["n_disks"], spec["r_min"], spec["r_max"],
                         spec["post_w"], spec["post_h"], spec["post_period"], spec["vmax"],
                         spec["sigma"], spec["seed"])
    else:
        raise ValueError(spec["kind"])
    return sim, spec


def mixed_fields(n: int = 64, seed: int = 4, l_min: int = 256, l_max: int = 2048):
    """Independent sequences of uneven sizes for one batch: square sides
    log-uniform in [l_min, l_max], half disk emulsions (1000 disks per 1024^2,
    radii U(10,16), jitter 0.2, shear 5e-4, threshold 0.5), half random fields
    (smoothing 6, AR(1) 0.98, threshold +1 std).  Returns [(sim, spec)]."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        L = int(round(np.exp(rng.uniform(np.log(l_min), np.log(l_max)))))
        if rng.random() < 0.5:
            nd = max(4, int(round(1000 * L * L / 1024 ** 2)))
            spec = dict(kind="disks", lx=L, ly=L, n_disks=nd, r_min=10.0, r_max=16.0, sigma=0.2,
                        shear=5e-4, seed=seed * 1000 + i, threshold=0.5, phase=0,
                        k_expect=nd)
            sim = DiskSim(L, L, nd, 10.0, 16.0, 0.2, 5e-4, spec["seed"])
        else:
            spec = dict(kind="grf", lx=L, ly=L, sigma=6.0, rho=0.98, seed=seed * 1000 + i,
                        threshold=1.0, phase=0, k_expect=int(9000 * L * L / 4096 ** 2) + 16)
            sim = GRFSim(L, L, 6.0, 0.98, spec["seed"])
        out.append((sim, spec))
    return out
