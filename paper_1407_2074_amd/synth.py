"""Seeded synthetic inputs: multi-channel fluorescence-like volumes, transfer functions, cameras.

This module holds only input generation.  It contains none of the method's arithmetic (no
down-sampling, no octree logic, no ray casting), so both the HIP path and the CPU oracle can be
fed from it without sharing any computation.

The paper evaluates on private SPIM mouse-embryo scans (three uint16 channels; Table 1).  Those
are not available, so the stand-in is a per-channel sum of anisotropic Gaussian blobs plus
Poisson photon noise, generated deterministically from a seed:

* blob centres uniform in the volume, per-axis sigma uniform in [2, 8] voxels, peak uniform in
  [1000, 4000]; each blob is evaluated at voxel centres (index + 1/2) in float64 and truncated to
  4 sigma per axis;
* noise ~ Poisson(50), drawn by inverse CDF from a counter-based uniform keyed by
  (seed, channel, linear voxel index), so any z-slab can be regenerated on its own;
* voxel = min(65535, floor(blob + 1/2) + noise), uint16.  Float volumes are uint16 * 2**-16.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "blob_params", "gen_volume", "gen_slab", "poisson_noise", "gen_tf", "orbit_camera",
    "View", "default_window",
]

_MASK64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea & Flood 2014) applied element-wise to uint64 keys."""
    with np.errstate(over="ignore"):
        z = (x + np.uint64(0x9E3779B97F4A7C15)) & _MASK64
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _MASK64
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _MASK64
        z = z ^ (z >> np.uint64(31))
    return z


def _poisson_cdf(mean: float = 50.0, kmax: int = 200) -> np.ndarray:
    pmf = np.empty(kmax + 1, dtype=np.float64)
    pmf[0] = math.exp(-mean)
    for k in range(1, kmax + 1):
        pmf[k] = pmf[k - 1] * mean / k
    return np.cumsum(pmf)


_CDF50 = _poisson_cdf()


def poisson_noise(seed: int, channel: int, lin_index: np.ndarray) -> np.ndarray:
    """Poisson(50) counts for the given linear voxel indices (counter-based, order free)."""
    key = (np.uint64(seed) * np.uint64(16) + np.uint64(channel)) << np.uint64(40)
    u = (_splitmix64(lin_index.astype(np.uint64) + key) >> np.uint64(11)).astype(np.float64)
    u *= 2.0 ** -53
    return np.searchsorted(_CDF50, u, side="right").astype(np.int64)


def blob_params(dims, seed: int, channel: int, n_blobs: int):
    """Blob centres (x,y,z), sigmas (x,y,z) and peaks for one channel."""
    dx, dy, dz = dims
    rng = np.random.Generator(np.random.PCG64(1000 * seed + channel))
    mu = rng.uniform(0.0, 1.0, size=(n_blobs, 3)) * np.array([dx, dy, dz], dtype=np.float64)
    sigma = rng.uniform(2.0, 8.0, size=(n_blobs, 3))
    peak = rng.uniform(1000.0, 4000.0, size=n_blobs)
    return mu, sigma, peak


def _blob_field(dims, z0: int, z1: int, mu, sigma, peak) -> np.ndarray:
    dx, dy, dz = dims
    out = np.zeros((z1 - z0, dy, dx), dtype=np.float64)
    for b in range(len(peak)):
        lo = np.ceil(mu[b] - 4.0 * sigma[b] - 0.5).astype(np.int64)
        hi = np.floor(mu[b] + 4.0 * sigma[b] - 0.5).astype(np.int64)
        xa, ya = max(lo[0], 0), max(lo[1], 0)
        xb, yb = min(hi[0], dx - 1), min(hi[1], dy - 1)
        za, zb = max(lo[2], z0), min(hi[2], z1 - 1)
        if xa > xb or ya > yb or za > zb:
            continue
        gx = np.exp(-0.5 * (((np.arange(xa, xb + 1) + 0.5) - mu[b, 0]) / sigma[b, 0]) ** 2)
        gy = np.exp(-0.5 * (((np.arange(ya, yb + 1) + 0.5) - mu[b, 1]) / sigma[b, 1]) ** 2)
        gz = np.exp(-0.5 * (((np.arange(za, zb + 1) + 0.5) - mu[b, 2]) / sigma[b, 2]) ** 2)
        out[za - z0:zb - z0 + 1, ya:yb + 1, xa:xb + 1] += \
            peak[b] * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    return out


def gen_slab(dims, channels: int, seed: int, n_blobs: int, z0: int, z1: int,
             dtype: str = "u16") -> np.ndarray:
    """Planar slab [C][z1-z0][Dy][Dx] of the synthetic volume (independently regenerable)."""
    dx, dy, dz = dims
    assert 0 <= z0 <= z1 <= dz
    out = np.empty((channels, z1 - z0, dy, dx), dtype=np.uint16)
    lin = (np.arange(z0 * dy * dx, z1 * dy * dx, dtype=np.uint64)).reshape(z1 - z0, dy, dx)
    for c in range(channels):
        mu, sigma, peak = blob_params(dims, seed, c, n_blobs)
        f = np.floor(_blob_field(dims, z0, z1, mu, sigma, peak) + 0.5).astype(np.int64)
        v = f + poisson_noise(seed, c, lin)
        out[c] = np.minimum(v, 65535).astype(np.uint16)
    if dtype == "f32":
        return (out.astype(np.float32) * np.float32(2.0 ** -16)).astype(np.float32)
    return out


def _slab_job(args):
    dims, channels, seed, n_blobs, z0, z1, dtype = args
    return z0, gen_slab(dims, channels, seed, n_blobs, z0, z1, dtype)


def gen_volume(dims, channels: int, seed: int, n_blobs: int, dtype: str = "u16",
               workers: int = 1) -> np.ndarray:
    """Whole planar volume [C][Dz][Dy][Dx]; with workers > 1 the z-slabs are generated in
    parallel processes (identical result: every voxel depends only on its index)."""
    if workers <= 1:
        return gen_slab(dims, channels, seed, n_blobs, 0, dims[2], dtype)
    import multiprocessing as mp
    dz = dims[2]
    step = max(1, -(-dz // (4 * workers)))
    jobs = [(dims, channels, seed, n_blobs, z, min(z + step, dz), dtype) for z in range(0, dz, step)]
    out = np.empty((channels, dz, dims[1], dims[0]), np.uint16 if dtype == "u16" else np.float32)
    with mp.get_context("fork").Pool(workers) as pool:
        for z0, slab in pool.imap_unordered(_slab_job, jobs):
            out[:, z0:z0 + slab.shape[1]] = slab
    return out


def default_window(dtype: str = "u16"):
    """Per-channel intensity window (lo, hi): the nominal 12-bit range of the detector."""
    return (0.0, 4095.0) if dtype == "u16" else (0.0, 4095.0 * 2.0 ** -16)


def gen_tf(seed: int, channel: int):
    """8 control points: positions [8] ascending in [0,1] and RGBA [8][4].

    The first two control points are fully transparent so that noise-level intensities are
    invisible (this is what makes empty-space skipping effective)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = np.empty(8, dtype=np.float64)
    pos[0], pos[7] = 0.0, 1.0
    pos[1] = rng.uniform(0.02, 0.10)
    pos[2:7] = np.sort(rng.uniform(pos[1], 1.0, size=5))
    rgba = np.empty((8, 4), dtype=np.float64)
    rgba[:, :3] = rng.uniform(0.0, 1.0, size=(8, 3))
    rgba[:, 3] = 0.0
    rgba[2:, 3] = rng.uniform(0.0, 0.05, size=6)
    return pos.astype(np.float32), rgba.astype(np.float32)


def orbit_camera(dims, az_deg: float, el_deg: float, fov_y_deg: float = 30.0,
                 dist_scale: float = 1.0):
    """Eye/target/up for an orbit around the volume centre that fits the bounding sphere."""
    c = np.array(dims, dtype=np.float64) / 2.0
    r = float(np.linalg.norm(np.array(dims, dtype=np.float64))) / 2.0
    dist = dist_scale * 1.05 * r / math.sin(math.radians(fov_y_deg / 2.0))
    az, el = math.radians(az_deg), math.radians(el_deg)
    eye = c + dist * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az),
                               math.sin(el)])
    return eye.astype(np.float32), c.astype(np.float32), np.array([0, 0, 1], np.float32)


@dataclass
class View:
    """One render request: camera, image size, sampling, clipping and per-channel TFs."""
    eye: np.ndarray
    target: np.ndarray
    up: np.ndarray
    width: int
    height: int
    tf_pos: np.ndarray            # [C][8] float32, ascending
    tf_rgba: np.ndarray           # [C][8][4] float32
    window: np.ndarray            # [C][2] float32 (lo, hi)
    fov_y_deg: float = 30.0
    step: float = 0.5
    ert_alpha: float = 1.0
    lod: int = 0                  # -1 = per-ray footprint LOD
    clips: list = field(default_factory=list)   # up to 3 (nx, ny, nz, d): keep n.p >= d
    tile_begin: int = 0
    tile_count: int = -1          # -1 = all tiles from tile_begin
    depth_segments: int = 0       # 0 = automatic (by ray length), 1 = one pass per ray
    no_skip: int = 0              # 1 = march every position (no empty-space skipping)
    mode: int = 0                 # 0 = emission-absorption (DVR), 1 = maximum intensity projection
    missing: int = 0              # non-resident bricks: 0 = AVG, 1 = full-frame fallback to the
                                  # two coarser levels, 2 = refinement (rays wait for the brick)
    xform: np.ndarray = None      # None, or [C][3][4] float32: channel c samples at M p + b

    @property
    def channels(self) -> int:
        return int(self.tf_pos.shape[0])


def make_view(dims, channels: int, cfg_seed: int, az: float, el: float, width: int,
              height: int, dtype: str = "u16", **kw) -> View:
    """Orbit view with the seeded per-channel TFs of a configuration."""
    eye, target, up = orbit_camera(dims, az, el, kw.pop("fov_y_deg", 30.0),
                                   kw.pop("dist_scale", 1.0))
    pos = np.empty((channels, 8), np.float32)
    rgba = np.empty((channels, 8, 4), np.float32)
    for c in range(channels):
        pos[c], rgba[c] = gen_tf(1000 * cfg_seed + 100 + c, c)
    win = np.array([default_window(dtype)] * channels, np.float32)
    return View(eye=eye, target=target, up=up, width=width, height=height, tf_pos=pos,
                tf_rgba=rgba, window=win, **kw)
