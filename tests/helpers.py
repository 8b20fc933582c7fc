"""Test-side helpers: independent brute-force references used to pin the oracle.

Nothing here is imported by the product or by the oracle.  The references are deliberately
different implementations of the definitions: numpy reshape-sums for the mipmap,
scipy.ndimage.map_coordinates for trilinear sampling and numpy.interp for the transfer function.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import ndimage

from paper_1407_2074_amd.synth import View


def np_halfsample(level: np.ndarray) -> np.ndarray:
    """One 2x2x2 down-sampling step over the valid children only (reshape-sum)."""
    C, ez, ey, ex = level.shape
    pz, py, px = ez + ez % 2, ey + ey % 2, ex + ex % 2
    v = np.zeros((C, pz, py, px), np.float64)
    v[:, :ez, :ey, :ex] = level
    n = np.zeros((pz, py, px), np.int64)
    n[:ez, :ey, :ex] = 1
    s = v.reshape(C, pz // 2, 2, py // 2, 2, px // 2, 2).sum(axis=(2, 4, 6))
    cnt = n.reshape(pz // 2, 2, py // 2, 2, px // 2, 2).sum(axis=(1, 3, 5))
    if level.dtype == np.uint16:
        si = s.astype(np.int64)
        return ((2 * si + cnt) // (2 * cnt)).astype(np.uint16)
    return (s / cnt).astype(np.float32)


def np_mip(v0: np.ndarray, brick: int):
    dmax = max(v0.shape[1:])
    N = 0
    while brick << N < dmax:
        N += 1
    levels = [v0]
    for _ in range(N):
        levels.append(np_halfsample(levels[-1]))
    return levels


def np_lut(pos, rgba) -> np.ndarray:
    """256-entry table at x = k/255 by numpy.interp (end values held outside)."""
    x = np.arange(256, dtype=np.float64) / 255.0
    return np.stack([np.interp(x, np.asarray(pos, np.float64), np.asarray(rgba, np.float64)[:, q])
                     for q in range(4)], axis=1)


def f32_camera(view: View):
    e = np.asarray(view.eye, np.float64)
    f = np.asarray(view.target, np.float64) - e
    f = f / math.sqrt((f[0] * f[0] + f[1] * f[1]) + f[2] * f[2])
    up = np.asarray(view.up, np.float64)
    r = np.array([f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2],
                  f[0] * up[1] - f[1] * up[0]])
    r = r / math.sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2])
    u = np.array([r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2],
                  r[0] * f[1] - r[1] * f[0]])
    th = math.tan(view.fov_y_deg * (math.pi / 360.0))
    return dict(eye=np.asarray(view.eye, np.float32), f=f.astype(np.float32),
                r=r.astype(np.float32), u=u.astype(np.float32),
                kx=np.float32(th * view.width / view.height), ky=np.float32(th),
                klod=np.float32(2.0 * th / view.height))


def f32_rays(view: View, dims, N: int):
    """Vectorised float32 ray set-up (same written operation order as the renderers)."""
    cm = f32_camera(view)
    W, H = view.width, view.height
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    f32 = np.float32
    a = (2 * ii + 1).astype(f32) / f32(W)
    b = (2 * jj + 1).astype(f32) / f32(H)
    sx = (a - f32(1)) * cm["kx"]
    sy = (f32(1) - b) * cm["ky"]
    d = np.stack([(cm["f"][k] + sx * cm["r"][k]) + sy * cm["u"][k] for k in range(3)], -1)
    n2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    inv = f32(1) / np.sqrt(n2)
    d = d * inv[..., None]
    o = np.broadcast_to(cm["eye"], d.shape).astype(f32)
    t0 = np.zeros((H, W), f32)
    t1 = np.full((H, W), np.inf, f32)
    hit = np.ones((H, W), bool)
    with np.errstate(divide="ignore", invalid="ignore"):
        for k in range(3):
            D = f32(dims[k])
            nz = d[..., k] != 0
            rk = f32(1) / np.where(nz, d[..., k], f32(1))
            ta = (f32(0) - o[..., k]) * rk
            tb = (D - o[..., k]) * rk
            t0 = np.where(nz, np.maximum(t0, np.minimum(ta, tb)), t0)
            t1 = np.where(nz, np.minimum(t1, np.maximum(ta, tb)), t1)
            hit &= nz | ((o[..., k] >= 0) & (o[..., k] <= D))
        for pl in view.clips:
            n = np.asarray(pl[:3], f32)
            nd = (n[0] * d[..., 0] + n[1] * d[..., 1]) + n[2] * d[..., 2]
            no = (n[0] * o[..., 0] + n[1] * o[..., 1]) + n[2] * o[..., 2]
            num = f32(pl[3]) - no
            q = num / np.where(nd != 0, nd, f32(1))
            t0 = np.where(nd > 0, np.maximum(t0, q), t0)
            t1 = np.where(nd < 0, np.minimum(t1, q), t1)
            hit &= ~((nd == 0) & (no < f32(pl[3])))
    hit &= t0 < t1
    if view.lod >= 0:
        L = np.full((H, W), min(view.lod, N), np.int32)
    else:
        w = t0 * cm["klod"]
        e = np.frexp(w)[1] - 1
        L = np.where(w > 0, np.clip(e, 0, N), 0).astype(np.int32)
    return o, d, t0, t1, L, hit


def bf_render_dense(levels, dims, view: View, N: int):
    """Regular-grid ray casting on dense level arrays (no octree): trilinear by
    scipy.ndimage.map_coordinates with edge clamping, numpy.interp transfer function."""
    o, d, t0, t1, L, hit = f32_rays(view, dims, N)
    C = levels[0].shape[0]
    H, W = view.height, view.width
    luts = [np_lut(view.tf_pos[c], view.tf_rgba[c]) for c in range(C)]
    img = np.zeros((H, W, 4), np.float64)
    A = np.zeros((H, W))
    Cc = np.zeros((H, W, 3))
    step = np.float32(view.step)
    k = 0
    active = hit.copy()
    while active.any():
        t = t0 + np.float32(k) * step
        active &= t < t1
        if not active.any():
            break
        idx = np.nonzero(active)
        p = o[idx] + t[idx][:, None] * d[idx]
        Ls = L[idx]
        vals = np.zeros((C, len(Ls)))
        for lv in np.unique(Ls):
            sel = Ls == lv
            q = p[sel] * np.float32(2.0 ** -int(lv)) - np.float32(0.5)
            coords = np.stack([q[:, 2], q[:, 1], q[:, 0]]).astype(np.float64)
            for c in range(C):
                vals[c, sel] = ndimage.map_coordinates(levels[lv][c].astype(np.float64), coords,
                                                       order=1, mode="nearest", prefilter=False)
        a_ = A[idx]
        c_ = Cc[idx]
        for c in range(C):
            lo, hi = float(view.window[c][0]), float(view.window[c][1])
            x = np.clip((vals[c] - lo) / (hi - lo), 0.0, 1.0)
            u = 255.0 * x
            i = np.minimum(np.floor(u), 254).astype(np.int64)
            fr = u - i
            rgba = luts[c][i] + fr[:, None] * (luts[c][i + 1] - luts[c][i])
            wgt = (1.0 - a_) * rgba[:, 3]
            c_ = c_ + wgt[:, None] * rgba[:, :3]
            a_ = a_ + wgt
        A[idx] = a_
        Cc[idx] = c_
        k += 1
    img[..., :3] = Cc
    img[..., 3] = A
    return img


def const_tf(C: int, alpha, rgb):
    """TF whose table is the same RGBA everywhere (all control points equal)."""
    pos = np.tile(np.linspace(0, 1, 8, dtype=np.float32), (C, 1))
    rgba = np.zeros((C, 8, 4), np.float32)
    for c in range(C):
        rgba[c, :, :3] = rgb[c]
        rgba[c, :, 3] = alpha[c]
    return pos, rgba


def np_channel_positions(p: np.ndarray, xform, c: int) -> np.ndarray:
    """Position channel c samples at: p itself, or ((m0 p0 + m1 p1) + m2 p2) + b per row, in
    float32 element-wise numpy arithmetic (each operation rounded once, nothing fused)."""
    if xform is None:
        return p
    m = np.asarray(xform, np.float32)[c]
    f32 = np.float32
    rows = []
    for a in range(3):
        s0 = m[a, 0] * p[:, 0]
        s1 = m[a, 1] * p[:, 1]
        s2 = m[a, 2] * p[:, 2]
        rows.append(((s0 + s1) + s2) + f32(m[a, 3]))
    return np.stack(rows, -1).astype(f32)


def np_node_avg(levels, L: int, M: int, b) -> np.ndarray:
    """AVG of the level-L node b: the data type's rounded mean over its valid voxels."""
    blk = levels[L][:, b[2] * M:(b[2] + 1) * M, b[1] * M:(b[1] + 1) * M, b[0] * M:(b[0] + 1) * M]
    n = blk[0].size
    if levels[L].dtype == np.uint16:
        s = blk.reshape(blk.shape[0], -1).astype(np.int64).sum(axis=1)
        return ((2 * s + n) // (2 * n)).astype(np.float64)
    return (blk.reshape(blk.shape[0], -1).astype(np.float64).sum(axis=1) / n).astype(
        np.float32).astype(np.float64)


def bf_render_general(levels, dims, view: View, N: int, M: int = 0, resident=None):
    """Regular-grid ray casting on dense level arrays for every node a brick (threshold 0):
    DVR or MIP (view.mode), per-channel affine positions (view.xform), and, when `resident`
    is given (a function (level, bx, by, bz) -> bool), the full-frame choice per sample of the
    ray's level, else the next coarser resident one of the two above it, else the AVG of the
    node at the ray's level (view.missing == 1), or that AVG directly (view.missing == 0).
    Trilinear by scipy.ndimage.map_coordinates with edge clamping, numpy.interp tables."""
    o, d, t0, t1, L, hit = f32_rays(view, dims, N)
    C = levels[0].shape[0]
    H, W = view.height, view.width
    luts = [np_lut(view.tf_pos[c], view.tf_rgba[c]) for c in range(C)]
    xform = getattr(view, "xform", None)
    mip = getattr(view, "mode", 0) == 1
    ff = getattr(view, "missing", 0) == 1
    A = np.zeros((H, W))
    Cc = np.zeros((H, W, 3))
    mx = np.full((C, H, W), -np.inf)
    step = np.float32(view.step)
    ert = (not mip) and view.ert_alpha < 1.0

    def classify(c, s):
        lo, hi = float(view.window[c][0]), float(view.window[c][1])
        x = np.clip((s - lo) / (hi - lo), 0.0, 1.0)
        u = 255.0 * x
        i = np.minimum(np.floor(u), 254).astype(np.int64)
        fr = u - i
        return luts[c][i] + fr[:, None] * (luts[c][i + 1] - luts[c][i])

    def sample(c, pc, Ls):
        vals = np.zeros(len(Ls))
        for lv in np.unique(Ls):
            sel = Ls == lv
            q = pc[sel] * np.float32(2.0 ** -int(lv)) - np.float32(0.5)
            coords = np.stack([q[:, 2], q[:, 1], q[:, 0]]).astype(np.float64)
            vals[sel] = ndimage.map_coordinates(levels[lv][c].astype(np.float64), coords,
                                                order=1, mode="nearest", prefilter=False)
        return vals

    k = 0
    active = hit.copy()
    while active.any():
        t = t0 + np.float32(k) * step
        active &= t < t1
        if ert:
            active &= ~(A >= view.ert_alpha)
        if not active.any():
            break
        idx = np.nonzero(active)
        p = o[idx] + t[idx][:, None] * d[idx]
        a_, c_ = A[idx], Cc[idx]
        for c in range(C):
            pc = np_channel_positions(p, xform, c)
            Lr = L[idx].astype(np.int64)
            if resident is None:
                s = sample(c, pc, Lr)
            else:
                vox = np.clip(np.floor(pc).astype(np.int64), 0, np.array(dims) - 1)
                s = np.zeros(len(Lr))
                for n in range(len(Lr)):
                    lv0 = int(Lr[n])
                    cands = [lv0] + ([lv0 + 1, lv0 + 2] if ff else [])
                    used = None
                    for lv in cands:
                        if lv > N:
                            break
                        b = tuple(int(x) for x in ((vox[n] >> lv) // M))
                        if resident(lv, *b):
                            used = lv
                            break
                    if used is None:
                        b = tuple(int(x) for x in ((vox[n] >> lv0) // M))
                        s[n] = np_node_avg(levels, lv0, M, b)[c]
                    else:
                        s[n] = sample(c, pc[n:n + 1], np.array([used]))[0]
            if mip:
                sel = (idx[0], idx[1])
                mx[c][sel] = np.maximum(mx[c][sel], s)
                continue
            rgba = classify(c, s)
            wgt = (1.0 - a_) * rgba[:, 3]
            c_ = c_ + wgt[:, None] * rgba[:, :3]
            a_ = a_ + wgt
        A[idx], Cc[idx] = a_, c_
        k += 1
    if mip:
        for c in range(C):
            sel = np.nonzero(hit)
            rgba = classify(c, mx[c][sel])
            wgt = (1.0 - A[sel]) * rgba[:, 3]
            Cc[sel] += wgt[:, None] * rgba[:, :3]
            A[sel] += wgt
    img = np.zeros((H, W, 4), np.float64)
    img[..., :3] = Cc
    img[..., 3] = A
    return img
