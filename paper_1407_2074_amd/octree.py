"""Thin ctypes binding of liboctree_rc.so (declared in include/octree_rc.h).

Only argument marshalling happens here: every step of construction and rendering runs in the
HIP kernels behind the C ABI.  PyTorch provides device memory and the current HIP stream.
If the library is missing this module raises at import time -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboctree_rc.so")

OCT_OK, OCT_INCOMPLETE = 0, 1
OCT_EINVAL, OCT_ENOMEM, OCT_ERANGE, OCT_EDEVICE, OCT_EBUSY = -1, -2, -3, -4, -5
OCT_U16, OCT_F32 = 0, 1
OCT_MODE_DVR, OCT_MODE_MIP = 0, 1
OCT_MISSING_AVG, OCT_MISSING_FALLBACK, OCT_MISSING_REFINE = 0, 1, 2
MAXC = 4

EXPORTS = ["octree_create", "octree_destroy", "octree_clear", "octree_insert_block",
           "octree_insert_slices", "brick_pool_upload", "render_views", "render_views_noalloc",
           "render_ckpt_bytes", "render_refine_bytes",
           "render_views_backward", "octree_dump_canonical", "octree_read_level", "octree_info",
           "octree_render_timing", "octree_build_timing", "octree_disk_stats", "oct_last_error"]
OCT_MASTER_HBM, OCT_MASTER_HOST, OCT_MASTER_DISK = 0, 1, 2
OCT_FRAMES_HOST, OCT_FRAMES_DEVICE = 0, 1


class CreateParams(ct.Structure):
    _fields_ = [("dims", ct.c_int32 * 3), ("channels", ct.c_int32), ("brick_size", ct.c_int32),
                ("dtype", ct.c_int32), ("background", ct.c_double),
                ("homog_threshold", ct.c_double), ("device_pool_bytes", ct.c_uint64),
                ("master_on_host", ct.c_int32), ("page_cells", ct.c_int32),
                ("host_bricks", ct.c_int32), ("disk_frames", ct.c_int32),
                ("host_cache_bytes", ct.c_uint64),
                ("disk_path", ct.c_char_p)]


class OctView(ct.Structure):
    _fields_ = [("eye", ct.c_float * 3), ("target", ct.c_float * 3), ("up", ct.c_float * 3),
                ("fov_y_deg", ct.c_float), ("width", ct.c_int32), ("height", ct.c_int32),
                ("tile_begin", ct.c_int32), ("tile_count", ct.c_int32), ("step", ct.c_float),
                ("ert_alpha", ct.c_float), ("lod", ct.c_int32), ("n_clip", ct.c_int32),
                ("clip", (ct.c_float * 4) * 3), ("tf_pos", (ct.c_float * 8) * MAXC),
                ("tf_rgba", ((ct.c_float * 4) * 8) * MAXC), ("window", (ct.c_float * 2) * MAXC),
                ("no_skip", ct.c_int32), ("depth_segments", ct.c_int32),
                ("mode", ct.c_int32), ("missing", ct.c_int32), ("n_xform", ct.c_int32),
                ("reserved", ct.c_int32), ("xform", ((ct.c_float * 4) * 3) * MAXC),
                ("refine_state", ct.c_void_p)]


class UploadStats(ct.Structure):
    _fields_ = [("bricks_gathered", ct.c_uint64), ("bricks_resident", ct.c_uint64),
                ("bricks_total", ct.c_uint64), ("nodes_changed", ct.c_uint64),
                ("bytes_written", ct.c_uint64), ("requests_seen", ct.c_uint64),
                ("evictions", ct.c_uint64), ("bricks_from_store", ct.c_uint64)]


class DiskStats(ct.Structure):
    _fields_ = [(k, ct.c_uint64) for k in ("pages", "frames", "hits", "loads", "fills", "writebacks",
                                           "evictions", "waits", "bytes_read", "bytes_written")]


class RenderStats(ct.Structure):
    _fields_ = [("rays", ct.c_uint64), ("positions_nominal", ct.c_uint64),
                ("positions_composited", ct.c_uint64), ("positions_trilinear", ct.c_uint64),
                ("rays_waiting", ct.c_uint64)]


def _load():
    # torch ships its own HIP runtime; loading it first makes the library's libamdhip64.so.7
    # dependency resolve to that same runtime instead of a second copy from /opt/rocm.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(hipcc, gfx950) -- there is no fallback implementation")
    L = ct.CDLL(LIB_PATH)
    vp, i32, u64, sz = ct.c_void_p, ct.c_int32, ct.c_uint64, ct.c_size_t
    L.octree_create.argtypes = [ct.POINTER(CreateParams), vp, ct.POINTER(vp)]
    L.octree_destroy.argtypes = [vp]
    L.octree_clear.argtypes = [vp, vp]
    L.octree_insert_block.argtypes = [vp, i32, ct.POINTER(i32), ct.POINTER(i32), vp, i32, vp]
    L.octree_insert_slices.argtypes = [vp, i32, i32, i32, vp, i32, vp]
    L.brick_pool_upload.argtypes = [vp, u64, vp, ct.POINTER(UploadStats)]
    L.render_views.argtypes = [vp, i32, ct.POINTER(OctView), ct.POINTER(vp), vp, vp,
                               ct.POINTER(RenderStats)]
    L.render_views_noalloc.argtypes = L.render_views.argtypes
    L.render_ckpt_bytes.restype = sz
    L.render_ckpt_bytes.argtypes = [vp, i32, ct.POINTER(OctView)]
    L.render_refine_bytes.restype = sz
    L.render_refine_bytes.argtypes = [vp, ct.POINTER(OctView)]
    L.render_views_backward.argtypes = [vp, i32, ct.POINTER(OctView), ct.POINTER(vp), vp, vp, vp,
                                        vp]
    L.octree_dump_canonical.argtypes = [vp, vp, sz, ct.POINTER(sz)]
    L.octree_read_level.argtypes = [vp, i32, vp, sz, ct.POINTER(i32)]
    L.octree_info.argtypes = [vp, ct.POINTER(i32), ct.POINTER(u64), ct.POINTER(u64)]
    L.octree_render_timing.argtypes = [vp, i32, ct.POINTER(ct.c_double), ct.POINTER(u64)]
    L.octree_build_timing.argtypes = [vp, i32, ct.POINTER(ct.c_double), ct.POINTER(ct.c_double)]
    L.octree_disk_stats.argtypes = [vp, ct.POINTER(DiskStats)]
    L.oct_last_error.restype = ct.c_char_p
    L.oct_last_error.argtypes = [vp]
    return L


lib = _load()


class OctError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"octree_rc error {code}: {msg}")
        self.code = code


def _stream(stream=None):
    """A torch.cuda.Stream, a raw hipStream_t as an int, or None (torch's current stream)."""
    if stream is not None:
        return ct.c_void_p(int(getattr(stream, "cuda_stream", stream)))
    import torch
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


_VIEW_DTYPE = np.dtype(OctView)   # the C layout of oct_view, derived from the ctypes mirror


def to_oct_views(views) -> np.ndarray:
    """Marshal synth.View-like objects into a numpy array with the C layout of oct_view (one
    vectorised fill per field; a few microseconds per view)."""
    n = len(views)
    a = np.zeros(n, _VIEW_DTYPE)
    if n == 0:
        return a
    f32 = np.float32
    a["eye"] = np.array([v.eye for v in views], f32)
    a["target"] = np.array([v.target for v in views], f32)
    a["up"] = np.array([v.up for v in views], f32)
    a["fov_y_deg"] = [v.fov_y_deg for v in views]
    a["width"] = [v.width for v in views]
    a["height"] = [v.height for v in views]
    a["tile_begin"] = [getattr(v, "tile_begin", 0) for v in views]
    a["tile_count"] = [getattr(v, "tile_count", -1) for v in views]
    a["step"] = [v.step for v in views]
    a["ert_alpha"] = [v.ert_alpha for v in views]
    a["lod"] = [v.lod for v in views]
    nc = [len(v.clips) for v in views]
    a["n_clip"] = nc
    if any(nc):             # one fill: every view's planes padded to three
        pad = (0.0, 0.0, 0.0, 0.0)
        a["clip"] = np.asarray([[tuple(pl[:4]) for pl in v.clips] + [pad] * (3 - len(v.clips))
                                for v in views], f32)
    cs = {len(v.tf_pos) for v in views}
    if len(cs) == 1:        # one stacked fill per field
        C = cs.pop()
        a["tf_pos"][:, :C] = np.asarray([v.tf_pos for v in views], f32)
        a["tf_rgba"][:, :C] = np.asarray([v.tf_rgba for v in views], f32)
        a["window"][:, :C] = np.asarray([v.window for v in views], f32)
    else:
        for k, v in enumerate(views):
            C = len(v.tf_pos)
            a["tf_pos"][k, :C] = v.tf_pos
            a["tf_rgba"][k, :C] = v.tf_rgba
            a["window"][k, :C] = v.window
    a["no_skip"] = [getattr(v, "no_skip", 0) for v in views]
    a["depth_segments"] = [getattr(v, "depth_segments", 0) for v in views]
    a["mode"] = [getattr(v, "mode", 0) for v in views]
    a["missing"] = [getattr(v, "missing", 0) for v in views]
    for k, v in enumerate(views):
        xf = getattr(v, "xform", None)
        if xf is not None:
            xf = np.asarray(xf, f32)
            a["n_xform"][k] = xf.shape[0]
            a["xform"][k, :xf.shape[0]] = xf
    return a


def to_oct_view(v) -> OctView:
    """Marshal one synth.View (or any object with the same attributes) field by field."""
    o = OctView()
    for a in range(3):
        o.eye[a], o.target[a], o.up[a] = float(v.eye[a]), float(v.target[a]), float(v.up[a])
    o.fov_y_deg = float(v.fov_y_deg)
    o.width, o.height = int(v.width), int(v.height)
    o.tile_begin, o.tile_count = int(getattr(v, "tile_begin", 0)), int(getattr(v, "tile_count", -1))
    o.step, o.ert_alpha, o.lod = float(v.step), float(v.ert_alpha), int(v.lod)
    o.n_clip = len(v.clips)
    for i, pl in enumerate(v.clips):
        for k in range(4):
            o.clip[i][k] = float(pl[k])
    pos, rgba, win = np.asarray(v.tf_pos), np.asarray(v.tf_rgba), np.asarray(v.window)
    for c in range(pos.shape[0]):
        for j in range(8):
            o.tf_pos[c][j] = float(pos[c, j])
            for q in range(4):
                o.tf_rgba[c][j][q] = float(rgba[c, j, q])
        o.window[c][0], o.window[c][1] = float(win[c, 0]), float(win[c, 1])
    o.no_skip = int(getattr(v, "no_skip", 0))
    o.depth_segments = int(getattr(v, "depth_segments", 0))
    o.mode, o.missing = int(getattr(v, "mode", 0)), int(getattr(v, "missing", 0))
    xf = getattr(v, "xform", None)
    if xf is not None:
        xf = np.asarray(xf, np.float32)
        o.n_xform = xf.shape[0]
        for c in range(xf.shape[0]):
            for a in range(3):
                for k in range(4):
                    o.xform[c][a][k] = float(xf[c, a, k])
    return o


class Octree:
    """A device-resident incrementally built multi-channel brick octree."""

    def __init__(self, dims, channels: int, brick: int, dtype: str = "u16",
                 background: float = 0.0, threshold: float = 0.0, pool_bytes: int = 0,
                 master_on_host: bool = False, stream=None, disk_path: str | None = None,
                 host_cache_bytes: int = 0, page_cells: int = 0, host_bricks: bool = False,
                 device_frames: bool = False):
        """disk_path: keep the mipmap in pages in this file with host_cache_bytes of page
        frames (the disk tier), in pinned host memory or, with device_frames, in device
        memory; master_on_host: in pinned host memory; else in HBM.
        host_bricks: keep gathered bricks in a host brick store (capped pools)."""
        p = CreateParams()
        for a in range(3):
            p.dims[a] = int(dims[a])
        p.channels, p.brick_size = int(channels), int(brick)
        p.dtype = OCT_U16 if dtype == "u16" else OCT_F32
        p.background, p.homog_threshold = float(background), float(threshold)
        p.device_pool_bytes = int(pool_bytes)
        p.host_bricks = 1 if host_bricks else 0
        if disk_path is not None:
            p.master_on_host = OCT_MASTER_DISK
            p.disk_path = os.fsencode(disk_path)
            p.host_cache_bytes = int(host_cache_bytes)
            p.page_cells = int(page_cells)
            p.disk_frames = OCT_FRAMES_DEVICE if device_frames else OCT_FRAMES_HOST
        else:
            p.master_on_host = OCT_MASTER_HOST if master_on_host else OCT_MASTER_HBM
        h = ct.c_void_p()
        rc = lib.octree_create(ct.byref(p), _stream(stream), ct.byref(h))
        if rc != OCT_OK:
            raise OctError(rc, lib.oct_last_error(None).decode())
        self.h = h
        self.dims, self.C, self.M, self.dtype = tuple(int(d) for d in dims), channels, brick, dtype
        self.pool_bytes = int(pool_bytes)          # 0: uncapped (every brick resident)
        lv, bb, ns = ct.c_int32(), ct.c_uint64(), ct.c_uint64()
        lib.octree_info(self.h, ct.byref(lv), ct.byref(bb), ct.byref(ns))
        self.levels, self.brick_bytes, self.pool_slots = lv.value, bb.value, ns.value

    def _check(self, rc: int, ok=(OCT_OK,)):
        if rc not in ok:
            raise OctError(rc, lib.oct_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            lib.octree_destroy(self.h)
            self.h = None

    __del__ = close

    def clear(self, stream=None):
        self._check(lib.octree_clear(self.h, _stream(stream)))

    def insert_block(self, channel: int, origin, data, stream=None):
        """data: planar [Cb][nz][ny][nx] torch CUDA tensor or numpy array (host)."""
        size = data.shape[1:][::-1]
        o = (ct.c_int32 * 3)(*[int(x) for x in origin])
        n = (ct.c_int32 * 3)(*[int(x) for x in size])
        ptr, dev = self._data_ptr(data)
        self._check(lib.octree_insert_block(self.h, int(channel), o, n, ptr, dev, _stream(stream)))

    def insert_slices(self, channel: int, z0: int, data, stream=None):
        ptr, dev = self._data_ptr(data)
        self._check(lib.octree_insert_slices(self.h, int(channel), int(z0), int(data.shape[1]),
                                             ptr, dev, _stream(stream)))

    def _data_ptr(self, data):
        want = np.uint16 if self.dtype == "u16" else np.float32
        if isinstance(data, np.ndarray):
            if data.dtype != want or not data.flags.c_contiguous:
                raise TypeError("block must be C-contiguous " + np.dtype(want).name)
            return ct.c_void_p(data.ctypes.data), 0
        import torch
        tw = (torch.uint16, torch.int16) if self.dtype == "u16" else (torch.float32,)
        if data.dtype not in tw or not data.is_contiguous() or not data.is_cuda:
            raise TypeError("device block must be a contiguous CUDA tensor of the volume dtype")
        return ct.c_void_p(data.data_ptr()), 1

    def upload(self, byte_budget: int = 0, stream=None) -> dict:
        st = UploadStats()
        rc = self._check(lib.brick_pool_upload(self.h, int(byte_budget), _stream(stream),
                                               ct.byref(st)), ok=(OCT_OK, OCT_INCOMPLETE))
        d = {k: getattr(st, k) for k, _ in UploadStats._fields_}
        d["complete"] = rc == OCT_OK
        return d

    @staticmethod
    def _check_buffer(t, what: str, dtype, shape=None, min_bytes=None):
        """The C ABI takes raw device pointers without sizes: check every buffer here."""
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
            raise TypeError(f"{what} must be a contiguous CUDA tensor")
        if dtype is not None and t.dtype != dtype:
            raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"{what} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        if min_bytes is not None and t.numel() * t.element_size() < min_bytes:
            raise ValueError(f"{what} holds {t.numel() * t.element_size()} bytes, "
                             f"needs {min_bytes}")

    def render(self, views, images=None, stats: bool = False, stream=None, ckpt=None,
               noalloc: bool = False, refine=None):
        """Render views into torch CUDA images [H][W][4] float32 (allocated when not given).
        noalloc=True calls render_views_noalloc (no allocation inside the library).
        refine: per view None or the refinement-state tensor of a refinement view (see
        refine_state())."""
        import torch
        if images is None:
            images = [torch.zeros((v.height, v.width, 4), dtype=torch.float32, device="cuda")
                      for v in views]
        if len(images) != len(views):
            raise ValueError("one image per view")
        f32 = torch.float32
        for k, (v, im) in enumerate(zip(views, images)):
            # one expression for the common case; the full check names what is wrong
            if not (type(im) is torch.Tensor and im.is_cuda and im.dtype is f32
                    and im.shape == (v.height, v.width, 4) and im.is_contiguous()):
                self._check_buffer(im, f"images[{k}]", f32, (v.height, v.width, 4))
        ova = to_oct_views(views)
        if refine is not None:
            if len(refine) != len(views):
                raise ValueError("one refinement state (or None) per view")
            for k, (v, r) in enumerate(zip(views, refine)):
                if r is None:
                    continue
                self._check_buffer(r, f"refine[{k}]", None, min_bytes=self.refine_bytes(v))
                ova["refine_state"][k] = r.data_ptr()
        ov = ova.ctypes.data_as(ct.POINTER(OctView))
        if ckpt is not None:
            self._check_buffer(ckpt, "ckpt", None, min_bytes=self.ckpt_bytes(views))
        ptrs = (ct.c_void_p * len(views))(*[im.data_ptr() for im in images])
        rs = RenderStats()
        fn = lib.render_views_noalloc if noalloc else lib.render_views
        self._check(fn(self.h, len(views), ov, ptrs,
                       ct.c_void_p(ckpt.data_ptr()) if ckpt is not None else None,
                       _stream(stream), ct.byref(rs) if stats else None))
        if stats:
            return images, {k: getattr(rs, k) for k, _ in RenderStats._fields_}
        return images

    def refine_bytes(self, view) -> int:
        """Bytes of refinement state one refinement view needs."""
        o = to_oct_view(view)
        return int(lib.render_refine_bytes(self.h, ct.byref(o)))

    def refine_state(self, view):
        """A zero-filled refinement state for `view` (every ray starts from its entry)."""
        import torch
        return torch.zeros(self.refine_bytes(view), dtype=torch.uint8, device="cuda")

    def ckpt_bytes(self, views) -> int:
        """Bytes of the checkpoint workspace a differentiable render of these views needs."""
        ova = to_oct_views(views)
        ov = ova.ctypes.data_as(ct.POINTER(OctView))
        return int(lib.render_ckpt_bytes(self.h, len(views), ov))

    def render_backward(self, views, dL_dimages, ckpt, dctrl, dvox=None, stream=None):
        """Accumulate dL/dctrl [n][C][8][4] (and dL/dvoxel [C][Dz][Dy][Dx]) for the loss whose
        image gradients are dL_dimages, using the workspace of the forward render."""
        import torch
        if len(dL_dimages) != len(views):
            raise ValueError("one image gradient per view")
        f32 = torch.float32
        for k, (v, g) in enumerate(zip(views, dL_dimages)):
            if not (type(g) is torch.Tensor and g.is_cuda and g.dtype is f32
                    and g.shape == (v.height, v.width, 4) and g.is_contiguous()):
                self._check_buffer(g, f"dL_dimages[{k}]", f32, (v.height, v.width, 4))
        self._check_buffer(ckpt, "ckpt", None, min_bytes=self.ckpt_bytes(views))
        self._check_buffer(dctrl, "dctrl", torch.float32, min_bytes=len(views) * self.C * 8 * 4 * 4)
        if dvox is not None:
            self._check_buffer(dvox, "dvox", torch.float32, (self.C,) + tuple(self.dims[::-1]))
        ova = to_oct_views(views)
        ov = ova.ctypes.data_as(ct.POINTER(OctView))
        gp = (ct.c_void_p * len(views))(*[g.data_ptr() for g in dL_dimages])
        self._check(lib.render_views_backward(
            self.h, len(views), ov, gp, ct.c_void_p(ckpt.data_ptr()), ct.c_void_p(dctrl.data_ptr()),
            ct.c_void_p(dvox.data_ptr()) if dvox is not None else None, _stream(stream)))

    def render_timing(self, enable: bool):
        """(total ms, launches) of the render kernels recorded so far (waits for them); then
        enable=True restarts recording from zero, False stops it."""
        ms, n = ct.c_double(), ct.c_uint64()
        self._check(lib.octree_render_timing(self.h, 1 if enable else 0, ct.byref(ms), ct.byref(n)))
        return ms.value, n.value

    def build_timing(self, enable: bool):
        """Per phase (insert, downsample, stats, gather): summed kernel ms and algorithmic
        bytes of the build work recorded so far (waits for it); then enable=True restarts
        recording from zero, False stops it."""
        ms, by = (ct.c_double * 4)(), (ct.c_double * 4)()
        self._check(lib.octree_build_timing(self.h, 1 if enable else 0, ms, by))
        return list(ms), list(by)

    def disk_stats(self) -> dict:
        """Disk-tier counters: pages, frames, hits, loads, fills, writebacks, evictions, waits,
        bytes_read, bytes_written."""
        st = DiskStats()
        self._check(lib.octree_disk_stats(self.h, ct.byref(st)))
        return {k: getattr(st, k) for k, _ in DiskStats._fields_}

    def dump(self) -> bytes:
        need = ct.c_size_t()
        lib.octree_dump_canonical(self.h, None, 0, ct.byref(need))
        buf = np.empty(need.value, np.uint8)
        self._check(lib.octree_dump_canonical(self.h, ct.c_void_p(buf.ctypes.data), need.value,
                                              ct.byref(need)))
        return buf.tobytes()

    def read_level(self, L: int) -> np.ndarray:
        ext = (ct.c_int32 * 3)()
        lib.octree_read_level(self.h, int(L), ct.c_void_p(1), 0, ext)   # size query
        ex, ey, ez = ext[0], ext[1], ext[2]
        out = np.empty((self.C, ez, ey, ex), np.uint16 if self.dtype == "u16" else np.float32)
        self._check(lib.octree_read_level(self.h, int(L), ct.c_void_p(out.ctypes.data),
                                          out.nbytes, ext))
        return out
