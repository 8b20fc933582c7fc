"""FP64 CPU oracle for the brick-octree ray caster -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this package.
It shares no code with the HIP path: the C source ``oracle.c`` is compiled on its own with gcc,
and this module only marshals numpy arrays into it.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MAXC = 4
ST_NONE, ST_EMPTY, ST_HOMOG_LEAF, ST_HOMOG, ST_BRICK = -1, 0, 1, 2, 3
F_HAS_CHILDREN, F_COMPLETE, F_POPULATED, F_RESIDENT = 1, 2, 4, 8


def num_threads() -> int:
    """OpenMP threads the oracle's renderer uses."""
    return int(lib().orc_num_threads())


def build(force: bool = True) -> str:
    """Compile the oracle (gcc, OpenMP, no floating-point contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ct.Structure):
    _fields_ = [("dims", ct.c_int32 * 3), ("channels", ct.c_int32), ("brick", ct.c_int32),
                ("dtype", ct.c_int32), ("background", ct.c_double), ("threshold", ct.c_double)]


class OrcView(ct.Structure):
    _fields_ = [("eye", ct.c_float * 3), ("target", ct.c_float * 3), ("up", ct.c_float * 3),
                ("fov_y_deg", ct.c_float), ("width", ct.c_int32), ("height", ct.c_int32),
                ("step", ct.c_float), ("ert_alpha", ct.c_float), ("lod", ct.c_int32),
                ("n_clip", ct.c_int32), ("clip", (ct.c_float * 4) * 3),
                ("tf_pos", (ct.c_float * 8) * MAXC), ("tf_rgba", ((ct.c_float * 4) * 8) * MAXC),
                ("window", (ct.c_float * 2) * MAXC), ("mode", ct.c_int32),
                ("fullframe", ct.c_int32), ("n_xform", ct.c_int32),
                ("xform", ((ct.c_float * 4) * 3) * MAXC)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ct.CDLL(_LIB)
        L.orc_build.restype = ct.c_void_p
        L.orc_build.argtypes = [ct.POINTER(_Params), ct.c_void_p, ct.c_void_p]
        L.orc_free.argtypes = [ct.c_void_p]
        L.orc_num_levels.argtypes = [ct.c_void_p]
        L.orc_tree_depth.argtypes = [ct.POINTER(ct.c_int32), ct.c_int]
        L.orc_level_extent.argtypes = [ct.c_void_p, ct.c_int, ct.c_void_p]
        L.orc_read_level.argtypes = [ct.c_void_p, ct.c_int, ct.c_void_p]
        L.orc_dump.restype = ct.c_size_t
        L.orc_dump.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_size_t]
        L.orc_render.argtypes = [ct.c_void_p, ct.c_int, ct.POINTER(OrcView), ct.c_void_p,
                                 ct.c_void_p, ct.c_void_p]
        L.orc_render_grad.argtypes = [ct.c_void_p, ct.c_int, ct.POINTER(OrcView), ct.c_void_p,
                                      ct.c_void_p, ct.c_void_p]
        L.orc_rays.argtypes = [ct.c_void_p, ct.POINTER(OrcView), ct.c_void_p, ct.c_void_p]
        L.orc_render_aux.argtypes = [ct.c_void_p, ct.POINTER(OrcView), ct.c_void_p, ct.c_void_p,
                                     ct.c_void_p, ct.c_void_p]
        L.orc_render_pixels.argtypes = [ct.c_void_p, ct.POINTER(OrcView), ct.c_void_p,
                                        ct.c_int64, ct.c_void_p, ct.c_void_p, ct.c_void_p]
        L.orc_render_rows.argtypes = [ct.c_void_p, ct.POINTER(OrcView), ct.c_void_p,
                                      ct.c_void_p, ct.c_int, ct.c_int]
        L.orc_render_window.argtypes = [ct.c_void_p, ct.POINTER(OrcView), ct.c_void_p, ct.c_int,
                                        ct.c_int, ct.c_int, ct.c_int]
        L.orc_poke_level0.argtypes = [ct.c_void_p, ct.c_int, ct.c_int, ct.c_int, ct.c_int,
                                      ct.c_double]
        L.orc_num_threads.restype = ct.c_int
        L.orc_node_info.argtypes = [ct.c_void_p, ct.c_int, ct.c_int, ct.c_int, ct.c_int,
                                    ct.c_void_p, ct.c_void_p, ct.c_void_p]
        L.orc_set_nonresident.argtypes = [ct.c_void_p, ct.c_int, ct.c_int, ct.c_int, ct.c_int,
                                          ct.c_int]
        _lib = L
    return _lib


def to_orc_view(v) -> OrcView:
    """Marshal any object with the View attributes (eye, target, up, width, ...)."""
    o = OrcView()
    for a in range(3):
        o.eye[a], o.target[a], o.up[a] = float(v.eye[a]), float(v.target[a]), float(v.up[a])
    o.fov_y_deg = float(v.fov_y_deg)
    o.width, o.height = int(v.width), int(v.height)
    o.step, o.ert_alpha, o.lod = float(v.step), float(v.ert_alpha), int(v.lod)
    o.n_clip = len(v.clips)
    for i, pl in enumerate(v.clips):
        for k in range(4):
            o.clip[i][k] = float(pl[k])
    C = np.asarray(v.tf_pos).shape[0]
    for c in range(C):
        for j in range(8):
            o.tf_pos[c][j] = float(v.tf_pos[c][j])
            for q in range(4):
                o.tf_rgba[c][j][q] = float(v.tf_rgba[c][j][q])
        o.window[c][0], o.window[c][1] = float(v.window[c][0]), float(v.window[c][1])
    o.mode = int(getattr(v, "mode", 0))
    o.fullframe = 1 if int(getattr(v, "missing", 0)) == 1 else 0
    xf = getattr(v, "xform", None)
    if xf is not None:
        xf = np.asarray(xf, np.float32)
        assert xf.shape == (C, 3, 4)
        o.n_xform = C
        for c in range(C):
            for a in range(3):
                for k in range(4):
                    o.xform[c][a][k] = float(xf[c, a, k])
    return o


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ct.c_void_p)


class Tree:
    """The oracle's octree over a fully specified level-0 volume and insertion mask.

    v0:   planar [C][Dz][Dy][Dx] uint16 or float32 (background where nothing was inserted)
    mask: [Dz][Dy][Dx] uint8, bit c set where channel c was inserted
    """

    def __init__(self, v0: np.ndarray, mask: np.ndarray, brick: int, background: float = 0.0,
                 threshold: float = 0.0):
        v0 = np.ascontiguousarray(v0)
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        C, Dz, Dy, Dx = v0.shape
        assert mask.shape == (Dz, Dy, Dx)
        self.dtype = "u16" if v0.dtype == np.uint16 else "f32"
        assert v0.dtype in (np.uint16, np.float32)
        p = _Params()
        p.dims[0], p.dims[1], p.dims[2] = Dx, Dy, Dz
        p.channels, p.brick = C, brick
        p.dtype = 0 if self.dtype == "u16" else 1
        p.background, p.threshold = float(background), float(threshold)
        self._keep = (v0, mask)
        self.h = lib().orc_build(ct.byref(p), _ptr(v0), _ptr(mask))
        if not self.h:
            raise ValueError("oracle rejected the parameters")
        self.C, self.dims, self.M = C, (Dx, Dy, Dz), brick
        self.levels = lib().orc_num_levels(self.h)
        self.N = self.levels - 1

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_free(self.h)
            self.h = None

    def extent(self, L: int):
        e = np.zeros(3, np.int32)
        lib().orc_level_extent(self.h, L, _ptr(e))
        return tuple(int(x) for x in e)

    def level(self, L: int) -> np.ndarray:
        ex, ey, ez = self.extent(L)
        out = np.empty((self.C, ez, ey, ex), np.uint16 if self.dtype == "u16" else np.float32)
        assert lib().orc_read_level(self.h, L, _ptr(out)) == 0
        return out

    def dump(self) -> bytes:
        need = lib().orc_dump(self.h, None, 0)
        if need == 0:
            raise ValueError("no dump after an in-place level-0 replacement")
        buf = np.empty(need, np.uint8)
        lib().orc_dump(self.h, _ptr(buf), need)
        return buf.tobytes()

    def node(self, L: int, bx: int, by: int, bz: int):
        st, fl = np.zeros(1, np.int32), np.zeros(1, np.int32)
        avg = np.zeros(MAXC, np.float64)
        assert lib().orc_node_info(self.h, L, bx, by, bz, _ptr(st), _ptr(fl), _ptr(avg)) == 0
        return int(st[0]), int(fl[0]), avg[:self.C].copy()

    def set_nonresident(self, nodes, nonresident: bool = True):
        """Mark brick nodes (level, bx, by, bz) whose brick the renderer does not have: they
        are sampled with their AVG."""
        for (L, bx, by, bz) in nodes:
            assert lib().orc_set_nonresident(self.h, int(L), int(bx), int(by), int(bz),
                                             1 if nonresident else 0) == 0

    def render(self, views, want_info: bool = False):
        """Images [H][W][4] float64 per view (plus nominal sample counts and ERT margins)."""
        ov = (OrcView * len(views))(*[to_orc_view(v) for v in views])
        imgs = [np.zeros((v.height, v.width, 4), np.float64) for v in views]
        ns = [np.zeros((v.height, v.width), np.int32) for v in views]
        mg = [np.zeros((v.height, v.width), np.float64) for v in views]
        P = ct.c_void_p * len(views)
        rc = lib().orc_render(self.h, len(views), ov, P(*[i.ctypes.data for i in imgs]),
                              P(*[a.ctypes.data for a in ns]), P(*[a.ctypes.data for a in mg]))
        if rc != 0:
            raise ValueError("oracle render rejected the views")
        return (imgs, ns, mg) if want_info else imgs

    def render_aux(self, view):
        """One view: image, nominal counts, margins (ERT / MIP arg-max ambiguity) and the
        number of channel samples that approximated a non-resident brick by its AVG."""
        ov = to_orc_view(view)
        img = np.zeros((view.height, view.width, 4), np.float64)
        ns = np.zeros((view.height, view.width), np.int32)
        mg = np.zeros((view.height, view.width), np.float64)
        na = np.zeros((view.height, view.width), np.int32)
        if lib().orc_render_aux(self.h, ct.byref(ov), _ptr(img), _ptr(ns), _ptr(mg),
                                _ptr(na)) != 0:
            raise ValueError("oracle render rejected the view")
        return img, ns, mg, na

    def render_pixels(self, view, px, want_info: bool = False):
        """RGBA of the listed pixels (px: [n][2] column, row) of one view (plus their nominal
        counts and margins)."""
        ov = to_orc_view(view)
        px = np.ascontiguousarray(px, np.int32)
        out = np.zeros((len(px), 4), np.float64)
        ns = np.zeros(len(px), np.int32)
        mg = np.zeros(len(px), np.float64)
        if lib().orc_render_pixels(self.h, ct.byref(ov), _ptr(px), len(px), _ptr(out), _ptr(ns),
                                   _ptr(mg)) != 0:
            raise ValueError("oracle render rejected the pixels")
        return (out, ns, mg) if want_info else out

    def render_grad(self, views, dL_dI, want_voxels: bool = True):
        """Gradient of a loss with image adjoints dL_dI w.r.t. control RGBA and level-0 voxels."""
        ov = (OrcView * len(views))(*[to_orc_view(v) for v in views])
        gI = [np.ascontiguousarray(g, dtype=np.float64) for g in dL_dI]
        dctrl = np.zeros((len(views), self.C, 8, 4), np.float64)
        Dx, Dy, Dz = self.dims
        dvox = np.zeros((self.C, Dz, Dy, Dx), np.float64) if want_voxels else None
        P = ct.c_void_p * len(views)
        if lib().orc_render_grad(self.h, len(views), ov, P(*[g.ctypes.data for g in gI]),
                                 _ptr(dctrl), _ptr(dvox) if dvox is not None else None) != 0:
            raise ValueError("oracle gradient rejected the views")
        return dctrl, dvox

    def render_rows(self, view, row_begin: int, row_step: int):
        """Render only rows row_begin, row_begin + row_step, ... of one view.  Returns the image
        (other rows zero) and the nominal sample count per pixel."""
        ov = to_orc_view(view)
        img = np.zeros((view.height, view.width, 4), np.float64)
        ns = np.zeros((view.height, view.width), np.int32)
        if lib().orc_render_rows(self.h, ct.byref(ov), _ptr(img), _ptr(ns), row_begin,
                                 row_step) != 0:
            raise ValueError("oracle render rejected the view")
        return img, ns

    def poke_level0(self, c: int, x: int, y: int, z: int, value: float):
        """Replace one level-0 value in place (threshold 0, brick node): for finite differences
        of LOD-0 renders; afterwards only LOD-0 renders and gradients are allowed."""
        if lib().orc_poke_level0(self.h, int(c), int(x), int(y), int(z), float(value)) != 0:
            raise ValueError("oracle refused the level-0 replacement")

    def render_window(self, view, x0: int, y0: int, x1: int, y1: int):
        """Render only the pixels x0 <= i < x1, y0 <= j < y1 (others zero)."""
        ov = to_orc_view(view)
        img = np.zeros((view.height, view.width, 4), np.float64)
        if lib().orc_render_window(self.h, ct.byref(ov), _ptr(img), int(x0), int(y0), int(x1),
                                   int(y1)) != 0:
            raise ValueError("oracle render rejected the window")
        return img

    def rays(self, view):
        ov = to_orc_view(view)
        out = np.zeros((view.height, view.width, 8), np.float32)
        lh = np.zeros((view.height, view.width, 2), np.int32)
        lib().orc_rays(self.h, ct.byref(ov), _ptr(out), _ptr(lh))
        return out, lh


def tree_depth(dims, brick: int) -> int:
    """N of Eq. 1 for these dimensions and brick size (no volume needed)."""
    d = (ct.c_int32 * 3)(*[int(x) for x in dims])
    return int(lib().orc_tree_depth(d, int(brick)))


def apply_inserts(dims, channels: int, inserts, dtype="u16", background=0.0):
    """Compose the level-0 volume and insertion mask from a list of inserts, in order.

    Each insert is (channel or -1 for all, (x0, y0, z0), block) with block planar
    [C or 1][nz][ny][nx].  Later inserts overwrite earlier ones."""
    Dx, Dy, Dz = dims
    npdt = np.uint16 if dtype == "u16" else np.float32
    v0 = np.full((channels, Dz, Dy, Dx), background, dtype=npdt)
    mask = np.zeros((Dz, Dy, Dx), np.uint8)
    for ch, (x0, y0, z0), blk in inserts:
        blk = np.asarray(blk)
        nz, ny, nx = blk.shape[1:]
        sl = (slice(z0, z0 + nz), slice(y0, y0 + ny), slice(x0, x0 + nx))
        chans = range(channels) if ch < 0 else [ch]
        for k, c in enumerate(chans):
            v0[(c,) + sl] = blk[k]
            mask[sl] |= np.uint8(1 << c)
    return v0, mask


def parse_dump(buf: bytes):
    """Split a canonical dump into (header dict, node records array, brick bytes)."""
    assert buf[:8] == b"OCTDUMP1", buf[:8]
    h = np.frombuffer(buf, np.int32, 9, 8)
    hdr = dict(dims=tuple(h[:3]), C=int(h[3]), M=int(h[4]), N=int(h[5]), dtype=int(h[6]),
               n_nodes=int(h[7]), n_bricks=int(h[8]))
    rec_t = np.dtype([("head", np.int32, 8), ("avg", np.float64, 4), ("bmin", np.float64, 4),
                      ("bmax", np.float64, 4), ("smin", np.float64, 4), ("smax", np.float64, 4)])
    assert rec_t.itemsize == 192
    recs = np.frombuffer(buf, rec_t, hdr["n_nodes"], 64)
    bricks = buf[64 + 192 * hdr["n_nodes"]:]
    return hdr, recs, bricks
