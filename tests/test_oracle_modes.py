"""Pins for the oracle's other compositing and sampling modes (CPU only).

* Maximum intensity projection ("Basic Ray-Casting": the traversal serves other compositing
  modes too; Fig. 6 and Table 1 render every data set in MIP): closed form on a constant
  volume, a regular-grid brute force, early termination not applying, and central differences
  for its arg-max adjoint.
* Full-frame fallback ("Full-Frame Ray-Casting"): a missing brick is drawn from the resident
  brick of one of the two coarser levels, else its AVG -- against plain renders at the coarser
  LOD, a per-sample brute force over a random residency, and the paper's statement that no AVG
  is used while the bricks two levels up fit (1/64 of the data).
* Chromatic-aberration correction ("Correction of Chromatic Aberration"): per-channel affine
  sample positions -- identity = no transform, brute force with random affine maps, and
  central differences of the adjoint.
"""
import numpy as np
import pytest

from helpers import bf_render_dense, bf_render_general, np_lut, np_mip
from paper_1407_2074_amd import synth


def _full(C, dims):
    Dx, Dy, Dz = dims
    return np.full((Dz, Dy, Dx), (1 << C) - 1, np.uint8)


def _bright(v):
    v.tf_pos[:, 1] = 0.005
    return v


def _brick_nodes(orc, t):
    hdr, recs, _ = orc.parse_dump(t.dump())
    return [tuple(int(x) for x in r["head"][:4]) for r in recs if r["head"][4] == orc.ST_BRICK]


def _xforms(C, rng, shift=2.5, scale=0.08, rot=0.06):
    out = np.zeros((C, 3, 4), np.float32)
    for c in range(C):
        a = rng.uniform(-rot, rot)
        ca, sa = np.cos(a), np.sin(a)
        R = np.array([[ca, -sa, 0], [sa, ca, 0], [0, 0, 1]])
        S = np.diag(1.0 + rng.uniform(-scale, scale, 3))
        out[c, :, :3] = R @ S
        out[c, :, 3] = rng.uniform(-shift, shift, 3)
    return out


# ------------------------------------------------------------------------ MIP

def test_mip_constant_volume_closed_form(orc):
    """Every sample of channel c equals v_c, so a hit pixel is the composite of the C
    classified constants in channel order; missed pixels stay zero."""
    dims, C = (20, 16, 12), 3
    vals = np.array([700, 1900, 3300], np.uint16)
    v0 = np.empty((C, 12, 16, 20), np.uint16)
    for c in range(C):
        v0[c] = vals[c]
    t = orc.Tree(v0, _full(C, dims), 4, 0, 1)
    v = synth.make_view(dims, C, 1, az=30, el=25, width=24, height=20, mode=1)
    img, ns, _, _ = t.render_aux(v)
    hit = ns > 0
    assert hit.any() and (~hit).any()
    A, col = 0.0, np.zeros(3)
    for c in range(C):
        lut = np_lut(v.tf_pos[c], v.tf_rgba[c])
        lo, hi = float(v.window[c][0]), float(v.window[c][1])
        u = 255.0 * ((float(vals[c]) - lo) / (hi - lo))
        i = min(int(np.floor(u)), 254)
        rgba = lut[i] + (u - i) * (lut[i + 1] - lut[i])
        w = (1 - A) * rgba[3]
        col += w * rgba[:3]
        A += w
    assert A > 0.01
    assert np.abs(img[hit][:, :3] - col).max() < 1e-14
    assert np.abs(img[hit][:, 3] - A).max() < 1e-14
    assert not img[~hit].any()


@pytest.mark.parametrize("lod", [0, 1, -1])
def test_mip_dense_bruteforce(orc, lod):
    dims, M, C = (30, 22, 17), 4, 3
    vol = synth.gen_volume(dims, C, seed=5, n_blobs=6)
    t = orc.Tree(vol, _full(C, dims), M, 0, 0)
    v = _bright(synth.make_view(dims, C, 1, az=37.0, el=18.0, width=40, height=33, lod=lod,
                                clips=[(1.0, 0.0, 0.0, 6.0)],
                                dist_scale=0.7 if lod < 0 else 1.0, mode=1))
    (img,) = t.render([v])
    ref = bf_render_general(np_mip(vol, M), dims, v, t.N)
    assert img[..., 3].max() > 0.05
    assert np.max(np.abs(img - ref)) < 1e-10
    # MIP differs from DVR on the same inputs, and early termination does not apply to it
    v.mode = 0
    (dvr,) = t.render([v])
    assert np.abs(dvr - img).max() > 1e-3
    v.mode, v.ert_alpha = 1, 0.3
    (img_ert,) = t.render([v])
    assert np.array_equal(img_ert, img)


def test_mip_adjoint_matches_central_differences(orc):
    """Arg-max adjoint vs central differences of the FP64 MIP forward, over the pixels whose
    largest sample leads the next one by more than twice the perturbation (there the arg max
    cannot move): 20 control-point components and 20 voxels."""
    dims, M, C = (14, 12, 10), 4, 2
    vol = synth.gen_volume(dims, C, seed=3, n_blobs=6, dtype="f32")
    rng = np.random.default_rng(1)
    v = synth.make_view(dims, C, 4, az=30, el=20, width=14, height=12, dtype="f32", mode=1)
    v.tf_pos[:] = np.linspace(0, 1, 8, dtype=np.float32)
    for c in range(C):
        v.tf_rgba[c] = np.linspace([0.1, 0.2, 0.3, 0.05], [0.9, 0.6, 0.4, 0.6], 8)
    v.window[:, 1] = float(vol.max()) * 1.01
    eps = 2e-5

    def loss(vv, vol_):
        t = orc.Tree(vol_, _full(C, dims), M, 0, 0)
        img, _, mg, _ = t.render_aux(vv)
        return t, img, mg

    t, img, mg = loss(v, vol)
    safe = mg > 4 * eps
    assert safe.mean() > 0.5
    tgt = np.zeros_like(img)
    w = safe[..., None].astype(np.float64)

    def L(img_):
        return float((w * (img_ - tgt) ** 2).sum())

    dctrl, dvox = t.render_grad([v], [2 * w * (img - tgt)])
    for _ in range(20):
        c, j, q = rng.integers(C), rng.integers(8), rng.integers(4)
        x = float(v.tf_rgba[c, j, q])
        hi, lo = np.float32(x + 1e-3), np.float32(x - 1e-3)
        v.tf_rgba[c, j, q] = hi
        Lp = L(loss(v, vol)[1])
        v.tf_rgba[c, j, q] = lo
        Lm = L(loss(v, vol)[1])
        v.tf_rgba[c, j, q] = x
        fd = (Lp - Lm) / (float(hi) - float(lo))
        assert abs(fd - dctrl[0, c, j, q]) <= 1e-4 * max(abs(fd), 1e-2), (c, j, q, fd)
    flat = np.argsort(-np.abs(dvox).ravel())[:100]
    assert np.abs(dvox).max() > 0
    for k in rng.choice(flat, 20, replace=False):
        idx = np.unravel_index(k, dvox.shape)
        x = float(vol[idx])
        vol[idx] = np.float32(x + eps)
        hi = float(vol[idx])
        Lp = L(loss(v, vol)[1])
        vol[idx] = np.float32(x - eps)
        lo = float(vol[idx])
        Lm = L(loss(v, vol)[1])
        vol[idx] = np.float32(x)
        fd = (Lp - Lm) / (hi - lo)
        assert abs(fd - dvox[idx]) <= 1e-4 * max(abs(fd), 1e-3), (idx, fd, dvox[idx])


# ------------------------------------------------------------------------ full-frame fallback

def test_fullframe_with_everything_resident_is_the_plain_render(orc):
    dims, M, C = (24, 20, 16), 4, 2
    vol = synth.gen_volume(dims, C, seed=6, n_blobs=5)
    t = orc.Tree(vol, _full(C, dims), M, 0, 205)
    v = _bright(synth.make_view(dims, C, 1, az=50, el=20, width=22, height=18, lod=0))
    (a,) = t.render([v])
    v.missing = 1
    (b,) = t.render([v])
    assert np.array_equal(a, b)


def test_fullframe_falls_back_to_the_two_coarser_levels(orc):
    """LOD 0 with every level-0 brick missing draws the level-1 bricks: the image is the
    LOD-1 image (bit for bit) and the regular-grid LOD-1 brute force; with levels 0 and 1
    missing it is the LOD-2 image; with levels 0-2 missing every sample is the level-0 node's
    AVG, as without the fallback."""
    dims, M, C = (32, 28, 24), 4, 2
    vol = synth.gen_volume(dims, C, seed=7, n_blobs=6)
    levels = np_mip(vol, M)
    t = orc.Tree(vol, _full(C, dims), M, 0, 0)
    assert t.N == 3
    nodes = _brick_nodes(orc, t)
    v = _bright(synth.make_view(dims, C, 2, az=35, el=25, width=26, height=22, lod=0,
                                missing=1))
    ref = {}
    for lod in (1, 2):
        w = synth.make_view(dims, C, 2, az=35, el=25, width=26, height=22, lod=lod)
        _bright(w)
        ref[lod] = t.render([w])[0]
    for gone, want in (((0,), 1), ((0, 1), 2)):
        t.set_nonresident([n for n in nodes if n[0] in gone])
        img, _, _, navg = t.render_aux(v)
        assert np.array_equal(img, ref[want])
        w = _bright(synth.make_view(dims, C, 2, az=35, el=25, width=26, height=22, lod=want))
        assert np.abs(img - bf_render_dense(levels, dims, w, t.N)).max() < 1e-10
        assert not navg.any()
        t.set_nonresident(nodes, False)
    t.set_nonresident([n for n in nodes if n[0] <= 2])
    img, ns, _, navg = t.render_aux(v)
    v.missing = 0
    img_avg, _, _, navg0 = t.render_aux(v)
    assert np.array_equal(img, img_avg)
    assert np.array_equal(navg, navg0) and np.array_equal(navg, C * ns)


def test_fullframe_random_residency_bruteforce(orc):
    """Random residency over levels 0-2: each sample comes from its level-0 brick if resident,
    else the level-1, else the level-2 brick on its path, else the level-0 node's AVG."""
    dims, M, C = (30, 26, 20), 4, 2
    vol = synth.gen_volume(dims, C, seed=8, n_blobs=6)
    levels = np_mip(vol, M)
    t = orc.Tree(vol, _full(C, dims), M, 0, 0)
    rng = np.random.default_rng(3)
    nodes = _brick_nodes(orc, t)
    gone = {n for n in nodes if n[0] <= 2 and rng.random() < 0.6}
    t.set_nonresident(sorted(gone))
    v = _bright(synth.make_view(dims, C, 3, az=125, el=-20, width=24, height=20, lod=0,
                                missing=1))
    img, _, _, navg = t.render_aux(v)
    ref = bf_render_general(levels, dims, v, t.N, M, resident=lambda *n: n not in gone)
    assert img[..., 3].max() > 0.02
    assert np.abs(img - ref).max() < 1e-10
    assert navg.any()      # some samples had no resident brick on their path
    v.missing = 0
    img0 = t.render([v])[0]
    ref0 = bf_render_general(levels, dims, v, t.N, M, resident=lambda *n: n not in gone)
    assert np.abs(img0 - ref0).max() < 1e-10
    assert np.abs(img0 - img).max() > 1e-4


def test_fullframe_needs_no_avg_once_bricks_two_levels_up_fit(orc):
    """"No AVG values are used as long as at least 1/64th of the data set size fits into the
    brick buffer": with only the bricks of levels >= 2 resident -- about 1/64 of the level-0
    bricks plus the levels above -- a full-frame render at LOD 0 draws no AVG."""
    dims, M, C = (64, 64, 64), 4, 1
    vol = synth.gen_volume(dims, C, seed=9, n_blobs=8)
    t = orc.Tree(vol, _full(C, dims), M, 0, 0)
    nodes = _brick_nodes(orc, t)
    n0 = sum(1 for n in nodes if n[0] == 0)
    kept = [n for n in nodes if n[0] >= 2]
    assert len(kept) <= n0 / 64 * 8 / 7 + 1
    t.set_nonresident([n for n in nodes if n[0] < 2])
    v = _bright(synth.make_view(dims, C, 1, az=20, el=30, width=32, height=32, lod=0,
                                missing=1))
    img, ns, _, navg = t.render_aux(v)
    assert ns.sum() > 0 and not navg.any()
    v.missing = 0
    _, _, _, navg0 = t.render_aux(v)
    assert navg0.sum() == ns.sum()    # without the fallback every sample is an AVG


# ------------------------------------------------------------------------ channel transforms

def test_identity_channel_transforms_change_nothing(orc):
    dims, M, C = (26, 22, 18), 4, 3
    vol = synth.gen_volume(dims, C, seed=10, n_blobs=6)
    t = orc.Tree(vol, _full(C, dims), M, 0, 205)
    v = _bright(synth.make_view(dims, C, 1, az=40, el=15, width=24, height=20, lod=-1,
                                clips=[(0.0, 1.0, 0.0, 5.0)]))
    (a,) = t.render([v])
    v.xform = np.tile(np.eye(3, 4, dtype=np.float32), (C, 1, 1))
    (b,) = t.render([v])
    assert np.array_equal(a, b)
    v.mode = 1
    (c,) = t.render([v])
    v.xform = None
    (d,) = t.render([v])
    assert np.array_equal(c, d)


@pytest.mark.parametrize("mode,lod", [(0, 0), (0, 1), (1, 0), (0, -1)])
def test_channel_transforms_dense_bruteforce(orc, mode, lod):
    dims, M, C = (30, 24, 20), 4, 3
    vol = synth.gen_volume(dims, C, seed=11, n_blobs=7)
    t = orc.Tree(vol, _full(C, dims), M, 0, 0)
    v = _bright(synth.make_view(dims, C, 1, az=65.0, el=22.0, width=30, height=26, lod=lod,
                                mode=mode, dist_scale=0.75 if lod < 0 else 1.0,
                                clips=[(0.0, 0.0, 1.0, 3.0)]))
    v.xform = _xforms(C, np.random.default_rng(lod + 5 * mode + 7))
    (img,) = t.render([v])
    ref = bf_render_general(np_mip(vol, M), dims, v, t.N)
    assert img[..., 3].max() > 0.05
    assert np.max(np.abs(img - ref)) < 1e-10
    v.xform = None
    (plain,) = t.render([v])
    assert np.abs(plain - img).max() > 1e-3


def test_channel_transform_adjoint_matches_central_differences(orc):
    dims, M, C = (12, 10, 8), 4, 2
    vol = synth.gen_volume(dims, C, seed=12, n_blobs=5, dtype="f32")
    rng = np.random.default_rng(2)
    v = synth.make_view(dims, C, 4, az=30, el=20, width=12, height=10, dtype="f32")
    v.tf_pos[:] = np.linspace(0, 1, 8, dtype=np.float32)
    for c in range(C):
        v.tf_rgba[c] = np.linspace([0.1, 0.2, 0.3, 0.0], [0.9, 0.6, 0.4, 0.3], 8)
    v.window[:, 1] = float(vol.max()) * 1.01
    v.xform = _xforms(C, rng, shift=1.5)
    tgt = np.zeros((10, 12, 4))

    def L(vol_):
        t = orc.Tree(vol_, _full(C, dims), M, 0, 0)
        (img,) = t.render([v])
        return t, img, float(((img - tgt) ** 2).sum())

    t, img, _ = L(vol)
    _, dvox = t.render_grad([v], [2 * (img - tgt)])
    eps = 1e-3
    flat = np.argsort(-np.abs(dvox).ravel())[:100]
    for k in rng.choice(flat, 20, replace=False):
        idx = np.unravel_index(k, dvox.shape)
        x = float(vol[idx])
        vol[idx] = np.float32(x + eps)
        hi = float(vol[idx])
        Lp = L(vol)[2]
        vol[idx] = np.float32(x - eps)
        lo = float(vol[idx])
        Lm = L(vol)[2]
        vol[idx] = np.float32(x)
        fd = (Lp - Lm) / (hi - lo)
        assert abs(fd - dvox[idx]) <= 1e-4 * max(abs(fd), 1e-3), (idx, fd, dvox[idx])


def test_listed_pixels_equal_the_full_render(orc):
    dims, M, C = (24, 20, 16), 4, 3
    vol = synth.gen_volume(dims, C, seed=13, n_blobs=5)
    t = orc.Tree(vol, _full(C, dims), M, 0, 205)
    v = _bright(synth.make_view(dims, C, 1, az=70, el=10, width=21, height=17, lod=-1,
                                mode=1))
    (full,) = t.render([v])
    rng = np.random.default_rng(4)
    px = np.stack([rng.integers(0, 21, 60), rng.integers(0, 17, 60)], -1)
    out = t.render_pixels(v, px)
    assert np.array_equal(out, full[px[:, 1], px[:, 0]])
