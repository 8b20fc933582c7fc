"""GPU parity of the other compositing and sampling modes against the FP64 oracle.

* MIP ("Basic Ray-Casting", Fig. 6, Table 1): images within 1e-4, bit-identical with skipping
  on and off and for any depth-segment count (a maximum is exact), mixed with DVR views in one
  launch, and its arg-max adjoint against the oracle's gradient.
* Full-frame fallback ("Full-Frame Ray-Casting") at partial residency against the oracle with
  the residency the library reports.
* Refinement ("Refinement Ray-Casting"): the image is written only by the pass in which no ray
  waited, and then equals the in-core image bit for bit.
* Per-channel sample transforms ("Correction of Chromatic Aberration"): DVR and MIP, u16 and
  f32, against the oracle; identity transforms and skipping on/off change no bit.
"""
import dataclasses

import numpy as np
import pytest

from paper_1407_2074_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _dev(a):
    import torch
    if a.dtype == np.uint16:
        return torch.from_numpy(np.ascontiguousarray(a).view(np.int16)).cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _full(C, dims):
    return np.full((dims[2], dims[1], dims[0]), (1 << C) - 1, np.uint8)


def _build(dims, C, M, vol, thr, dtype="u16", pool_slots=0):
    from paper_1407_2074_amd.octree import Octree
    bb = 0
    if pool_slots:
        probe = Octree(dims, C, M, dtype, 0, thr)
        bb = probe.brick_bytes
        probe.close()
    t = Octree(dims, C, M, dtype, 0, thr, pool_bytes=pool_slots * bb)
    t.insert_block(-1, (0, 0, 0), _dev(vol))
    t.upload()
    return t


def _err(gpu, ref, ok=None):
    d = np.abs(gpu.cpu().numpy().astype(np.float64) - ref)
    if ok is not None:
        d = d[ok]
    return float(d.max()) if d.size else 0.0


def _xforms(C, rng, shift=2.5, scale=0.08, rot=0.06):
    out = np.zeros((C, 3, 4), np.float32)
    for c in range(C):
        a = rng.uniform(-rot, rot)
        ca, sa = np.cos(a), np.sin(a)
        R = np.array([[ca, -sa, 0], [sa, ca, 0], [0, 0, 1]])
        out[c, :, :3] = R @ np.diag(1.0 + rng.uniform(-scale, scale, 3))
        out[c, :, 3] = rng.uniform(-shift, shift, 3)
    return out


def _missing_nodes(orc, dump):
    _, recs, _ = orc.parse_dump(dump)
    return [tuple(int(x) for x in r["head"][:4]) for r in recs
            if r["head"][4] == orc.ST_BRICK and not (r["head"][5] & orc.F_RESIDENT)]


@pytest.fixture(scope="module")
def cfg1():
    dims, C, M = (64, 64, 64), 3, 16
    return dims, C, M, synth.gen_volume(dims, C, seed=1, n_blobs=20)


# ------------------------------------------------------------------------ MIP

@pytest.mark.parametrize("thr,lod", [(205, 0), (0, -1), (205, 1)])
def test_mip_parity(orc, cfg1, thr, lod):
    import torch
    dims, C, M, vol = cfg1
    t = _build(dims, C, M, vol, thr)
    ref = orc.Tree(vol, _full(C, dims), M, 0, thr)
    v = synth.make_view(dims, C, 1, az=30.0, el=20.0, width=131, height=121, lod=lod,
                        clips=[(1.0, 0.0, 0.0, 24.0)], mode=1,
                        dist_scale=0.6 if lod < 0 else 1.0)
    (img,) = t.render([v])
    (want,) = ref.render([v])
    assert want[..., 3].max() > 0.05
    assert _err(img, want) <= TOL
    # skipping and depth segments change no bit (maxima are exact)
    for kw in (dict(no_skip=1), dict(depth_segments=1), dict(depth_segments=7)):
        w = synth.make_view(dims, C, 1, az=30.0, el=20.0, width=131, height=121, lod=lod,
                            clips=[(1.0, 0.0, 0.0, 24.0)], mode=1,
                            dist_scale=0.6 if lod < 0 else 1.0, **kw)
        (b,) = t.render([w])
        assert torch.equal(img, b), kw
    t.close()


def test_mip_f32_and_mixed_launch(orc):
    """f32 bricks; MIP and DVR views of different sizes in one launch equal their single
    launches bit for bit."""
    import torch
    dims, C, M = (40, 36, 30), 2, 8
    vol = synth.gen_volume(dims, C, seed=4, n_blobs=10, dtype="f32")
    t = _build(dims, C, M, vol, 0.0, "f32")
    ref = orc.Tree(vol, _full(C, dims), M, 0.0, 0.0)
    views = []
    for k, (mode, az) in enumerate(((1, 20.0), (0, 80.0), (1, 140.0), (0, 200.0), (1, 260.0))):
        v = synth.make_view(dims, C, 4, az=az, el=15.0, width=37 + 8 * k, height=29 + 4 * k,
                            lod=0, dtype="f32", mode=mode)
        v.tf_pos[:, 1] = 0.005
        views.append(v)
    imgs = t.render(views)
    wants = ref.render(views)
    for g, w in zip(imgs, wants):
        assert _err(g, w) <= TOL
    for v, g in zip(views, imgs):
        (one,) = t.render([v])
        assert torch.equal(one, g)
    t.close()


@pytest.mark.parametrize("dtype", ["f32", "u16"])
def test_mip_adjoint_matches_oracle(orc, dtype):
    """Gradients of an L2 loss through the arg max: table (control-point) and voxel groups
    within 1e-3 relative of the oracle, over the pixels whose maximum leads the next sample
    clearly (near-ties may pick a different position in float32)."""
    import torch
    dims, C, M = (30, 26, 22), 3, 8
    vol = synth.gen_volume(dims, C, seed=6, n_blobs=10, dtype=dtype)
    t = _build(dims, C, M, vol, 0, dtype)
    ref = orc.Tree(vol, _full(C, dims), M, 0, 0)
    v = synth.make_view(dims, C, 4, az=35.0, el=25.0, width=45, height=38, lod=0, dtype=dtype,
                        mode=1)
    v.tf_pos[:] = np.linspace(0, 1, 8, dtype=np.float32)
    for c in range(C):
        v.tf_rgba[c] = np.linspace([0.1, 0.2, 0.3, 0.05], [0.9, 0.6, 0.4, 0.6], 8)
    v.window[:, 1] = float(vol.max()) * 1.01
    want, _, mg, _ = ref.render_aux(v)
    ck = torch.zeros(t.ckpt_bytes([v]), dtype=torch.uint8, device="cuda")
    (img,) = t.render([v], ckpt=ck)
    assert _err(img, want) <= TOL
    safe = mg > 1e-4 * float(vol.max())
    assert safe.mean() > 0.8
    tgt = want * 0.5
    gI = 2 * (want - tgt) * safe[..., None]
    dctrl = torch.zeros((1, C, 8, 4), dtype=torch.float32, device="cuda")
    dvox = torch.zeros((C,) + dims[::-1], dtype=torch.float32, device="cuda")
    t.render_backward([v], [torch.from_numpy(gI.astype(np.float32)).cuda()], ck, dctrl, dvox)
    rc, rv = ref.render_grad([v], [gI])
    gc, gv = dctrl.cpu().numpy().astype(np.float64), dvox.cpu().numpy().astype(np.float64)

    def rel(a, b):
        return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))

    assert np.abs(rv).max() > 0
    assert rel(gc, rc) <= 1e-3, rel(gc, rc)
    assert rel(gv, rv) <= 1e-3, rel(gv, rv)
    t.close()


# ------------------------------------------------------------------------ full-frame fallback

def test_fullframe_fallback_matches_oracle(orc):
    """Capped pool, small upload budgets: at each partial residency the full-frame image (a
    missing brick drawn from a resident brick one or two levels up, else the AVG) equals the
    oracle with the residency the library reports; converged it equals the AVG-mode image."""
    import torch
    dims, C, M = (96, 80, 72), 3, 8
    vol = synth.gen_volume(dims, C, seed=21, n_blobs=40)
    full = _build(dims, C, M, vol, 205)
    t = _build(dims, C, M, vol, 205, pool_slots=full.pool_slots - 1)
    v = synth.make_view(dims, C, 21, az=50.0, el=25.0, width=75, height=67, lod=0, missing=1)
    v.tf_pos[:, 1] = 0.01
    fell_back = False
    for it in range(60):
        (img,) = t.render([v])
        ref = orc.Tree(vol, _full(C, dims), M, 0, 205)
        miss = _missing_nodes(orc, t.dump())
        ref.set_nonresident(miss)
        want, _, _, navg = ref.render_aux(v)
        assert _err(img, want) <= TOL, it
        _, _, _, navg0 = ref.render_aux(dataclasses.replace(v, missing=0))
        if navg.sum() < navg0.sum():
            fell_back = True    # some missing bricks were drawn from a coarser resident one
        st = t.upload(byte_budget=(40 if it else 6) * t.brick_bytes)
        if st["requests_seen"] == 0:
            break
    else:
        pytest.fail("paging did not converge")
    assert fell_back
    # converged: nothing is missing, so the one-pass AVG-mode image of the in-core tree
    v.missing, v.depth_segments = 0, 1
    (b,) = full.render([v])
    v.missing = 1
    (a,) = t.render([v])
    assert torch.equal(a, b)


# ------------------------------------------------------------------------ refinement

@pytest.mark.parametrize("mode", [0, 1])
def test_refinement_equals_in_core_image(orc, mode):
    """Rays stop at missing bricks and resume in the next pass from their cached state; the
    image is replaced only by the pass in which no ray waited, and then equals the in-core
    one-pass image bit for bit (and the oracle within 1e-4)."""
    import torch
    dims, C, M = (96, 80, 72), 3, 8
    vol = synth.gen_volume(dims, C, seed=22, n_blobs=40)
    full = _build(dims, C, M, vol, 205)
    t = _build(dims, C, M, vol, 205, pool_slots=full.pool_slots - 1)
    v = synth.make_view(dims, C, 22, az=130.0, el=-20.0, width=70, height=61, lod=0,
                        missing=2, mode=mode, ert_alpha=0.97 if mode == 0 else 1.0)
    v.tf_pos[:, 1] = 0.01
    state = t.refine_state(v)
    img = torch.full((v.height, v.width, 4), -7.0, device="cuda")
    passes = 0
    while True:
        _, st = t.render([v], images=[img], refine=[state], stats=True)
        passes += 1
        if st["rays_waiting"] == 0:
            break
        assert bool((img == -7.0).all()), "image written while rays still wait"
        t.upload(byte_budget=25 * t.brick_bytes)
        assert passes < 100
    assert passes > 2
    w = synth.make_view(dims, C, 22, az=130.0, el=-20.0, width=70, height=61, lod=0,
                        mode=mode, depth_segments=1, ert_alpha=0.97 if mode == 0 else 1.0)
    w.tf_pos[:, 1] = 0.01
    (want,) = full.render([w])
    assert torch.equal(img, want)
    ref = orc.Tree(vol, _full(C, dims), M, 0, 205)
    r, _, mg, _ = ref.render_aux(w)
    ok = mg >= 1e-5 if mode == 0 else None
    assert _err(img, r, ok) <= TOL
    # a finished state renders the same image again without marching
    img2 = torch.zeros_like(img)
    _, st = t.render([v], images=[img2], refine=[state], stats=True)
    assert st["rays_waiting"] == 0 and st["positions_composited"] == 0
    assert torch.equal(img2, img)


# ------------------------------------------------------------------------ channel transforms

@pytest.mark.parametrize("dtype,mode,lod", [("u16", 0, 0), ("u16", 1, -1), ("f32", 0, 1),
                                            ("f32", 1, 0)])
def test_channel_transforms_parity(orc, dtype, mode, lod):
    import torch
    dims, C, M = (56, 48, 40), 3, 8
    vol = synth.gen_volume(dims, C, seed=23, n_blobs=25, dtype=dtype)
    thr = 205 if dtype == "u16" else 0.0
    t = _build(dims, C, M, vol, thr, dtype)
    ref = orc.Tree(vol, _full(C, dims), M, 0, thr)
    v = synth.make_view(dims, C, 23, az=65.0, el=22.0, width=77, height=59, lod=lod,
                        dtype=dtype, mode=mode, clips=[(0.0, 0.0, 1.0, 3.0)],
                        dist_scale=0.7 if lod < 0 else 1.0)
    v.tf_pos[:, 1] = 0.01
    v.xform = _xforms(C, np.random.default_rng(5 + mode))
    (img,) = t.render([v])
    want, _, mg, _ = ref.render_aux(v)
    assert want[..., 3].max() > 0.05
    assert _err(img, want) <= TOL
    v.no_skip = 1
    (b,) = t.render([v])
    assert torch.equal(img, b)
    # the identity transform gives the plain image, bit for bit
    v.no_skip = 0
    v.xform = np.tile(np.eye(3, 4, dtype=np.float32), (C, 1, 1))
    (ident,) = t.render([v])
    v.xform = None
    v.depth_segments = 1
    (plain,) = t.render([v])
    assert torch.equal(ident, plain)
    t.close()


def test_mip_with_transforms_adjoint_matches_oracle(orc):
    import torch
    dims, C, M = (30, 26, 22), 2, 8
    vol = synth.gen_volume(dims, C, seed=7, n_blobs=10, dtype="f32")
    t = _build(dims, C, M, vol, 0, "f32")
    ref = orc.Tree(vol, _full(C, dims), M, 0, 0)
    v = synth.make_view(dims, C, 4, az=55.0, el=15.0, width=41, height=35, lod=0, dtype="f32",
                        mode=1)
    v.tf_pos[:] = np.linspace(0, 1, 8, dtype=np.float32)
    for c in range(C):
        v.tf_rgba[c] = np.linspace([0.1, 0.2, 0.3, 0.05], [0.9, 0.6, 0.4, 0.6], 8)
    v.window[:, 1] = float(vol.max()) * 1.01
    v.xform = _xforms(C, np.random.default_rng(9), shift=1.5)
    want, _, mg, _ = ref.render_aux(v)
    ck = torch.zeros(t.ckpt_bytes([v]), dtype=torch.uint8, device="cuda")
    (img,) = t.render([v], ckpt=ck)
    assert _err(img, want) <= TOL
    safe = mg > 1e-4 * float(vol.max())
    gI = 2 * (want - want * 0.5) * safe[..., None]
    dctrl = torch.zeros((1, C, 8, 4), dtype=torch.float32, device="cuda")
    dvox = torch.zeros((C,) + dims[::-1], dtype=torch.float32, device="cuda")
    t.render_backward([v], [torch.from_numpy(gI.astype(np.float32)).cuda()], ck, dctrl, dvox)
    rc, rv = ref.render_grad([v], [gI])
    for g, r in ((dctrl, rc), (dvox, rv)):
        g = g.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(g - r) <= 1e-3 * np.linalg.norm(r)
    t.close()


def test_views_that_the_adjoint_does_not_cover_are_refused(cfg1):
    import torch
    from paper_1407_2074_amd.octree import OctError
    dims, C, M, vol = cfg1
    t = _build(dims, C, M, vol, 205)
    v = synth.make_view(dims, C, 1, az=30.0, el=20.0, width=32, height=32, lod=0)
    v.xform = np.tile(np.eye(3, 4, dtype=np.float32), (C, 1, 1))
    ck = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda")
    with pytest.raises(OctError):
        t.render([v], ckpt=ck)
    v.xform, v.missing = None, 1
    with pytest.raises(OctError):
        t.render([v], ckpt=ck)
    v.missing = 2
    with pytest.raises(OctError):
        t.render([v])            # a refinement view needs its state
    t.close()
