"""GPU parity of the adjoint: gradients of an L2 image loss with respect to the control-point
RGBA values and the level-0 voxels, against the FP64 oracle's reverse-mode gradient and against
central finite differences (eps 1e-3) of the FP64 oracle forward."""
import numpy as np
import pytest

from paper_1407_2074_amd import synth

pytestmark = pytest.mark.gpu


def _full(C, dims):
    return np.full((dims[2], dims[1], dims[0]), (1 << C) - 1, np.uint8)


def _tree(dims, C, M, vol, dtype="f32"):
    from paper_1407_2074_amd.octree import Octree
    t = Octree(dims, C, M, dtype, 0.0, 0.0)
    t.insert_block(-1, (0, 0, 0), vol)
    t.upload()
    return t


def _views(dims, C, n, w, h, seed=4, dtype="f32"):
    rng = np.random.default_rng(seed)
    vs = []
    for i in range(n):
        v = synth.make_view(dims, C, seed, az=float(rng.uniform(0, 360)),
                            el=float(rng.uniform(-40, 40)), width=w, height=h, dtype=dtype)
        v.tf_pos[:, 1] = 0.01
        v.tf_rgba[:, 2:, 3] = 0.15
        vs.append(v)
    return vs


def _gpu_grads(t, views, dL, want_vox=True, ck_out=None):
    import torch
    ck = torch.zeros(t.ckpt_bytes(views), dtype=torch.uint8, device="cuda")
    imgs = t.render(views, ckpt=ck)
    g = [torch.from_numpy(x.astype(np.float32)).cuda() for x in dL(imgs)]
    dctrl = torch.zeros((len(views), t.C, 8, 4), dtype=torch.float32, device="cuda")
    Dx, Dy, Dz = t.dims
    dvox = torch.zeros((t.C, Dz, Dy, Dx), dtype=torch.float32, device="cuda") if want_vox else None
    t.render_backward(views, g, ck, dctrl, dvox)
    torch.cuda.synchronize()
    if ck_out is not None:
        ck_out.append(ck.cpu().numpy())
    return imgs, dctrl.cpu().numpy(), (dvox.cpu().numpy() if want_vox else None)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_adjoint_matches_oracle_gradient(orc):
    dims, C, M = (40, 36, 30), 3, 16
    vol = synth.gen_volume(dims, C, seed=4, n_blobs=10, dtype="f32")
    t = _tree(dims, C, M, vol)
    views = _views(dims, C, 2, 48, 40)
    rng = np.random.default_rng(1)
    tgt = [rng.uniform(0, 0.3, size=(v.height, v.width, 4)) for v in views]

    def dL(imgs):
        return [2 * (im.cpu().numpy().astype(np.float64) - g) for im, g in zip(imgs, tgt)]

    imgs, dctrl, dvox = _gpu_grads(t, views, dL)
    ref = orc.Tree(vol, _full(C, dims), M, 0.0, 0.0)
    want = ref.render(views)
    gI = [2 * (w - g) for w, g in zip(want, tgt)]
    rc, rv = ref.render_grad(views, gI)
    assert _rel(dctrl, rc) <= 1e-3, _rel(dctrl, rc)
    assert _rel(dvox, rv) <= 1e-3, _rel(dvox, rv)
    for c in range(C):        # each channel's group on its own
        assert _rel(dctrl[:, c], rc[:, c]) <= 1e-3
        assert _rel(dvox[c], rv[c]) <= 1e-3


@pytest.mark.parametrize("step", [0.5, 1.0, 2.5])
def test_voxel_gradient_along_axes_and_steps(orc, step):
    """Rays close to each axis in both directions, at steps that move a sample's corner cube
    by at most one voxel per axis (the shared corners' sums are kept) or jump further: voxel
    by voxel against the oracle, volume faces included (clamped corner indices)."""
    import dataclasses
    dims, C, M = (34, 30, 28), 3, 8
    vol = synth.gen_volume(dims, C, seed=9, n_blobs=10, dtype="f32")
    t = _tree(dims, C, M, vol)
    base = _views(dims, C, 1, 40, 36, seed=9)[0]
    base.tf_rgba[:, 2:, 3] = 0.03      # semi-transparent: gradient reaches every depth
    views = []
    for az, el in ((0.0, 0.0), (90.0, 0.0), (180.0, 0.0), (270.0, 0.0), (30.0, 80.0),
                   (210.0, -80.0)):
        v = synth.make_view(dims, C, 9, az=az, el=el, width=40, height=36, dtype="f32")
        views.append(dataclasses.replace(v, tf_pos=base.tf_pos, tf_rgba=base.tf_rgba, step=step))
    rng = np.random.default_rng(2)
    tgt = [rng.uniform(0, 0.3, size=(v.height, v.width, 4)) for v in views]

    def dL(imgs):
        return [2 * (im.cpu().numpy().astype(np.float64) - g) for im, g in zip(imgs, tgt)]

    _, dctrl, dvox = _gpu_grads(t, views, dL)
    ref = orc.Tree(vol, _full(C, dims), M, 0.0, 0.0)
    gI = [2 * (w - g) for w, g in zip(ref.render(views), tgt)]
    rc, rv = ref.render_grad(views, gI)
    assert np.abs(rv).max() > 0
    assert _rel(dctrl, rc) <= 1e-3
    assert _rel(dvox, rv) <= 1e-3, _rel(dvox, rv)
    err = np.abs(dvox - rv).max()
    assert err <= 1e-3 * np.abs(rv).max(), (err, np.abs(rv).max())
    # every face of the volume receives gradient (rays enter through each of them)
    for sl in (np.s_[:, 0], np.s_[:, -1], np.s_[:, :, 0], np.s_[:, :, -1], np.s_[..., 0],
               np.s_[..., -1]):
        assert np.abs(rv[sl]).max() > 0


def test_adjoint_matches_finite_differences(orc):
    """50 parameters: 25 control-point components and 25 voxels, central differences of the
    FP64 oracle forward with eps 1e-3; voxels are taken where the table is linear across the
    perturbation (a linear TF: the table has no kinks inside the window)."""
    dims, C, M = (20, 18, 16), 3, 8
    vol = synth.gen_volume(dims, C, seed=9, n_blobs=6, dtype="f32")
    views = _views(dims, C, 1, 24, 20, seed=9)
    v = views[0]
    rng = np.random.default_rng(2)
    tgt = rng.uniform(0, 0.2, size=(v.height, v.width, 4))

    def loss(vol_, view_):
        tr = orc.Tree(vol_, _full(C, dims), M, 0.0, 0.0)
        (im,) = tr.render([view_])
        return float(((im - tgt) ** 2).sum())

    t = _tree(dims, C, M, vol)
    _, dctrl, _ = _gpu_grads(t, [v], lambda ims: [2 * (ims[0].cpu().numpy() - tgt)],
                             want_vox=False)
    eps = 1e-3
    for _ in range(25):
        c, j, q = int(rng.integers(C)), int(rng.integers(8)), int(rng.integers(4))
        x = float(v.tf_rgba[c, j, q])
        v.tf_rgba[c, j, q] = np.float32(x + eps)
        hi = float(v.tf_rgba[c, j, q])
        lp = loss(vol, v)
        v.tf_rgba[c, j, q] = np.float32(x - eps)
        lo = float(v.tf_rgba[c, j, q])
        lm = loss(vol, v)
        v.tf_rgba[c, j, q] = np.float32(x)
        fd = (lp - lm) / (hi - lo)
        assert abs(dctrl[0, c, j, q] - fd) <= 1e-3 * max(abs(fd), 1e-2), (c, j, q, fd,
                                                                          dctrl[0, c, j, q])
    # voxels, with a linear transfer function
    lin = _views(dims, C, 1, 24, 20, seed=9)[0]
    lin.tf_pos[:] = np.linspace(0, 1, 8, dtype=np.float32)
    for c in range(C):
        lin.tf_rgba[c] = np.linspace([0.1, 0.2, 0.3, 0.0], [0.9, 0.6, 0.4, 0.3], 8)
    lin.window[:, 1] = float(vol.max()) * 1.01
    _, _, dvox = _gpu_grads(t, [lin], lambda ims: [2 * (ims[0].cpu().numpy() - tgt)])
    big = np.argsort(-np.abs(dvox).ravel())[:300]
    for k in rng.choice(big, 25, replace=False):
        idx = np.unravel_index(k, dvox.shape)
        x = float(vol[idx])
        vol[idx] = np.float32(x + eps)
        hi = float(vol[idx])
        lp = loss(vol, lin)
        vol[idx] = np.float32(x - eps)
        lo = float(vol[idx])
        lm = loss(vol, lin)
        vol[idx] = np.float32(x)
        fd = (lp - lm) / (hi - lo)
        assert abs(dvox[idx] - fd) <= 1e-3 * max(abs(fd), 1e-2 * np.abs(dvox).max()), (idx, fd,
                                                                                     dvox[idx])


def test_adjoint_with_early_termination_and_skipping(orc):
    """ERT is part of the function; skipping in the forward does not change the gradient."""
    dims, C, M = (32, 32, 32), 3, 8
    vol = synth.gen_volume(dims, C, seed=5, n_blobs=8, dtype="f32")
    vol[:, :, :, 20:] = np.minimum(vol[:, :, :, 20:], np.float32(60 * 2 ** -16))
    t = _tree(dims, C, M, vol)
    (v,) = _views(dims, C, 1, 40, 40, seed=5)
    v.tf_rgba[:, 2:, 3] = 0.6
    v.ert_alpha = 0.9
    rng = np.random.default_rng(3)
    tgt = rng.uniform(0, 0.5, size=(40, 40, 4))

    def dL(imgs):
        return [2 * (imgs[0].cpu().numpy().astype(np.float64) - tgt)]

    cks = []
    _, c_skip, v_skip = _gpu_grads(t, [v], dL, ck_out=cks)
    v.no_skip = 1
    _, c_full, v_full = _gpu_grads(t, [v], dL, ck_out=cks)
    # every transmittance the forward recorded with skipping (it skips transparent positions),
    # and every end position, is bit-identical to the one recorded without; the gradients then
    # differ only by the order of float atomics
    a, b = cks[0].view(np.uint32), cks[1].view(np.uint32)
    rec = a != 0
    assert rec.sum() > 0 and rec.sum() <= (b != 0).sum()
    np.testing.assert_array_equal(a[rec], b[rec])
    assert _rel(c_skip, c_full) <= 1e-5 and _rel(v_skip, v_full) <= 1e-5
    ref = orc.Tree(vol, _full(C, dims), M, 0.0, 0.0)
    want, _, mg = ref.render([v], want_info=True)
    assert (mg[0] < 1e-5).sum() == 0          # no ambiguous termination in this case
    rc, rv = ref.render_grad([v], [2 * (want[0] - tgt)])
    assert _rel(c_skip, rc) <= 1e-3 and _rel(v_skip, rv) <= 1e-3


def test_autograd_function(orc):
    import torch
    from paper_1407_2074_amd.autograd import render
    dims, C, M = (24, 24, 24), 3, 8
    vol = synth.gen_volume(dims, C, seed=6, n_blobs=5, dtype="f32")
    t = _tree(dims, C, M, vol)
    views = _views(dims, C, 2, 16, 16, seed=6)
    tf = torch.tensor(np.stack([v.tf_rgba for v in views]), requires_grad=True)
    vox = torch.from_numpy(vol).cuda().requires_grad_(True)
    imgs = render(t, views, tf, vox)
    loss = sum((im ** 2).sum() for im in imgs)
    loss.backward()
    ref = orc.Tree(vol, _full(C, dims), M, 0.0, 0.0)
    want = ref.render(views)
    rc, rv = ref.render_grad(views, [2 * w for w in want])
    assert tf.grad is not None and tf.grad.shape == (2, C, 8, 4)
    assert _rel(tf.grad.numpy(), rc) <= 1e-3
    assert _rel(vox.grad.cpu().numpy(), rv) <= 1e-3


def test_voxel_gradient_preconditions():
    import torch
    from paper_1407_2074_amd.octree import OCT_EINVAL, Octree, OctError
    dims, C, M = (16, 16, 16), 1, 8
    vol = synth.gen_volume(dims, C, seed=6, n_blobs=2, dtype="f32")
    t = Octree(dims, C, M, "f32", 0.0, 0.0)
    t.insert_block(-1, (0, 0, 0), np.ascontiguousarray(vol[:, :8]))   # half inserted
    t.upload()
    (v,) = _views(dims, C, 1, 8, 8)
    ck = torch.empty(t.ckpt_bytes([v]), dtype=torch.uint8, device="cuda")
    (im,) = t.render([v], ckpt=ck)
    dctrl = torch.zeros((1, C, 8, 4), device="cuda")
    dvox = torch.zeros((C, 16, 16, 16), device="cuda")
    with pytest.raises(OctError) as e:
        t.render_backward([v], [torch.ones_like(im)], ck, dctrl, dvox)
    assert e.value.code == OCT_EINVAL
    t.render_backward([v], [torch.ones_like(im)], ck, dctrl)          # TF gradients still fine


def test_adjoint_with_depth_segments(orc):
    """Rays split into depth segments (forward and adjoint walk each segment in its own waves;
    with checkpoints the segment bounds are whole 64-position blocks): the images match the
    plain and the one-pass renders up to compositing rounding, and the gradients match the
    oracle and the one-pass adjoint."""
    import dataclasses

    import torch
    dims, C, M = (40, 36, 30), 3, 16
    vol = synth.gen_volume(dims, C, seed=4, n_blobs=10, dtype="f32")
    t = _tree(dims, C, M, vol)
    base = _views(dims, C, 2, 48, 40)
    rng = np.random.default_rng(1)
    tgt = [rng.uniform(0, 0.3, size=(v.height, v.width, 4)) for v in base]

    def dL(imgs):
        return [2 * (im.cpu().numpy().astype(np.float64) - g) for im, g in zip(imgs, tgt)]

    split = [dataclasses.replace(v, depth_segments=3) for v in base]
    one = [dataclasses.replace(v, depth_segments=1) for v in base]
    imgs_s, dctrl_s, dvox_s = _gpu_grads(t, split, dL)
    imgs_1, dctrl_1, dvox_1 = _gpu_grads(t, one, dL)
    for a, b, c in zip(imgs_s, t.render(split), imgs_1):
        assert float((a - b).abs().max()) <= 2e-6 and float((a - c).abs().max()) <= 2e-6
    assert _rel(dctrl_s, dctrl_1) <= 1e-4 and _rel(dvox_s, dvox_1) <= 1e-4
    ref = orc.Tree(vol, _full(C, dims), M, 0.0, 0.0)
    want = ref.render(base)
    rc, rv = ref.render_grad(base, [2 * (w - g) for w, g in zip(want, tgt)])
    assert _rel(dctrl_s, rc) <= 1e-3 and _rel(dvox_s, rv) <= 1e-3
