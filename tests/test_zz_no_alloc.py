"""render_views_noalloc against render_views, through the C ABI: the allocation-free entry point
renders the same images (bit for bit where both march rays in one pass) on two calls in a row,
the second with fewer and smaller views, and rejects launches beyond its limits."""
import numpy as np
import pytest

from paper_1407_2074_amd import synth

pytestmark = pytest.mark.gpu

DIMS, C, M = (48, 40, 32), 3, 8


def _tree():
    import torch
    from paper_1407_2074_amd.octree import Octree
    vol = synth.gen_volume(DIMS, C, seed=11, n_blobs=14)
    t = Octree(DIMS, C, M, "u16", 0, 205)
    dev = torch.from_numpy(vol.view(np.int16)).cuda()
    t.insert_slices(-1, 0, dev)
    t.upload()
    return t


def _views(n, w, h, **kw):
    out = []
    for k in range(n):
        v = synth.make_view(DIMS, C, 20 + k, az=37.0 * k + 10.0, el=25.0 - 9.0 * k, width=w + 3 * k,
                            height=h + 5 * k, lod=(-1 if k % 2 else 0),
                            clips=[(1.0, 0.0, 0.0, 10.0)] if k == 1 else (), **kw)
        out.append(v)
    return out


def _one_pass(views):
    for v in views:
        v.depth_segments = 1
    return views


def _render(t, views, noalloc, stats=False):
    import torch
    imgs = [torch.full((v.height, v.width, 4), -1.0, dtype=torch.float32, device="cuda")
            for v in views]
    r = t.render(views, images=imgs, noalloc=noalloc, stats=stats)
    torch.cuda.synchronize()
    if stats:
        imgs, st = r
        return [im.cpu() for im in imgs], st
    return [im.cpu() for im in imgs]


def test_noalloc_equals_render_views_on_two_calls():
    import torch
    t = _tree()
    big = _one_pass(_views(5, 64, 48))
    big[3].ert_alpha = 0.9
    small = _one_pass(_views(2, 24, 16))
    for views in (big, small):          # second call: fewer, smaller views
        want, st_want = _render(t, views, False, stats=True)
        got, st_got = _render(t, views, True, stats=True)
        assert st_got == st_want
        for a, b in zip(got, want):
            assert torch.equal(a, b)
    t.close()


def test_noalloc_with_default_segments_within_rounding():
    """render_views splits long rays into depth segments; the no-alloc call marches them in one
    pass, so only the compositing rounding differs."""
    t = _tree()
    for views in (_views(3, 96, 80), _views(1, 40, 24)):
        for v in views:
            v.depth_segments = 3
        want = _render(t, views, False)
        got = _render(t, views, True)
        for a, b in zip(got, want):
            assert float((a - b).abs().max()) <= 1e-5
    t.close()


def test_noalloc_with_checkpoints_drives_the_adjoint():
    """With a checkpoint workspace the no-alloc forward fills it as render_views does: the
    backward after either gives the same gradients."""
    import torch
    from paper_1407_2074_amd.octree import Octree
    vol = synth.gen_volume(DIMS, C, seed=12, n_blobs=10).astype(np.float32) / 65536.0
    t = Octree(DIMS, C, M, "f32", 0, 0)
    t.insert_slices(-1, 0, torch.from_numpy(vol).cuda())
    t.upload()
    views = _views(2, 32, 24, dtype="f32")
    for v in views:
        v.lod = 0
    res = []
    for noalloc in (False, True):
        ck = torch.zeros(t.ckpt_bytes(views), dtype=torch.uint8, device="cuda")
        imgs = t.render(views, ckpt=ck, noalloc=noalloc)
        g = [torch.ones_like(im) * 0.5 for im in imgs]
        dctrl = torch.zeros((len(views), C, 8, 4), dtype=torch.float32, device="cuda")
        dvox = torch.zeros((C,) + DIMS[::-1], dtype=torch.float32, device="cuda")
        t.render_backward(views, g, ck, dctrl, dvox)
        torch.cuda.synchronize()
        res.append(([im.cpu() for im in imgs], dctrl.cpu(), dvox.cpu()))
    for a, b in zip(res[0][0], res[1][0]):
        assert torch.equal(a, b)
    # the gradients are sums of float atomics, whose order varies from run to run
    for k in (1, 2):
        a, b = res[0][k], res[1][k]
        assert float((a - b).abs().max()) <= 1e-5 * float(a.abs().max())
    t.close()


def test_noalloc_rejects_too_many_views():
    from paper_1407_2074_amd.octree import OCT_ERANGE, OctError
    t = _tree()
    views = _views(1, 8, 8) * 65
    with pytest.raises(OctError) as e:
        t.render(views, noalloc=True)
    assert e.value.code == OCT_ERANGE
    # the handle stays usable
    (img,) = _render(t, _views(1, 16, 16), True)
    assert bool((img >= 0).all())
    t.close()
