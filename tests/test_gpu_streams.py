"""Calls on different HIP streams: the library orders their device work as if they had been
issued on one stream in call order, so a streamed build on one stream with renders on another
gives the same images after every batch, and the same octree, as everything on one stream."""
import numpy as np
import pytest

from paper_1407_2074_amd import synth

pytestmark = pytest.mark.gpu

DIMS, C, M = (48, 40, 32), 3, 8


def _stream_build(vol, views, bstream, rstream):
    import torch
    from paper_1407_2074_amd.octree import Octree
    t = Octree(DIMS, C, M, "u16", 0, 205)
    dev = torch.from_numpy(vol.view(np.int16)).cuda()
    slabs = [dev[:, z:z + 4].contiguous() for z in range(0, DIMS[2], 4)]
    imgs = [torch.empty((v.height, v.width, 4), dtype=torch.float32, device="cuda")
            for v in views]
    torch.cuda.synchronize()
    out = []
    for b, sl in enumerate(slabs):
        t.insert_slices(-1, 4 * b, sl, stream=bstream)
        t.upload(stream=bstream)
        t.render(views, images=imgs, stream=rstream)
        # the host copies run on the render stream, after the render
        with torch.cuda.stream(rstream if rstream is not None else torch.cuda.current_stream()):
            out.append([im.to("cpu", non_blocking=False) for im in imgs])
    torch.cuda.synchronize()
    dump = t.dump()
    t.close()
    return out, dump


def _views():
    return [synth.make_view(DIMS, C, 7, az=az, el=el, width=40, height=32, lod=lod)
            for az, el, lod in ((20.0, 30.0, 0), (200.0, -20.0, -1))]


def test_build_and_render_on_two_streams_match_one_stream():
    import torch
    vol = synth.gen_volume(DIMS, C, seed=7, n_blobs=12)
    views = _views()
    ref_imgs, ref_dump = _stream_build(vol, views, None, None)
    b, r = torch.cuda.Stream(), torch.cuda.Stream()
    imgs, dump = _stream_build(vol, views, b, r)
    assert dump == ref_dump
    for k, (x, y) in enumerate(zip(imgs, ref_imgs)):
        for i, (a, w) in enumerate(zip(x, y)):
            assert torch.equal(a, w), (k, i)


def test_paged_upload_on_another_stream_reads_the_render_flags():
    """With a capped pool the upload reads the flags the renders wrote: on another stream it
    must wait for them, and refinement converges exactly as on one stream."""
    import torch
    vol = synth.gen_volume(DIMS, C, seed=8, n_blobs=12)
    views = _views()

    def refine(bstream, rstream):
        from paper_1407_2074_amd.octree import Octree
        probe = Octree(DIMS, C, M, "u16", 0, 205)
        bb, n_all = probe.brick_bytes, probe.pool_slots
        probe.close()
        # one slot short of every brick: paging on request, and both views fit
        t = Octree(DIMS, C, M, "u16", 0, 205, pool_bytes=(n_all - 1) * bb)
        t.insert_block(-1, (0, 0, 0), vol, stream=bstream)
        t.upload(stream=bstream)
        imgs = [torch.empty((v.height, v.width, 4), dtype=torch.float32, device="cuda")
                for v in views]
        seq = []
        for it in range(40):
            t.render(views, images=imgs, stream=rstream)
            up = t.upload(stream=bstream)
            seq.append((up["requests_seen"], up["bricks_gathered"], up["evictions"]))
            if up["requests_seen"] == 0:
                break
        torch.cuda.synchronize()
        res = [im.cpu() for im in imgs]
        t.close()
        return seq, res

    seq1, img1 = refine(None, None)
    seq2, img2 = refine(torch.cuda.Stream(), torch.cuda.Stream())
    assert seq1 == seq2
    assert seq1[-1][0] == 0
    for a, w in zip(img2, img1):
        assert torch.equal(a, w)


def test_upload_during_a_render_keeps_that_render_s_octree():
    """A render issued before an upload reads the octree as it was when it was issued, even
    while the upload runs on another stream: the upload rebuilds the bricks that render reads
    into other pool slots and switches node tables, and the next render sees the new data."""
    import dataclasses

    import torch
    from paper_1407_2074_amd.octree import Octree
    vol = synth.gen_volume(DIMS, C, seed=12, n_blobs=14)
    vol2 = vol.copy()
    vol2[:, 8:24] = synth.gen_volume(DIMS, C, seed=13, n_blobs=14)[:, 8:24]
    # slow render: 1024^2 rays, every position of the whole ray in one pass
    v = dataclasses.replace(synth.make_view(DIMS, C, 7, az=35.0, el=25.0, width=1024,
                                            height=1024), step=0.1, no_skip=1,
                            depth_segments=1)

    def tree(data):
        t = Octree(DIMS, C, M, "u16", 0, 205)
        t.insert_block(-1, (0, 0, 0), data)
        t.upload()
        return t

    ref_old, ref_new = tree(vol), tree(vol2)
    (want_old,) = ref_old.render([v])
    (want_new,) = ref_new.render([v])
    torch.cuda.synchronize()
    assert not torch.equal(want_old, want_new)
    t = tree(vol)
    slab = torch.from_numpy(vol2[:, 8:24].view(np.int16)).cuda()
    torch.cuda.synchronize()
    r, b = torch.cuda.Stream(), torch.cuda.Stream()
    img_old = torch.empty_like(want_old)
    img_new = torch.empty_like(want_old)
    t.render([v], images=[img_old], stream=r)           # in flight while the upload runs
    t.insert_slices(-1, 8, slab, stream=b)
    up = t.upload(stream=b)
    t.render([v], images=[img_new], stream=r)
    torch.cuda.synchronize()
    assert up["bricks_gathered"] > 0
    assert torch.equal(img_old, want_old)
    assert torch.equal(img_new, want_new)
    for x in (ref_old, ref_new, t):
        x.close()


def _grad_tree():
    import torch
    from paper_1407_2074_amd.octree import Octree
    dims = (24, 20, 16)
    vol = synth.gen_volume(dims, C, seed=9, n_blobs=6).astype(np.float32) / 65536.0
    t = Octree(dims, C, 8, "f32", 0, 0)
    t.insert_slices(-1, 0, torch.from_numpy(vol).cuda())
    t.upload()
    views = [synth.make_view(dims, C, 9, az=30.0, el=20.0, width=24, height=16, lod=0,
                             dtype="f32")]
    return t, views, vol


def _backward(t, views, ck, imgs, stream=None):
    import torch
    g = [im * 2.0 - 0.25 for im in imgs]
    dctrl = torch.zeros((len(views), C, 8, 4), dtype=torch.float32, device="cuda")
    dvox = torch.zeros((C,) + tuple(t.dims[::-1]), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t.render_backward(views, g, ck, dctrl, dvox, stream=stream)
    torch.cuda.synchronize()
    return dctrl.cpu(), dvox.cpu()


def test_forward_and_backward_on_two_streams_match_one_stream():
    """A backward on another stream than its forward waits for the forward's checkpoints, and two
    backwards on two streams do not share their temporaries while running."""
    import torch
    t, views, _ = _grad_tree()
    ck = torch.zeros(t.ckpt_bytes(views), dtype=torch.uint8, device="cuda")
    imgs = t.render(views, ckpt=ck)
    ref = _backward(t, views, ck, imgs)
    a, b = torch.cuda.Stream(), torch.cuda.Stream()
    for _ in range(3):
        ck2 = torch.zeros_like(ck)
        imgs2 = t.render(views, ckpt=ck2, stream=a)     # no host synchronisation in between
        g = [im * 2.0 - 0.25 for im in imgs]
        d1 = torch.zeros((1, C, 8, 4), dtype=torch.float32, device="cuda")
        d2 = torch.zeros_like(d1)
        torch.cuda.synchronize()
        t.render_backward(views, g, ck2, d1, None, stream=b)
        t.render_backward(views, g, ck2, d2, None, stream=a)
        torch.cuda.synchronize()
        for im, w in zip(imgs2, imgs):
            assert torch.equal(im, w)
        for d in (d1, d2):
            assert float((d.cpu() - ref[0]).abs().max()) <= 1e-5 * float(ref[0].abs().max())
    t.close()


def test_backward_refuses_a_changed_octree_or_other_views():
    import torch
    from paper_1407_2074_amd.octree import OCT_EINVAL, OctError
    t, views, vol = _grad_tree()
    ck = torch.zeros(t.ckpt_bytes(views), dtype=torch.uint8, device="cuda")
    imgs = t.render(views, ckpt=ck)
    other = [synth.make_view(t.dims, C, 9, az=50.0, el=20.0, width=24, height=16, lod=0,
                             dtype="f32")]
    with pytest.raises(OctError) as e:
        _backward(t, other, ck, imgs)
    assert e.value.code == OCT_EINVAL
    _backward(t, views, ck, imgs)                       # the matching views are accepted
    # an upload that changes the octree invalidates the checkpoints
    t.insert_block(-1, (0, 0, 0), torch.from_numpy(vol[:, :4, :4, :4] * 0.5).cuda())
    t.upload()
    with pytest.raises(OctError) as e:
        _backward(t, views, ck, imgs)
    assert e.value.code == OCT_EINVAL
    imgs = t.render(views, ckpt=ck)                     # a new forward makes it valid again
    _backward(t, views, ck, imgs)
    t.close()
