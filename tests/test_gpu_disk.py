"""Disk tier ("Brick Upload from Disk to RAM"): the mipmap lives in pages in a file with a small
RAM set of frames.  Whatever the frames hold, the octree built through it is bit-identical to
the one built with the mipmap in HBM (and to the oracle), after every batch; modified pages are
written back and read again; a capped device pool pages bricks in through it and converges to
the in-core image.  Every case runs with the frames in pinned host memory and in device
memory."""
import numpy as np
import pytest

from paper_1407_2074_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.parametrize("frames", ["host", "device"])]


def _dev(a):
    import torch
    if a.dtype == np.uint16:
        return torch.from_numpy(np.ascontiguousarray(a).view(np.int16)).cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _octree(*a, **k):
    from paper_1407_2074_amd.octree import Octree
    return Octree(*a, **k)


def _page_bytes(M, page_cells, C, esz):
    P = M * page_cells
    return P ** 3 * C * esz


def _full(C, dims):
    return np.full((dims[2], dims[1], dims[0]), (1 << C) - 1, np.uint8)


@pytest.mark.parametrize("dtype", ["u16", "f32"])
def test_streamed_build_through_small_page_cache(orc, tmp_path, dtype, frames):
    """96x80x64 x 3, 8^3 bricks, 16^3-voxel pages, 20 RAM frames for 148 pages: every batch of
    slices evicts; dumps and levels equal the in-HBM octree's after every upload."""
    dims, C, M, thr = (96, 80, 64), 3, 8, (205 if dtype == "u16" else 0.0)
    vol = synth.gen_volume(dims, C, seed=21, n_blobs=30, dtype=dtype)
    esz = 2 if dtype == "u16" else 4
    n_frames = 20
    disk = _octree(dims, C, M, dtype, 0, thr, disk_path=str(tmp_path / "pages.bin"),
                   host_cache_bytes=n_frames * _page_bytes(M, 2, C, esz),
                   device_frames=frames == "device")
    ref = _octree(dims, C, M, dtype, 0, thr)
    dv = _dev(vol)
    for z0 in range(0, dims[2], 8):
        for t in (disk, ref):
            t.insert_slices(-1, z0, dv[:, z0:z0 + 8].contiguous())
            t.upload()
        assert disk.dump() == ref.dump(), z0
    for L in range(ref.levels):
        assert np.array_equal(disk.read_level(L), ref.read_level(L)), L
    st = disk.disk_stats()
    assert st["frames"] == n_frames and st["pages"] > n_frames
    assert st["writebacks"] > 0 and st["loads"] > 0 and st["evictions"] > 0, st
    assert st["bytes_written"] == st["writebacks"] * _page_bytes(M, 2, C, esz)
    # and the oracle
    want = orc.Tree(vol, _full(C, dims), M, 0, thr)
    assert disk.dump() == want.dump()
    disk.close()
    assert not (tmp_path / "pages.bin").exists()


def test_odd_shapes_blocks_and_channel_split(orc, tmp_path, frames):
    """37x29x23 (ragged pages and cells), 4^3 bricks, 8^3-voxel pages, blocks at odd offsets
    inserted per channel, overwrites: equal to the oracle."""
    dims, C, M = (37, 29, 23), 2, 4
    vol = synth.gen_volume(dims, C, seed=22, n_blobs=8)
    other = synth.gen_volume(dims, C, seed=23, n_blobs=8)
    t = _octree(dims, C, M, "u16", 17, 150, disk_path=str(tmp_path / "p.bin"),
                host_cache_bytes=16 * _page_bytes(M, 2, C, 2), device_frames=frames == "device")
    t.insert_block(-1, (0, 0, 0), other)
    t.upload()
    rng = np.random.default_rng(3)
    for c in range(C):
        for z0 in range(0, dims[2], 7):
            for x0 in (0, 13, 26):
                blk = vol[c:c + 1, z0:z0 + 7, :, x0:x0 + 13]
                t.insert_block(c, (x0, 0, z0), np.ascontiguousarray(blk))
            if rng.random() < 0.5:
                t.upload()
    t.upload()
    want = orc.Tree(vol, _full(C, dims), M, 17, 150)
    for L in range(want.levels):
        assert np.array_equal(t.read_level(L), want.level(L)), L
    assert t.dump() == want.dump()
    assert t.disk_stats()["writebacks"] > 0


def test_clear_returns_every_page_to_the_background(tmp_path, frames):
    dims, C, M = (64, 48, 32), 3, 8
    vol = synth.gen_volume(dims, C, seed=24, n_blobs=10)
    t = _octree(dims, C, M, "u16", 0, 100, disk_path=str(tmp_path / "p.bin"),
                host_cache_bytes=16 * _page_bytes(M, 2, C, 2), device_frames=frames == "device")
    fresh = _octree(dims, C, M, "u16", 0, 100)
    empty = fresh.dump()
    t.insert_block(-1, (0, 0, 0), vol)
    t.upload()
    t.clear()
    t.upload()
    assert t.dump() == empty
    for L in range(fresh.levels):
        assert np.array_equal(t.read_level(L), fresh.read_level(L)), L


def test_capped_pool_pages_through_the_disk_tier(tmp_path, frames):
    """Device pool of a quarter of the bricks, pages from the disk tier: the converged image
    equals the in-core image bit for bit."""
    dims, C, M = (128, 128, 96), 3, 16
    vol = synth.gen_volume(dims, C, seed=12, n_blobs=60)
    ref = _octree(dims, C, M, "u16", 0, 205)
    ref.insert_block(-1, (0, 0, 0), vol)
    ref.upload()
    bb = ref.brick_bytes
    t = _octree(dims, C, M, "u16", 0, 205, pool_bytes=(ref.pool_slots // 4) * bb,
                disk_path=str(tmp_path / "p.bin"), host_cache_bytes=24 * _page_bytes(M, 2, C, 2),
                device_frames=frames == "device")
    t.insert_block(-1, (0, 0, 0), vol)
    t.upload()
    v = synth.make_view(dims, C, 12, az=30.0, el=25.0, width=64, height=64, lod=1)
    for _ in range(80):
        (img,) = t.render([v])
        if t.upload()["requests_seen"] == 0:
            break
    else:
        raise AssertionError("paging did not converge")
    (img,) = t.render([v])
    (want,) = ref.render([v])
    import torch
    assert torch.equal(img, want)
    assert t.disk_stats()["loads"] > 0
