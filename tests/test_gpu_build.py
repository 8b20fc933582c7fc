"""GPU parity of incremental construction: the canonical dump (node states, AVG/min/max,
bordered bricks) and every mipmap level must equal the oracle's bit for bit, after every
insert batch, for any chunking, order, overwrite pattern, channel split and data type."""
import numpy as np
import pytest

from paper_1407_2074_amd import synth

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    if a.dtype == np.uint16:
        return torch.from_numpy(np.ascontiguousarray(a).view(np.int16)).cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _Octree(*a, **k):
    from paper_1407_2074_amd.octree import Octree
    return Octree(*a, **k)


def _full(C, dims):
    return np.full((dims[2], dims[1], dims[0]), (1 << C) - 1, np.uint8)


def _diff_dump(orc, a: bytes, b: bytes):
    """Human-readable first difference between two dumps."""
    if a == b:
        return "equal"
    ha, ra, ba = orc.parse_dump(a)
    hb, rb, bb = orc.parse_dump(b)
    if ha != hb:
        return f"headers {ha} vs {hb}"
    for i in range(len(ra)):
        if ra[i].tobytes() != rb[i].tobytes():
            return f"record {i}: {ra[i]} vs {rb[i]}"
    return f"brick bytes differ at {np.nonzero(np.frombuffer(ba, np.uint8) != np.frombuffer(bb, np.uint8))[0][:5]}"


@pytest.mark.parametrize("thr", [0, 205])
def test_cfg1_whole_volume_bit_exact(orc, thr):
    """64^3 x 3 uint16, 16^3 bricks, 3 levels: one host block insert."""
    dims, C, M = (64, 64, 64), 3, 16
    vol = synth.gen_volume(dims, C, seed=1, n_blobs=20)
    t = _Octree(dims, C, M, "u16", 0, thr)
    t.insert_block(-1, (0, 0, 0), vol)
    t.upload()
    ref = orc.Tree(vol, _full(C, dims), M, 0, thr)
    assert t.levels == ref.levels == 3
    for L in range(ref.levels):
        assert np.array_equal(t.read_level(L), ref.level(L)), L
    a, b = t.dump(), ref.dump()
    assert a == b, _diff_dump(orc, a, b)


@pytest.mark.parametrize("thr", [0, 205])
def test_streamed_slabs_bit_exact_after_every_batch(orc, thr):
    """Slices arrive 8 at a time from device memory; after each brick_pool_upload the octree
    equals the oracle's for exactly the data inserted so far (incomplete nodes included)."""
    dims, C, M = (96, 80, 64), 3, 16
    vol = synth.gen_volume(dims, C, seed=2, n_blobs=40)
    dv = _dev(vol)
    t = _Octree(dims, C, M, "u16", 0, thr)
    for z0 in range(0, dims[2], 8):
        t.insert_slices(-1, z0, dv[:, z0:z0 + 8].contiguous())
        t.upload()
        v0 = np.zeros_like(vol)
        v0[:, :z0 + 8] = vol[:, :z0 + 8]
        mask = np.zeros((dims[2], dims[1], dims[0]), np.uint8)
        mask[:z0 + 8] = 7
        ref = orc.Tree(v0, mask, M, 0, thr)
        a, b = t.dump(), ref.dump()
        assert a == b, (z0, _diff_dump(orc, a, b))


def test_chunking_order_and_channel_split_independence(orc):
    """Different insertion schedules of the same data give the same octree (only complete
    nodes are merged, so nothing depends on the order of arrival)."""
    dims, C, M = (40, 36, 30), 3, 8
    vol = synth.gen_volume(dims, C, seed=3, n_blobs=15)
    ref = orc.Tree(vol, _full(C, dims), M, 0, 205).dump()
    rng = np.random.default_rng(0)
    # (a) shuffled single slices, all channels
    t = _Octree(dims, C, M, "u16", 0, 205)
    for z in rng.permutation(dims[2]):
        t.insert_slices(-1, int(z), vol[:, z:z + 1].copy())
        if rng.random() < 0.3:
            t.upload()
    t.upload()
    assert t.dump() == ref
    # (b) per channel, reversed slabs of 7, uploads in between
    t = _Octree(dims, C, M, "u16", 0, 205)
    for c in range(C):
        for z0 in reversed(range(0, dims[2], 7)):
            z1 = min(z0 + 7, dims[2])
            t.insert_slices(c, z0, _dev(vol[c:c + 1, z0:z1]))
            t.upload()
    assert t.dump() == ref
    # (c) random cuboids covering the volume twice
    t = _Octree(dims, C, M, "u16", 0, 205)
    for _ in range(2):
        for z0 in range(0, dims[2], 10):
            for y0 in range(0, dims[1], 13):
                for x0 in range(0, dims[0], 11):
                    blk = vol[:, z0:z0 + 10, y0:y0 + 13, x0:x0 + 11]
                    t.insert_block(-1, (x0, y0, z0), np.ascontiguousarray(blk))
        t.upload()
    assert t.dump() == ref


def test_overwrite_replaces_data(orc):
    dims, C, M = (32, 32, 32), 2, 8
    vol = synth.gen_volume(dims, C, seed=4, n_blobs=10)
    other = synth.gen_volume(dims, C, seed=5, n_blobs=10)
    t = _Octree(dims, C, M, "u16", 0, 100)
    t.insert_block(-1, (0, 0, 0), other)
    t.upload()
    blk = np.ascontiguousarray(vol[:, 5:20, 3:30, 9:17])
    t.insert_block(-1, (9, 3, 5), blk)
    t.upload()
    final = other.copy()
    final[:, 5:20, 3:30, 9:17] = blk
    assert t.dump() == orc.Tree(final, _full(C, dims), M, 0, 100).dump()


@pytest.mark.parametrize("dims,M", [((13, 9, 7), 4), ((20, 17, 33), 6), ((31, 5, 12), 2),
                                    ((64, 8, 16), 16)])
def test_odd_shapes_and_brick_sizes(orc, dims, M):
    """Virtual extension (non power-of-two dims), non power-of-two even M, ragged bricks."""
    C = 2
    vol = synth.gen_volume(dims, C, seed=6, n_blobs=6)
    t = _Octree(dims, C, M, "u16", 17, 150)
    half = dims[2] // 2
    t.insert_block(0, (0, 0, 0), np.ascontiguousarray(vol[0:1]))
    t.insert_block(1, (0, 0, 0), np.ascontiguousarray(vol[1:2, :half]))
    t.upload()
    v0 = vol.copy()
    v0[1, half:] = 17
    mask = np.ones((dims[2], dims[1], dims[0]), np.uint8)
    mask[:half] |= 2
    ref = orc.Tree(v0, mask, M, 17, 150)
    for L in range(ref.levels):
        assert np.array_equal(t.read_level(L), ref.level(L)), L
    a, b = t.dump(), ref.dump()
    assert a == b, _diff_dump(orc, a, b)


def test_float32_volume_bit_exact(orc):
    """Float data (uint16 * 2^-16): float32-rounded means of exact double sums."""
    dims, C, M = (48, 40, 36), 3, 16
    vol = synth.gen_volume(dims, C, seed=4, n_blobs=12, dtype="f32")
    t = _Octree(dims, C, M, "f32", 0.0, 0.0)
    dv = _dev(vol)
    for z0 in range(0, dims[2], 12):
        t.insert_slices(-1, z0, dv[:, z0:z0 + 12].contiguous())
    t.upload()
    ref = orc.Tree(vol, _full(C, dims), M, 0.0, 0.0)
    for L in range(ref.levels):
        assert np.array_equal(t.read_level(L), ref.level(L)), L
    assert t.dump() == ref.dump()


def test_clear_returns_to_initial_state(orc):
    dims, C, M = (24, 24, 24), 1, 8
    vol = synth.gen_volume(dims, C, seed=7, n_blobs=5)
    t = _Octree(dims, C, M, "u16", 9, 0)
    empty = orc.Tree(np.full_like(vol, 9), np.zeros((24, 24, 24), np.uint8), M, 9, 0).dump()
    assert t.dump() == empty
    t.insert_block(-1, (0, 0, 0), vol)
    t.upload()
    t.clear()
    t.upload()
    assert t.dump() == empty


def test_invalid_inserts_are_rejected(orc):
    from paper_1407_2074_amd.octree import OCT_EINVAL, OCT_ERANGE, OctError
    t = _Octree((16, 16, 16), 2, 8, "u16", 0, 0)
    blk = np.zeros((1, 4, 4, 4), np.uint16)
    with pytest.raises(OctError) as e:
        t.insert_block(2, (0, 0, 0), blk)
    assert e.value.code == OCT_EINVAL
    with pytest.raises(OctError) as e:
        t.insert_block(0, (14, 0, 0), blk)
    assert e.value.code == OCT_ERANGE
    with pytest.raises(OctError) as e:
        t.insert_slices(-1, 15, np.zeros((2, 2, 16, 16), np.uint16))
    assert e.value.code == OCT_ERANGE
