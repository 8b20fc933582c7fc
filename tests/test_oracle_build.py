"""Pins for the oracle's octree construction (CPU only).

Each test checks the oracle against something other than itself: a numpy reshape-sum mipmap,
the geometric-series brick count of the paper's brick pool, the narrative of the paper's
incremental-construction example (Fig. 3), the homogeneity rules and a Python brute force of the
represented field with clamped borders."""
import numpy as np
import pytest

from helpers import np_mip
from paper_1407_2074_amd import synth


def _full_mask(C, dims):
    Dx, Dy, Dz = dims
    return np.full((Dz, Dy, Dx), (1 << C) - 1, np.uint8)


@pytest.mark.parametrize("dims,M,dtype", [((13, 9, 7), 4, "u16"), ((20, 17, 33), 6, "u16"),
                                          ((16, 16, 16), 4, "f32"), ((31, 5, 12), 2, "u16"),
                                          ((40, 24, 10), 8, "f32")])
def test_mip_equals_numpy_reshape_sum(orc, dims, M, dtype):
    """Half-sampling over valid children, integer round-half-up (u16) / rounded mean (f32)."""
    rng = np.random.default_rng(7)
    C = 3
    Dx, Dy, Dz = dims
    if dtype == "u16":
        v0 = rng.integers(0, 65536, size=(C, Dz, Dy, Dx), dtype=np.uint16)
    else:
        v0 = (rng.integers(0, 65536, size=(C, Dz, Dy, Dx)).astype(np.float32)
              * np.float32(2 ** -16))
    t = orc.Tree(v0, _full_mask(C, dims), M, 0.0, 0.0)
    ref = np_mip(v0, M)
    assert t.N == len(ref) - 1
    assert M << t.N >= max(dims) and (t.N == 0 or M << (t.N - 1) < max(dims))
    for L in range(t.levels):
        assert np.array_equal(t.level(L), ref[L]), L


def test_rounding_half_up_small_cases(orc):
    """Partial 2x2x2 cells: 1, 2 and 4 valid children; halves round up."""
    v0 = np.zeros((1, 1, 1, 5), np.uint16)       # Dx=5, Dy=Dz=1, M=2 -> N=2
    v0[0, 0, 0] = [1, 2, 7, 9, 4]
    t = orc.Tree(v0, _full_mask(1, (5, 1, 1)), 2, 0, 0)
    assert t.N == 2
    # level 1: mean(1,2)=1.5 -> 2 ; mean(7,9)=8 ; lone child 4
    assert t.level(1)[0, 0, 0].tolist() == [2, 8, 4]
    # level 2: mean(2,8)=5 ; lone child 4
    assert t.level(2)[0, 0, 0].tolist() == [5, 4]
    v0[0, 0, 0] = [1, 2, 2, 2, 0]
    t = orc.Tree(v0, _full_mask(1, (5, 1, 1)), 2, 0, 0)
    # (1+2)/2 = 1.5 -> 2, (2+2)/2 = 2 ; then (2+2)/2 = 2 and 0
    assert t.level(2)[0, 0, 0].tolist() == [2, 0]
    v3 = np.zeros((1, 2, 2, 4), np.uint16)          # Dx=4, M=2 -> N=1, two full cells
    v3[0, 0, 0, 0], v3[0, 1, 1, 1] = 1, 2           # sum 3 over 8 = 0.375 -> 0
    v3[0, 0, 0, 2], v3[0, 1, 1, 3] = 2, 2           # sum 4 over 8 = 0.5 -> 1 (half up)
    t = orc.Tree(v3, _full_mask(1, (4, 2, 2)), 2, 0, 0)
    assert t.N == 1 and t.level(1)[0, 0, 0].tolist() == [0, 1]


def _states(t):
    hdr, recs, _ = __import__("oracle").parse_dump(t.dump())
    return {tuple(r["head"][:4]): (int(r["head"][4]), int(r["head"][5])) for r in recs}


def test_brick_pool_geometric_series(orc):
    """Dense data, no merging: every node of the complete tree holds a brick and the pool is
    sum_i 8^-i of the volume (about 8/7)."""
    M, N = 4, 3
    D = M << N
    rng = np.random.default_rng(1)
    v0 = rng.integers(0, 65536, size=(1, D, D, D), dtype=np.uint16)
    t = orc.Tree(v0, _full_mask(1, (D, D, D)), M, 0, 0)
    hdr, recs, bricks = orc.parse_dump(t.dump())
    assert hdr["n_nodes"] == sum(8 ** i for i in range(N + 1))
    assert hdr["n_bricks"] == hdr["n_nodes"]
    ratio = hdr["n_bricks"] * M ** 3 / D ** 3
    assert abs(ratio - sum(0.125 ** i for i in range(N + 1))) < 1e-12
    assert abs(ratio - 8 / 7) < 0.01


def test_virtual_extension_counts(orc):
    """Arbitrary dims are padded virtually to M*2^N; nodes beyond the volume stay EMPTY and
    only in-volume bricks are created."""
    dims, M = (20, 12, 9), 4
    rng = np.random.default_rng(2)
    v0 = rng.integers(100, 60000, size=(2, 9, 12, 20), dtype=np.uint16)
    t = orc.Tree(v0, _full_mask(2, dims), M, 0, 0)
    assert t.N == 3
    hdr, recs, _ = orc.parse_dump(t.dump())
    st = recs["head"][:, 4]
    for L in range(t.levels):
        ext = t.extent(L)
        nb = np.prod([-(-e // M) for e in ext])
        sel = recs["head"][:, 0] == L
        assert (st[sel] == orc.ST_BRICK).sum() == nb
        # every other existing node of the level lies outside the volume and is EMPTY
        assert np.all(st[sel & (st != orc.ST_BRICK)] == orc.ST_EMPTY)


def test_out_of_volume_voxels_do_not_enter_statistics(orc):
    """A partly-outside brick's min/max/avg use only its valid voxels."""
    dims, M = (6, 4, 4), 4         # second x-brick has only 2 valid columns
    v0 = np.full((1, 4, 4, 6), 10, np.uint16)
    v0[0, :, :, 4:] = 30
    t = orc.Tree(v0, _full_mask(1, dims), M, background=999, threshold=5)
    st, fl, avg = t.node(0, 1, 0, 0)
    assert st == orc.ST_HOMOG_LEAF and avg[0] == 30
    st, fl, avg = t.node(0, 0, 0, 0)
    assert st == orc.ST_HOMOG_LEAF and avg[0] == 10


def _golden(name):
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)) as f:
        return json.load(f)


def test_fig3_incremental_example(orc):
    """The paper's 1-D example (tests/golden/fig3_incremental_1d.json): brick resolution 4,
    homogeneity threshold 1, the printed blocks [1,5,2], [3,3,2,2], [4,3,3].

    Facts pinned from the narrative: data need not be coherent; a brick with min 3 and max 3 is
    homogeneous, deleted and represented by its AVG 3; a homogeneous parent keeps its subtree
    while a leaf below has min 1 and max 5; after the volume is complete the root is homogeneous
    but no subtree is deleted.  (Block positions are ours; the figure is not available.)"""
    gd = _golden("fig3_incremental_1d.json")
    M, thr = gd["brick_resolution"], gd["homogeneity_threshold"]
    pb, ours = gd["printed_blocks"], gd["ours"]
    dims = (ours["volume_length"], 1, 1)
    vals = [pb[0], pb[1], pb[2] + ours["block_3_padding"], ours["block_4"]]
    blocks = list(zip(ours["block_starts"], vals))
    ins = []
    expect = [
        {(2, 0, 0, 0): orc.ST_BRICK, (1, 0, 0, 0): orc.ST_BRICK, (1, 1, 0, 0): orc.ST_EMPTY,
         (0, 0, 0, 0): orc.ST_BRICK, (0, 1, 0, 0): orc.ST_EMPTY},
        {(1, 1, 0, 0): orc.ST_BRICK, (0, 2, 0, 0): orc.ST_BRICK, (0, 3, 0, 0): orc.ST_EMPTY},
        {(0, 0, 0, 0): orc.ST_BRICK, (0, 1, 0, 0): orc.ST_HOMOG_LEAF, (1, 0, 0, 0): orc.ST_HOMOG,
         (2, 0, 0, 0): orc.ST_BRICK},
        {(2, 0, 0, 0): orc.ST_HOMOG, (1, 0, 0, 0): orc.ST_HOMOG, (1, 1, 0, 0): orc.ST_BRICK,
         (0, 0, 0, 0): orc.ST_BRICK, (0, 1, 0, 0): orc.ST_HOMOG_LEAF,
         (0, 2, 0, 0): orc.ST_BRICK, (0, 3, 0, 0): orc.ST_BRICK},
    ]
    for step, (x0, vals) in enumerate(blocks):
        ins.append((-1, (x0, 0, 0), np.array(vals, np.uint16).reshape(1, 1, 1, -1)))
        v0, mask = orc.apply_inserts(dims, 1, ins)
        t = orc.Tree(v0, mask, M, background=0, threshold=thr)
        for key, st in expect[step].items():
            assert t.node(*key)[0] == st, (step, key)
        if step == 0:
            assert t.node(0, 2, 0, 0)[0] == orc.ST_NONE      # below an EMPTY leaf
        if step == 2:
            out = gd["printed_outcomes"]["after_block_3"]
            _, recs, _ = orc.parse_dump(t.dump())
            homog = [r for r in recs if r["head"][4] in (orc.ST_HOMOG_LEAF, orc.ST_HOMOG)]
            assert len(homog) == out["homogeneous_bricks"]
            for r in homog:
                assert (r["bmin"][0], r["bmax"][0], r["avg"][0]) == \
                    (out["their_min"], out["their_max"], out["their_avg"])
            leaf = [r for r in recs if tuple(r["head"][:4]) == (0, 0, 0, 0)][0]
            assert (leaf["bmin"][0], leaf["bmax"][0]) == (out["leftmost_leaf_min"],
                                                        out["leftmost_leaf_max"])
            assert bool(t.node(1, 0, 0, 0)[1] & orc.F_HAS_CHILDREN) == \
                (not out["left_subtree_deleted"])
    out = gd["printed_outcomes"]["after_block_4"]
    # homogeneous nodes carry AVG 3; the root's subtree survives
    assert t.node(0, 1, 0, 0)[2][0] == 3
    assert t.node(1, 0, 0, 0)[2][0] == 3
    assert t.node(2, 0, 0, 0)[2][0] == 3
    st, fl, _ = t.node(2, 0, 0, 0)
    assert (st in (orc.ST_HOMOG, orc.ST_HOMOG_LEAF)) == out["root_homogeneous"]
    assert fl & orc.F_HAS_CHILDREN and fl & orc.F_COMPLETE
    _, recs, _ = orc.parse_dump(t.dump())
    deleted = [r for r in recs if r["head"][4] == orc.ST_HOMOG_LEAF and r["head"][0] > 0]
    assert len(deleted) == out["subtrees_deleted"]


def test_printed_overheads_and_virtual_extension(orc):
    """Numbers the paper prints (tests/golden/paper_numbers.json): the brick pool is about 14%
    larger than the volume; one voxel of border per side costs about 20% at 32^3; and
    3865 x 1966 x 2893 with 32^3 bricks is extended virtually to 4096^3 (N = 7)."""
    gd = _golden("paper_numbers.json")
    # pool: the oracle's brick count for a dense volume over 7 levels, relative to level 0
    M, N = 2, 6
    D = M << N
    rng = np.random.default_rng(5)
    v0 = rng.integers(0, 65536, size=(1, D, D, D), dtype=np.uint16)
    t = orc.Tree(v0, _full_mask(1, (D, D, D)), M, 0, 0)
    hdr, _, bricks = orc.parse_dump(t.dump())
    overhead = hdr["n_bricks"] * M ** 3 / D ** 3 - 1.0
    assert abs(overhead - gd["brick_pool_overhead"]["fraction"]) < 0.005, overhead
    # borders: bordered bricks in the oracle's dump are (M+2)^3
    Mb = gd["border_overhead_32"]["brick"]
    v1 = rng.integers(0, 65536, size=(1, Mb, Mb, Mb), dtype=np.uint16)
    t1 = orc.Tree(v1, _full_mask(1, (Mb, Mb, Mb)), Mb, 0, 0)
    hdr1, _, b1 = orc.parse_dump(t1.dump())
    per_brick = len(b1) // (hdr1["n_bricks"] * 2)     # uint16 voxels of one bordered brick
    assert per_brick == (Mb + 2) ** 3
    assert abs(per_brick / Mb ** 3 - 1.0 - gd["border_overhead_32"]["fraction"]) < 0.005
    # virtual extension
    ve = gd["virtual_extension"]
    n = orc.tree_depth(ve["dims"], ve["brick"])
    assert ve["brick"] << n == ve["virtual_edge"] and n == 7


def test_threshold_is_strict_and_per_channel(orc):
    dims = (4, 4, 4)
    v0 = np.full((2, 4, 4, 4), 100, np.uint16)
    v0[0, 0, 0, 0] = 105                       # channel 0 range 5
    for thr, expect in [(5, orc.ST_BRICK), (5.5, orc.ST_HOMOG_LEAF)]:
        t = orc.Tree(v0, _full_mask(2, dims), 4, 0, thr)
        assert t.node(0, 0, 0, 0)[0] == expect
    v0[1, 3, 3, 3] = 200                       # channel 1 not homogeneous
    t = orc.Tree(v0, _full_mask(2, dims), 4, 0, 50)
    assert t.node(0, 0, 0, 0)[0] == orc.ST_BRICK


def test_incomplete_nodes_are_never_merged(orc):
    """A partly inserted constant brick keeps its brick until it is complete (and a brick
    missing one channel is incomplete)."""
    dims = (8, 8, 8)
    ins = [(-1, (0, 0, 0), np.full((2, 4, 8, 8), 7, np.uint16))]
    v0, mask = orc.apply_inserts(dims, 2, ins)
    t = orc.Tree(v0, mask, 8, background=7, threshold=3)
    st, fl, _ = t.node(0, 0, 0, 0)
    assert st == orc.ST_BRICK and not fl & orc.F_COMPLETE
    ins.append((0, (0, 0, 4), np.full((1, 4, 8, 8), 7, np.uint16)))
    v0, mask = orc.apply_inserts(dims, 2, ins)
    t = orc.Tree(v0, mask, 8, background=7, threshold=3)
    assert t.node(0, 0, 0, 0)[0] == orc.ST_BRICK      # channel 1 still missing
    ins.append((1, (0, 0, 4), np.full((1, 4, 8, 8), 7, np.uint16)))
    v0, mask = orc.apply_inserts(dims, 2, ins)
    t = orc.Tree(v0, mask, 8, background=7, threshold=3)
    assert t.node(0, 0, 0, 0)[0] == orc.ST_HOMOG_LEAF


def test_constant_volume_prunes_to_root(orc):
    dims = (32, 24, 20)
    v0 = np.full((3, 20, 24, 32), 1234, np.uint16)
    t = orc.Tree(v0, _full_mask(3, dims), 4, 0, 1)
    hdr, recs, _ = orc.parse_dump(t.dump())
    assert hdr["n_nodes"] == 1 and recs["head"][0, 4] == orc.ST_HOMOG_LEAF
    assert list(recs["avg"][0, :3]) == [1234.0] * 3


def _represented_bf(levels, recs, M, C):
    """Brute force of R_L from the dump's node list: the deepest existing node at level >= L."""
    ex = {tuple(r["head"][:4]): (int(r["head"][4]), r["avg"][:C]) for r in recs}
    out = []
    for L, V in enumerate(levels):
        R = np.empty(V.shape, np.float64)
        _, ez, ey, exx = V.shape
        for z in range(ez):
            for y in range(ey):
                for x in range(exx):
                    b = (x // M, y // M, z // M)
                    l = L
                    while (l,) + b not in ex:
                        l += 1
                        b = (b[0] // 2, b[1] // 2, b[2] // 2)
                    st, avg = ex[(l,) + b]
                    R[:, z, y, x] = V[:, z, y, x] if (l == L and st == 3) else avg
        out.append(R)
    return out


@pytest.mark.parametrize("thr", [0, 90])
def test_bordered_bricks_bruteforce(orc, thr):
    """Every brick node's bordered brick equals R_L at the clamped neighbour indices."""
    dims, M, C = (13, 10, 9), 4, 2
    vol = synth.gen_volume(dims, C, seed=11, n_blobs=3)
    vol[:, :4, :, 4:8] = 60                  # one flat level-0 brick
    vol[:, :, 8:, :] = 70                    # flat bricks along the y border
    # insert part of the volume only, so EMPTY, homogeneous and brick nodes all occur
    ins = [(-1, (0, 0, 0), vol[:, :6]), (1, (0, 0, 6), vol[1:2, 6:])]
    v0, mask = orc.apply_inserts(dims, C, ins, background=50)
    t = orc.Tree(v0, mask, M, background=50, threshold=thr)
    hdr, recs, bricks = orc.parse_dump(t.dump())
    levels = np_mip(v0, M)
    R = _represented_bf(levels, recs, M, C)
    S = M + 2
    bk = np.frombuffer(bricks, np.uint16).reshape(-1, S, S, S, C)
    assert bk.shape[0] == hdr["n_bricks"]
    k = 0
    for r in recs:
        L, bx, by, bz, st = (int(v) for v in r["head"][:5])
        if st != orc.ST_BRICK:
            continue
        e = R[L].shape[1:]
        zz = np.clip(np.arange(S) + bz * M - 1, 0, e[0] - 1)
        yy = np.clip(np.arange(S) + by * M - 1, 0, e[1] - 1)
        xx = np.clip(np.arange(S) + bx * M - 1, 0, e[2] - 1)
        ref = R[L][:, zz][:, :, yy][:, :, :, xx].transpose(1, 2, 3, 0)
        assert np.array_equal(bk[k].astype(np.float64), ref), (L, bx, by, bz)
        k += 1
    assert k == hdr["n_bricks"]
    if thr == 0:
        assert (recs["head"][:, 4] == orc.ST_HOMOG_LEAF).sum() == 0
    else:
        assert (recs["head"][:, 4] == orc.ST_HOMOG_LEAF).sum() > 0
