"""Pins for the oracle's per-node statistics and states on non-constant volumes (CPU only).

Every existing node of the oracle's canonical dump is compared, record by record, with an
independent recomputation written here from the definitions (section "CPU Data Structure" for
homogeneity and AVG, "Handling Multi-Channel Data" for per-channel completeness, "Handling
Volumes of Arbitrary Dimensions" for the valid extents):

* the mipmap comes from the numpy reshape-sum of ``helpers.np_mip`` (pinned on its own);
* bmin / bmax / bsum: numpy reductions over the node's own level-L brick, valid voxels only;
* AVG: u16 -- the exact rational mean of that brick rounded half up (``fractions.Fraction``);
  f32 -- a float32 value within half a float32 ulp of the exact rational mean;
* smin / smax: numpy reductions of level 0 over the node's level-0 region;
* populated / complete: any / every valid level-0 voxel inserted in every channel (mask bits);
* states by a recursive descent from the root: the first complete node whose subtree range is
  below the threshold in every channel is a homogeneous leaf; a complete node whose own brick
  range is below it keeps its children; other populated nodes hold bricks; unpopulated nodes are
  empty leaves with the background as AVG.
"""
import zlib
from fractions import Fraction

import numpy as np
import pytest

from helpers import np_mip

ST_EMPTY, ST_HOMOG_LEAF, ST_HOMOG, ST_BRICK = 0, 1, 2, 3


def _depth(dims, M):
    n = 0
    while M << n < max(dims):
        n += 1
    return n


def _avg_u16(bsum: int, count: int) -> int:
    q = Fraction(bsum, count) + Fraction(1, 2)
    return q.numerator // q.denominator        # floor of mean + 1/2: halves round up


def _f32_ulp(x: float) -> float:
    x32 = np.float32(x)
    return float(np.spacing(np.abs(x32)))


def expected_nodes(v0, mask, M, background, thr):
    """{(L, bx, by, bz): dict(state, flags, avg, bmin, bmax, smin, smax)} for existing nodes."""
    C, Dz, Dy, Dx = v0.shape
    dims = (Dx, Dy, Dz)
    N = _depth(dims, M)
    levels = np_mip(v0, M)
    allbits = (1 << C) - 1
    info = {}
    for L in range(N + 1):
        G = 1 << (N - L)
        lev = levels[L]
        span = M << L
        for bz in range(G):
            for by in range(G):
                for bx in range(G):
                    b = (bx, by, bz)
                    own = tuple(slice(b[a] * M, min((b[a] + 1) * M, lev.shape[3 - a]))
                                for a in (2, 1, 0))
                    reg = tuple(slice(b[a] * span, min((b[a] + 1) * span, dims[a]))
                                for a in (2, 1, 0))
                    blk = lev[(slice(None),) + own]
                    r0 = v0[(slice(None),) + reg]
                    m0 = mask[reg]
                    d = dict(count=blk[0].size, nvalid=m0.size)
                    if d["count"]:
                        if v0.dtype == np.uint16:
                            d["bsum"] = [int(blk[c].astype(np.int64).sum()) for c in range(C)]
                        else:   # every value is a multiple of 2^-16: Fraction sums are exact
                            d["bsum"] = [sum(Fraction(float(x)) for x in blk[c].ravel())
                                         for c in range(C)]
                        d["bmin"] = [float(blk[c].min()) for c in range(C)]
                        d["bmax"] = [float(blk[c].max()) for c in range(C)]
                        d["smin"] = [float(r0[c].min()) for c in range(C)]
                        d["smax"] = [float(r0[c].max()) for c in range(C)]
                    d["populated"] = bool(m0.size) and bool((m0 != 0).any())
                    d["complete"] = bool(m0.size) and bool((m0 == allbits).all())
                    info[(L,) + b] = d

    out = {}

    def visit(L, b):
        d = info[(L,) + b]
        rec = dict(bmin=[0.0] * C, bmax=[0.0] * C, smin=[0.0] * C, smax=[0.0] * C)
        flags = (2 if d["complete"] else 0) | (4 if d["populated"] else 0)
        if not d["populated"]:
            bg = float(background) if v0.dtype == np.uint16 else float(np.float32(background))
            rec.update(state=ST_EMPTY, flags=flags, avg=[bg] * C, exact=None)
            out[(L,) + b] = rec
            return
        if v0.dtype == np.uint16:
            avg = [float(_avg_u16(s, d["count"])) for s in d["bsum"]]
            exact = None
        else:
            exact = [s / d["count"] for s in d["bsum"]]
            avg = None
        rec.update(bmin=d["bmin"], bmax=d["bmax"], smin=d["smin"], smax=d["smax"], avg=avg,
                   exact=exact)
        sub = d["complete"] and all(d["smax"][c] - d["smin"][c] < thr for c in range(C))
        own = d["complete"] and all(d["bmax"][c] - d["bmin"][c] < thr for c in range(C))
        if sub:
            rec.update(state=ST_HOMOG_LEAF, flags=flags)
            out[(L,) + b] = rec
            return
        kids = L > 0
        rec.update(state=ST_HOMOG if own else ST_BRICK, flags=flags | (1 if kids else 0))
        out[(L,) + b] = rec
        if kids:
            for dz in (0, 1):
                for dy in (0, 1):
                    for dx in (0, 1):
                        visit(L - 1, (2 * b[0] + dx, 2 * b[1] + dy, 2 * b[2] + dz))

    visit(N, (0, 0, 0))
    return out


def check_dump_against(orc, dump: bytes, v0, mask, M, background, thr):
    hdr, recs, _ = orc.parse_dump(dump)
    C = v0.shape[0]
    want = expected_nodes(v0, mask, M, background, thr)
    got = {tuple(int(v) for v in r["head"][:4]): r for r in recs}
    assert set(got) == set(want), sorted(set(got) ^ set(want))[:8]
    n_checked = 0
    for key, w in want.items():
        r = got[key]
        assert int(r["head"][4]) == w["state"], (key, int(r["head"][4]), w["state"])
        assert int(r["head"][5]) & 7 == w["flags"], (key, int(r["head"][5]), w["flags"])
        for f in ("bmin", "bmax", "smin", "smax"):
            assert list(r[f][:C]) == w[f], (key, f, list(r[f][:C]), w[f])
        if w["exact"] is None:
            assert list(r["avg"][:C]) == w["avg"], (key, list(r["avg"][:C]), w["avg"])
        else:
            for c in range(C):
                a = float(r["avg"][c])
                assert float(np.float32(a)) == a, (key, "AVG is not a float32 value")
                assert abs(Fraction(a) - w["exact"][c]) <= Fraction(_f32_ulp(a)) / 2, (key, c)
        n_checked += 1
    return want, n_checked


def _patchy_volume(rng, C, dims, dtype):
    """Noise whose amplitude varies per 3x3x3 patch (0 .. 400), on a per-channel offset, so
    that homogeneous and inhomogeneous bricks and subtrees occur at every level."""
    Dx, Dy, Dz = dims
    amp = rng.choice([0, 0, 3, 20, 400], size=(C, -(-Dz // 3), -(-Dy // 3), -(-Dx // 3)))
    amp = amp.repeat(3, 1).repeat(3, 2).repeat(3, 3)[:, :Dz, :Dy, :Dx]
    base = rng.integers(200, 3000, size=(C, 1, 1, 1))
    v = base + (rng.random((C, Dz, Dy, Dx)) * (amp + 1)).astype(np.int64)
    v = v.astype(np.uint16)
    if dtype == "f32":
        return (v.astype(np.float32) * np.float32(2.0 ** -16)).astype(np.float32)
    return v


CASES = [
    # dims, M, dtype, threshold (in u16 units)
    ((13, 9, 7), 2, "u16", 0),
    ((13, 9, 7), 2, "u16", 30),
    ((21, 17, 11), 4, "u16", 25),
    ((19, 14, 25), 6, "u16", 25),
    ((12, 11, 9), 4, "f32", 25),
    ((23, 7, 10), 6, "f32", 0),
]


@pytest.mark.parametrize("dims,M,dtype,thr", CASES)
def test_node_statistics_full_insert(orc, dims, M, dtype, thr):
    rng = np.random.default_rng(zlib.crc32(repr((dims, M, dtype, thr)).encode()))
    C = 3
    v0 = _patchy_volume(rng, C, dims, dtype)
    Dx, Dy, Dz = dims
    mask = np.full((Dz, Dy, Dx), (1 << C) - 1, np.uint8)
    t_thr = thr if dtype == "u16" else thr * 2.0 ** -16
    t = orc.Tree(v0, mask, M, background=0, threshold=t_thr)
    want, n = check_dump_against(orc, t.dump(), v0, mask, M, 0, t_thr)
    states = {w["state"] for w in want.values()}
    assert ST_BRICK in states
    if thr > 0:
        assert ST_HOMOG_LEAF in states
    # non-constant nodes are the point of this test: most have bmin < bmax
    nonconst = sum(1 for w in want.values() if w["state"] != ST_EMPTY
                   and any(a < b for a, b in zip(w["bmin"], w["bmax"])))
    assert nonconst >= n // 3


@pytest.mark.parametrize("dims,M,thr", [((17, 13, 11), 4, 0), ((17, 13, 11), 4, 40),
                                        ((15, 10, 9), 2, 40), ((19, 9, 14), 6, 40)])
def test_node_statistics_partial_and_per_channel_inserts(orc, dims, M, thr):
    """Partly inserted volumes (cuboid blocks, single channels, overwrites): background
    voxels, incomplete and unpopulated nodes, and homogeneous merges only where complete."""
    rng = np.random.default_rng(sum(dims) * 7 + M + thr)
    C, bg = 3, 150
    vol = _patchy_volume(rng, C, dims, "u16")
    Dx, Dy, Dz = dims
    ins = [
        (-1, (0, 0, 0), vol[:, :Dz // 2]),                                  # lower half, all
        (1, (0, 0, Dz // 2), vol[1:2, Dz // 2:]),                           # upper half, ch 1
        (0, (Dx // 3, 0, Dz // 2), vol[0:1, Dz // 2:, :, Dx // 3:]),        # part of ch 0
        (-1, (1, 2, 1), np.full((C, 3, 4, 5), 999, np.uint16)),             # overwrite a box
    ]
    v0, mask = orc.apply_inserts(dims, C, ins, background=bg)
    t = orc.Tree(v0, mask, M, background=bg, threshold=thr)
    want, _ = check_dump_against(orc, t.dump(), v0, mask, M, bg, thr)
    flags = [w["flags"] for w in want.values()]
    assert any(not f & 4 for f in flags)             # unpopulated nodes
    assert any(f & 4 and not f & 2 for f in flags)   # populated but incomplete
