"""Out-of-core rendering with a capped brick pool: renders request missing bricks (sampled with
their AVG meanwhile), brick_pool_upload pages them in (least recently used slots first,
coarser levels first), and the image converges to the in-core image.  Partially resident
images match the oracle rendering with the same residency set."""
import numpy as np
import pytest

from paper_1407_2074_amd import synth

pytestmark = pytest.mark.gpu

DIMS, C, M, THR = (128, 128, 96), 3, 16, 205


@pytest.fixture(scope="module")
def vol():
    return synth.gen_volume(DIMS, C, seed=12, n_blobs=60)


def _full(C, dims):
    return np.full((dims[2], dims[1], dims[0]), (1 << C) - 1, np.uint8)


def _tree(vol, slots=0, host=False):
    from paper_1407_2074_amd.octree import Octree
    probe = Octree(DIMS, C, M, "u16", 0, THR)
    bb = probe.brick_bytes
    probe.close()
    t = Octree(DIMS, C, M, "u16", 0, THR, pool_bytes=slots * bb, master_on_host=host)
    t.insert_block(-1, (0, 0, 0), vol)
    t.upload()
    return t


def _views():
    # alternating fixed levels: the views need different bricks, so a pool holding the largest
    # single working set cannot hold them all and switching views has to evict
    return [synth.make_view(DIMS, C, 12, az=az, el=25.0, width=64, height=64, lod=lod)
            for az, lod in ((10.0, 1), (100.0, 0), (190.0, 1), (280.0, 0))]


def _converge(t, v, max_iter=80):
    for it in range(max_iter):
        (img,) = t.render([v])
        st = t.upload()
        if st["requests_seen"] == 0:
            return img, st
    raise AssertionError("paging did not converge")


def _oracle_with_residency(orc, vol, dump):
    ref = orc.Tree(vol, _full(C, DIMS), M, 0, THR)
    _, recs, _ = orc.parse_dump(dump)
    missing = [tuple(int(x) for x in r["head"][:4]) for r in recs
               if r["head"][4] == orc.ST_BRICK and not (r["head"][5] & orc.F_RESIDENT)]
    ref.set_nonresident(missing)
    return ref, len(missing)


def test_paging_converges_to_in_core_image(orc, vol):
    import torch
    full = _tree(vol)
    views = _views()
    # working set of each view alone: a fresh tree whose pool is one slot short of holding
    # every brick, so that it pages on request
    n_all = full.pool_slots - 1
    ws = []
    for v in views:
        t = _tree(vol, slots=n_all)
        _, st = _converge(t, v)
        ws.append(st["bricks_resident"])
        t.close()
    cap = max(ws)
    assert cap < sum(ws)
    t = _tree(vol, slots=cap)
    total_evictions = 0
    checked_partial = False
    for v in views:
        (want,) = full.render([v])
        for it in range(80):
            (img,) = t.render([v])
            if not checked_partial:
                # nothing is resident yet: the first image uses AVG for every brick node
                ref, n_missing = _oracle_with_residency(orc, vol, t.dump())
                assert n_missing > 0
                (r,) = ref.render([v])
                assert np.abs(img.cpu().numpy() - r).max() <= 1e-4
                checked_partial = True
            st = t.upload()
            total_evictions += st["evictions"]
            if st["requests_seen"] == 0:
                break
        else:
            pytest.fail("paging did not converge")
        assert torch.equal(img, want)
    assert total_evictions > 0


def test_partial_residency_matches_oracle(orc, vol):
    """Mid-way through paging (small byte budget per upload), the image equals the oracle's
    rendering with exactly the residency the library reports."""
    t = _tree(vol, slots=200)
    v = _views()[1]
    for it in range(4):
        (img,) = t.render([v])
        ref, n_missing = _oracle_with_residency(orc, vol, t.dump())
        (r,) = ref.render([v])
        assert np.abs(img.cpu().numpy() - r).max() <= 1e-4, it
        t.upload(byte_budget=6 * t.brick_bytes)


def test_zero_budget_keeps_avg_rendering(orc, vol):
    t = _tree(vol, slots=64)
    v = _views()[2]
    (a,) = t.render([v])
    st = t.upload(byte_budget=1)            # less than one brick: nothing is paged in
    assert st["bricks_gathered"] == 0 and st["requests_seen"] > 0 and not st["complete"]
    (b,) = t.render([v])
    ref, _ = _oracle_with_residency(orc, vol, t.dump())
    (r,) = ref.render([v])
    assert np.abs(b.cpu().numpy() - r).max() <= 1e-4
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_master_in_pinned_host_memory(orc, vol):
    """The full-resolution mipmap in pinned host memory: same octree, same images."""
    import torch
    t = _tree(vol, host=True)
    ref = orc.Tree(vol, _full(C, DIMS), M, 0, THR)
    assert t.dump() == ref.dump()
    full = _tree(vol)
    for v in _views()[:2]:
        (a,) = t.render([v])
        (b,) = full.render([v])
        assert torch.equal(a, b)


@pytest.fixture(scope="module")
def cap(vol):
    """The largest working set of the four views (bricks resident once a view converged)."""
    full = _tree(vol)
    n_all = full.pool_slots - 1
    ws = []
    for v in _views():
        t = _tree(vol, slots=n_all)
        _, st = _converge(t, v)
        ws.append(st["bricks_resident"])
        t.close()
    return max(ws)


def _paged(vol, slots, **kw):
    from paper_1407_2074_amd.octree import Octree
    probe = Octree(DIMS, C, M, "u16", 0, THR)
    bb = probe.brick_bytes
    probe.close()
    return Octree(DIMS, C, M, "u16", 0, THR, pool_bytes=slots * bb, **kw)


def test_host_brick_store_pages_bricks_back_as_copies(orc, vol, cap):
    """With a host brick store the upload after an insert gathers every changed brick into the
    store (resident or not), so paging only copies stored bricks; every converged view equals
    the in-core image and the image equals the oracle's at the reported residency."""
    import torch
    full = _tree(vol)
    views = _views()
    t = _paged(vol, cap, host_bricks=True, master_on_host=True)
    t.insert_block(-1, (0, 0, 0), vol)
    t.upload()
    copied = gathered = 0
    for v in views + views:            # the second round re-requests evicted bricks
        (want,) = full.render([v])
        for it in range(80):
            (img,) = t.render([v])
            st = t.upload()
            copied += st["bricks_from_store"]
            gathered += st["bricks_gathered"] - st["bricks_from_store"]
            if st["requests_seen"] == 0:
                break
        else:
            pytest.fail("paging did not converge")
        assert torch.equal(img, want)
    assert copied > 0 and gathered == 0
    ref, _ = _oracle_with_residency(orc, vol, t.dump())
    (r,) = ref.render([views[0]])
    (img,) = t.render([views[0]])
    assert np.abs(img.cpu().numpy() - r).max() <= 1e-4


def test_host_brick_store_follows_new_data(orc, cap):
    """Bricks stored before more data arrives are not reused once their data (or a neighbour's
    border data) changed: after the second half of the volume is inserted, paging converges to
    the in-core image of the whole volume."""
    import torch
    vol = synth.gen_volume(DIMS, C, seed=13, n_blobs=60)
    half = DIMS[2] // 2
    t = _paged(vol, cap + 40, host_bricks=True)
    full = _tree(vol)
    views = _views()
    t.insert_slices(-1, 0, np.ascontiguousarray(vol[:, :half]))
    t.upload()
    for v in views:                    # page (and store) bricks of the half volume
        for it in range(80):
            t.render([v])
            if t.upload()["requests_seen"] == 0:
                break
    t.insert_slices(-1, half, np.ascontiguousarray(vol[:, half:]))
    t.upload()
    copied = 0
    for v in views:
        (want,) = full.render([v])
        for it in range(80):
            (img,) = t.render([v])
            st = t.upload()
            copied += st["bricks_from_store"]
            if st["requests_seen"] == 0:
                break
        else:
            pytest.fail("paging did not converge")
        assert torch.equal(img, want)
    want_dump = orc.Tree(vol, _full(C, DIMS), M, 0, THR)
    ref, _ = _oracle_with_residency(orc, vol, t.dump())
    (r,) = ref.render([views[1]])
    (img,) = t.render([views[1]])
    assert np.abs(img.cpu().numpy() - r).max() <= 1e-4
    assert want_dump.levels == t.levels
