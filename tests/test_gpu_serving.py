"""Continuous batching: every request's image is bit-identical whether rendered alone or in the
mix, the framebuffer cap is respected, and the latency accounting is consistent."""
import numpy as np
import pytest

from paper_1407_2074_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def served_tree():
    import torch
    from paper_1407_2074_amd.octree import Octree
    dims, C, M = (128, 128, 64), 3, 16
    vol = synth.gen_volume(dims, C, seed=2, n_blobs=60)
    t = Octree(dims, C, M, "u16", 0, 205)
    t.insert_block(-1, (0, 0, 0), torch.from_numpy(vol.view(np.int16)).cuda())
    t.upload()
    torch.cuda.synchronize()
    return dims, C, t


def test_alone_equals_mix(served_tree):
    import torch
    from paper_1407_2074_amd.serving import Server, poisson_requests
    dims, C, t = served_tree
    reqs = poisson_requests(dims, C, 40, rate=2000.0, seed=5, sizes=(16, 40, 64, 128))
    got = {}
    srv = Server(t, streams=3, tiles_per_launch=300, chunk_tiles=64, fb_cap_bytes=600_000)
    st = srv.run(reqs, realtime=True, on_complete=lambda r: got.__setitem__(r.rid, r.image.clone()))
    torch.cuda.synchronize()
    assert st.completed == len(reqs) == len(got)
    assert st.launches > 1 and st.max_in_flight >= 2
    biggest = max(r.fb_bytes for r in reqs)
    assert st.max_fb_bytes_in_use <= max(600_000, biggest)
    for r in reqs:
        v = r.view
        (alone,) = t.render([v])
        assert torch.equal(alone, got[r.rid]), r.rid
        assert r.done >= r.admitted >= r.arrival - 1e-3
    assert st.latency_p99_ms >= st.latency_p50_ms > 0


def test_closed_loop_throughput(served_tree):
    from paper_1407_2074_amd.serving import Server, poisson_requests
    dims, C, t = served_tree
    reqs = poisson_requests(dims, C, 24, rate=1e6, seed=6, sizes=(32, 64, 128, 256))
    st = Server(t, streams=2).run(reqs, realtime=False)
    assert st.completed == 24 and st.requests_per_s > 0
