"""Continuous-batching render server over a device-resident octree.

Requests (camera, image size, transfer functions, clipping planes) arrive over time.  Each is
split into 8x8-pixel tiles; every scheduler tick builds ONE render_views launch from the tile
chunks of all admitted requests (oldest first, round-robin over requests within the tick's
tile budget) and enqueues it on the next of K HIP streams, so launches of different ticks run
concurrently and a small request is never stuck behind a large one.  A request completes when
the event of the last launch holding one of its tiles has fired.  Latency is arrival ->
completion.

Admission is by device memory:
  * framebuffer: the images of the admitted requests stay under `fb_cap_bytes`;
  * brick pool: the bricks the admitted requests sample stay under `pool_cap_bytes` (default:
    the octree's pool cap; none for an uncapped, fully resident octree).  Requests at the same level of detail share bricks, so the demand of a
    set of requests is the sum, over the distinct levels they render at, of the level's brick
    nodes (the cells of that level inside the volume -- an upper bound) times the brick size.
    A request's level is its fixed LOD, or for the per-ray footprint LOD the level whose voxel
    projects to about one pixel at the distance from its eye to the volume centre.
A request that alone exceeds a cap is admitted when nothing else is in flight.

Each pixel depends only on its own ray, so a request's image is the same whether it is
rendered alone or inside any mix (bit-identical).
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time

import numpy as np

from .octree import Octree

TILE = 8


@dataclasses.dataclass(eq=False)          # requests compare and hash by identity
class Request:
    rid: int
    view: object            # synth.View (or same attributes)
    arrival: float          # seconds from the start of the run
    image: object = None    # torch CUDA tensor [H][W][4] once admitted
    next_tile: int = 0
    pending: int = 0        # launches in flight that hold tiles of this request
    admitted: float = -1.0
    done: float = -1.0
    lod_level: int = 0      # level of detail it renders at (set on admission)

    @property
    def n_tiles(self) -> int:
        return math.ceil(self.view.width / TILE) * math.ceil(self.view.height / TILE)

    @property
    def fb_bytes(self) -> int:
        return self.view.width * self.view.height * 16

    def level(self, N: int, dims) -> int:
        """The level of detail the request renders at (see the module docstring)."""
        v = self.view
        if v.lod >= 0:
            return min(int(v.lod), N)
        centre = np.array(dims, np.float64) / 2
        dist = float(np.linalg.norm(np.asarray(v.eye, np.float64) - centre))
        w = 2.0 * dist * math.tan(math.radians(v.fov_y_deg) / 2) / v.height
        return int(min(max(math.floor(math.log2(w)), 0), N)) if w > 0 else 0


@dataclasses.dataclass
class ServeStats:
    completed: int
    makespan_s: float
    requests_per_s: float
    latency_p50_ms: float
    latency_p99_ms: float
    latency_mean_ms: float
    launches: int
    max_fb_bytes_in_use: int
    max_in_flight: int
    max_pool_bytes_in_use: int = 0

    def as_dict(self):
        return dataclasses.asdict(self)


class Server:
    """Tile-level continuous batching on `streams` HIP streams.

    tiles_per_launch: upper bound on the 8x8 tiles one launch carries (4 tiles per workgroup;
    a full MI355X wants a few thousand workgroups); fb_cap_bytes: framebuffer memory cap for
    admitted requests; chunk_tiles: largest tile range of one request inside one launch."""

    def __init__(self, tree: Octree, streams: int = 3, tiles_per_launch: int = 16384,
                 chunk_tiles: int = 4096, fb_cap_bytes: int = 2 << 30, max_in_flight: int = 3,
                 pool_cap_bytes: int | None = None):
        import torch
        self.torch = torch
        self.tree = tree
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.tiles_per_launch = tiles_per_launch
        self.chunk_tiles = chunk_tiles
        self.fb_cap = fb_cap_bytes
        self.max_in_flight = min(max_in_flight, streams)
        # default: the octree's capped pool; an uncapped octree holds every brick, so no set
        # of requests can exceed it
        if pool_cap_bytes is None:
            pool_cap_bytes = tree.pool_bytes if tree.pool_bytes > 0 else float("inf")
        self.pool_cap = pool_cap_bytes
        # brick nodes per level at most: the level's cells inside the volume
        M, N = tree.M, tree.levels - 1
        self.N = N
        self.level_bytes = []
        for L in range(N + 1):
            cells = 1
            for d in tree.dims:
                ext = -(-d // (1 << L))          # valid extent of level L along this axis
                cells *= -(-ext // M)            # its cells, rounded up
            self.level_bytes.append(cells * tree.brick_bytes)

    def pool_demand(self, levels) -> int:
        """Brick-pool bytes of requests rendering at these levels (each level's bricks once)."""
        return sum(self.level_bytes[L] for L in set(levels))

    def run(self, requests, realtime: bool = True, on_complete=None) -> ServeStats:
        """Serve `requests` (sorted by arrival).  With realtime=False arrivals are taken as
        already due (closed-loop throughput); otherwise a request cannot be admitted before
        its arrival time on the wall clock."""
        torch = self.torch
        queue = collections.deque(sorted(requests, key=lambda r: r.arrival))
        active: list[Request] = []
        inflight = collections.deque()        # (event, [requests], stream)
        fb_used = max_fb = max_pool = 0
        launches = max_inflight = 0
        level_use = collections.Counter()     # admitted requests per level of detail
        done: list[Request] = []
        si = 0
        t_start = time.perf_counter()

        def now():
            return time.perf_counter() - t_start

        while queue or active or inflight:
            # retire finished launches (in order per stream; any order across streams)
            progressed = False
            for _ in range(len(inflight)):
                ev, reqs, _s = inflight[0]
                if not ev.query():
                    inflight.rotate(-1)
                    continue
                inflight.popleft()
                progressed = True
                for r in reqs:
                    r.pending -= 1
                    if r.pending == 0 and r.next_tile >= r.n_tiles:
                        r.done = now()
                        active.remove(r)
                        fb_used -= r.fb_bytes
                        level_use[r.lod_level] -= 1
                        if level_use[r.lod_level] == 0:
                            del level_use[r.lod_level]
                        done.append(r)
                        if on_complete:
                            on_complete(r)
            # admit arrivals while framebuffer and brick-pool memory allow
            t = now()
            while queue and (not realtime or queue[0].arrival <= t):
                r = queue[0]
                r.lod_level = r.level(self.N, self.tree.dims)
                pool = self.pool_demand(list(level_use) + [r.lod_level])
                if active and (fb_used + r.fb_bytes > self.fb_cap or pool > self.pool_cap):
                    break
                queue.popleft()
                level_use[r.lod_level] += 1
                max_pool = max(max_pool, pool)
                r.image = torch.empty((r.view.height, r.view.width, 4), dtype=torch.float32,
                                      device="cuda")
                r.admitted = t
                fb_used += r.fb_bytes
                max_fb = max(max_fb, fb_used)
                active.append(r)
            # build one launch from the tiles not yet scheduled
            todo = [r for r in active if r.next_tile < r.n_tiles]
            if todo and len(inflight) < self.max_in_flight:
                budget = self.tiles_per_launch
                views, images, owners = [], [], []
                while budget > 0 and todo:
                    for r in list(todo):
                        n = min(self.chunk_tiles, r.n_tiles - r.next_tile, budget)
                        v = dataclasses.replace(r.view, tile_begin=r.next_tile, tile_count=n) \
                            if dataclasses.is_dataclass(r.view) else r.view
                        views.append(v)
                        images.append(r.image)
                        owners.append(r)
                        r.next_tile += n
                        budget -= n
                        if r.next_tile >= r.n_tiles:
                            todo.remove(r)
                        if budget <= 0:
                            break
                stream = self.streams[si]
                si = (si + 1) % len(self.streams)
                with torch.cuda.stream(stream):
                    self.tree.render(views, images=images, stream=stream.cuda_stream)
                    ev = torch.cuda.Event()
                    ev.record(stream)
                for im in images:
                    im.record_stream(stream)   # framebuffers stay reserved until the launch ends
                uniq = list(dict.fromkeys(owners))
                for r in uniq:
                    r.pending += 1
                inflight.append((ev, uniq, stream))
                launches += 1
                max_inflight = max(max_inflight, len(inflight))
                progressed = True
            if not progressed:
                if inflight:
                    time.sleep(0.0002)
                elif queue and realtime:
                    time.sleep(max(0.0, min(0.002, queue[0].arrival - now())))
        torch.cuda.synchronize()
        makespan = now()
        lat = np.array([(r.done - r.arrival) * 1e3 for r in done]) if done else np.zeros(1)
        return ServeStats(completed=len(done), makespan_s=makespan,
                          requests_per_s=len(done) / makespan if makespan > 0 else 0.0,
                          latency_p50_ms=float(np.percentile(lat, 50)),
                          latency_p99_ms=float(np.percentile(lat, 99)),
                          latency_mean_ms=float(lat.mean()), launches=launches,
                          max_fb_bytes_in_use=max_fb, max_in_flight=max_inflight,
                          max_pool_bytes_in_use=max_pool)


def poisson_requests(dims, channels: int, n: int, rate: float, seed: int = 5,
                     sizes=(256, 512, 1024, 2048)):
    """Seeded request mix: Poisson arrivals, image size uniform in `sizes`, orbit cameras
    (az ~ U[0, 360), el ~ U[-60, 60], distance x U[0.9, 1.1]), per-request transfer functions
    and 0-3 clipping planes with random normals through centre + U[-1/4, 1/4] * D."""
    from . import synth
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    centre = np.array(dims, np.float64) / 2
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        s = int(rng.choice(sizes))
        v = synth.make_view(dims, channels, 1000 + i, az=float(rng.uniform(0, 360)),
                            el=float(rng.uniform(-60, 60)), width=s, height=s, lod=-1,
                            dist_scale=float(rng.uniform(0.9, 1.1)))
        clips = []
        for _ in range(int(rng.integers(0, 4))):
            nrm = rng.normal(size=3)
            nrm /= np.linalg.norm(nrm)
            pt = centre + rng.uniform(-0.25, 0.25, size=3) * np.array(dims)
            clips.append((float(nrm[0]), float(nrm[1]), float(nrm[2]), float(nrm @ pt)))
        v.clips = clips
        out.append(Request(rid=i, view=v, arrival=t))
    return out
