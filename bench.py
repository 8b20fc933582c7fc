"""Benchmark: streamed octree build + render of a 3-channel 512x512x256 uint16 volume.

One step is the whole streamed workload: the octree is cleared, then 32 batches of 8 z-slices
(already resident in HBM) are inserted; after each batch brick_pool_upload applies the changes
and one 1024x1024 view (orbit az 45 el 30, step 0.5, per-ray footprint LOD) is rendered.
Insertion and uploads run on a stream of their own (the library orders it against the render
stream), so the next batch is inserted and analysed while the current one renders.  32^3 bricks,
homogeneity threshold 205, seeded synthetic blob + Poisson data (stand-in for the paper's SPIM
scans).

Prints one JSON line.  `value` is composited sample positions per second over the whole step
(build time included); render-only, nominal and frame rates are reported beside it, with the
render kernel's roofline (VALU-bound: algorithmic FP32 flops per second against the published
FP32 peak), the CPU oracle timed on a bounded sample, and further legs: the build kernels'
algorithmic GB/s (streamed and whole-volume), MIP on the final octree, the adjoint at 256^3
f32, and the out-of-core 2048x2048x1024 orbit-and-dolly path with its own oracle sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP32 flops per composited position (FMA = 2): position 8 + compositing 3x8
# for every position; a position interpolated inside a brick adds local coordinates 12,
# trilinear 3x21 and classification 3x15.
FLOPS_ANY = 8 + 24
FLOPS_TRILINEAR = 12 + 63 + 45
# MI355X's published FP32 vector peak (it counts packed two-wide FMAs) -- the roofline's peak
PEAK_FP32_TFLOPS = 157.3
# 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz x 2 (FMA): the ceiling of FP32 without packed math,
# which this build never emits (reported beside the published peak)
NONPACKED_FP32_TFLOPS = 78.6
PEAK_HBM_GBPS = 8000.0

# HBM bytes per render launch of the default workload, from FETCH_SIZE / WRITE_SIZE counter
# runs scaled by the same counters over a plain 1 GiB copy; valid only for the kernel code
# they were taken on (its sources are hashed without comments, with the compile flags)
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_render_u16_hbm_traffic_stream_512x512x256.md")
RENDER_SOURCES = ("render_kernels.hip", "raycommon.h", "internal.h")
# the workload those counters were taken on (the default streamed configuration)
TRAFFIC_WORKLOAD = "stream 512x512x256x3 u16 M32 1024x1024"


def render_code_hash() -> str:
    import hashlib
    import re
    from paper_1407_2074_amd import build
    h = hashlib.sha256(" ".join(build.HIPCC_FLAGS).encode())
    for name in RENDER_SOURCES:
        txt = open(os.path.join(ROOT, "paper_1407_2074_amd", "csrc", name)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        txt = re.sub(r"//[^\n]*", "", txt)
        h.update(" ".join(txt.split()).encode())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per render launch from the committed counter profile, when it was taken on
    this workload and on the current kernel code; else None."""
    import re
    try:
        txt = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    b = re.search(r"traffic_bytes_per_launch:\s*(\d+)", txt)
    h = re.search(r"kernel_code_sha256:\s*([0-9a-f]{64})", txt)
    w = re.search(r"workload_key:\s*(.+)", txt)
    if not b or not h or not w or h.group(1) != render_code_hash():
        return None
    if w.group(1).strip() != workload:
        return None
    return int(b.group(1))

CFG = {
    2: dict(dims=(512, 512, 256), C=3, M=32, seed=2, blobs=2000, thr=205, batch=8,
            width=1024, height=1024, az=45.0, el=30.0, lod=-1),
    1: dict(dims=(64, 64, 64), C=3, M=16, seed=1, blobs=20, thr=205, batch=8,
            width=128, height=128, az=30.0, el=20.0, lod=0),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2, choices=sorted(CFG))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="stream workload: skip the adjoint leg (256^3 f32, 512x512)")
    ap.add_argument("--no-paging", action="store_true",
                    help="stream workload: skip the out-of-core leg (2048x2048x1024)")
    ap.add_argument("--no-build", action="store_true",
                    help="stream workload: skip the whole-volume build and MIP legs")
    ap.add_argument("--no-disk", action="store_true",
                    help="leave out the disk-tier leg (streamed build through a page file)")
    ap.add_argument("--no-serve", action="store_true",
                    help="stream workload: skip the serving leg (2000 Poisson requests)")
    ap.add_argument("--serve-only", action="store_true",
                    help="serve workload: skip the one-view-per-launch comparison loop")
    ap.add_argument("--streams", type=int, default=2, choices=[1, 2],
                    help="stream workload: 2 = build and render on separate streams")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    ap.add_argument("--no-host-bricks", action="store_true",
                    help="paging workload / leg: no host brick store (every paged brick is "
                         "gathered from the pinned mipmap)")
    ap.add_argument("--scale", type=int, default=1, choices=[1, 2, 4],
                    help="paging workload / leg: 1 = 2048x2048x1024, 2 = half and 4 = quarter "
                         "size per axis")
    ap.add_argument("--workload", default="stream",
                    choices=["stream", "adjoint", "serve", "views", "paging", "build", "mip",
                             "disk"],
                    help="stream: streamed build+render (default); adjoint: 256^3 f32 forward + "
                         "adjoint at 512x512; serve: Poisson request mix; views: 64 views of "
                         "the 64^3 volume in one launch vs one launch per view; paging: the "
                         "out-of-core path alone; build: whole-volume build of the 512x512x256 "
                         "volume; mip: MIP renders of the 512x512x256 octree; disk: the streamed "
                         "step, then the same step with the mipmap in the disk tier")
    args = ap.parse_args()
    if args.workload == "disk":   # the streamed step and the disk-tier leg only
        args.workload = "stream"
        args.no_cpu_baseline = args.no_adjoint = args.no_build = True
        args.no_serve = args.no_paging = True
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU design is described but not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1407_2074_amd import synth
    from paper_1407_2074_amd.octree import Octree

    if args.workload not in ("stream", "build", "mip"):
        {"adjoint": bench_adjoint, "serve": bench_serve, "views": bench_views,
         "paging": bench_paging}[args.workload](args)
        return

    cfg = CFG[args.config]
    dims, C, M = cfg["dims"], cfg["C"], cfg["M"]
    torch.cuda.set_device(0)
    t_gen = time.perf_counter()
    vol = synth.gen_volume(dims, C, seed=cfg["seed"], n_blobs=cfg["blobs"])
    print(f"[bench] generated {dims} x{C} in {time.perf_counter() - t_gen:.1f}s", file=sys.stderr,
          flush=True)
    dev = torch.from_numpy(vol.view(np.int16)).cuda()
    if args.copy_probe_mib:
        # a plain device copy of known size: calibrates the FETCH_SIZE / WRITE_SIZE counters
        a = torch.empty(args.copy_probe_mib << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.workload == "build":
        print(json.dumps(measure_build(dev, cfg, args)), flush=True)
        return
    if args.workload == "mip":
        t = Octree(dims, C, M, "u16", background=0, threshold=cfg["thr"])
        t.insert_block(-1, (0, 0, 0), dev)
        t.upload()
        print(json.dumps(measure_mip(t, cfg, args)), flush=True)
        return
    nb = dims[2] // cfg["batch"]
    slabs = [dev[:, b * cfg["batch"]:(b + 1) * cfg["batch"]].contiguous() for b in range(nb)]
    tree = Octree(dims, C, M, "u16", background=0, threshold=cfg["thr"])
    view = synth.make_view(dims, C, cfg["seed"], az=cfg["az"], el=cfg["el"], width=cfg["width"],
                           height=cfg["height"], lod=cfg["lod"])
    img = torch.zeros((view.height, view.width, 4), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    # insertion and uploads on their own stream: the library orders the two streams, and the
    # next batch's insertion and statistics run while the current batch renders
    bstream = torch.cuda.Stream() if args.streams == 2 else stream

    def step(stats=None, events=None):
        tree.clear(stream=bstream)
        for b in range(nb):
            tree.insert_slices(-1, b * cfg["batch"], slabs[b], stream=bstream)
            tree.upload(stream=bstream)
            if events is not None:
                # the render waits for this upload anyway; waiting before the start event
                # keeps the timed interval to the render itself
                stream.wait_stream(bstream)
                events[b][0].record(stream)
            if stats is not None:
                _, st = tree.render([view], images=[img], stats=True, stream=stream)
                stats.append(st)
            else:
                tree.render([view], images=[img], stream=stream)
            if events is not None:
                events[b][1].record(stream)

    # warm-up; the first warm-up step also counts positions (deterministic per step)
    per_batch = []
    for w in range(max(args.warmup, 1)):
        step(stats=per_batch if w == 0 else None)
    torch.cuda.synchronize()
    nominal = sum(s["positions_nominal"] for s in per_batch)
    composited = sum(s["positions_composited"] for s in per_batch)
    trilinear = sum(s["positions_trilinear"] for s in per_batch)
    flops_step = FLOPS_ANY * composited + FLOPS_TRILINEAR * trilinear

    evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in range(nb)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    tree.render_timing(True)   # HIP events around each ray-casting kernel, on its stream
    tree.build_timing(True)    # and around the build kernels, on theirs
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events=evs[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms, kernel_n = tree.render_timing(False)
    build_ms, build_bytes = tree.build_timing(False)
    render_ms = sum(e[0].elapsed_time(e[1]) for ev in evs for e in ev)   # whole render calls
    n_launch = args.steps * nb
    assert kernel_n == n_launch, (kernel_n, n_launch)
    render_s = render_ms / 1e3
    ms_per_step = elapsed / args.steps * 1e3

    value = composited * args.steps / elapsed / 1e9
    achieved_tflops = flops_step * args.steps / (kernel_ms / 1e3) / 1e12
    workload_key = (f"stream {dims[0]}x{dims[1]}x{dims[2]}x{C} u16 M{M} "
                    f"{cfg['width']}x{cfg['height']}")
    traffic = measured_traffic(workload_key) if args.streams == 2 else None
    out = {
        "metric": "Gsamples/s + frames/s, 3-ch octree raycast fwd & adjoint, % HBM peak",
        "value": round(value, 3),
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded blobs + Poisson noise; stand-in for the paper's SPIM scans)",
        "config": {"workload": f"streamed build+render {dims[0]}x{dims[1]}x{dims[2]}x{C} u16, "
                               f"{M}^3 bricks, {nb} batches of {cfg['batch']} slices, one "
                               f"{cfg['width']}x{cfg['height']} view per batch",
                   "threshold": cfg["thr"], "step_voxels": 0.5, "lod": "per-ray footprint"
                   if cfg["lod"] < 0 else cfg["lod"]},
        "frames_per_s": round(nb * args.steps / elapsed, 2),
        "render_only_gsamples_per_s": round(composited * args.steps / render_s / 1e9, 3),
        "render_frames_per_s": round(n_launch / render_s, 2),
        "nominal_positions_per_step": nominal,
        "composited_positions_per_step": composited,
        "trilinear_positions_per_step": trilinear,
        "render_ms_per_launch": round(render_ms / n_launch, 4),
        "render_kernel_ms_per_launch": round(kernel_ms / n_launch, 4),
        "streams": args.streams,
        "non_render_ms_per_step": round(ms_per_step - render_ms / args.steps, 3),
        "hbm_pct_of_peak": (round(100.0 * traffic / (kernel_ms / n_launch / 1e3) /
                                  (PEAK_HBM_GBPS * 1e9), 2) if traffic else None),
        "roofline": {"bound": "alu", "achieved": round(achieved_tflops, 3),
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved_tflops / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
                     "kernel": "k_render_u16<3, true, false>",
                     "flops_per_launch": flops_step // nb,
                     "nonpacked_fp32_ceiling": NONPACKED_FP32_TFLOPS,
                     "frac_of_nonpacked_ceiling": round(achieved_tflops / NONPACKED_FP32_TFLOPS, 4)},
        "build_streamed": build_summary(build_ms, build_bytes, args.steps),
    }

    if not args.no_cpu_baseline:
        # the FP64 oracle renders the full frame of four states of the stream (after a quarter,
        # half, three quarters and all of the batches), each on an oracle octree of that state
        import numpy as np
        import oracle
        states = sorted({max(1, nb * q // 4) for q in (1, 2, 3, 4)})
        pos, dt, t_all = 0, 0.0, time.perf_counter()
        for nbat in states:
            zf = min(nbat * cfg["batch"], dims[2])
            v0 = np.zeros_like(vol)
            v0[:, :zf] = vol[:, :zf]
            mask = np.zeros((dims[2], dims[1], dims[0]), np.uint8)
            mask[:zf] = (1 << C) - 1
            ref = oracle.Tree(v0, mask, M, background=0, threshold=cfg["thr"])
            tc = time.perf_counter()
            img_ref, ns = ref.render_rows(view, 0, 1)
            dt += time.perf_counter() - tc
            pos += int(ns.sum())
            del ref, v0, mask
        err = float(np.abs(img.cpu().numpy().astype(np.float64) - img_ref).max())
        out["cpu_baseline"] = {
            "value": round(pos / dt / 1e9, 5), "unit": "Gsamples/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"FP64 oracle renders of the full {cfg['width']}x{cfg['height']} frame "
                      f"after batches {states} of the stream, each on an oracle octree of that "
                      f"state ({pos} positions in {dt:.1f} s of rendering; the oracle builds, "
                      f"excluded from the value, bring the sample to "
                      f"{time.perf_counter() - t_all:.1f} s)"}
        out["final_frame_max_abs_err_vs_oracle"] = err
    if not args.no_adjoint:
        out["adjoint"] = {k: v for k, v in measure_adjoint(args).items()
                          if k in ("value", "unit", "forward_ms", "adjoint_ms", "adjoint_tf_only_ms",
                                   "kernel_ms", "config")}
    final_img = img.clone()
    if not args.no_build:
        out["mip"] = measure_mip(tree, cfg, args)
        tree.close()
        out["build_whole_volume"] = measure_build(dev, cfg, args)
    tree.close()
    if not args.no_disk:
        torch.cuda.empty_cache()
        out["disk_tier"] = measure_disk(slabs, cfg, args, final_img, composited, ms_per_step)
    del slabs, dev
    if not args.no_serve:
        torch.cuda.empty_cache()
        out["serving"] = {k: v for k, v in measure_serve(args).items()
                          if k not in ("metric", "n_gpus", "higher_is_better", "data")}
    if not args.no_paging:
        torch.cuda.empty_cache()
        out["out_of_core"] = measure_paging(args)
    print(json.dumps(out), flush=True)


def build_summary(ms, by, steps: int = 1) -> dict:
    """Per build phase: kernel ms (per step), algorithmic GB, GB/s and % of HBM peak."""
    names = ("insert", "downsample", "stats", "gather")
    out = {}
    for k, n in enumerate(names):
        gbps = by[k] / (ms[k] / 1e3) / 1e9 if ms[k] > 0 else 0.0
        out[n] = {"ms": round(ms[k] / steps, 3), "gb": round(by[k] / steps / 1e9, 4),
                  "gb_per_s": round(gbps, 1), "hbm_pct": round(100.0 * gbps / PEAK_HBM_GBPS, 2)}
    tot_ms, tot_b = sum(ms), sum(by)
    g = tot_b / (tot_ms / 1e3) / 1e9 if tot_ms > 0 else 0.0
    out["all"] = {"ms": round(tot_ms / steps, 3), "gb": round(tot_b / steps / 1e9, 4),
                  "gb_per_s": round(g, 1), "hbm_pct": round(100.0 * g / PEAK_HBM_GBPS, 2)}
    return out


def measure_build(dev, cfg, args) -> dict:
    """Whole-volume build from HBM: one insert of the full volume (level 0 + every level above)
    and one brick_pool_upload (statistics of every cell, every bordered brick gathered); build
    kernel time and algorithmic bytes per phase, median of the timed repetitions."""
    import torch

    from paper_1407_2074_amd.octree import Octree
    dims, C, M = cfg["dims"], cfg["C"], cfg["M"]
    t = Octree(dims, C, M, "u16", background=0, threshold=cfg["thr"])
    runs = []
    reps = max(args.steps, 3)
    for r in range(reps + 1):
        t.clear()
        torch.cuda.synchronize()
        t.build_timing(True)
        t.insert_block(-1, (0, 0, 0), dev)
        t.upload()
        torch.cuda.synchronize()
        ms, by = t.build_timing(False)
        if r:
            runs.append((ms, by))
    t.close()
    runs.sort(key=lambda x: sum(x[0]))
    ms, by = runs[len(runs) // 2]
    res = build_summary(ms, by)
    res["config"] = (f"{dims[0]}x{dims[1]}x{dims[2]}x{C} u16 from HBM, {M}^3 bricks, "
                     f"threshold {cfg['thr']}: one insert + one upload, median of {reps}")
    return res


def _fs_type(path: str) -> str:
    """File system of `path` (the longest mount point above it in /proc/mounts)."""
    best, kind = "", "unknown"
    try:
        for line in open("/proc/mounts"):
            f = line.split()
            if len(f) >= 3 and path.startswith(f[1]) and len(f[1]) > len(best):
                best, kind = f[1], f[2]
    except OSError:
        pass
    return kind


def measure_disk(slabs, cfg, args, want, composited, hbm_ms_per_step) -> dict:
    """Disk tier: the streamed build + render step of the headline configuration with the
    mipmap kept in pages in a file (pages of 2x2x2 cells = 64^3 voxels, all channels) and RAM
    frames for half of the pages (about what one batch's insertion, half-sampling, statistics
    and border gathers touch); one warm-up step, then one timed step.  Reports the
    step's rate, the page traffic of the timed step, and the final image against the in-HBM
    run's (the octree is the same, so the image must be equal)."""
    import shutil
    import tempfile

    import numpy as np
    import torch

    from paper_1407_2074_amd import synth
    from paper_1407_2074_amd.octree import Octree
    dims, C, M = cfg["dims"], cfg["C"], cfg["M"]
    P, page_cells = 2 * M, 2
    N = 0
    while (M << N) < max(dims):
        N += 1
    n_pages = 0
    for L in range(N + 1):
        ext = [-(-d // (1 << L)) for d in dims]
        n_pages += int(np.prod([-(-e // P) for e in ext]))
    page_bytes = P ** 3 * C * 2
    frames = max(16, n_pages // 2)
    tmp = tempfile.mkdtemp(prefix="octree_pages_")
    path = os.path.join(tmp, "pages.bin")
    try:
        t = Octree(dims, C, M, "u16", background=0, threshold=cfg["thr"], disk_path=path,
                   host_cache_bytes=frames * page_bytes, page_cells=page_cells)
        view = synth.make_view(dims, C, cfg["seed"], az=cfg["az"], el=cfg["el"],
                               width=cfg["width"], height=cfg["height"], lod=cfg["lod"])
        img = torch.zeros((view.height, view.width, 4), dtype=torch.float32, device="cuda")

        def step(tree):
            tree.clear()
            for b, slab in enumerate(slabs):
                tree.insert_slices(-1, b * cfg["batch"], slab)
                tree.upload()
                tree.render([view], images=[img])

        def timed(tree):
            step(tree)   # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            step(tree)
            torch.cuda.synchronize()
            return time.perf_counter() - t0

        step(t)
        torch.cuda.synchronize()
        s0 = t.disk_stats()
        t0 = time.perf_counter()
        step(t)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        s1 = t.disk_stats()
        err = float((img - want).abs().max().item())
        t.close()
        # the same with the frames in device memory (pages copied through a staging page)
        td = Octree(dims, C, M, "u16", background=0, threshold=cfg["thr"], disk_path=path,
                    host_cache_bytes=frames * page_bytes, page_cells=page_cells, device_frames=True)
        el_dev = timed(td)
        err_dev = float((img - want).abs().max().item())
        sd = td.disk_stats()
        td.close()
        # the same step with the whole mipmap in pinned host memory: what the kernels' traffic
        # over the host link costs without the page file
        th = Octree(dims, C, M, "u16", background=0, threshold=cfg["thr"], master_on_host=True)
        el_host = timed(th)
        th.close()
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    d = {k: s1[k] - s0[k] for k in ("hits", "loads", "fills", "writebacks", "evictions", "waits",
                                   "bytes_read", "bytes_written")}
    return {
        "config": (f"streamed build+render {dims[0]}x{dims[1]}x{dims[2]}x{C} u16, {M}^3 bricks, "
                   f"{len(slabs)} batches of {cfg['batch']} slices, one {cfg['width']}x"
                   f"{cfg['height']} view per batch; mipmap in {n_pages} pages of {P}^3 voxels "
                   f"({page_bytes / 2**20:.1f} MiB) in a file on {_fs_type(tmp)}, {frames} frames in "
                   f"pinned host memory (device_frames: in device memory)"),
        "ms_per_step": round(el * 1e3, 2),
        "gsamples_per_s": round(composited / el / 1e9, 3),
        "hbm_master_ms_per_step": round(hbm_ms_per_step, 2),
        "host_master_ms_per_step": round(el_host * 1e3, 2),
        "page_traffic": d,
        "file_read_gb_per_s": round(d["bytes_read"] / el / 1e9, 3),
        "file_write_gb_per_s": round(d["bytes_written"] / el / 1e9, 3),
        "final_image_max_abs_diff_vs_hbm_master": err,
        "device_frames": {"ms_per_step": round(el_dev * 1e3, 2),
                          "gsamples_per_s": round(composited / el_dev / 1e9, 3),
                          "loads_two_steps": sd["loads"], "writebacks_two_steps": sd["writebacks"],
                          "final_image_max_abs_diff_vs_hbm_master": err_dev},
    }


def measure_mip(tree, cfg, args) -> dict:
    """MIP of the complete octree: one 1024x1024 view (same camera as the streamed frames)."""
    import torch

    from paper_1407_2074_amd import synth
    dims, C = cfg["dims"], cfg["C"]
    v = synth.make_view(dims, C, cfg["seed"], az=cfg["az"], el=cfg["el"], width=cfg["width"],
                        height=cfg["height"], lod=cfg["lod"], mode=1)
    d = synth.make_view(dims, C, cfg["seed"], az=cfg["az"], el=cfg["el"], width=cfg["width"],
                        height=cfg["height"], lod=cfg["lod"])
    img = torch.empty((v.height, v.width, 4), dtype=torch.float32, device="cuda")
    _, st = tree.render([v], images=[img], stats=True)
    _, sd = tree.render([d], images=[img], stats=True)
    reps = max(10, args.steps)
    tm = _sync_time(lambda: tree.render([v], images=[img]), reps)
    td = _sync_time(lambda: tree.render([d], images=[img]), reps)
    return {"config": f"MIP, {cfg['width']}x{cfg['height']}, final octree of the stream",
            "ms_per_frame": round(tm * 1e3, 4), "frames_per_s": round(1.0 / tm, 1),
            "gsamples_per_s": round(st["positions_composited"] / tm / 1e9, 3),
            "positions_composited": st["positions_composited"],
            "dvr_ms_per_frame": round(td * 1e3, 4),
            "dvr_positions_composited": sd["positions_composited"]}


def _sync_time(fn, reps):
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps


def bench_adjoint(args):
    """256^3 x 3 f32 (u16 * 2^-16), 64^3 bricks, 512x512 at LOD 0, threshold 0: differentiable
    forward (with checkpoints) and adjoint of an L2 loss against a target rendered with
    perturbed transfer functions."""
    print(json.dumps(measure_adjoint(args)), flush=True)


def measure_adjoint(args) -> dict:
    import numpy as np
    import torch

    from paper_1407_2074_amd import synth
    from paper_1407_2074_amd.octree import Octree
    dims, C, M = (256, 256, 256), 3, 64
    vol = synth.gen_volume(dims, C, seed=4, n_blobs=2000, dtype="f32")
    t = Octree(dims, C, M, "f32", 0.0, 0.0)
    t.insert_block(-1, (0, 0, 0), torch.from_numpy(vol).cuda())
    t.upload()
    v = synth.make_view(dims, C, 4, az=30.0, el=20.0, width=512, height=512, lod=0, dtype="f32")
    tv = synth.make_view(dims, C, 4, az=30.0, el=20.0, width=512, height=512, lod=0, dtype="f32")
    rng = np.random.default_rng(4 * 1000 + 300)
    tv.tf_rgba = np.clip(tv.tf_rgba + rng.normal(0, 0.05, tv.tf_rgba.shape), 0, 1).astype(np.float32)
    (tgt,) = t.render([tv])
    ck = torch.empty(t.ckpt_bytes([v]), dtype=torch.uint8, device="cuda")
    img = torch.empty((512, 512, 4), dtype=torch.float32, device="cuda")
    dctrl = torch.zeros((1, C, 8, 4), dtype=torch.float32, device="cuda")
    dvox = torch.zeros((C, 256, 256, 256), dtype=torch.float32, device="cuda")
    _, st = t.render([v], images=[img], ckpt=ck, stats=True)

    def fwd():
        t.render([v], images=[img], ckpt=ck)

    gI = [2 * (img - tgt)]

    def bwd():
        t.render_backward([v], gI, ck, dctrl, dvox)

    def bwd_tf_only():
        t.render_backward([v], gI, ck, dctrl, None)

    for _ in range(max(args.warmup, 1)):
        fwd()
        gI[0] = 2 * (img - tgt)
        bwd()
        bwd_tf_only()
    tf = _sync_time(fwd, args.steps)
    tb = _sync_time(bwd, args.steps)
    tb_tf = _sync_time(bwd_tf_only, args.steps)
    # kernel time alone (HIP events around the ray-casting / adjoint kernel of each call); the
    # wall times above also hold each call's record copy and host work between kernels
    kms = {}
    for name, fn in (("forward", fwd), ("adjoint", bwd), ("adjoint_tf_only", bwd_tf_only)):
        t.render_timing(True)
        for _ in range(args.steps):
            fn()
        ms, n = t.render_timing(False)
        kms[name] = round(ms / max(n, 1), 3)
    nom, comp = st["positions_nominal"], st["positions_composited"]
    out = {"metric": "adjoint Gsamples/s", "value": round(nom / (tf + tb) / 1e9, 3),
           "unit": "Gsamples/s (nominal positions per forward+adjoint)", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round((tf + tb) * 1e3, 3), "higher_is_better": True,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "256^3x3 f32, 64^3 bricks, 512x512, LOD 0, L2 loss vs "
                                  "perturbed-TF target; forward recording transmittances + adjoint"},
           "forward_ms": round(tf * 1e3, 3), "adjoint_ms": round(tb * 1e3, 3),
           "adjoint_tf_only_ms": round(tb_tf * 1e3, 3),
           "kernel_ms": kms,
           "forward_gsamples_per_s": round(comp / tf / 1e9, 3),
           "adjoint_gsamples_per_s": round(nom / tb / 1e9, 3),
           "positions_nominal": nom, "positions_composited": comp,
           "voxel_atomics_per_s": round(nom * C * 8 / tb / 1e9, 2)}
    return out


def bench_serve(args):
    """Serving alone (see measure_serve)."""
    print(json.dumps(measure_serve(args)), flush=True)


def measure_serve(args, n: int = 2000) -> dict:
    """Serving: the 512x512x256 streamed-config octree resident; 2000 Poisson requests (200/s)
    with image sizes uniform in {256, 512, 1024, 2048}^2, random orbits, per-request TFs and 0-3
    clipping planes; admission by framebuffer (2 GB cap) and brick-pool memory.  Reported:
    requests/s, p50/p99 latency (arrival -> completion), the closed-loop rate, the same views
    one launch per view, and 1024 random pixels of 8 served images against the FP64 oracle."""
    import numpy as np
    import torch

    import oracle
    from paper_1407_2074_amd import synth
    from paper_1407_2074_amd.octree import Octree
    from paper_1407_2074_amd.serving import Server, poisson_requests
    dims, C, M = (512, 512, 256), 3, 32
    vol = synth.gen_volume(dims, C, seed=2, n_blobs=2000)
    t = Octree(dims, C, M, "u16", 0, 205)
    t.insert_block(-1, (0, 0, 0), torch.from_numpy(vol.view(np.int16)).cuda())
    t.upload()
    reqs = poisson_requests(dims, C, n, rate=200.0, seed=5)
    # positions per request, counted once (deterministic), not part of the timed run
    pos = 0
    for k in range(0, len(reqs), 16):
        _, st = t.render([r.view for r in reqs[k:k + 16]], stats=True)
        pos += st["positions_composited"]
    warm = poisson_requests(dims, C, 8, rate=1e6, seed=55)
    Server(t).run(warm, realtime=False)
    keep = {r.rid for r in reqs[:: max(1, n // 8)][:8]}
    kept = {}

    def grab(r):
        if r.rid in keep:
            kept[r.rid] = r.image.cpu()
    st = Server(t).run(reqs, realtime=True, on_complete=grab)
    closed = Server(t).run(poisson_requests(dims, C, n, rate=1e9, seed=5), realtime=False)
    torch.cuda.synchronize()
    alone = None
    if not getattr(args, "serve_only", False):
        t0 = time.perf_counter()
        for r in reqs:
            t.render([r.view])
        torch.cuda.synchronize()
        alone = time.perf_counter() - t0
    t.close()
    # the oracle on 1024 random pixels of each kept image
    ref = oracle.Tree(vol, np.full((dims[2], dims[1], dims[0]), (1 << C) - 1, np.uint8), M,
                      background=0, threshold=205)
    rng = np.random.default_rng(5)
    worst = 0.0
    for r in reqs:
        if r.rid not in kept:
            continue
        v = r.view
        px = np.stack([rng.integers(0, v.width, 1024), rng.integers(0, v.height, 1024)], -1)
        want = ref.render_pixels(v, px)
        got = kept[r.rid].numpy().astype(np.float64)[px[:, 1], px[:, 0]]
        worst = max(worst, float(np.abs(got - want).max()))
    return {"metric": "serving requests/s, p50/p99 latency", "value": round(st.requests_per_s, 2),
            "unit": "requests/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
            "config": {"workload": f"{n} Poisson requests at 200/s, sizes {{256..2048}}^2, "
                                   "0-3 clip planes, per-request TFs, 512x512x256x3 octree "
                                   "resident, admission by framebuffer (2 GB) and brick-pool "
                                   "memory"},
            "offered_rate": 200.0, "completed": st.completed,
            "latency_p50_ms": round(st.latency_p50_ms, 2),
            "latency_p99_ms": round(st.latency_p99_ms, 2),
            "gsamples_per_s": round(pos / st.makespan_s / 1e9, 3),
            "closed_loop_requests_per_s": round(closed.requests_per_s, 2),
            "closed_loop_gsamples_per_s": round(pos / closed.makespan_s / 1e9, 3),
            "closed_loop_latency_p50_ms": round(closed.latency_p50_ms, 2),
            "closed_loop_latency_p99_ms": round(closed.latency_p99_ms, 2),
            "one_view_per_launch_gsamples_per_s": round(pos / alone / 1e9, 3) if alone else None,
            "launches": st.launches, "max_in_flight": st.max_in_flight,
            "max_fb_bytes": st.max_fb_bytes_in_use,
            "sampled_parity": {"images": len(kept), "pixels_each": 1024,
                               "max_abs_err_vs_oracle": worst, "tolerance": 1e-4,
                               "pass": bool(kept and worst <= 1e-4)}}


def bench_views(args):
    """64 views (orbit) of the 64^3 x 3 volume at 128x128 in one launch vs one launch each."""
    import numpy as np
    import torch

    from paper_1407_2074_amd import synth
    from paper_1407_2074_amd.octree import Octree
    dims, C, M = (64, 64, 64), 3, 16
    vol = synth.gen_volume(dims, C, seed=1, n_blobs=20)
    t = Octree(dims, C, M, "u16", 0, 205)
    t.insert_block(-1, (0, 0, 0), vol)
    t.upload()
    views = [synth.make_view(dims, C, 1, az=360.0 * i / 64, el=20.0, width=128, height=128,
                             clips=[(1.0, 0.0, 0.0, 24.0)]) for i in range(64)]
    imgs = [torch.empty((128, 128, 4), dtype=torch.float32, device="cuda") for _ in views]
    _, st = t.render(views, images=imgs, stats=True)
    for _ in range(3):
        t.render(views, images=imgs)
    reps = max(args.steps, 10)
    t.render_timing(True)      # ray-casting kernel time (HIP events), beside the wall time
    tb = _sync_time(lambda: t.render(views, images=imgs), reps)
    kb_ms, kb_n = t.render_timing(False)

    def single():
        for v, im in zip(views, imgs):
            t.render([v], images=[im])

    single()
    t.render_timing(True)
    ts = _sync_time(single, reps)
    ks_ms, ks_n = t.render_timing(False)
    comp = st["positions_composited"]
    out = {"metric": "Gsamples/s, 64 views of 64^3 x 3 at 128x128", "value": round(comp / tb / 1e9, 3),
           "unit": "Gsamples/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
           "config": {"workload": "64 orbit views, 128x128, clip x >= 24, LOD 0, thr 205"},
           "batched_us_per_launch": round(tb * 1e6, 1), "us_per_frame": round(tb * 1e6 / 64, 2),
           "batched_kernel_us_per_launch": round(kb_ms * 1e3 / kb_n, 1),
           "one_view_per_launch_us_per_frame": round(ts * 1e6 / 64, 2),
           "one_view_kernel_us_per_launch": round(ks_ms * 1e3 / ks_n, 1),
           "one_view_per_launch_gsamples_per_s": round(comp / ts / 1e9, 3),
           "positions_composited": comp}
    print(json.dumps(out), flush=True)


def bench_paging(args):
    """The out-of-core path alone (see measure_paging)."""
    print(json.dumps(measure_paging(args)), flush=True)


def h2d_peak_gb_per_s(nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Plain pinned-host to device copy rate (hipMemcpyAsync through torch), median of reps."""
    import torch
    h = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    d = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    d.copy_(h, non_blocking=True)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        d.copy_(h, non_blocking=True)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    del h, d
    return nbytes / sorted(ts)[len(ts) // 2] / 1e9


def measure_paging(args) -> dict:
    """Out-of-core: 3-channel u16 2048x2048x1024 (100k blobs) at --scale 1, 32^3 bricks, the
    full-resolution mipmap in pinned host memory, device brick pool capped (16 GiB at scale 1,
    divided by scale^3), 1920x1080 views along a 64-frame orbit that dollies from 1.0 to 0.5 of
    the fitting distance (per-ray LOD, step 0.5, ERT 0.99).  At --scale s the image shrinks by s
    too, so per-ray LODs and the working set relative to the pool match the full-size case.
    Each frame = render + one brick_pool_upload with a byte budget (bricks are paged in on
    request).  Afterwards four frames of the path (the last one among them) are refined until
    no brick is missing, and 4096 random pixels of each converged image are compared with the
    FP64 oracle, whose time on those rays is the CPU baseline."""
    import numpy as np
    import torch

    import oracle
    from paper_1407_2074_amd import synth
    from paper_1407_2074_amd.octree import Octree
    sc = args.scale
    dims, C, M = (2048 // sc, 2048 // sc, 1024 // sc), 3, 32
    blobs = 100000 // (sc ** 3)
    workers = min(16, os.cpu_count() or 1)
    t_gen = time.perf_counter()
    vol = synth.gen_volume(dims, C, seed=3, n_blobs=blobs, workers=workers)
    t_gen = time.perf_counter() - t_gen
    print(f"[bench] out-of-core volume {dims} x{C} generated in {t_gen:.1f}s", file=sys.stderr,
          flush=True)
    h2d = h2d_peak_gb_per_s()
    pool_bytes = (16 << 30) // (sc ** 3)
    store = not args.no_host_bricks
    tree = Octree(dims, C, M, "u16", 0, 205, pool_bytes=pool_bytes, master_on_host=True,
                  host_bricks=store)
    t_ins = time.perf_counter()
    zc = 64 // sc
    for z0 in range(0, dims[2], zc):
        tree.insert_slices(-1, z0, np.ascontiguousarray(vol[:, z0:z0 + zc]))
    tree.upload()
    torch.cuda.synchronize()
    t_ins = time.perf_counter() - t_ins
    print(f"[bench] out-of-core octree built in {t_ins:.1f}s", file=sys.stderr, flush=True)
    n_frames = 64
    W, H = 1920 // sc, 1080 // sc
    budget = (1 << 30) // sc
    views = []
    for k in range(n_frames):
        v = synth.make_view(dims, C, 3, az=360.0 * k / n_frames, el=20.0, width=W,
                            height=H, lod=-1, dist_scale=1.0 - 0.5 * k / (n_frames - 1))
        v.ert_alpha = 0.99
        views.append(v)
    img = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
    tree.render([views[0]], images=[img])       # warm-up (also the first requests)
    tree.upload(byte_budget=budget)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(n_frames)]
    comp = gathered = requests = evictions = copied = 0
    tree.build_timing(True)    # gather kernel time of the frames' uploads (HIP events)
    t0 = time.perf_counter()
    up_s = 0.0
    stream = torch.cuda.current_stream()
    for k, v in enumerate(views):
        ev[k][0].record(stream)
        _, st = tree.render([v], images=[img], stats=True)
        ev[k][1].record(stream)
        comp += st["positions_composited"]
        tu = time.perf_counter()
        up = tree.upload(byte_budget=budget)
        up_s += time.perf_counter() - tu
        gathered += up["bricks_gathered"]
        copied += up["bricks_from_store"]
        requests += up["requests_seen"]
        evictions += up["evictions"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    bt_ms, _ = tree.build_timing(False)
    gather_s = bt_ms[3] / 1e3
    render_s = sum(a.elapsed_time(b) for a, b in ev) / 1e3
    # host-link bytes per gathered brick: the bordered brick's source voxels, all channels
    src_bytes = (M + 2) ** 3 * C * 2
    # refine four frames of the path to convergence (untimed), keep their images
    checks = sorted({0, n_frames // 3, 2 * n_frames // 3, n_frames - 1})
    converged, passes_last, unserved_last, resident_last = {}, 0, 0, 0
    for k in checks:
        v = views[k]
        for passes in range(1, 400):
            _, st = tree.render([v], images=[img], stats=True)
            up = tree.upload()
            unserved, resident = up["requests_seen"], up["bricks_resident"]
            if unserved == 0 or (up["bricks_gathered"] == 0 and up["evictions"] == 0):
                break       # converged, or the pool holds what it can
        (img,) = tree.render([v], images=[img])
        converged[k] = (img.cpu().numpy().astype(np.float64), unserved)
        passes_last, unserved_last, resident_last = passes, unserved, resident
    slots = tree.pool_slots
    tree.close()
    torch.cuda.empty_cache()
    # oracle: the same volume, everything inserted; 4096 random pixels per converged frame
    t_orc = time.perf_counter()
    mask = np.full((dims[2], dims[1], dims[0]), (1 << C) - 1, np.uint8)
    ref = oracle.Tree(vol, mask, M, background=0, threshold=205)
    del mask
    t_orc = time.perf_counter() - t_orc
    rng = np.random.default_rng(3)
    worst, n_px, n_amb, pos, dt = 0.0, 0, 0, 0, 0.0
    for k in checks:
        gimg, unserved = converged[k]
        if unserved:
            continue    # not converged (over-subscribed pool): no in-core image to compare
        px = np.stack([rng.integers(0, W, 4096), rng.integers(0, H, 4096)], -1)
        tc = time.perf_counter()
        want, ns, mg = ref.render_pixels(views[k], px, want_info=True)
        dt += time.perf_counter() - tc
        pos += int(ns.sum())
        ok = mg >= 1e-5          # early-termination decisions FP32 and FP64 may take apart
        got = gimg[px[:, 1], px[:, 0]]
        worst = max(worst, float(np.abs(got - want)[ok].max()))
        n_px += int(ok.sum())
        n_amb += int((~ok).sum())
    del ref
    # host-link bytes: a gathered brick's source voxels, a copied brick's store entry (the
    # bordered brick, channels unpadded) -- the same count for 3 channels
    paged_gbps = gathered * src_bytes / gather_s / 1e9 if gather_s > 0 else 0.0
    return {"metric": "out-of-core frames/s over a 64-frame orbit-and-dolly path",
            "value": round(n_frames / elapsed, 2), "unit": "frames/s", "n_gpus": 1,
            "higher_is_better": True, "data": "synthetic",
            "config": {"workload": f"{dims[0]}x{dims[1]}x{dims[2]}x3 u16, {blobs} blobs, 32^3 "
                       f"bricks, master in pinned host memory"
                       f"{', host brick store' if store else ''}, device pool {pool_bytes >> 20} "
                       f"MiB, {W}x{H}, ERT 0.99, per-ray LOD, {budget >> 20} MiB upload budget "
                       "per frame"},
            "render_only_gsamples_per_s": round(comp / render_s / 1e9, 3),
            "render_ms_per_frame": round(render_s / n_frames * 1e3, 3),
            "upload_host_ms_per_frame": round(up_s / n_frames * 1e3, 3),
            "gather_kernel_ms_per_frame": round(gather_s / n_frames * 1e3, 3),
            "paged_bricks": gathered,
            "paged_bricks_from_store": copied,
            "paged_gb_per_s": round(paged_gbps, 2),
            "h2d_peak_gb_per_s": round(h2d, 2),
            "paged_frac_of_h2d_peak": round(paged_gbps / h2d, 3) if h2d > 0 else None,
            "requests": requests, "evictions": evictions, "pool_slots": slots,
            "refined_frames": checks, "refine_passes_last_frame": passes_last,
            "last_frame_resident_bricks": resident_last,
            "last_frame_unserved_requests": unserved_last,
            "sampled_parity": {"pixels": n_px, "excluded_near_ert": n_amb,
                               "max_abs_err_vs_oracle": worst, "tolerance": 1e-4,
                               "pass": bool(n_px > 0 and worst <= 1e-4)},
            "cpu_baseline": {"value": round(pos / dt / 1e9, 5) if dt > 0 else None,
                             "unit": "Gsamples/s", "cores": oracle.num_threads(),
                             "kind": "oracle",
                             "sample": f"FP64 oracle on 4096 random rays of each converged frame "
                                       f"{checks} ({pos} positions in {dt:.1f} s; its octree "
                                       f"build took {t_orc:.1f} s, not counted)"},
            "generation_s": round(t_gen, 1), "insert_s": round(t_ins, 2)}


if __name__ == "__main__":
    main()
