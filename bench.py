"""Benchmark: streamed octree build + render of a 3-channel 512x512x256 uint16 volume.

One step is the whole streamed workload: the octree is cleared, then 32 batches of 8 z-slices
(already resident in HBM) are inserted; after each batch brick_pool_upload applies the changes
and one 1024x1024 view (orbit az 45 el 30, step 0.5, per-ray footprint LOD) is rendered.
32^3 bricks, homogeneity threshold 205, seeded synthetic blob + Poisson data (stand-in for the
paper's SPIM scans).

Prints one JSON line.  `value` is composited sample positions per second over the whole step
(build time included); render-only, nominal and frame rates are reported beside it, with the
render kernel's roofline (VALU-bound: algorithmic FP32 flops per second vs the non-packed FP32
peak) and the CPU oracle timed on a bounded sample.
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
# 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz x 2 (FMA) -- FP32 without packed math
PEAK_FP32_TFLOPS = 78.6

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
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU design is described but not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1407_2074_amd import synth
    from paper_1407_2074_amd.octree import Octree

    cfg = CFG[args.config]
    dims, C, M = cfg["dims"], cfg["C"], cfg["M"]
    torch.cuda.set_device(0)
    t_gen = time.perf_counter()
    vol = synth.gen_volume(dims, C, seed=cfg["seed"], n_blobs=cfg["blobs"])
    print(f"[bench] generated {dims} x{C} in {time.perf_counter() - t_gen:.1f}s", file=sys.stderr,
          flush=True)
    dev = torch.from_numpy(vol.view(np.int16)).cuda()
    nb = dims[2] // cfg["batch"]
    slabs = [dev[:, b * cfg["batch"]:(b + 1) * cfg["batch"]].contiguous() for b in range(nb)]
    del dev
    tree = Octree(dims, C, M, "u16", background=0, threshold=cfg["thr"])
    view = synth.make_view(dims, C, cfg["seed"], az=cfg["az"], el=cfg["el"], width=cfg["width"],
                           height=cfg["height"], lod=cfg["lod"])
    img = torch.zeros((view.height, view.width, 4), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    if args.copy_probe_mib:
        a = torch.empty(args.copy_probe_mib << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    def step(stats=None, events=None):
        tree.clear()
        for b in range(nb):
            tree.insert_slices(-1, b * cfg["batch"], slabs[b])
            tree.upload()
            if events is not None:
                events[b][0].record(stream)
            if stats is not None:
                _, st = tree.render([view], images=[img], stats=True)
                stats.append(st)
            else:
                tree.render([view], images=[img])
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
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events=evs[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    render_ms = sum(e[0].elapsed_time(e[1]) for ev in evs for e in ev)   # all render launches
    n_launch = args.steps * nb
    render_s = render_ms / 1e3
    ms_per_step = elapsed / args.steps * 1e3

    value = composited * args.steps / elapsed / 1e9
    achieved_tflops = flops_step * args.steps / render_s / 1e12
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
        "dtype": "u16 data, f32 compute",
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
        "build_ms_per_step": round(ms_per_step - render_ms / args.steps, 3),
        "roofline": {"bound": "alu", "achieved": round(achieved_tflops, 3),
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved_tflops / PEAK_FP32_TFLOPS, 4), "traffic": None,
                     "kernel": "k_render<u16,3>",
                     "flops_per_launch": flops_step // nb},
    }

    if not args.no_cpu_baseline:
        import numpy as np
        import oracle
        full = np.full((dims[2], dims[1], dims[0]), (1 << C) - 1, np.uint8)
        ref = oracle.Tree(vol, full, M, background=0, threshold=cfg["thr"])
        row_step = 4 if args.config == 2 else 1
        tc = time.perf_counter()
        img_ref, ns = ref.render_rows(view, 0, row_step)
        dt = time.perf_counter() - tc
        pos = int(ns.sum())
        got = img.cpu().numpy().astype(np.float64)[::row_step]
        err = float(np.abs(got - img_ref[::row_step]).max())
        out["cpu_baseline"] = {
            "value": round(pos / dt / 1e9, 5), "unit": "Gsamples/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"FP64 oracle render of every {row_step}th row of the final "
                      f"{cfg['width']}x{cfg['height']} frame on the fully built octree "
                      f"({pos} positions, {dt:.2f}s; oracle build excluded)"}
        out["final_frame_max_abs_err_vs_oracle_rows"] = err
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
