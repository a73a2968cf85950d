"""Dynamic point-cloud sequence: per frame, estimate every point's ellipsoid (the learned
estimator in BF16: the paper's UNet by default, or the plain eight-layer network; or the kNN-PCA
plain path) and render two views, reporting p50/p99 latency per frame and PSNR against a dense
ground-truth render (Section 4.3's video setting, at 30 frames of a deforming procedural surface).

    python -m paper_2409_16504_amd.sequence [--estimator unet|plain] [--weights path.pt]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from synthetic import look_at_camera  # noqa: E402
from synthetic.scenes import ProceduralSurface  # noqa: E402

from . import Renderer, RenderState, default_options  # noqa: E402
from .estimator import SparseEstimator, UNetEstimator, Voxels, adaptive_grid, psnr  # noqa: E402


SEQUENCE_SEED = 1005
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "estimator_surface.pt")
UNET_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "unet_surface.pt")


def make_sequence(n_frames: int, points: int, seed: int = SEQUENCE_SEED):
    """The deforming surface and its frames: radii scaled by 1 + 0.2 sin(2 pi t / 30 + phase), points
    sampled area-uniformly plus N(0, 0.002^2) position noise, value-noise colour. Returns the
    surface and a list of dicts with xyz (3, n) and rgb (3, n) float32 arrays and the radius scale."""
    rng = np.random.default_rng(seed)
    surf = ProceduralSurface(rng, margin_scale=1.2)
    frames = []
    for t in range(n_frames):
        scale = 1.0 + 0.2 * np.sin(2.0 * math.pi * t / 30 + surf.phase)
        p = surf.sample(points, rng, radius_scale=scale)
        p = p + rng.normal(0.0, 0.002, size=p.shape)
        rgb = surf.color(p)
        frames.append(dict(xyz=np.ascontiguousarray(p, np.float32), rgb=np.ascontiguousarray(rgb, np.float32),
                           scale=scale))
    return surf, frames


def sequence_cameras(width: int, height: int) -> list:
    """The two views of every frame: eye at radius 3, 0.3 above the centre, 90 degrees apart."""
    return [look_at_camera([3.0 * math.sin(a), 0.3, 3.0 * math.cos(a)], width=width, height=height)
            for a in (0.0, math.pi / 2)]


def load_estimator(R: Renderer, weights: str | None = WEIGHTS, kind: str = "plain"):
    """The estimator ("unet": the paper's UNet-like network; "plain": the eight-layer sparse
    network) with the shipped (or given) trained weights."""
    est = UNetEstimator(R, seed=0) if kind == "unet" else SparseEstimator(R, seed=0)
    est.grid_neighbours = 6.0               # the voxel-grid rule (see estimator.adaptive_grid)
    if weights:
        ck = torch.load(weights, weights_only=True)
        est.load_params(ck["params"])
        est.grid_neighbours = ck.get("report", {}).get("grid_neighbours", 6.0)
    return est


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--frames", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--points", type=int, default=1_000_000)
    ap.add_argument("--width", type=int, default=1440)
    ap.add_argument("--height", type=int, default=1600)
    ap.add_argument("--estimator", choices=("unet", "plain"), default="unet",
                    help="the learned estimator: the paper's UNet or the plain eight-layer network")
    ap.add_argument("--weights", default=None, help="trained weights (default: the shipped ones)")
    ap.add_argument("--kappa", type=float, default=1.0)
    ap.add_argument("--psnr-frames", type=int, default=3)
    args = ap.parse_args(argv)

    R = Renderer(0)
    dev = torch.device("cuda", 0)
    t0 = time.time()
    surf, raw = make_sequence(args.frames + args.warmup, args.points)
    frames = [dict(xyz=torch.from_numpy(f["xyz"]).to(dev), rgb=torch.from_numpy(f["rgb"]).to(dev),
                   scale=f["scale"]) for f in raw]
    print(f"[sequence] {len(frames)} frames ready in {time.time() - t0:.1f}s", flush=True)
    cams = sequence_cameras(args.width, args.height)
    if args.weights is None:
        args.weights = UNET_WEIGHTS if args.estimator == "unet" else WEIGHTS
    est = load_estimator(R, args.weights, args.estimator)
    opts = default_options()
    # the density is the sequence's; the grid rule is the estimator's
    grid = adaptive_grid(R, frames[0]["xyz"], frames[0]["rgb"], est.grid_neighbours).grid
    vox = Voxels(R)
    out = R.render(dict(mean=frames[0]["xyz"], quat=torch.zeros((4, args.points), device=dev),
                        scale=torch.full((3, args.points), 0.002, device=dev),
                        opacity=torch.full((args.points,), 0.9, device=dev), rgb=frames[0]["rgb"],
                        normal=torch.zeros((3, args.points), device=dev)), cams, opts)

    levels = []                         # the UNet's pooled voxel sets, rebuilt in place per frame

    def learned(f):
        vox.build(f["xyz"], f["rgb"], grid)
        if args.estimator == "unet":
            levels[:] = UNetEstimator.levels(R, vox, levels or None)
            return est.forward(levels)
        return est.forward(vox)

    def plain(f):
        e = R.knn_pca(f["xyz"], k=16, kappa=args.kappa, floor=0.1)
        return dict(mean=f["xyz"], quat=e["quat"], scale=e["scale"],
                    opacity=torch.full((f["xyz"].shape[1],), 0.9, device=dev), rgb=f["rgb"], normal=e["normal"])

    report = {}
    for name, fn in (("learned_bf16", learned), ("knn_pca", plain)):
        times = []
        for i, f in enumerate(frames):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            g = fn(f)
            R.render(g, cams, opts, out=out)
            torch.cuda.synchronize()
            if i >= args.warmup:
                times.append((time.perf_counter() - t1) * 1e3)
        report[name] = dict(p50_ms=float(np.percentile(times, 50)), p99_ms=float(np.percentile(times, 99)),
                            max_ms=float(np.max(times)), frames=len(times))
        print(f"[sequence] {name}: {report[name]}", flush=True)

    # Pipelined: the estimate of frame t + 1 (its own context and stream) overlaps the render of
    # frame t (another context and stream; both streams at the default priority). The render runs
    # in capacity mode, so the host never waits on it and can queue the next estimate at once.
    # Throughput is the steady-state time per frame; the first frame's estimate is not overlapped.
    # "graph": the render of both views is captured once in a HIP graph (capacity mode: it neither
    # waits nor allocates) reading the Gaussians from fixed buffers; per frame they are copied in
    # and the graph is replayed on the render stream.
    s_est, s_ren = torch.cuda.Stream(), torch.cuda.Stream()
    static = {k: v.clone() for k, v in plain(frames[0]).items()}
    # the eager capacity-mode renders and the captured one each have their own context and state:
    # a captured graph keeps the addresses of its context's and state's buffers
    R2, R3 = Renderer(0), Renderer(0)
    st2, st3 = RenderState(R2), RenderState(R3)
    out2, out3 = R2.render(static, cams, opts), R3.render(static, cams, opts)
    # size both states' capacity over every frame of both estimates (an overflowing frame resizes
    # the next render, so each frame is rendered until it fits)
    for fn in (learned, plain):
        for f in frames:
            g = fn(f)
            for k in static:
                static[k].copy_(g[k])
            for Rx, stx, outx in ((R2, st2, out2), (R3, st3, out3)):
                for _ in range(3):
                    Rx.render(static, cams, opts, state=stx, out=outx, capacity=True)
                    if stx.status()[0] == 0:
                        break
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    s_ren.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s_ren):
        R3.render(static, cams, opts, state=st3, out=out3, capacity=True)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=s_ren):
        R3.render(static, cams, opts, state=st3, out=out3, capacity=True)
    torch.cuda.synchronize()

    def render_capacity(g):
        R2.render(g, cams, opts, state=st2, out=out2, capacity=True)

    def render_graph(g):
        for k in static:
            static[k].copy_(g[k])
        graph.replay()

    for name, fn, render, stx in (("learned_bf16_pipelined", learned, render_capacity, st2),
                                  ("knn_pca_pipelined", plain, render_capacity, st2),
                                  ("learned_bf16_graph", learned, render_graph, st3),
                                  ("knn_pca_graph", plain, render_graph, st3)):
        torch.cuda.synchronize()
        with torch.cuda.stream(s_est):
            g_cur = fn(frames[0])
            ev = torch.cuda.Event()
            ev.record(s_est)
        t1 = None
        for i in range(len(frames)):
            if i == args.warmup:
                torch.cuda.synchronize()
                t1 = time.perf_counter()
            g_next = ev_next = None
            if i + 1 < len(frames):
                with torch.cuda.stream(s_est):
                    g_next = fn(frames[i + 1])
                    ev_next = torch.cuda.Event()
                    ev_next.record(s_est)
            with torch.cuda.stream(s_ren):
                s_ren.wait_event(ev)
                render(g_cur)
                for t in g_cur.values():                # produced on s_est, last used on s_ren
                    t.record_stream(s_ren)
            g_cur, ev = g_next, ev_next
        torch.cuda.synchronize()
        n_timed = len(frames) - args.warmup
        ms = (time.perf_counter() - t1) * 1e3 / n_timed
        rc, _ = stx.status()                            # the last frame's status
        report[name] = dict(ms_per_frame=ms, fps=1e3 / ms, frames=n_timed, last_frame_status=rc)
        print(f"[sequence] {name}: {report[name]}", flush=True)

    # PSNR on a few frames against the plain render of an 8x dense sample of the clean surface
    ps = {"learned_bf16": [], "knn_pca": []}
    for f in frames[args.warmup:args.warmup + args.psnr_frames]:
        pd = surf.sample(8 * args.points, np.random.default_rng(5), radius_scale=f["scale"])
        xd = torch.from_numpy(np.ascontiguousarray(pd, np.float32)).to(dev)
        e = R.knn_pca(xd, k=16, kappa=1.0, floor=0.1)
        dense = dict(mean=xd, quat=e["quat"], scale=e["scale"], opacity=torch.full((xd.shape[1],), 0.9, device=dev),
                     rgb=torch.from_numpy(np.ascontiguousarray(surf.color(pd), np.float32)).to(dev), normal=e["normal"])
        gt = R.render(dense, cams, opts, want=("rgb",))["rgb"].clone()
        for name, fn in (("learned_bf16", learned), ("knn_pca", plain)):
            img = R.render(fn(f), cams, opts, want=("rgb",))["rgb"]
            ps[name].append(psnr(img, gt))
    for name in ps:
        report[name]["psnr_db"] = float(np.mean(ps[name]))
    report["config"] = dict(frames=args.frames, points=args.points, views=2, width=args.width, height=args.height,
                            estimator=args.estimator,
                            weights=os.path.relpath(args.weights, ROOT) if args.weights else None)
    print(json.dumps(report), flush=True)
    return report


if __name__ == "__main__":
    main()
