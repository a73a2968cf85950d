"""Benchmark of the splatting renderer on one MI355X.

Workload (default): 1,000,000 surfel Gaussians at 1920x1080, RGB + normal + depth + alpha. The
cloud is a procedural union of 6 spheres and 4 tori (radii U(0.2, 0.6)) normalised into [-1,1]^3,
sampled area-uniformly, quantised to the 10-bit lattice, coloured with 3-octave value noise; its
ellipsoids come from kNN-PCA (k = 16, kappa = 1) computed on the GPU; opacity 0.9; one pinhole
camera at (0, 0, 3) looking at the origin with a 60 degree vertical field of view.

A step is one frame of the renderer: projection, instance scan, binning, radix sort, tile ranges
and compositing (all inputs resident in HBM). `value` is Gaussians per second = N / frame time.
Per-stage times come from HIP events the library records on the launch stream; the roofline
entry is computed for the stage that dominates the frame. The CPU oracle renders the same
workload once on the host cores for the `cpu_baseline` entry.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms/frame @1M Gaussians 1080p; Gaussians/s; learned-vs-kNN-PCA PSNR gap"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3         # MI355X FP32 vector peak (packed FP32: 256 CUs x 4 SIMD x 32 x 2 x 2.4 GHz)
FP32_VALU_PEAK_TFLOPS = 78.6     # the same without packed FP32 (the build disables it)
BF16_MFMA_PEAK_TFLOPS = 2500.0   # dense BF16 matrix cores
# Compositing work as the method defines it: 25 FLOP per evaluated (pixel, list entry) pair (the
# quadratic form, one exp, the 7-channel blend), E pairs counted by the oracle.
COMPOSITE_FLOP_PER_VISIT = 25
# Backward compositing per (pixel, list entry) walked back from the last contributor: the
# quadratic form (9 FLOP); per blended splat about 45 more (transmittance recovered with a
# reciprocal and a product, the blend weight, the 7-channel dot products with the pixel gradient,
# dL/dalpha, the behind-sum update, 7 weight gradients, opacity, q, conic and position partials).
COMPOSITE_BWD_VISIT_FLOP = 9
COMPOSITE_BWD_BLEND_FLOP = 45

# Algorithmic bytes per unit (stated in the design doc):
PROJECT_READ_B = 68      # mean 12 + quat 16 + scale 12 + opacity 4 + rgb 12 + normal 12
PROJECT_WRITE_VIS_B = 76  # 64 B splat record + 4 B depth bits + 8 B tile rectangle
PROJECT_WRITE_CULL_B = 12  # depth bits and rectangle, zero
NARROW_RECT_TILES = 255    # up to this many tile columns and rows a tile rectangle takes 4 B, not 8


def rect_bytes(W, H):
    """Bytes of one stored tile rectangle for a W x H frame."""
    return 4 if max((W + 15) // 16, (H + 15) // 16) <= NARROW_RECT_TILES else 8
SORT_PASS_B = 16         # read + write of a 4 B key and a 4 B value
# Compositing FLOP per (pixel, list entry) visit and per blended splat.
COMPOSITE_VISIT_FLOP = 9     # offset (2), conic quadratic form (7)
COMPOSITE_BLEND_FLOP = 21    # -q/2, exp, o*e, w = a*T, 7 fused multiply-adds (14), 1 - a, T update


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1080)
    ap.add_argument("--seed", type=int, default=1006)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras-only", action="store_true",
                    help="run only the secondary workloads (64 views forward + backward, estimator) "
                         "and print their JSON; for profiling them apart from the headline frame")
    ap.add_argument("--estimator-only", action="store_true",
                    help="run only the sparse estimator workload (for profiling its kernels)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device copy of this size (for scaling HBM byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (this renderer "
              "runs on a single MI355X; multi-GPU sharding is design only)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2409_16504_amd as P
    from synthetic import look_at_camera, make_surface

    if args.extras_only or args.estimator_only:
        print(json.dumps({"extras": extra_workloads(P.Renderer(0), estimator_only=args.estimator_only)}),
              flush=True)
        return
    t0 = time.time()
    _, xyz, rgb = make_surface(args.n, args.seed, quantize=True)
    cams = [look_at_camera([0, 0, 3], width=args.width, height=args.height)]
    print(f"[bench] inputs ready in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    R = P.Renderer(0)
    dev = torch.device("cuda", 0)
    txyz = torch.from_numpy(xyz).to(dev)
    est = R.knn_pca(txyz, k=16, kappa=1.0, floor=0.1)
    g = dict(mean=txyz, quat=est["quat"], scale=est["scale"],
             opacity=torch.full((args.n,), 0.9, device=dev), rgb=torch.from_numpy(rgb).to(dev),
             normal=est["normal"])
    torch.cuda.synchronize()
    # kNN-PCA time (ellipsoid estimation, reported separately from the frame)
    R.timing(True)
    for _ in range(3):
        R.knn_pca(txyz, k=16, kappa=1.0, floor=0.1, out=est)
    knn_ms = R.timings()["knn_pca"][0] / 3.0

    if args.copy_calibration_mib:
        # a plain elementwise kernel (negation) that reads and writes the stated size once
        src = torch.ones((args.copy_calibration_mib << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: {args.copy_calibration_mib} MiB read + written", file=sys.stderr,
              flush=True)
        del src, dst
    opts = P.default_options()
    out = R.render(g, cams, opts)
    for _ in range(args.warmup):
        R.render(g, cams, opts, out=out)
    # timed frames: the compositing kernel's dispatch (the roofline's kernel) stamps its start and
    # end into HIP events, so the frame time carries no per-stage instrumentation
    torch.cuda.synchronize()
    R.timing(True, stages=["composite"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        R.render(g, cams, opts, out=out)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    composite_ms = R.timings()["composite"][0] / args.steps
    ms_per_step = (t2 - t1) * 1e3 / args.steps
    print(f"[bench] {args.steps} frames: {ms_per_step:.3f} ms/frame", file=sys.stderr, flush=True)
    R.timing(False)
    modes = frame_modes(R, g, cams, opts, args.steps)
    # per-stage breakdown from a separate run of the same frames with events around every stage
    R.timing(True)
    for _ in range(args.steps):
        R.render(g, cams, opts, out=out)
    stages = R.timings()

    # instance count and visible splats of this frame (from a state export)
    st = P.RenderState(R)
    R.render(g, cams, opts, state=st)
    bins = R.bins(st)
    m = int(bins["keys"].size)
    # per frame: a stage may run as several timed sections (the sort runs twice per frame)
    per_stage = {k: v[0] / args.steps for k, v in stages.items() if v[1] > 0}

    cpu = None
    visits = blends = None
    if not args.no_cpu_baseline:
        cpu, visits, blends = cpu_baseline(xyz, rgb, cams)

    lds_peak = R.lds_bandwidth()
    print(f"[bench] measured LDS read peak {lds_peak / 1e3:.1f} TB/s", file=sys.stderr, flush=True)
    roof = roofline(dict(per_stage, composite=composite_ms), args.n, m, bins, visits, blends, lds_peak)
    roof_bwd = backward_roofline(R, g, cams, opts, bins, blends)
    stage_roof = stage_rooflines(per_stage, args.n, m, bins, args.width, args.height)
    extras = None if args.no_extras else extra_workloads(R)
    gap = None if args.no_extras else psnr_gap(R)
    unet = None if args.no_extras else unet_gap(R)
    if extras is not None:
        extras["psnr_gap"] = gap
        extras["unet"] = unet
        extras["late_shading"] = late_shading(R, out, cams)
    line = dict(
        metric=METRIC, value=args.n / (ms_per_step * 1e-3), unit="Gaussians/s", n_gpus=1,
        steps=args.steps, warmup=args.warmup, ms_per_step=ms_per_step, higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload=f"{args.n} surfel Gaussians (procedural sphere/torus surface, kNN-PCA "
                             f"ellipsoids), {args.width}x{args.height}, RGB+normal+depth",
                    n_gaussians=args.n, width=args.width, height=args.height, cameras=1),
        ms_per_frame=ms_per_step, instances=m, knn_pca_ms=knn_ms,
        stage_ms={k: round(v, 5) for k, v in per_stage.items()},
        frame_modes=modes, roofline=roof, roofline_backward=roof_bwd, stage_roofline=stage_roof,
        cpu_baseline=cpu, psnr_gap_db=(unet["gap_db"] if unet is not None else None if gap is None else gap["gap_db"]), extras=extras,
    )
    print(json.dumps(line), flush=True)


def extra_workloads(R, estimator_only=False):
    """Secondary measurements (not the headline value): the 64-camera 1024^2 forward + backward of
    the 800k-point surface in one launch, and the sparse estimator on that cloud."""
    import torch
    import paper_2409_16504_amd as P
    from paper_2409_16504_amd.estimator import SparseEstimator, adaptive_grid
    from synthetic import make_surface, orbit_cameras
    dev = torch.device("cuda", 0)
    _, xyz, rgb = make_surface(800_000, 1002, quantize=True)
    txyz, trgb = torch.from_numpy(xyz).to(dev), torch.from_numpy(rgb).to(dev)
    est = R.knn_pca(txyz, k=16, kappa=1.0, floor=0.1)
    g = dict(mean=txyz, quat=est["quat"], scale=est["scale"], opacity=torch.full((xyz.shape[1],), 0.9, device=dev),
             rgb=trgb, normal=est["normal"])
    many = None
    reps = 3
    if not estimator_only:
        cams = orbit_cameras(64, np.random.default_rng(1003), width=1024, height=1024)
        st = P.RenderState(R)
        opts = P.default_options()
        out = R.render(g, cams, opts, state=st)
        gen = torch.Generator(device=dev).manual_seed(0)
        go = dict(rgb=torch.randn(out["rgb"].shape, device=dev, generator=gen),
                  normal=torch.randn(out["normal"].shape, device=dev, generator=gen),
                  depth=torch.randn(out["depth"].shape, device=dev, generator=gen))
        R.render_backward(st, go)
        torch.cuda.synchronize()
        R.timing(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            R.render(g, cams, opts, state=st, out=out)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            R.render_backward(st, go)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        stages = {k: round(v[0] / reps, 4) for k, v in R.timings().items() if v[1] > 0}
        many = dict(workload="800k surfel Gaussians x 64 orbit cameras at 1024x1024, one launch",
                    forward_ms=(t1 - t0) * 1e3 / reps, backward_ms=(t2 - t1) * 1e3 / reps, stage_ms=stages)
        del st, out, go
    # sparse estimator (BF16 MFMA) on the same cloud: voxelise + 8 convolutions + head
    E = SparseEstimator(R, seed=0)
    vox = adaptive_grid(R, txyz, trgb)
    E.forward(vox)
    torch.cuda.synchronize()
    R.timing(True)
    t3 = time.perf_counter()
    for _ in range(reps):
        E.forward(vox.build(txyz, trgb, vox.grid))
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    est_stages = {k: round(v[0] / reps, 4) for k, v in R.timings().items() if v[1] > 0}
    from paper_2409_16504_amd.estimator import IN_CHANNELS, LAYERS
    # the method's own work: 2 FLOP per multiply-add over the present (voxel, neighbour) pairs (the
    # voxel itself included) and the used channels (6 inputs in the first layer); the kernels also
    # multiply absent neighbours' zero rows and the first layer's padding, counted apart
    pairs = int((vox.arrays()["nbr"] >= 0).sum().item())
    used = sum((IN_CHANNELS if i == 0 else ci) * co for i, (ci, co) in enumerate(LAYERS))
    conv_flop = 2 * pairs * used
    dense_flop = 2 * 27 * vox.V * sum(ci * co for ci, co in LAYERS)
    conv_ms = est_stages.get("conv", float("nan"))
    ok = conv_ms == conv_ms
    estimator = dict(workload=f"sparse estimator on {xyz.shape[1]} points ({vox.V} voxels, grid {vox.grid}^3, "
                              f"{vox.mean_neighbours():.1f} occupied neighbours per voxel)",
                     ms_per_cloud=(t4 - t3) * 1e3 / reps, stage_ms=est_stages, neighbour_pairs=pairs,
                     conv_flop=conv_flop,
                     conv_tflops=conv_flop / (conv_ms * 1e-3) / 1e12 if ok else None,
                     conv_frac_bf16=conv_flop / (conv_ms * 1e-3) / 1e12 / BF16_MFMA_PEAK_TFLOPS if ok else None,
                     conv_dense_equivalent_tflops=dense_flop / (conv_ms * 1e-3) / 1e12 if ok else None)
    del E, vox
    if estimator_only:
        return dict(estimator=estimator)
    # dynamic sequence (10 timed frames here; the full 30 run with python -m paper_2409_16504_amd.sequence)
    from paper_2409_16504_amd import sequence
    t5 = time.time()
    import contextlib
    with contextlib.redirect_stdout(sys.stderr):        # stdout carries the bench line alone
        seq = sequence.main(["--frames", "10", "--warmup", "3", "--psnr-frames", "1"])
    print(f"[bench] sequence in {time.time() - t5:.1f}s", file=sys.stderr, flush=True)
    seq["workload"] = ("deforming procedural surface, 10 timed frames after 3 warm-up frames, ~1M points per "
                       "frame, estimate + 2 views at 1440x1600; p99 over 10 frames is their maximum")
    return dict(many_cameras=many, estimator=estimator, sequence=seq)


def frame_modes(R, g, cams, opts, steps):
    """The same frame in capacity mode (no host wait: frames queue back to back) and replayed from a
    HIP graph captured in capacity mode; ms per frame by wall clock over `steps` frames."""
    import torch
    import paper_2409_16504_amd as P
    st = P.RenderState(R)
    out = R.render(g, cams, opts, state=st, capacity=True)      # sizes the capacity (waits once)
    for _ in range(3):
        R.render(g, cams, opts, state=st, out=out, capacity=True)
    assert st.status() == (0, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        R.render(g, cams, opts, state=st, out=out, capacity=True)
    torch.cuda.synchronize()
    cap_ms = (time.perf_counter() - t0) * 1e3 / steps
    assert st.status() == (0, 0)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        R.render(g, cams, opts, state=st, out=out, capacity=True)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        R.render(g, cams, opts, state=st, out=out, capacity=True)
    torch.cuda.synchronize()
    for _ in range(3):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - t0) * 1e3 / steps
    assert st.status() == (0, 0)
    print(f"[bench] capacity mode {cap_ms:.3f} ms/frame, graph replay {graph_ms:.3f} ms/frame",
          file=sys.stderr, flush=True)
    return dict(capacity_ms=cap_ms, graph_replay_ms=graph_ms, capacity=st.capacity,
                note="same frame and outputs as the headline loop; capacity mode queues frames without "
                     "a host wait, the graph replays the captured capacity-mode frame")


def backward_roofline(R, g, cams, opts, bins, blends, reps=10):
    """Roofline entry of the backward compositing kernel on the headline frame (upstream gradient
    N(0,1) on rgb, normal, depth): FLOP = 9 per (pixel, list entry) up to each pixel's last
    contributor (the sum of n_contrib) + 45 per blended splat (the oracle's blend count)."""
    import torch
    import paper_2409_16504_amd as P
    st = P.RenderState(R)
    out = R.render(g, cams, opts, state=st)
    gen = torch.Generator(device="cuda").manual_seed(0)
    go = {k: torch.randn(out[k].shape, device="cuda", generator=gen) for k in ("rgb", "normal", "depth")}
    R.render_backward(st, go)
    torch.cuda.synchronize()
    R.timing(True, stages=["backward_composite", "backward_project"])
    for _ in range(reps):
        R.render_backward(st, go)
    t = R.timings()
    ms = t["backward_composite"][0] / reps
    walked = int(bins["n_contrib"].astype(np.int64).sum())
    entry = dict(kernel="composite_backward", bound="alu", avg_ms=ms, peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                 project_backward_ms=t["backward_project"][0] / reps, walked_pairs=walked)
    if blends is not None:
        flop = COMPOSITE_BWD_VISIT_FLOP * walked + COMPOSITE_BWD_BLEND_FLOP * blends
        entry.update(flop=flop, achieved=flop / (ms * 1e-3) / 1e12,
                     frac=flop / (ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS)
    return entry


def late_shading(R, out, cams, reps=20):
    """Blinn-Phong late shading of the headline frame's rgb / normal / alpha (one kernel, 28 B read
    and 12 B written per pixel)."""
    import torch
    light = dict(dir=(0.3, 0.8, 0.5), color=(1.0, 1.0, 1.0), ambient=0.15, diffuse=0.7, specular=0.3, shininess=24.0)
    shaded = R.shade(out, cams, light)
    torch.cuda.synchronize()
    R.timing(True, stages=["shade"])
    for _ in range(reps):
        R.shade(out, cams, light, out=shaded)
    ms = R.timings()["shade"][0] / reps
    W, H = cams[0].width, cams[0].height
    byts = W * H * 40
    return dict(workload=f"Blinn-Phong late shading of the {W}x{H} frame", ms=ms, bytes=byts,
                gbs=byts / (ms * 1e-3) / 1e9, frac=byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)


# Kernel source each stage's dominant kernel is built from (a counter summary applies only while
# this file is unchanged).
# Sources a stage's counters depend on: its kernel's, and the projection's where the tile lists
# it walks come from the projection's binning rule.
STAGE_SOURCES = {"composite": ("project.hip", "composite.hip"), "project": ("project.hip",),
                 "binning": ("project.hip", "scan_sort.hip"), "sort": ("project.hip", "scan_sort.hip"),
                 "ranges": ("project.hip", "scan_sort.hip")}


def sources_sha256(stage):
    """sha256 of the stage's sources (STAGE_SOURCES, concatenated in that order), or None."""
    import hashlib
    paths = [os.path.join(ROOT, "paper_2409_16504_amd", "csrc", f) for f in STAGE_SOURCES.get(stage, ())]
    if not paths or not all(os.path.isfile(q) for q in paths):
        return None
    h = hashlib.sha256()
    for q in paths:
        with open(q, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_lds(stage="composite"):
    """LDS bytes per launch of the stage's kernel (64 x SQ_INSTS_LDS_LOAD_BANDWIDTH +
    64 x SQ_INSTS_LDS_STORE_BANDWIDTH) and its bank-conflict cycles from the committed rocprofv3
    counter summary, or None when there is none or the stage's sources have changed since."""
    import re
    path = os.path.join(ROOT, "profiles", f"{stage}_1M_1080p_lds_counters.md")
    sha = sources_sha256(stage)
    if not os.path.exists(path) or sha is None:
        return None
    text = open(path).read()
    h = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    b = re.search(r"lds_bytes_per_launch:\s*([0-9.eE+]+)", text)
    c = re.search(r"bank_conflict_fraction:\s*([0-9.eE+-]+)", text)
    if not h or not b or sha != h.group(1):
        return None
    return dict(bytes=float(b.group(1)), bank_conflict_fraction=float(c.group(1)) if c else None)


def measured_traffic(stage):
    """HBM bytes per launch of the stage's kernel from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE scaled by a plain copy kernel's counters), or None when there is no
    summary or the stage's sources have changed since it was taken."""
    import re
    path = os.path.join(ROOT, "profiles", f"{stage}_1M_1080p_hbm_traffic.md")
    sha = sources_sha256(stage)
    if not os.path.exists(path) or sha is None:
        return None
    text = open(path).read()
    h = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not h or not b or sha != h.group(1):
        return None
    return float(b.group(1))


WEIGHTS = os.path.join(ROOT, "paper_2409_16504_amd", "weights", "estimator_surface.pt")


def psnr_gap(R):
    """PSNR of the plain sparse-convolution estimator (eight submanifold layers at one resolution,
    BF16, trained weights shipped with the package) against the kNN-PCA plain path on held-out
    clouds; ground truth is the plain render of each cloud's 8x denser unquantised sample (the
    evaluation of the training driver)."""
    if not os.path.exists(WEIGHTS):
        return None
    import torch
    from paper_2409_16504_amd.estimator import SparseEstimator
    from paper_2409_16504_amd.train import SIGMA_FACTORS, evaluate, make_cloud
    from synthetic import orbit_cameras
    ck = torch.load(WEIGHTS, weights_only=True)
    est = SparseEstimator(R, seed=0)
    with torch.no_grad():
        for p, v in zip(est.params, ck["params"]):
            p.copy_(v.to(p.device))
    rep = ck["report"]
    t0 = time.time()
    held = [make_cloud(R, 2000 + i, rep["points"]) for i in range(2)]
    cams = orbit_cameras(rep["views"], np.random.default_rng(2024), width=rep["res"], height=rep["res"])
    # the global-sigma baseline's factor: the one chosen on the training clouds when the weights'
    # report has it, else the best of the paper's three on these clouds (favours the baseline)
    if "sigma_factor" in rep:
        r = evaluate(R, est, held, cams, rep["kappa"], rep["sigma_factor"])
        r["sigma_factor"] = rep["sigma_factor"]
    else:
        runs = {f: evaluate(R, est, held, cams, rep["kappa"], f) for f in SIGMA_FACTORS}
        best = max(runs, key=lambda f: runs[f]["psnr_global_sigma"])
        r = dict(runs[best], sigma_factor=best,
                 psnr_global_sigma_by_factor={f: v["psnr_global_sigma"] for f, v in runs.items()})
    print(f"[bench] PSNR gap on held-out clouds in {time.time() - t0:.1f}s: {r}", file=sys.stderr, flush=True)
    return dict(r, kappa=rep["kappa"], train_steps=rep["steps"],
                workload=f"2 held-out procedural clouds ({rep['points']} points, seeds 2000-2001) x "
                         f"{rep['views']} orbit views at {rep['res']}x{rep['res']}; ground truth = plain render "
                         "of the 8x denser unquantised sample; kNN-PCA kappa chosen on the training clouds; "
                         "global-sigma baseline: isotropic sigma = factor x mean nearest-neighbour distance")


UNET_WEIGHTS = os.path.join(ROOT, "paper_2409_16504_amd", "weights", "unet_surface.pt")


def unet_gap(R):
    """The paper's UNet-like estimator (BF16, trained with Eq. 5 and the density augmentation;
    weights shipped with the package) against the kNN-PCA plain path and the global-sigma baseline
    on held-out clouds: at full density and over the augmentation's range (lattices coarsened by a,
    samples thinned to b); ground truth is the plain render of each cloud's 8x denser unquantised
    sample (the evaluation of the training driver). Also the estimate's time per cloud against
    kNN-PCA's on the same points."""
    if not os.path.exists(UNET_WEIGHTS):
        return None
    import torch
    from paper_2409_16504_amd import train_unet as TU
    from paper_2409_16504_amd.estimator import UNetEstimator
    from synthetic import orbit_cameras
    ck = torch.load(UNET_WEIGHTS, weights_only=True)
    est = UNetEstimator(R, seed=0)
    est.load_params(ck["params"])
    rep = ck["report"]
    gn = rep.get("grid_neighbours", 6.0)        # the voxel-grid rule the weights were trained with
    t0 = time.time()
    held = [TU.make_cloud(R, 2000 + i, rep["points"]) for i in range(2)]
    cams = orbit_cameras(rep["views"], np.random.default_rng(2024), width=rep["res"], height=rep["res"])
    runs = {}
    for a in (1.0, 0.5, 0.25):
        runs[f"a={a}"] = TU.evaluate(R, est, held, cams, rep["kappa"], rep["sigma_factor"], True, a=a,
                                     grid_neighbours=gn)
    for b in (0.5, 0.25, 0.125):
        runs[f"b={b}"] = TU.evaluate(R, est, held, cams, rep["kappa"], rep["sigma_factor"], False, b=b,
                                     grid_neighbours=gn)
    # time per cloud: voxelise + pool + network + head, against kNN-PCA of the same points
    x = TU.sample_input(R, held[0], np.random.default_rng(0), True, grid_neighbours=gn)
    vox, grid = x["vox"], x["vox"].grid
    with torch.no_grad():
        for _ in range(2):
            est.forward(UNetEstimator.levels(R, vox.build(x["xyz"], x["rgb"], grid)))
            R.knn_pca(x["xyz"], k=16, kappa=rep["kappa"], floor=0.1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(10):
            est.forward(UNetEstimator.levels(R, vox.build(x["xyz"], x["rgb"], grid)))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(10):
            R.knn_pca(x["xyz"], k=16, kappa=rep["kappa"], floor=0.1)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
    full = runs["a=1.0"]
    print(f"[bench] UNet on held-out clouds in {time.time() - t0:.1f}s: {full}", file=sys.stderr, flush=True)
    return dict(full, train_steps=rep["steps"], kappa=rep["kappa"], sigma_factor=rep["sigma_factor"],
                grid_neighbours=gn,
                gap_db_by_density={k: v["gap_db"] for k, v in runs.items()},
                psnr_by_density={k: dict(learned=v["psnr_learned"], knn_pca=v["psnr_knn_pca"],
                                         global_sigma=v["psnr_global_sigma"]) for k, v in runs.items()},
                estimate_ms_per_cloud=(t2 - t1) * 1e3 / 10, knn_pca_ms_per_cloud=(t3 - t2) * 1e3 / 10,
                points=int(x["xyz"].shape[1]),
                workload=f"2 held-out procedural clouds ({rep['points']} points, seeds 2000-2001) x "
                         f"{rep['views']} orbit views at {rep['res']}x{rep['res']}; a: integer lattice "
                         "coordinates x -> round(a x)/a, b: fraction of points kept; ground truth = plain "
                         "render of the 8x denser unquantised sample")


def stage_rooflines(per_stage, n, m, bins, W, H):
    """Algorithmic HBM bytes of every ordering stage (per frame) over its measured time, against the
    8 TB/s peak. Bytes per unit as stated in the design doc."""
    vis = int(np.unique(bins["vals"]).size) if m else 0
    z = (bins["keys"] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    depth_bits = int(z.max() - z.min()).bit_length() if m else 0
    tiles = int(bins["ranges"].shape[1])
    tile_bits = int(tiles - 1).bit_length()
    shrink = 8 - rect_bytes(W, H)                              # rectangle bytes saved per splat
    byts = {
        "project": n * PROJECT_READ_B + vis * (PROJECT_WRITE_VIS_B - shrink) +
                   (n - vis) * (PROJECT_WRITE_CULL_B - shrink),
        "binning": n * (4 + 8 - shrink) + m * 8,                   # order + gathered rectangle; key+value
        "sort": n * (12 + SORT_PASS_B * ((depth_bits + 7) // 8)) +      # depth keys, passes
                m * SORT_PASS_B * ((tile_bits + 7) // 8),                 # (histograms come fused)
        "ranges": tiles * 24,                                      # tile order: runs read twice, starts + order written
    }
    out = {}
    for k, b in byts.items():
        if k in per_stage and per_stage[k] > 0:
            gbs = b / (per_stage[k] * 1e-3) / 1e9
            out[k] = dict(ms=round(per_stage[k], 5), bytes=int(b), gbs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4))
    return out


def roofline(per_stage, n, m, bins, visits, blends, lds_peak=None):
    """Roofline entry of the frame's dominant kernel, from algorithmic work per launch. Every stage
    but compositing is a chain of short kernels (the sort alone runs about a dozen), so the longest
    single kernel is the compositing kernel; the other stages are in `stage_roofline`."""
    frame = {k: v for k, v in per_stage.items() if k in ("project", "binning", "sort", "ranges", "composite")}
    dom = "composite" if "composite" in frame else max(frame, key=frame.get)
    ms = frame[dom]
    if dom == "composite":
        if visits is None:
            # the FLOP count needs the oracle's visit and blend counts, which only the CPU
            # baseline leg computes: no achieved figure without them
            return dict(kernel=dom, bound="alu", achieved=None, peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                        frac=None, traffic=measured_traffic(dom), avg_ms=ms,
                        note="achieved needs the CPU baseline leg (run without --no-cpu-baseline)")
        flop = COMPOSITE_FLOP_PER_VISIT * visits
        ach = flop / (ms * 1e-3) / 1e12
        # the finer count (9 FLOP per visit, 21 more per blend) against the peak without packed FP32
        fine = COMPOSITE_VISIT_FLOP * visits + COMPOSITE_BLEND_FLOP * blends
        fine_ach = fine / (ms * 1e-3) / 1e12
        lds = measured_lds(dom)
        if lds is not None:
            gbs = lds["bytes"] / (ms * 1e-3) / 1e9
            lds.update(gbs=gbs, peak_gbs=lds_peak, frac=gbs / lds_peak if lds_peak else None)
        return dict(kernel=dom, bound="alu", achieved=ach, peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=ach / FP32_PEAK_TFLOPS, traffic=measured_traffic(dom), avg_ms=ms,
                    flop=flop, visits=visits, blends=blends, lds=lds,
                    fine_model=dict(flop=fine, achieved=fine_ach, peak=FP32_VALU_PEAK_TFLOPS,
                                    frac=fine_ach / FP32_VALU_PEAK_TFLOPS))
    if dom == "sort":
        # depth sort of the n splats (u32 keys) then tile sort of the m instances (u32 keys): per
        # pass a read and a write of key and value (the histograms are counted by the kernels that
        # write the keys)
        z = (bins["keys"] & np.uint64(0xFFFFFFFF)).astype(np.int64)
        depth_bits = int(z.max() - z.min()).bit_length() if m else 0
        tile_bits = int(bins["ranges"].shape[1] - 1).bit_length()
        byts = n * (12 + SORT_PASS_B * ((depth_bits + 7) // 8)) + m * SORT_PASS_B * ((tile_bits + 7) // 8)
    elif dom == "project":
        vis = int(np.unique(bins["vals"]).size)
        byts = n * PROJECT_READ_B + vis * PROJECT_WRITE_VIS_B + (n - vis) * PROJECT_WRITE_CULL_B
    elif dom == "binning":
        byts = n * 12 + m * 8
    else:
        byts = m * 8
    ach = byts / (ms * 1e-3) / 1e9
    return dict(kernel=dom, bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                traffic=measured_traffic(dom), avg_ms=ms)


def cpu_baseline(xyz, rgb, cams):
    """The oracle (exact-FP32 projection, FP64 compositing, OpenMP over pixels) renders one full
    frame of the same workload on the host cores; its own kNN-PCA supplies the ellipsoids."""
    import oracle
    from oracle import knn_pca as kp
    t0 = time.time()
    est = kp.knn_pca(xyz, k=16, kappa=1.0)
    g = dict(mean=xyz, quat=est["quat"].astype(np.float32), scale=est["scale"].astype(np.float32),
             opacity=np.full(xyz.shape[1], 0.9, np.float32), rgb=rgb, normal=est["normal"].astype(np.float32))
    print(f"[bench] oracle kNN-PCA {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    img = oracle.render(g, cams, mode="ref")
    t2 = time.perf_counter()
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    print(f"[bench] oracle frame {t2 - t1:.1f}s on {cores} threads", file=sys.stderr, flush=True)
    n = xyz.shape[1]
    return (dict(value=n / (t2 - t1), unit="Gaussians/s", cores=cores, kind="oracle",
                 sample="one full 1920x1080 frame of the 1M-Gaussian workload (FP32-exact projection, "
                        "FP64 compositing)", seconds=t2 - t1),
            int(img["visits"]), int(img["blends"]))


if __name__ == "__main__":
    main()
