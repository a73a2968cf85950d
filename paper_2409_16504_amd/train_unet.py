"""Train the paper's UNet-like estimator (Section 3.2) through the hand-written backward rasterizer
with the loss of Eq. 5 and the density augmentation of Section 3.3, and report its PSNR against
the kNN-PCA plain path and the global-sigma baseline, with a robustness curve over density.

Data (synthetic stand-ins for the paper's meshes): procedural clouds (6 spheres + 4 tori, value-noise
colour); the ground truth of a view is the plain render of an 8x denser unquantised sample of the
same surface (kNN-PCA ellipsoids, opacity 0.9) with the surfaces' analytic normals in its normal
channel. Training inputs mix quantised (10-bit lattice) and unquantised samples, augmented per step
as Section 3.3 describes: a quantised cloud's integer coordinates x become round(a x) / a with
a ~ U[0.25, 1], an unquantised cloud keeps a random b N of its N points with b ~ U[0.125, 1].
Loss (Eq. 5): w1 |I - I_hat|_1 + w2 (|n x n_hat|_2 + w3 min(|n - n_hat|_2, |n + n_hat|_2)) with
w1 = 1, w2 = 10, w3 = 0.1, the normal term over pixels covered in both normal maps.
Voxel size (Section 3.2: about one point per voxel): the finest power-of-two grid whose voxels have
on average at least --grid-neighbours occupied neighbours (1.5: a 300k-point cloud lands on 512^3
with 1.09 points per voxel); the value is stored in the checkpoint's report.

    python -m paper_2409_16504_amd.train_unet --steps 1500 --out gpurun_out/unet.pt
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

from synthetic import orbit_cameras  # noqa: E402
from synthetic.scenes import ProceduralSurface  # noqa: E402

from . import Renderer, RenderState, default_options  # noqa: E402
from .estimator import Adam, UNetEstimator, Voxels, adaptive_grid, psnr, train_step_unet  # noqa: E402
from .train import SIGMA_FACTORS  # noqa: E402

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "unet_surface.pt")


def quantised(p: np.ndarray) -> np.ndarray:
    """Integer 10-bit lattice coordinates of points in [-1,1]^3 (scale 512, Section 3.3)."""
    return np.clip(np.floor((p + 1.0) * 512.0), 0, 1023)


def make_cloud(R: Renderer, seed: int, n: int, dense_factor: int = 8) -> dict:
    """A surface with its sparse sample (kept in both forms) and its dense ground-truth Gaussians."""
    rng = np.random.default_rng(seed)
    surf = ProceduralSurface(rng)
    p = surf.sample(n, rng)
    pd, nd = surf.sample(n * dense_factor, rng, with_normals=True)
    dev = torch.device("cuda", R.device)
    xd = torch.from_numpy(np.ascontiguousarray(pd, np.float32)).to(dev)
    est = R.knn_pca(xd, k=16, kappa=1.0, floor=0.1)
    dense = dict(mean=xd, quat=est["quat"], scale=est["scale"], opacity=torch.full((xd.shape[1],), 0.9, device=dev),
                 rgb=torch.from_numpy(np.ascontiguousarray(surf.color(pd), np.float32)).to(dev),
                 normal=torch.from_numpy(np.ascontiguousarray(nd, np.float32)).to(dev))
    return dict(seed=seed, surf=surf, p=p, q=quantised(p), rgb=surf.color(p), dense=dense)


def sample_input(R: Renderer, c: dict, rng: np.random.Generator, quantise: bool, a: float = 1.0,
                 b: float = 1.0, grid_neighbours: float = 6.0) -> dict:
    """The network input of a cloud: quantised coordinates coarsened to round(a x) / a, or the
    unquantised sample thinned to a fraction b (points keep their colours); voxelised at the
    density-adaptive grid (the finest whose voxels have on average at least ``grid_neighbours``
    occupied neighbours) with its pooled levels."""
    if quantise:
        x = np.round(a * c["q"]) / a
        pts, rgb = (x + 0.5) / 512.0 - 1.0, c["rgb"]
    else:
        keep = np.sort(rng.permutation(c["p"].shape[1])[: max(64, int(round(b * c["p"].shape[1])))])
        pts, rgb = c["p"][:, keep], c["rgb"][:, keep]
    pts = np.clip(pts, -0.999, 0.999)
    dev = torch.device("cuda", R.device)
    xyz = torch.from_numpy(np.ascontiguousarray(pts, np.float32)).to(dev)
    col = torch.from_numpy(np.ascontiguousarray(rgb, np.float32)).to(dev)
    vox = adaptive_grid(R, xyz, col, grid_neighbours)
    return dict(xyz=xyz, rgb=col, vox=vox, levels=UNetEstimator.levels(R, vox))


def render_all(R: Renderer, g: dict, cams: list) -> dict:
    return R.render(g, cams, default_options(), want=("rgb", "normal", "alpha"))


def global_sigma(x: dict, factor: float, dbar: float) -> dict:
    n = x["xyz"].shape[1]
    dev = x["xyz"].device
    q = torch.zeros((4, n), device=dev)
    q[0] = 1.0
    return dict(mean=x["xyz"], quat=q, scale=torch.full((3, n), factor * dbar, device=dev),
                opacity=torch.full((n,), 0.9, device=dev), rgb=x["rgb"], normal=torch.zeros((3, n), device=dev))


def knn(R: Renderer, x: dict, kappa: float) -> dict:
    e = R.knn_pca(x["xyz"], k=16, kappa=kappa, floor=0.1)
    return dict(mean=x["xyz"], quat=e["quat"], scale=e["scale"],
                opacity=torch.full((x["xyz"].shape[1],), 0.9, device=x["xyz"].device), rgb=x["rgb"], normal=e["normal"])


def normal_angle(n_hat: torch.Tensor, n_gt: torch.Tensor, mask: torch.Tensor) -> float:
    """Mean angle (degrees) between per-pixel normalised normals over the mask, sign-agnostic."""
    a = n_hat / (n_hat.norm(dim=1, keepdim=True) + 1e-8)
    b = n_gt / (n_gt.norm(dim=1, keepdim=True) + 1e-8)
    cos = (a * b).sum(dim=1).abs().clamp(max=1.0)
    return float(torch.rad2deg(torch.acos(cos))[mask].mean().item())


def evaluate(R, est, clouds, cams, kappa, sigma_factor, quantise=True, a=1.0, b=1.0, seed=0,
             grid_neighbours=6.0) -> dict:
    rng = np.random.default_rng(seed)
    res = {k: [] for k in ("learned", "knn_pca", "global_sigma", "normal_learned", "normal_knn_pca")}
    with torch.no_grad():
        for c in clouds:
            x = sample_input(R, c, rng, quantise, a, b, grid_neighbours)
            gt = render_all(R, c["dense"], cams)
            mask = gt["alpha"] > 0.5
            dbar = float(R.knn_pca(x["xyz"], k=16, kappa=1.0, floor=0.1, nn_dist=True)["nn_dist"].mean().item())
            for name, g in (("learned", est.forward(x["levels"])), ("knn_pca", knn(R, x, kappa)),
                            ("global_sigma", global_sigma(x, sigma_factor, dbar))):
                img = render_all(R, g, cams)
                res[name].append(psnr(img["rgb"], gt["rgb"]))
                if name != "global_sigma":
                    m = mask & (img["alpha"] > 0.5)
                    res["normal_" + name].append(normal_angle(img["normal"], gt["normal"], m))
    out = {("psnr_" + k if not k.startswith("normal") else k + "_deg"): float(np.mean(v)) for k, v in res.items()}
    out["gap_db"] = out["psnr_learned"] - out["psnr_knn_pca"]
    out["gap_vs_global_sigma_db"] = out["psnr_learned"] - out["psnr_global_sigma"]
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--train-clouds", type=int, default=4)
    ap.add_argument("--eval-clouds", type=int, default=2)
    ap.add_argument("--points", type=int, default=300_000)
    ap.add_argument("--views", type=int, default=6)
    ap.add_argument("--res", type=int, default=512)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default=None)
    ap.add_argument("--curve", action="store_true", help="also the PSNR-versus-density curve")
    ap.add_argument("--head-residual", action="store_true",
                    help="train the head's weights on each point's residual (default: held at zero, one set "
                         "of parameters per voxel)")
    ap.add_argument("--grid-neighbours", type=float, default=1.5,
                    help="voxel grid: the finest whose voxels have on average this many occupied neighbours")
    ap.add_argument("--keep-frac", type=float, default=0.0,
                    help="fraction of training inputs left at full density (the rest are downsampled)")
    args = ap.parse_args(argv)

    R = Renderer(0)
    t0 = time.time()
    train = [make_cloud(R, 10040 + i, args.points) for i in range(args.train_clouds)]
    held = [make_cloud(R, 2000 + i, args.points) for i in range(args.eval_clouds)]
    print(f"[unet] clouds ready in {time.time() - t0:.1f}s", flush=True)
    sel_cams = orbit_cameras(args.views, np.random.default_rng(7), width=args.res, height=args.res)
    rng = np.random.default_rng(123)
    # the plain path's kappa and the global-sigma factor, chosen on the training clouds
    scores, sscores = {}, {}
    with torch.no_grad():
        xs = [sample_input(R, c, rng, True) for c in train]
        gts = [render_all(R, c["dense"], sel_cams)["rgb"] for c in train]
        for kappa in (0.8, 1.0, 1.2, 1.5):
            scores[kappa] = float(np.mean([psnr(render_all(R, knn(R, x, kappa), sel_cams)["rgb"], gt)
                                           for x, gt in zip(xs, gts)]))
        for fac in SIGMA_FACTORS:
            vals = []
            for x, gt in zip(xs, gts):
                dbar = float(R.knn_pca(x["xyz"], k=16, kappa=1.0, floor=0.1, nn_dist=True)["nn_dist"].mean().item())
                vals.append(psnr(render_all(R, global_sigma(x, fac, dbar), sel_cams)["rgb"], gt))
            sscores[fac] = float(np.mean(vals))
        del xs, gts
    kappa = max(scores, key=scores.get)
    sigma_factor = max(sscores, key=sscores.get)
    print(f"[unet] kappa {scores} -> {kappa}; global sigma {sscores} -> {sigma_factor}", flush=True)

    est = UNetEstimator(R, seed=0, head_residual=args.head_residual)
    opt = Adam(est.params, lr=args.lr)
    eval_cams = orbit_cameras(args.views, np.random.default_rng(2024), width=args.res, height=args.res)
    gn = args.grid_neighbours
    before = evaluate(R, est, held, eval_cams, kappa, sigma_factor, grid_neighbours=gn)
    print(f"[unet] before: {before}", flush=True)
    view_rng = np.random.default_rng(99)

    def views(c):
        cams = orbit_cameras(args.views, view_rng, width=args.res, height=args.res)
        rot = view_rng.uniform(0, 2 * math.pi)
        for cam in cams:
            cs, sn = math.cos(rot), math.sin(rot)
            Ry = np.array([[cs, 0, sn], [0, 1, 0], [-sn, 0, cs]], np.float32)
            cam.T = (cam.T @ Ry.T).astype(np.float32)
        with torch.no_grad():
            gt = render_all(R, c["dense"], cams)
        return cams, gt["rgb"], gt["normal"], gt["alpha"]

    losses = []
    torch.cuda.synchronize()
    t1 = time.time()
    for step in range(args.steps):
        opt.lr = args.lr * (0.1 + 0.45 * (1.0 + math.cos(math.pi * step / max(1, args.steps))))
        batch = []
        for c in train:
            quant = bool(rng.integers(2))
            full = rng.uniform() < args.keep_frac
            x = sample_input(R, c, rng, quant, a=1.0 if full else rng.uniform(0.25, 1.0),
                             b=1.0 if full else rng.uniform(0.125, 1.0), grid_neighbours=gn)
            x["dense"] = c["dense"]
            x["state"] = c.setdefault("state", RenderState(R))      # render buffers reused per cloud
            batch.append(x)
        loss = train_step_unet(est, opt, batch, views)
        losses.append(loss)
        if step % 50 == 0 or step == args.steps - 1:
            print(f"[unet] step {step} loss {loss:.5f} ({time.time() - t1:.1f}s)", flush=True)
    torch.cuda.synchronize()
    train_s = time.time() - t1
    after = evaluate(R, est, held, eval_cams, kappa, sigma_factor, grid_neighbours=gn)
    print(f"[unet] after: {after}", flush=True)
    curve = None
    if args.curve:
        curve = dict(quantised={}, subsampled={})
        for a in (1.0, 0.5, 0.25):
            curve["quantised"][a] = evaluate(R, est, held, eval_cams, kappa, sigma_factor, True, a=a, grid_neighbours=gn)
            print(f"[unet] a={a}: {curve['quantised'][a]}", flush=True)
        for b in (1.0, 0.5, 0.25, 0.125):
            curve["subsampled"][b] = evaluate(R, est, held, eval_cams, kappa, sigma_factor, False, b=b,
                                              grid_neighbours=gn)
            print(f"[unet] b={b}: {curve['subsampled'][b]}", flush=True)
    # inference time per cloud: voxelise (density-adaptive grid chosen once) + pool + network + head
    x = sample_input(R, held[0], rng, True, grid_neighbours=gn)
    vox, grid = x["vox"], x["vox"].grid
    for _ in range(2):
        est.forward(UNetEstimator.levels(R, vox.build(x["xyz"], x["rgb"], grid)))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    reps = 10
    for _ in range(reps):
        est.forward(UNetEstimator.levels(R, vox.build(x["xyz"], x["rgb"], grid)))
    torch.cuda.synchronize()
    infer_ms = (time.perf_counter() - t2) * 1e3 / reps
    report = dict(model="unet", steps=args.steps, train_seconds=train_s, ms_per_step=train_s * 1e3 / max(1, args.steps),
                  clouds_per_step=len(train), views=args.views, res=args.res, points=args.points, kappa=kappa,
                  kappa_scores=scores, sigma_factor=sigma_factor, sigma_scores=sscores, before=before, after=after,
                  curve=curve, loss_first=losses[0] if losses else None, loss_last=losses[-1] if losses else None,
                  inference_ms_per_cloud=infer_ms, loss="Eq. 5: 1 L1 + 10 (cross + 0.1 min(|n - n_hat|, |n + n_hat|))",
                  head_residual=args.head_residual, keep_frac=args.keep_frac, grid_neighbours=gn,
                  augmentation=f"quantised: round(a x)/a, a~U[0.25,1]; unquantised: b N points, b~U[0.125,1]; "
                               f"a fraction {args.keep_frac} of inputs kept at full density")
    print(json.dumps(report), flush=True)
    if args.out:
        torch.save(dict(params=[p.detach().cpu() for p in est.params], report=report), args.out)
    return report


if __name__ == "__main__":
    main()
