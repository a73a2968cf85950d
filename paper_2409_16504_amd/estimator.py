"""Sparse point-to-ellipsoid estimator (Section 3.2) on the HIP kernels of libpcsplat.

Network (the configuration-4 stand-in for the paper's UNet): eight submanifold 3x3x3 convolutions
32(6 used) -> 32 -> 32 -> 64 -> 64 -> 64 -> 64 -> 32 -> 32 with ReLU, BF16 activations and weights
on MFMA with FP32 accumulation, then a per-voxel linear head 32 -> 11 (scale 3, quaternion 4,
opacity 1, colour residual 3). Inputs per voxel: mean colour and mean coordinate residual
(Section 3.2). PyTorch holds the weights, the activations and the Adam state; every
convolution, the voxelisation, the head and the renderer run in the library's kernels.
"""
from __future__ import annotations

import ctypes
import math
import sys

import torch

from . import _lib
from ._lib import check
from .render import Renderer, RenderState, default_options

LAYERS = [(32, 32), (32, 32), (32, 64), (64, 64), (64, 64), (64, 64), (64, 32), (32, 32)]
IN_CHANNELS = 6          # mean rgb + mean residual (the first layer's input is padded to 32)
UNET_IN_CHANNELS = 9     # the UNet also reads the voxel's mean absolute position (channels 6-8)
HEAD_OUT = 11


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _s():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class _DevArray:
    """Zero-copy view of a library-owned device array (``__cuda_array_interface__``)."""

    def __init__(self, ptr: int, shape, typestr: str):
        self.__cuda_array_interface__ = dict(shape=tuple(shape), typestr=typestr, data=(ptr, False),
                                             version=2, strides=None)


class Voxels:
    """Voxelised cloud and kernel map (owned by the library)."""

    def __init__(self, renderer: Renderer):
        self.renderer = renderer
        self.handle = ctypes.c_void_p()
        L = _lib.load()
        check(L.pcs_voxels_create(renderer.ctx, ctypes.byref(self.handle)))
        # held by the instance: module globals may already be cleared when __del__ runs
        self._destroy = L.pcs_voxels_destroy
        self._finalizing = sys.is_finalizing
        self.V = 0
        self.n = 0

    def build(self, xyz: torch.Tensor, rgb: torch.Tensor, grid: int = 1024) -> "Voxels":
        n = xyz.shape[1]
        V = ctypes.c_int64()
        check(_lib.load().pcs_voxelize(self.renderer.ctx, _p(xyz), _p(rgb), n, int(grid), self.handle,
                                       ctypes.byref(V), _s()))
        self.V, self.n, self.grid = int(V.value), n, int(grid)
        self.xyz, self.rgb = xyz, rgb
        return self

    def mean_neighbours(self) -> float:
        """Mean number of occupied voxels among the 26 around each voxel."""
        nbr = self.arrays()["nbr"]
        return float((nbr >= 0).sum(dim=0).float().mean().item()) - 1.0


    def arrays(self) -> dict:
        """Zero-copy tensors: coords (3,V) int32, nbr (27,V) int32, point_voxel (n,) int32,
        features (V,32) bf16."""
        c, nb, pv, f = (ctypes.c_void_p() for _ in range(4))
        V = ctypes.c_int64()
        check(_lib.load().pcs_voxels_get(self.handle, ctypes.byref(c), ctypes.byref(nb), ctypes.byref(pv),
                                         ctypes.byref(f), ctypes.byref(V)))
        dev = torch.device("cuda", self.renderer.device)
        coords = torch.as_tensor(_DevArray(c.value, (3, self.V), "<i4"), device=dev)
        nbr = torch.as_tensor(_DevArray(nb.value, (27, self.V), "<i4"), device=dev)
        pvox = torch.as_tensor(_DevArray(pv.value, (self.n,), "<i4"), device=dev)
        feat = torch.as_tensor(_DevArray(f.value, (self.V, 32), "<i2"), device=dev).view(torch.bfloat16)
        return dict(coords=coords, nbr=nbr, point_voxel=pvox, features=feat)

    def __del__(self):
        # at interpreter exit the HIP runtime may be shutting down; process exit frees the memory
        finalizing = getattr(self, "_finalizing", None)
        if finalizing is None or finalizing():
            return
        if getattr(self, "handle", None) and self.handle.value:
            self._destroy(self.handle)
            self.handle = ctypes.c_void_p()


def adaptive_grid(R: Renderer, xyz: torch.Tensor, rgb: torch.Tensor, target: float = 6.0) -> Voxels:
    """Density-adaptive voxel size (Section 3.2 scales the cloud to about one point per voxel so
    that voxelisation keeps neighbouring points in neighbouring voxels): the finest power-of-two
    grid, at most 1024^3, whose voxels have on average at least ``target`` occupied neighbours."""
    vox = None
    for grid in (1024, 512, 256, 128, 64):
        vox = Voxels(R).build(xyz, rgb, grid)
        if vox.mean_neighbours() >= target:
            return vox
    return vox


def conv_forward(R: Renderer, vox: Voxels, x: torch.Tensor, w_bf16: torch.Tensor, bias, relu: bool,
                 out: torch.Tensor | None = None) -> torch.Tensor:
    cin, cout = x.shape[1], w_bf16.shape[1]
    y = out if out is not None else torch.empty((vox.V, cout), device=x.device, dtype=torch.bfloat16)
    check(_lib.load().pcs_subm_conv_forward(R.ctx, vox.handle, _p(x), cin, _p(w_bf16), _p(bias), cout,
                                            int(relu), _p(y), _s()))
    return y


def conv_forward_cat(R: Renderer, vox: Voxels, x1: torch.Tensor, x2: torch.Tensor, w_bf16: torch.Tensor,
                     bias, relu: bool) -> torch.Tensor:
    """conv_forward of the channel concatenation [x1 | x2], which the kernel reads in place."""
    c1, c2, cout = x1.shape[1], x2.shape[1], w_bf16.shape[1]
    y = torch.empty((vox.V, cout), device=x1.device, dtype=torch.bfloat16)
    check(_lib.load().pcs_subm_conv_forward_cat(R.ctx, vox.handle, _p(x1), c1, _p(x2), c2, _p(w_bf16),
                                                _p(bias), cout, int(relu), _p(y), _s()))
    return y


def conv_backward(R: Renderer, vox: Voxels, x, w_bf16, y, dy, want_dx=True, dw=None, db=None):
    cin, cout = x.shape[1], w_bf16.shape[1]
    dx = torch.empty((vox.V, cin), device=x.device, dtype=torch.bfloat16) if want_dx else None
    check(_lib.load().pcs_subm_conv_backward(R.ctx, vox.handle, _p(x), cin, _p(w_bf16), cout, _p(y), _p(dy),
                                             _p(dx), _p(dw), _p(db), _s()))
    return dx


def head_forward(R: Renderer, vox: Voxels, f, wh, bh, xyz, rgb) -> dict:
    n = xyz.shape[1]
    dev = xyz.device
    g = dict(mean=xyz, quat=torch.empty((4, n), device=dev), scale=torch.empty((3, n), device=dev),
             opacity=torch.empty((n,), device=dev), rgb=torch.empty((3, n), device=dev),
             normal=torch.empty((3, n), device=dev))
    check(_lib.load().pcs_estimator_head_forward(R.ctx, vox.handle, _p(f), _p(wh), _p(bh), _p(xyz), _p(rgb),
                                                 _p(g["quat"]), _p(g["scale"]), _p(g["opacity"]), _p(g["rgb"]),
                                                 _p(g["normal"]), _s()))
    return g


def head_backward(R: Renderer, vox: Voxels, f, wh, bh, grads: dict, dwh, dbh) -> torch.Tensor:
    df = torch.empty((vox.V, 32), device=f.device, dtype=torch.bfloat16)
    check(_lib.load().pcs_estimator_head_backward(R.ctx, vox.handle, _p(f), _p(wh), _p(bh),
                                                  _p(grads["quat"].contiguous()), _p(grads["scale"].contiguous()),
                                                  _p(grads["opacity"].contiguous()), _p(grads["rgb"].contiguous()),
                                                  _p(df), _p(dwh), _p(dbh), _s()))
    return df


class SparseEstimator:
    """Weights (FP32 masters, BF16 copies for the kernels) and the forward/backward passes."""

    def __init__(self, renderer: Renderer, seed: int = 0, opacity_init: float = 0.9):
        self.R = renderer
        dev = torch.device("cuda", renderer.device)
        gen = torch.Generator(device="cpu").manual_seed(seed)
        self.w, self.b = [], []
        for li, (cin, cout) in enumerate(LAYERS):
            fan_in = 27 * (IN_CHANNELS if li == 0 else cin)
            w = torch.randn((27, cout, cin), generator=gen) * math.sqrt(2.0 / fan_in)
            if li == 0:
                w[:, :, IN_CHANNELS:] = 0.0
            self.w.append(w.to(dev))
            self.b.append(torch.zeros(cout, device=dev))
        self.wh = (torch.randn((HEAD_OUT, 32), generator=gen) * 1e-3).to(dev)
        self.bh = torch.zeros(HEAD_OUT, device=dev)
        self.bh[7] = math.log(opacity_init / (1.0 - opacity_init))
        self.bh[0:3] = math.log(2.3)            # initial scale ~2.3 voxels
        self.params = self.w + self.b + [self.wh, self.bh]

    def load_params(self, params: list):
        """Copy saved parameters (order of ``params``)."""
        with torch.no_grad():
            for p, v in zip(self.params, params):
                p.copy_(v.to(p.device))

    def bf16_weights(self):
        return [w.to(torch.bfloat16).contiguous() for w in self.w]

    def forward(self, vox: Voxels, save=False):
        """Per-point Gaussians of the voxelised cloud (mean = the points)."""
        arr = vox.arrays()
        wb = self.bf16_weights()
        acts = [arr["features"]]
        x = arr["features"]
        for li in range(len(LAYERS)):
            x = conv_forward(self.R, vox, x, wb[li], self.b[li], relu=True)
            acts.append(x)
        g = head_forward(self.R, vox, x, self.wh, self.bh, vox.xyz, vox.rgb)
        if save:
            return g, dict(acts=acts, wb=wb)
        return g

    def backward(self, vox: Voxels, saved: dict, grads: dict):
        """Weight gradients (FP32, same order as ``params``) from per-point Gaussian gradients."""
        dws = [torch.zeros_like(w) for w in self.w]
        dbs = [torch.zeros_like(b) for b in self.b]
        dwh = torch.zeros_like(self.wh)
        dbh = torch.zeros_like(self.bh)
        acts, wb = saved["acts"], saved["wb"]
        dy = head_backward(self.R, vox, acts[-1], self.wh, self.bh, grads, dwh, dbh)
        for li in reversed(range(len(LAYERS))):
            dy = conv_backward(self.R, vox, acts[li], wb[li], acts[li + 1], dy, want_dx=li > 0,
                               dw=dws[li], db=dbs[li])
        dws[0][:, :, IN_CHANNELS:] = 0.0      # this estimator reads colour and residual only
        return dws + dbs + [dwh, dbh]


def ssim(a: torch.Tensor, b: torch.Tensor, window=11, sigma=1.5, c1=0.01 ** 2, c2=0.03 ** 2):
    """Mean SSIM (Wang et al. 2004) of image batches (N,3,H,W) with a Gaussian window."""
    x = torch.arange(window, device=a.device, dtype=a.dtype) - window // 2
    g = torch.exp(-(x ** 2) / (2 * sigma ** 2))
    g = g / g.sum()
    k = (g[:, None] * g[None, :]).expand(a.shape[1], 1, window, window).contiguous()
    f = lambda t: torch.nn.functional.conv2d(t, k, groups=a.shape[1])  # noqa: E731
    mu_a, mu_b = f(a), f(b)
    saa = f(a * a) - mu_a ** 2
    sbb = f(b * b) - mu_b ** 2
    sab = f(a * b) - mu_a * mu_b
    s = ((2 * mu_a * mu_b + c1) * (2 * sab + c2)) / ((mu_a ** 2 + mu_b ** 2 + c1) * (saa + sbb + c2))
    return s.mean()


def psnr(a: torch.Tensor, b: torch.Tensor) -> float:
    mse = torch.mean((a.clamp(0, 1) - b.clamp(0, 1)) ** 2).item()
    return 10.0 * math.log10(1.0 / max(mse, 1e-12))


class Adam:
    def __init__(self, params, lr=1e-3, betas=(0.9, 0.999), eps=1e-8):
        self.params, self.lr, self.b1, self.b2, self.eps = params, lr, betas[0], betas[1], eps
        self.m = [torch.zeros_like(p) for p in params]
        self.v = [torch.zeros_like(p) for p in params]
        self.t = 0

    def step(self, grads):
        self.t += 1
        c1, c2 = 1 - self.b1 ** self.t, 1 - self.b2 ** self.t
        for p, g, m, v in zip(self.params, grads, self.m, self.v):
            m.mul_(self.b1).add_(g, alpha=1 - self.b1)
            v.mul_(self.b2).addcmul_(g, g, value=1 - self.b2)
            p.addcdiv_(m / c1, (v / c2).sqrt_().add_(self.eps), value=-self.lr)


def render_views(R: Renderer, g: dict, cams: list, state: RenderState | None = None):
    return R.render(g, cams, default_options(), state=state, want=("rgb",))["rgb"]


def train_step(est: SparseEstimator, opt: Adam, clouds: list, view_fn, w_l1=0.8, w_ssim=0.2) -> float:
    """One optimisation step over a batch of clouds. ``clouds`` holds dicts with a built ``vox``;
    ``view_fn(cloud)`` returns (cameras, ground-truth images (C,3,H,W))."""
    R = est.R
    total = [torch.zeros_like(p) for p in est.params]
    loss_sum = 0.0
    for c in clouds:
        cams, gt = view_fn(c)
        g, saved = est.forward(c["vox"], save=True)
        st = c.get("state")
        if st is None:                       # one render state per cloud, its buffers reused
            st = c["state"] = RenderState(R)
        img = render_views(R, g, cams, st).requires_grad_(True)
        loss = w_l1 * (img - gt).abs().mean() + w_ssim * (1.0 - ssim(img, gt))
        loss.backward()
        gg = R.render_backward(st, dict(rgb=img.grad))
        grads = est.backward(c["vox"], saved, gg)
        for t, gr in zip(total, grads):
            t.add_(gr, alpha=1.0 / len(clouds))
        loss_sum += float(loss.item())
    opt.step(total)
    return loss_sum / len(clouds)


# ---- the paper's UNet-like estimator (Section 3.2) --------------------------------------------
# (name, kind, cin, cout): encoder at levels 0-3, decoder back to level 0 with skip connections
# (concatenated channels); every convolution is followed by ReLU. Head: MLP 32 -> 32 -> 14.
UNET_LAYOUT = [
    ("e0a", "subm", 32, 32), ("e0b", "subm", 32, 32),
    ("e1", "subm", 32, 64), ("e2", "subm", 64, 64), ("e3", "subm", 64, 64),
    ("u3", "up", 64, 64), ("d2", "subm", 128, 64),
    ("u2", "up", 64, 64), ("d1", "subm", 128, 64),
    ("u1", "up", 64, 32), ("d0", "subm", 64, 32),
]
UNET_HEAD_HIDDEN, UNET_HEAD_OUT = 32, 14
UNET_HEAD_IN = 35         # per point: its voxel's 32 decoder features and its own residual (3)


def pool(R: Renderer, child: Voxels, parent: Voxels | None = None) -> Voxels:
    """Parent voxels of ``child`` on the grid of half the resolution (Section 3.2's pooling),
    holding the child -> parent map and the upsampling tables. A given ``parent`` is rebuilt in
    place (its device buffers are reused)."""
    parent = parent if parent is not None else Voxels(R)
    Vp = ctypes.c_int64()
    check(_lib.load().pcs_pool(R.ctx, child.handle, parent.handle, ctypes.byref(Vp), _s()))
    parent.V, parent.n, parent.grid = int(Vp.value), child.V, child.grid // 2
    parent.child = child                      # the parent's tables refer to the child's numbering
    return parent


def pool_features(R: Renderer, parent: Voxels, x: torch.Tensor) -> torch.Tensor:
    C = x.shape[1]
    y = torch.empty((parent.V, C), device=x.device, dtype=torch.bfloat16)
    check(_lib.load().pcs_pool_features(R.ctx, parent.handle, _p(x), C, _p(y), _s()))
    return y


def pool_features_backward(R: Renderer, parent: Voxels, dy: torch.Tensor) -> torch.Tensor:
    C = dy.shape[1]
    dx = torch.empty((parent.n, C), device=dy.device, dtype=torch.bfloat16)
    check(_lib.load().pcs_pool_features_backward(R.ctx, parent.handle, _p(dy.contiguous()), C, _p(dx), _s()))
    return dx


def up_conv_forward(R: Renderer, parent: Voxels, x, w_bf16, bias, relu=True) -> torch.Tensor:
    cin, cout = x.shape[1], w_bf16.shape[1]
    y = torch.empty((parent.n, cout), device=x.device, dtype=torch.bfloat16)
    check(_lib.load().pcs_up_conv_forward(R.ctx, parent.handle, _p(x), cin, _p(w_bf16), _p(bias), cout,
                                          int(relu), _p(y), _s()))
    return y


def up_conv_backward(R: Renderer, parent: Voxels, x, w_bf16, y, dy, dw=None, db=None) -> torch.Tensor:
    cin, cout = x.shape[1], w_bf16.shape[1]
    dx = torch.empty((parent.V, cin), device=x.device, dtype=torch.bfloat16)
    check(_lib.load().pcs_up_conv_backward(R.ctx, parent.handle, _p(x), cin, _p(w_bf16), cout, _p(y),
                                           _p(dy.contiguous()), _p(dx), _p(dw), _p(db), _s()))
    return dx


def unet_head_forward(R: Renderer, vox: Voxels, f, w1, b1, w2, b2, xyz, rgb) -> dict:
    n = xyz.shape[1]
    dev = xyz.device
    g = dict(mean=torch.empty((3, n), device=dev), quat=torch.empty((4, n), device=dev),
             scale=torch.empty((3, n), device=dev), opacity=torch.empty((n,), device=dev),
             rgb=torch.empty((3, n), device=dev), normal=torch.empty((3, n), device=dev))
    check(_lib.load().pcs_unet_head_forward(R.ctx, vox.handle, _p(f), _p(w1), _p(b1), _p(w2), _p(b2), _p(xyz),
                                            _p(rgb), _p(g["mean"]), _p(g["quat"]), _p(g["scale"]),
                                            _p(g["opacity"]), _p(g["rgb"]), _p(g["normal"]), _s()))
    return g


def unet_head_backward(R: Renderer, vox: Voxels, f, w1, b1, w2, b2, xyz, grads: dict, dws: list) -> torch.Tensor:
    df = torch.empty((vox.V, 32), device=f.device, dtype=torch.bfloat16)
    c = {k: (grads[k].contiguous() if grads.get(k) is not None else None)
         for k in ("mean", "quat", "scale", "opacity", "normal")}
    check(_lib.load().pcs_unet_head_backward(R.ctx, vox.handle, _p(f), _p(w1), _p(b1), _p(w2), _p(b2), _p(xyz),
                                             _p(c["mean"]), _p(c["quat"]), _p(c["scale"]), _p(c["opacity"]),
                                             _p(c["normal"]), _p(df), *(_p(t) for t in dws), _s()))
    return df


class UNetEstimator:
    """The paper's estimator (Section 3.2): a sparse UNet over three 2x2x2 poolings with pruned
    transposed convolutions and skip connections, and a shared MLP head predicting per point the
    offset, scale, rotation, opacity and normal. FP32 master weights, BF16 copies for the MFMA
    kernels; the head runs in FP32."""

    def __init__(self, renderer: Renderer, seed: int = 0, opacity_init: float = 0.9, head_residual: bool = False):
        """``head_residual`` False (the default) holds the head's weights on the point's residual at
        zero, so every point of a voxel gets the same parameters; True trains them too."""
        self.R = renderer
        self.head_residual = head_residual
        dev = torch.device("cuda", renderer.device)
        gen = torch.Generator(device="cpu").manual_seed(seed)
        self.w, self.b = {}, {}
        for name, kind, cin, cout in UNET_LAYOUT:
            k = 27 if kind == "subm" else 8
            fan_in = k * (UNET_IN_CHANNELS if name == "e0a" else cin)
            w = torch.randn((k, cout, cin), generator=gen) * math.sqrt(2.0 / fan_in)
            if name == "e0a":
                w[:, :, UNET_IN_CHANNELS:] = 0.0
            self.w[name] = w.to(dev)
            self.b[name] = torch.zeros(cout, device=dev)
        self.w1 = (torch.randn((UNET_HEAD_HIDDEN, UNET_HEAD_IN), generator=gen) * math.sqrt(2.0 / UNET_HEAD_IN)).to(dev)
        if not head_residual:
            self.w1[:, 32:] = 0.0
        self.b1 = torch.zeros(UNET_HEAD_HIDDEN, device=dev)
        w2 = torch.randn((UNET_HEAD_OUT, UNET_HEAD_HIDDEN), generator=gen) * 1e-3
        w2[11:14] = torch.randn((3, UNET_HEAD_HIDDEN), generator=gen) * 0.1    # varied initial normals
        self.w2 = w2.to(dev)
        self.b2 = torch.zeros(UNET_HEAD_OUT, device=dev)
        self.b2[3:6] = math.log(2.3)            # initial scale ~2.3 voxel edges
        self.b2[10] = math.log(opacity_init / (1.0 - opacity_init))
        names = [n for n, *_ in UNET_LAYOUT]
        self.params = [self.w[n] for n in names] + [self.b[n] for n in names] + [self.w1, self.b1, self.w2, self.b2]

    def load_params(self, params: list):
        """Copy saved parameters (order of ``params``). A head saved with only the 32 feature
        inputs gets zero weights on the residual inputs, which makes it the same per-voxel head."""
        with torch.no_grad():
            for p, v in zip(self.params, params):
                v = v.to(p.device)
                if p is self.w1 and v.shape[1] < p.shape[1]:
                    p.zero_()
                    p[:, :v.shape[1]] = v
                else:
                    p.copy_(v)

    def _bf16_weights(self) -> dict:
        """BF16 copies of the convolution weights, made again only for weights changed in place
        since (tracked by each tensor's version counter, which optimiser steps advance)."""
        cache = getattr(self, "_wb_cache", None)
        if cache is None:
            cache = self._wb_cache = {}
        out = {}
        for n, w in self.w.items():
            hit = cache.get(n)
            if hit is None or hit[0] is not w or hit[1] != w._version:
                hit = cache[n] = (w, w._version, w.to(torch.bfloat16).contiguous())
            out[n] = hit[2]
        return out

    @staticmethod
    def levels(R: Renderer, vox: Voxels, reuse: list | None = None) -> list:
        """Voxel sets of levels 0..3 of a voxelised cloud (level 0 is ``vox``). ``reuse``, the
        list of an earlier call, has its pooled levels rebuilt in place (no new device buffers)."""
        lv = [vox]
        for i in range(3):
            lv.append(pool(R, lv[-1], reuse[i + 1] if reuse is not None else None))
        return lv

    def forward(self, lv: list, save=False):
        R = self.R
        wb = self._bf16_weights()
        x0 = lv[0].arrays()["features"]
        a = {}

        def conv(name, x, level):
            a[name + ":in"] = x
            a[name] = conv_forward(R, lv[level], x, wb[name], self.b[name], relu=True)
            return a[name]

        def up(name, x, level):          # from level + 1 to the children at `level`
            a[name + ":in"] = x
            a[name] = up_conv_forward(R, lv[level + 1], x, wb[name], self.b[name], relu=True)
            return a[name]

        def conv_skip(name, x, skip, level):
            # the skip concatenation: training keeps the concatenated input for the weight gradient;
            # inference lets the convolution read the two parts where they lie
            if save:
                return conv(name, torch.cat([x, skip], dim=1), level)
            a[name] = conv_forward_cat(R, lv[level], x, skip, wb[name], self.b[name], relu=True)
            return a[name]

        s0 = conv("e0b", conv("e0a", x0, 0), 0)
        s1 = conv("e1", pool_features(R, lv[1], s0), 1)
        s2 = conv("e2", pool_features(R, lv[2], s1), 2)
        b3 = conv("e3", pool_features(R, lv[3], s2), 3)
        d2 = conv_skip("d2", up("u3", b3, 2), s2, 2)
        d1 = conv_skip("d1", up("u2", d2, 1), s1, 1)
        d0 = conv_skip("d0", up("u1", d1, 0), s0, 0)
        g = unet_head_forward(R, lv[0], d0, self.w1, self.b1, self.w2, self.b2, lv[0].xyz, lv[0].rgb)
        if save:
            return g, dict(acts=a, wb=wb)
        return g

    def backward(self, lv: list, saved: dict, grads: dict):
        """Weight gradients (FP32, order of ``params``) from per-point Gaussian gradients."""
        R = self.R
        a, wb = saved["acts"], saved["wb"]
        dw = {n: torch.zeros_like(w) for n, w in self.w.items()}
        db = {n: torch.zeros_like(b) for n, b in self.b.items()}
        dh = [torch.zeros_like(t) for t in (self.w1, self.b1, self.w2, self.b2)]
        g = unet_head_backward(R, lv[0], a["d0"], self.w1, self.b1, self.w2, self.b2, lv[0].xyz, grads, dh)
        if not self.head_residual:
            dh[0][:, 32:] = 0.0

        def conv_b(name, level, dy, want_dx=True):
            return conv_backward(R, lv[level], a[name + ":in"], wb[name], a[name], dy, want_dx=want_dx,
                                 dw=dw[name], db=db[name])

        def up_b(name, level, dy):
            return up_conv_backward(R, lv[level + 1], a[name + ":in"], wb[name], a[name], dy, dw=dw[name],
                                    db=db[name])

        dc0 = conv_b("d0", 0, g)                                  # (V0, 64): [u1 | s0]
        ds0 = dc0[:, 32:]
        dd1 = up_b("u1", 0, dc0[:, :32])
        dc1 = conv_b("d1", 1, dd1)                                # (V1, 128): [u2 | s1]
        ds1 = dc1[:, 64:]
        dd2 = up_b("u2", 1, dc1[:, :64])
        dc2 = conv_b("d2", 2, dd2)                                # (V2, 128): [u3 | s2]
        ds2 = dc2[:, 64:]
        db3 = up_b("u3", 2, dc2[:, :64])
        dp3 = conv_b("e3", 3, db3)
        ds2 = ds2 + pool_features_backward(R, lv[3], dp3)
        dp2 = conv_b("e2", 2, ds2)
        ds1 = ds1 + pool_features_backward(R, lv[2], dp2)
        dp1 = conv_b("e1", 1, ds1)
        ds0 = ds0 + pool_features_backward(R, lv[1], dp1)
        de0 = conv_b("e0b", 0, ds0)
        conv_b("e0a", 0, de0, want_dx=False)
        names = [n for n, *_ in UNET_LAYOUT]
        return [dw[n] for n in names] + [db[n] for n in names] + dh


def normal_loss(n_hat: torch.Tensor, n_gt: torch.Tensor, mask: torch.Tensor, w3: float = 0.1) -> torch.Tensor:
    """Eq. 5's normal term over the pixels in ``mask``: |n x n_hat|_2 + w3 min(|n - n_hat|_2,
    |n + n_hat|_2), both normal maps normalised per pixel ((C,3,H,W) maps, (C,H,W) mask)."""
    eps = 1e-8
    a = n_hat / (n_hat.norm(dim=1, keepdim=True) + eps)
    b = n_gt / (n_gt.norm(dim=1, keepdim=True) + eps)
    cross = torch.linalg.cross(a, b, dim=1).norm(dim=1)
    sign = torch.minimum((a - b).norm(dim=1), (a + b).norm(dim=1))
    per = cross + w3 * sign
    m = mask.to(per.dtype)
    return (per * m).sum() / m.sum().clamp_min(1.0)


def train_step_unet(est: "UNetEstimator", opt: Adam, clouds: list, view_fn, w1=1.0, w2=10.0, w3=0.1) -> float:
    """One optimisation step with Eq. 5: L = w1 |I - I_hat|_1 + w2 L_n, L_n the normal term of
    ``normal_loss`` on the pixels covered in both the rendered and the ground-truth normal maps.
    ``view_fn(cloud)`` returns (cameras, gt rgb (C,3,H,W), gt normal (C,3,H,W), gt alpha (C,H,W))."""
    R = est.R
    total = [torch.zeros_like(p) for p in est.params]
    loss_sum = 0.0
    for c in clouds:
        cams, gt, gt_n, gt_a = view_fn(c)
        g, saved = est.forward(c["levels"], save=True)
        st = c.get("state")
        if st is None:
            st = c["state"] = RenderState(R)
        out = R.render(g, cams, default_options(), state=st, want=("rgb", "normal", "alpha"))
        img = out["rgb"].requires_grad_(True)
        nrm = out["normal"].requires_grad_(True)
        mask = (gt_a > 0.5) & (out["alpha"] > 0.5)
        loss = w1 * (img - gt).abs().mean() + w2 * normal_loss(nrm, gt_n, mask, w3)
        loss.backward()
        gg = R.render_backward(st, dict(rgb=img.grad, normal=nrm.grad))
        grads = est.backward(c["levels"], saved, gg)
        for t, gr in zip(total, grads):
            t.add_(gr, alpha=1.0 / len(clouds))
        loss_sum += float(loss.item())
    opt.step(total)
    return loss_sum / len(clouds)
