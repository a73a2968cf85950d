"""GPU parity of the paper's UNet-like estimator kernels (Section 3.2) against the FP64 oracle
(oracle/unet.py) run on the same BF16 values.

Bars: parent voxels, child -> parent maps and upsampling tables bit-exact; pooled features within
BF16 rounding of the FP64 mean; transposed-convolution outputs within 2^-8 relative plus 1e-5 of
the sum of absolute products (BF16 output rounding, FP32 accumulation), its gradients within 1e-4
of the sum of absolute terms (as the submanifold convolution's); the FP32 per-point head within
1e-4 relative (BF16 features and FP32 residuals in, FP32 arithmetic). The whole network's BF16 error against the FP64
chain is reported per output.
"""
import numpy as np
import pytest
import torch

from oracle import estimator as E
from oracle import unet as U
from synthetic import make_surface

pytestmark = pytest.mark.gpu
GRID = 128


@pytest.fixture(scope="module")
def R():
    import paper_2409_16504_amd as P
    return P.Renderer(0)


def bf16(a):
    t = torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(torch.bfloat16)
    return t.to(torch.float64).numpy(), t


@pytest.fixture(scope="module")
def cloud(R):
    from paper_2409_16504_amd.estimator import UNetEstimator, Voxels
    _, p, rgb = make_surface(40000, 21, quantize=False)
    p = np.clip(p, -0.999, 0.999).astype(np.float32)
    vox = Voxels(R).build(torch.from_numpy(p).cuda(), torch.from_numpy(rgb).cuda(), GRID)
    lv = UNetEstimator.levels(R, vox)
    ref = E.voxelize(p, rgb, GRID)
    olv = U.levels(ref["coords"], GRID)
    return p, rgb, vox, lv, ref, olv


def test_pooled_levels_and_tables(cloud):
    _, _, vox, lv, ref, olv = cloud
    for level in range(1, 4):
        arr = lv[level].arrays()
        assert lv[level].V == olv[level]["coords"].shape[0]
        assert np.array_equal(arr["coords"].cpu().numpy().T, olv[level]["coords"]), level
        assert np.array_equal(arr["point_voxel"].cpu().numpy(), olv[level]["parent_of"]), level
        assert np.array_equal(arr["nbr"].cpu().numpy(), olv[level]["nbr"]), level
    assert lv[3].V < lv[2].V < lv[1].V < vox.V


def test_pool_features_and_adjoint(R, cloud):
    from paper_2409_16504_amd.estimator import pool_features, pool_features_backward
    _, _, vox, lv, ref, olv = cloud
    rng = np.random.default_rng(3)
    for C in (32, 64, 128):
        x64, xt = bf16(rng.normal(size=(vox.V, C)))
        y = pool_features(R, lv[1], xt.cuda()).to(torch.float64).cpu().numpy()
        want = U.pool(olv[0]["coords"], x64)["feat"]
        assert np.all(np.abs(y - want) <= 2.0 ** -8 * np.abs(want) + 1e-6), C
        d64, dt = bf16(rng.normal(size=(lv[1].V, C)))
        dx = pool_features_backward(R, lv[1], dt.cuda()).to(torch.float64).cpu().numpy()
        cnt = olv[1]["count"][olv[1]["parent_of"]]
        want = d64[olv[1]["parent_of"]] / cnt[:, None]
        assert np.all(np.abs(dx - want) <= 2.0 ** -8 * np.abs(want) + 1e-12), C


@pytest.mark.parametrize("level,half,cout", [(0, 32, 32), (1, 64, 64), (2, 64, 64), (0, 64, 32)])
def test_skip_concatenation_is_read_in_place(R, cloud, level, half, cout):
    """The decoder's convolution over the skip concatenation [up | skip], read from the two arrays
    where they lie, equals the convolution over the concatenated rows bit for bit; unequal halves
    are refused."""
    from paper_2409_16504_amd import _lib
    from paper_2409_16504_amd.estimator import conv_forward, conv_forward_cat
    _, _, vox, lv, _, _ = cloud
    rng = np.random.default_rng(30 + level)
    V = lv[level].V
    _, x1 = bf16(rng.normal(size=(V, half)))
    _, x2 = bf16(rng.normal(size=(V, half)))
    _, wt = bf16(rng.normal(size=(27, cout, 2 * half)) * np.sqrt(2.0 / (27 * 2 * half)))
    bt = torch.from_numpy(rng.normal(size=cout).astype(np.float32) * 0.1).cuda()
    x1, x2, wt = x1.cuda(), x2.cuda(), wt.cuda()
    for relu in (False, True):
        want = conv_forward(R, lv[level], torch.cat([x1, x2], dim=1), wt, bt, relu)
        got = conv_forward_cat(R, lv[level], x1, x2, wt, bt, relu)
        torch.cuda.synchronize()
        assert torch.equal(got.view(torch.int16), want.view(torch.int16)), relu
    with pytest.raises(_lib.PcsError):
        conv_forward_cat(R, lv[level], x1, x2[:, :half // 2].contiguous(), wt, bt, True)


@pytest.mark.parametrize("level,cin,cout", [(0, 64, 32), (1, 64, 64), (2, 128, 64)])
def test_up_conv_forward_and_adjoint(R, cloud, level, cin, cout):
    """Children at `level` from their parents at level + 1."""
    from paper_2409_16504_amd.estimator import up_conv_backward, up_conv_forward
    _, _, vox, lv, ref, olv = cloud
    rng = np.random.default_rng(10 + level)
    par = lv[level + 1]
    child = olv[level]["coords"]
    parent_of = olv[level + 1]["parent_of"]
    x64, xt = bf16(rng.normal(size=(par.V, cin)))
    w64, wt = bf16(rng.normal(size=(8, cout, cin)) * np.sqrt(2.0 / cin))
    b = rng.normal(size=cout).astype(np.float32) * 0.1
    bt = torch.from_numpy(b).cuda()
    y = up_conv_forward(R, par, xt.cuda(), wt.cuda(), bt, relu=False)
    W = w64.transpose(0, 2, 1)                       # (8, Cin, Cout)
    want = U.up_conv(x64, W, b.astype(np.float64), child, parent_of, relu=False)
    sabs = np.einsum("vc,vco->vo", np.abs(x64[parent_of]), np.abs(W[U.child_offset(child)])) + np.abs(b)
    got = y.to(torch.float64).cpu().numpy()
    assert np.all(np.abs(got - want) <= 2.0 ** -8 * np.abs(want) + 1e-5 * sabs)
    # adjoint with a ReLU mask from the forward output
    yr = up_conv_forward(R, par, xt.cuda(), wt.cuda(), bt, relu=True)
    yr64 = yr.to(torch.float64).cpu().numpy()
    g64, gt = bf16(rng.normal(size=(lv[level].V, cout)))
    dw = torch.zeros((8, cout, cin), device="cuda")
    db = torch.zeros(cout, device="cuda")
    dx = up_conv_backward(R, par, xt.cuda(), wt.cuda(), yr, gt.cuda(), dw=dw, db=db)
    gm = g64 * (yr64 > 0)
    k = U.child_offset(child)
    dx_want = np.zeros_like(x64)
    np.add.at(dx_want, parent_of, np.einsum("vo,vco->vc", gm, W[k]))
    dx_abs = np.zeros_like(x64)
    np.add.at(dx_abs, parent_of, np.einsum("vo,vco->vc", np.abs(gm), np.abs(W[k])))
    dxg = dx.to(torch.float64).cpu().numpy()
    assert np.all(np.abs(dxg - dx_want) <= 2.0 ** -8 * np.abs(dx_want) + 1e-4 * dx_abs + 1e-6)
    dw_want = np.zeros((8, cin, cout))
    dw_abs = np.zeros((8, cin, cout))
    for o in range(8):
        m = k == o
        dw_want[o] = x64[parent_of[m]].T @ gm[m]
        dw_abs[o] = np.abs(x64[parent_of[m]]).T @ np.abs(gm[m])
    dwg = dw.cpu().numpy().astype(np.float64).transpose(0, 2, 1)
    assert np.all(np.abs(dwg - dw_want) <= 1e-4 * dw_abs + 1e-6)
    assert np.allclose(db.cpu().numpy(), gm.sum(axis=0), rtol=1e-4, atol=1e-3)


def test_head_forward_and_adjoint(R, cloud):
    from paper_2409_16504_amd.estimator import unet_head_backward, unet_head_forward
    p, rgb, vox, lv, ref, olv = cloud
    rng = np.random.default_rng(5)
    f64, ft = bf16(np.abs(rng.normal(size=(vox.V, 32))))
    W1 = (rng.normal(size=(32, 35)) * 0.3).astype(np.float32)
    b1 = (rng.normal(size=32) * 0.1).astype(np.float32)
    W2 = (rng.normal(size=(14, 32)) * 0.3).astype(np.float32)
    b2 = (rng.normal(size=14) * 0.1).astype(np.float32)
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    xyz, col = cu(p), cu(rgb)
    g = unet_head_forward(R, vox, ft.cuda(), cu(W1), cu(b1), cu(W2), cu(b2), xyz, col)
    want = U.head(f64, W1.T.astype(np.float64), b1, W2.T.astype(np.float64), b2, p, rgb, ref["point_voxel"], GRID,
                  ref["coords"])
    for k in ("mean", "quat", "scale", "opacity", "rgb", "normal"):
        got = g[k].cpu().numpy().astype(np.float64)
        assert np.allclose(got, want[k], rtol=1e-4, atol=1e-5), k
    # adjoint against FP64 autograd of the same head (per point: its voxel's features and its residual)
    tf = torch.from_numpy(f64).requires_grad_(True)
    tw = [torch.from_numpy(a.astype(np.float64)).requires_grad_(True) for a in (W1, b1, W2, b2)]
    pv = torch.from_numpy(ref["point_voxel"])
    res = torch.from_numpy((p.T.astype(np.float64) + 1.0) * (GRID / 2.0) - (ref["coords"][ref["point_voxel"]] + 0.5))
    x = torch.cat([tf[pv], res], dim=1)
    h = torch.relu(x @ tw[0].T + tw[1])
    raw = h @ tw[2].T + tw[3]
    e = 2.0 / GRID
    mean = torch.from_numpy(p.astype(np.float64)) + e * torch.tanh(raw[:, 0:3]).T
    scale = (e * torch.exp(raw[:, 3:6])).T
    q = raw[:, 6:10] + torch.tensor([1.0, 0, 0, 0], dtype=torch.float64)
    q = (q / q.norm(dim=1, keepdim=True)).T
    opac = torch.sigmoid(raw[:, 10])
    nrm = (raw[:, 11:14] / raw[:, 11:14].norm(dim=1, keepdim=True)).T
    up = {k: rng.normal(size=s) for k, s in dict(mean=(3, p.shape[1]), quat=(4, p.shape[1]),
                                                  scale=(3, p.shape[1]), opacity=(p.shape[1],),
                                                  normal=(3, p.shape[1])).items()}
    loss = sum((t * torch.from_numpy(up[k])).sum() for k, t in
               dict(mean=mean, quat=q, scale=scale, opacity=opac, normal=nrm).items())
    loss.backward()
    dws = [torch.zeros(a.shape, device="cuda") for a in (W1, b1, W2, b2)]
    df = unet_head_backward(R, vox, ft.cuda(), cu(W1), cu(b1), cu(W2), cu(b2), xyz,
                            {k: cu(v.astype(np.float32)) for k, v in up.items()}, dws)
    dfg = df.to(torch.float64).cpu().numpy()
    ref_df = tf.grad.numpy()
    assert np.all(np.abs(dfg - ref_df) <= 2.0 ** -8 * np.abs(ref_df) + 1e-3 * np.abs(ref_df).max())
    for got, t in zip(dws, tw):
        r = t.grad.numpy()
        assert np.allclose(got.cpu().numpy(), r, rtol=1e-3, atol=1e-4 * np.abs(r).max()), t.shape
    # a pooled level is not the points' voxels: refused
    from paper_2409_16504_amd import PcsError
    with pytest.raises(PcsError):
        unet_head_forward(R, lv[1], ft.cuda()[: lv[1].V], cu(W1), cu(b1), cu(W2), cu(b2), xyz, col)


def test_network_forward_error_against_fp64(R, cloud):
    """The whole network in BF16 on MFMA against the FP64 chain at the same (BF16) weights; the error
    is reported per output (no precision claim; the assertion only guards against gross errors)."""
    from paper_2409_16504_amd.estimator import UNET_LAYOUT, UNetEstimator
    p, rgb, vox, lv, ref, olv = cloud
    est = UNetEstimator(R, seed=4)
    g = est.forward(lv)
    weights = {}
    for name, kind, ci, co in UNET_LAYOUT:
        w = est.w[name].to(torch.bfloat16).to(torch.float64).cpu().numpy().transpose(0, 2, 1)
        weights[name] = (w, est.b[name].cpu().numpy().astype(np.float64))
    x0 = np.zeros((vox.V, 32))
    x0[:, :9] = vox.arrays()["features"][:, :9].to(torch.float64).cpu().numpy()
    f = U.forward(x0, olv, weights)
    want = U.head(f, est.w1.cpu().numpy().T.astype(np.float64), est.b1.cpu().numpy(),
                  est.w2.cpu().numpy().T.astype(np.float64), est.b2.cpu().numpy(), p, rgb, ref["point_voxel"], GRID,
                  ref["coords"])
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}
    errs = dict(mean=np.abs(got["mean"] - want["mean"]).max() / (2.0 / GRID),
                scale_rel=np.abs(got["scale"] / want["scale"] - 1).max(),
                opacity=np.abs(got["opacity"] - want["opacity"]).max(),
                angle_deg=np.degrees(2 * np.arccos(np.clip(np.abs((got["quat"] * want["quat"]).sum(0)), 0, 1))).max(),
                normal_deg=np.degrees(np.arccos(np.clip((got["normal"] * want["normal"]).sum(0), -1, 1))).max())
    print(f"UNet BF16 vs FP64: {errs}", flush=True)
    assert errs["scale_rel"] < 0.1 and errs["opacity"] < 0.05 and errs["mean"] < 0.1
