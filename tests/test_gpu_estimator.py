"""GPU parity of the sparse estimator kernels (voxelisation, kernel map, BF16 MFMA submanifold
convolution and its adjoint, head) against the FP64 oracle run on the same BF16 values.

Bars: voxel coordinates, point-to-voxel map and kernel map bit-exact; features within BF16
rounding; convolution outputs within 2^-8 relative (the BF16 rounding of the output) plus 1e-5 of
the sum of absolute products (FP32 accumulation); gradients within 1e-4 of the sum of absolute
terms (BF16 inputs, FP32 accumulation, float atomics).
"""
import numpy as np
import pytest
import torch

from oracle import estimator as E
from synthetic import make_surface

pytestmark = pytest.mark.gpu
GRID = 128


@pytest.fixture(scope="module")
def R():
    import paper_2409_16504_amd as P
    return P.Renderer(0)


def bf16_round(a):
    """Round FP32 values to BF16 (nearest even), returned as float64 and as a bf16 tensor."""
    t = torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(torch.bfloat16)
    return t.to(torch.float64).numpy(), t


@pytest.fixture(scope="module")
def cloud(R):
    from paper_2409_16504_amd.estimator import Voxels
    rng = np.random.default_rng(12)
    _, p, rgb = make_surface(40000, 21, quantize=False)
    p = p + rng.normal(0, 0.001, p.shape).astype(np.float32)
    p = np.clip(p, -0.999, 0.999).astype(np.float32)
    # 40k surface points: the 128^3 grid keeps neighbouring samples in neighbouring voxels
    vox = Voxels(R).build(torch.from_numpy(p).cuda(), torch.from_numpy(rgb).cuda(), GRID)
    ref = E.voxelize(p, rgb, GRID)
    return p, rgb, vox, ref


def test_voxelize_and_kernel_map(cloud):
    p, rgb, vox, ref = cloud
    arr = vox.arrays()
    assert vox.V == ref["coords"].shape[0]
    assert np.array_equal(arr["coords"].cpu().numpy().T, ref["coords"])
    assert np.array_equal(arr["point_voxel"].cpu().numpy(), ref["point_voxel"])
    nbr_ref = E.kernel_map(ref["coords"], GRID)
    assert np.array_equal(arr["nbr"].cpu().numpy(), nbr_ref)
    f = arr["features"].to(torch.float64).cpu().numpy()
    want = np.concatenate([ref["color"], ref["residual"], ref["position"]], axis=1)
    # BF16 rounding of the mean (2^-9 relative) plus, for the residual (p + 1) * G/2 - (c + 0.5),
    # the FP32 rounding of p + 1 amplified by G/2 (at most 2^-23 * G/2 per point) and the FP32
    # sums of at most a few points
    absolute = np.array([1e-6] * 3 + [2.0 ** -23 * GRID / 2 * 8] * 3 + [1e-6] * 3)
    assert np.all(np.abs(f[:, :9] - want) <= 2.0 ** -8 * np.abs(want) + absolute)
    assert np.all(f[:, 9:] == 0)
    assert (nbr_ref >= 0).sum(axis=0).mean() > 3          # neighbours exist (surface connectivity)


def test_voxelize_grids_and_adaptive_choice(R):
    """Every power-of-two grid voxelises bit-exactly; the adaptive choice is the finest grid whose
    voxels have at least six occupied neighbours on average."""
    from paper_2409_16504_amd.estimator import Voxels, adaptive_grid
    _, p, rgb = make_surface(20000, 33, quantize=True)
    tp, tr = torch.from_numpy(p).cuda(), torch.from_numpy(rgb).cuda()
    means = {}
    for g in (1024, 512, 256, 128, 64, 2):
        vox = Voxels(R).build(tp, tr, g)
        ref = E.voxelize(p, rgb, g)
        arr = vox.arrays()
        assert np.array_equal(arr["coords"].cpu().numpy().T, ref["coords"]), g
        assert np.array_equal(arr["point_voxel"].cpu().numpy(), ref["point_voxel"]), g
        nb = E.kernel_map(ref["coords"], g)
        assert np.array_equal(arr["nbr"].cpu().numpy(), nb), g
        means[g] = (nb >= 0).sum(axis=0).mean() - 1
        assert abs(vox.mean_neighbours() - means[g]) < 1e-6
    chosen = adaptive_grid(R, tp, tr)
    want = next((g for g in (1024, 512, 256, 128, 64) if means[g] >= 6.0), 64)
    assert chosen.grid == want
    with pytest.raises(RuntimeError):
        Voxels(R).build(tp, tr, 100)


@pytest.mark.parametrize("cin,cout", [(32, 32), (32, 64), (64, 64), (64, 32)])
def test_conv_forward_and_adjoint(R, cloud, cin, cout):
    from paper_2409_16504_amd.estimator import conv_backward, conv_forward
    _, _, vox, ref = cloud
    nbr = E.kernel_map(ref["coords"], GRID)
    rng = np.random.default_rng(cin * 100 + cout)
    V = vox.V
    x64, xt = bf16_round(rng.normal(size=(V, cin)))
    w64, wt = bf16_round(rng.normal(size=(27, cout, cin)) * 0.1)
    b = rng.normal(size=cout).astype(np.float32)
    W = w64.transpose(0, 2, 1)                         # oracle layout (27, cin, cout)
    y_ref = E.subm_conv(x64, W, b.astype(np.float64), nbr, relu=False)
    s_abs = E.subm_conv(np.abs(x64), np.abs(W), np.abs(b.astype(np.float64)), nbr, relu=False)
    y = conv_forward(R, vox, xt.cuda(), wt.cuda(), torch.from_numpy(b).cuda(), relu=False)
    y = y.to(torch.float64).cpu().numpy()
    assert np.all(np.abs(y - y_ref) <= 2.0 ** -8 * np.abs(y_ref) + 1e-5 * s_abs + 1e-6)
    yr = conv_forward(R, vox, xt.cuda(), wt.cuda(), torch.from_numpy(b).cuda(), relu=True).to(torch.float64).cpu().numpy()
    assert np.array_equal(yr, np.maximum(y, 0))
    # adjoint (no ReLU mask): dx, dW, db
    dy64, dyt = bf16_round(rng.normal(size=(V, cout)))
    dw = torch.zeros((27, cout, cin), device="cuda")
    db = torch.zeros(cout, device="cuda")
    dx = conv_backward(R, vox, xt.cuda(), wt.cuda(), None, dyt.cuda(), want_dx=True, dw=dw, db=db)
    dx_ref, dW_ref, db_ref = E.subm_conv_backward(x64, W, nbr, dy64)
    dxa, dWa, _ = E.subm_conv_backward(np.abs(x64), np.abs(W), nbr, np.abs(dy64))
    dx = dx.to(torch.float64).cpu().numpy()
    assert np.all(np.abs(dx - dx_ref) <= 2.0 ** -8 * np.abs(dx_ref) + 1e-5 * dxa + 1e-6)
    dW = dw.cpu().numpy().astype(np.float64).transpose(0, 2, 1)
    assert np.all(np.abs(dW - dW_ref) <= 1e-4 * dWa + 1e-5)
    assert np.allclose(db.cpu().numpy(), db_ref, rtol=1e-4, atol=1e-3)
    # ReLU mask: dy is zeroed where the forward output is not positive
    y_bf = torch.from_numpy(yr).to(torch.bfloat16).cuda()
    dw2 = torch.zeros((27, cout, cin), device="cuda")
    dx2 = conv_backward(R, vox, xt.cuda(), wt.cuda(), y_bf, dyt.cuda(), want_dx=True, dw=dw2, db=None)
    dym = np.where(yr > 0, dy64, 0.0)
    dx2_ref, dW2_ref, _ = E.subm_conv_backward(x64, W, nbr, dym)
    assert np.all(np.abs(dx2.to(torch.float64).cpu().numpy() - dx2_ref) <= 2.0 ** -8 * np.abs(dx2_ref) + 1e-5 * dxa + 1e-6)
    assert np.all(np.abs(dw2.cpu().numpy().astype(np.float64).transpose(0, 2, 1) - dW2_ref) <= 1e-4 * dWa + 1e-5)


def test_head_forward_and_adjoint(R, cloud):
    from paper_2409_16504_amd.estimator import head_backward, head_forward
    p, rgb, vox, ref = cloud
    rng = np.random.default_rng(9)
    V, n = vox.V, p.shape[1]
    f64, ft = bf16_round(np.abs(rng.normal(size=(V, 32))))
    wh = (rng.normal(size=(11, 32)) * 0.05).astype(np.float32)
    bh = (rng.normal(size=11) * 0.1).astype(np.float32)
    tp, tr = torch.from_numpy(p).cuda(), torch.from_numpy(rgb).cuda()
    g = head_forward(R, vox, ft.cuda(), torch.from_numpy(wh).cuda(), torch.from_numpy(bh).cuda(), tp, tr)
    out = E.head(f64, wh.T.astype(np.float64), bh.astype(np.float64), rgb, p, ref["point_voxel"], GRID)
    for k in ("quat", "scale", "opacity", "rgb"):
        a = g[k].cpu().numpy()
        assert np.allclose(a, out[k], rtol=1e-5, atol=1e-5), k
    dots = np.abs(np.einsum("kn,kn->n", g["normal"].cpu().numpy(), out["normal"]))
    s = np.sort(out["scale"], axis=0)
    sep = (s[1] - s[0]) > 1e-3 * s[1]
    assert np.all(dots[sep] > 1 - 1e-4)
    # adjoint against autograd of the FP64 torch head
    up = {k: torch.from_numpy(rng.normal(size=out[k].shape).astype(np.float32)) for k in ("quat", "scale", "opacity", "rgb")}
    dwh = torch.zeros((11, 32), device="cuda")
    dbh = torch.zeros(11, device="cuda")
    df = head_backward(R, vox, ft.cuda(), torch.from_numpy(wh).cuda(), torch.from_numpy(bh).cuda(),
                       {k: v.cuda() for k, v in up.items()}, dwh, dbh)
    F = torch.from_numpy(f64).requires_grad_(True)
    Wh = torch.from_numpy(wh.T.astype(np.float64)).requires_grad_(True)
    Bh = torch.from_numpy(bh.astype(np.float64)).requires_grad_(True)
    q, sc, o, c = E.head_torch(F, Wh, Bh, torch.from_numpy(rgb.astype(np.float64)), ref["point_voxel"], GRID)
    L = (q * up["quat"].double()).sum() + (sc * up["scale"].double()).sum() + (o * up["opacity"].double()).sum() + \
        (c * up["rgb"].double()).sum()
    L.backward()
    dfa = df.to(torch.float64).cpu().numpy()
    assert np.allclose(dfa, F.grad.numpy(), rtol=2.0 ** -7, atol=1e-3 * np.abs(F.grad.numpy()).max())
    assert np.allclose(dwh.cpu().numpy(), Wh.grad.numpy().T, rtol=1e-3, atol=1e-3 * np.abs(Wh.grad.numpy()).max())
    assert np.allclose(dbh.cpu().numpy(), Bh.grad.numpy(), rtol=1e-3, atol=1e-3 * np.abs(Bh.grad.numpy()).max())


def test_estimator_forward_error_vs_fp64(R, cloud):
    """Whole network in BF16 against the FP64 oracle with the same (BF16-rounded) weights: the
    error per output is reported, and bounded loosely (the network is random-initialised)."""
    from paper_2409_16504_amd.estimator import LAYERS, SparseEstimator
    p, rgb, vox, ref = cloud
    est = SparseEstimator(R, seed=3)
    g = est.forward(vox)
    nbr = E.kernel_map(ref["coords"], GRID)
    x = vox.arrays()["features"].to(torch.float64).cpu().numpy()
    for li in range(len(LAYERS)):
        W = est.w[li].to(torch.bfloat16).to(torch.float64).cpu().numpy().transpose(0, 2, 1)
        x = E.subm_conv(x, W, est.b[li].cpu().numpy().astype(np.float64), nbr, relu=True)
    out = E.head(x, est.wh.cpu().numpy().T.astype(np.float64), est.bh.cpu().numpy().astype(np.float64), rgb, p,
                 ref["point_voxel"], GRID)
    rel_s = np.abs(g["scale"].cpu().numpy() / out["scale"] - 1)
    ang = 2 * np.degrees(np.arccos(np.clip(np.abs(np.einsum("kn,kn->n", g["quat"].cpu().numpy(), out["quat"])), 0, 1)))
    do = np.abs(g["opacity"].cpu().numpy() - out["opacity"])
    dc = np.abs(g["rgb"].cpu().numpy() - out["rgb"])
    print(f"BF16 vs FP64: scale rel max {rel_s.max():.2e} p99 {np.percentile(rel_s, 99):.2e}; "
          f"quat angle max {ang.max():.2e} deg; opacity max {do.max():.2e}; rgb max {dc.max():.2e}")
    assert rel_s.max() < 0.05 and ang.max() < 2.0 and do.max() < 0.02 and dc.max() < 0.05
