"""GPU tests of the boundary conventions: capacity mode (no wait on the device, fixed-capacity tile
buffers, overflow reported), the error path of the ordering's bounded waits, HIP-graph capture of
a capacity-mode frame, and workspace from PyTorch's caching allocator.

Capacity-mode frames are compared with plain renders of the same inputs (bit-exact key lists,
tile ranges and images), and those with the oracle by the parity tests.
"""
import numpy as np
import pytest

import oracle
from helpers import c1_scene, surface_gaussians, to_torch
from synthetic import look_at_camera

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import paper_2409_16504_amd as P
    return P.Renderer(0)


def _render(R, tg, cams, capacity, state=None):
    import torch
    import paper_2409_16504_amd as P
    st = state if state is not None else P.RenderState(R)
    out = R.render(tg, cams, P.default_options(), state=st, capacity=capacity)
    torch.cuda.synchronize()
    return st, {k: v.cpu().numpy() for k, v in out.items()}


def _same(a_imgs, a_bins, b_imgs, b_bins):
    for k in a_imgs:
        assert np.array_equal(a_imgs[k], b_imgs[k]), k
    for k in ("keys", "vals", "ranges", "n_contrib", "t_final"):
        assert np.array_equal(a_bins[k], b_bins[k]), k


def test_capacity_mode_matches_plain_render(R):
    """The first capacity-mode frame of a state sizes it (1.25 x its instance total); the later ones
    reuse the capacity without waiting, and every frame equals the plain render."""
    g = surface_gaussians(1_000_000, 1006)
    tg = to_torch(g)
    cams = [look_at_camera([0, 0, 3], width=1920, height=1080)]
    print("capacity mode: 1M Gaussians at 1920x1080", flush=True)
    st0, plain = _render(R, tg, cams, False)
    ref_bins = R.bins(st0)
    import paper_2409_16504_amd as P
    st = P.RenderState(R)
    for it in range(3):
        _, imgs = _render(R, tg, cams, True, st)
        assert st.status() == (0, 0)
        _same(plain, ref_bins, imgs, R.bins(st))
    m = ref_bins["keys"].size
    assert m + m // 4 - 1 <= st.capacity <= m + m // 4 + 1


def test_capacity_overflow_is_reported_then_resized(R):
    """A frame with more instances than the capacity composites nothing (background), reports
    PCS_ERR_CAPACITY with the count it needs, and the next capacity-mode frame is sized for it."""
    import paper_2409_16504_amd as P
    from paper_2409_16504_amd import _lib
    g, cams = c1_scene()
    few = {k: v[..., :200].copy() for k, v in g.items()}
    st = P.RenderState(R)
    _render(R, to_torch(few), cams, True, st)             # sizes the capacity on 200 Gaussians
    assert st.status()[0] == _lib.PCS_OK
    cap0 = st.capacity
    print(f"capacity after 200 Gaussians: {cap0}", flush=True)
    _, imgs = _render(R, to_torch(g), cams, True, st)     # 2,000 Gaussians: more instances
    ref = oracle.render(g, cams, mode="ref")
    need = ref["keys"].size
    assert need > cap0
    rc, req = st.status()
    assert rc == _lib.PCS_ERR_CAPACITY and req == need
    assert np.all(imgs["rgb"] == 0) and np.all(imgs["alpha"] == 0)      # background only
    with pytest.raises(P.PcsError):
        R.bins(st)
    # the backward of the failed frame adds nothing
    import torch
    gr = R.render_backward(st, dict(rgb=torch.ones((1, 3, 128, 128), device="cuda")))
    assert float(gr["mean"].abs().sum()) == 0.0 and float(gr["rgb"].abs().sum()) == 0.0
    # the next frame is sized from the overflowing one's count and renders correctly
    _, imgs = _render(R, to_torch(g), cams, True, st)
    assert st.status() == (0, 0) and st.capacity >= need
    bins = R.bins(st)
    assert np.array_equal(bins["keys"], ref["keys"]) and np.array_equal(bins["vals"], ref["vals"])
    _, plain = _render(R, to_torch(g), cams, False)
    for k in plain:
        assert np.array_equal(plain[k], imgs[k]), k


@pytest.mark.parametrize("capacity", [False, True])
def test_wait_bound_running_out_fails_the_frame(R, capacity):
    """A look-back wait bound of one round makes the ordering's waits give up (the host forces it,
    every kernel still ends): the frame reports PCS_ERR_HIP, composites nothing and exports no lists.
    With the bound restored the same state renders correctly again."""
    import paper_2409_16504_amd as P
    from paper_2409_16504_amd import _lib
    g = surface_gaussians(1_000_000, 1006)
    tg = to_torch(g)
    cams = [look_at_camera([0, 0, 3], width=1920, height=1080)]
    _, plain = _render(R, tg, cams, False)
    st = P.RenderState(R)
    if capacity:
        _render(R, tg, cams, True, st)                     # size the capacity first
    print(f"wait bound 1 round, capacity mode {capacity}", flush=True)
    R.set_wait_limit(1)
    try:
        _, imgs = _render(R, tg, cams, capacity, st)
        rc, _ = st.status()
    finally:
        R.set_wait_limit(0)
    assert rc == _lib.PCS_ERR_HIP
    assert np.all(imgs["alpha"] == 0) and np.all(imgs["rgb"] == 0)
    with pytest.raises(P.PcsError):
        R.bins(st)
    _, imgs = _render(R, tg, cams, capacity, st)
    assert st.status() == (0, 0)
    for k in plain:
        assert np.array_equal(plain[k], imgs[k]), k


def test_graph_capture_replays_capacity_frame(R):
    """A capacity-mode frame captured in a HIP graph (through torch.cuda.CUDAGraph) and replayed
    gives the plain render's key lists and images bit for bit, on every replay, with eager work and
    synchronisations between the replays, one of them an eager render of another state on the same
    context (which must match its own reference too)."""
    import torch
    import paper_2409_16504_amd as P
    g = surface_gaussians(800_000, 1002)
    tg = to_torch(g)
    cams = [look_at_camera([0.4, 0.2, 3], width=1920, height=1080)]
    st0, plain = _render(R, tg, cams, False)
    ref_bins = R.bins(st0)
    st = P.RenderState(R)
    out = R.render(tg, cams, P.default_options(), state=st, capacity=True)    # sizes everything
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):                     # one more eager frame on the capture stream
        R.render(tg, cams, P.default_options(), state=st, out=out, capacity=True)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    gs, cs = c1_scene()
    tgs = to_torch(gs)
    st_small, small_ref = _render(R, tgs, cs, False)
    small_bins = R.bins(st_small)
    graph = torch.cuda.CUDAGraph()
    print("capturing a capacity-mode frame", flush=True)
    with torch.cuda.graph(graph):
        R.render(tg, cams, P.default_options(), state=st, out=out, capacity=True)
    for rep in range(3):
        if rep == 1:                                  # an eager frame between replays
            st_e, imgs_e = _render(R, tgs, cs, False)
            _same(small_ref, small_bins, imgs_e, R.bins(st_e))
        for v in out.values():
            v.fill_(-1.0)                             # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert st.status() == (0, 0)
        imgs = {k: v.cpu().numpy() for k, v in out.items()}
        _same(plain, ref_bins, imgs, R.bins(st))
        print(f"replay {rep}: bit-identical", flush=True)


def test_workspace_comes_from_the_torch_allocator():
    """With the default torch allocator the library's workspace shows up in PyTorch's allocated
    bytes; without it, it does not."""
    import torch
    import paper_2409_16504_amd as P
    g, cams = c1_scene()
    tg = to_torch(g)
    for use_torch in (True, False):
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        R2 = P.Renderer(0, torch_allocator=use_torch)
        st = P.RenderState(R2)
        out = R2.render(tg, cams, P.default_options(), state=st)
        torch.cuda.synchronize()
        outputs = sum(v.numel() * 4 for v in out.values())
        grew = torch.cuda.memory_allocated() - before - outputs
        print(f"torch allocator {use_torch}: {grew} bytes of workspace in torch's pool", flush=True)
        if use_torch:
            assert grew > 500_000                      # records, sort buffers, ...
        else:
            assert grew == 0
        del st, out
        R2.close()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
