"""Edge cases of the batched path against the FP64 oracle: the largest view
batch the library accepts (64 views in one launch), one more than that
(rejected), and degenerate image shapes (a single pixel, one row, one
column)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from synth import scenes
from tests.gpu_helpers import (GRAD_NAMES, TOL_G, check_forward, check_grad, cotangents, dev_scene, oracle_views,
                               rel)

pytestmark = pytest.mark.gpu

MAX_VIEWS = 64   # views one call accepts (GS_MAX_VIEWS)


@pytest.fixture(scope="module")
def ctx():
    import paper_2405_19614_amd as gs
    torch.cuda.set_device(0)
    return gs.Context(0)


def _check_forward_backward(ctx, s, seed):
    g, poses = dev_scene(s)
    color, depth, alpha, state, plan = ctx.forward(g, s.cams, poses)
    og, ref = oracle_views(s)
    print(f"  V={s.V} pairs={plan.n_pairs}", flush=True)
    label = f"edges V={s.V} {s.cams[0].width}x{s.cams[0].height}"
    check_forward(s, color, depth, alpha, ref, label)
    dC, dD, dA = cotangents(s, ref, seed=seed)
    t = lambda a: torch.tensor(a, device="cuda")
    grads, dpose = ctx.backward(g, s.cams, poses, state, plan, t(dC), t(dD), t(dA))
    torch.cuda.synchronize()
    rg = O.backward_views(og, s.cams, s.poses, dC, dD, dA)
    for nm in GRAD_NAMES:
        check_grad(label, nm, getattr(grads, nm), rg[nm])
    for v in range(s.V):
        if np.linalg.norm(rg["pose"][v]) > 0:
            check_grad(label, f"pose[{v}]", dpose[v], rg["pose"][v])


def test_max_views_in_one_launch(ctx):
    s = scenes.c3(n=8000, views=MAX_VIEWS, width=48, height=32)
    print(f"[max-views] V={s.V}", flush=True)
    _check_forward_backward(ctx, s, seed=31)


def test_one_view_too_many_is_rejected(ctx):
    import paper_2405_19614_amd as gs
    s = scenes.c3(n=500, views=MAX_VIEWS + 1, width=16, height=16)
    g, poses = dev_scene(s)
    with pytest.raises(gs.GSError):
        ctx.forward(g, s.cams, poses)


@pytest.mark.parametrize("wh", [(1, 1), (1, 19), (23, 1), (17, 3)])
def test_degenerate_image_shapes(ctx, wh):
    w, h = wh
    s = scenes.c1(n=400, width=w, height=h, seed=40 + w + h)
    print(f"[degenerate] {w}x{h}", flush=True)
    _check_forward_backward(ctx, s, seed=33)


def test_mapping_step_loss_per_view_at_max_views(ctx):
    """The fused loss reduction writes one (Lc, Ld, Lr, Ls) row per view for
    the largest batch; the colour and depth terms equal the oracle's."""
    import paper_2405_19614_amd as gs
    s = scenes.c3(n=8000, views=MAX_VIEWS, width=48, height=32, seed=13)
    og = O.Gaussians.from_scene(s)
    tgt = O.render_views(og, s.cams, s.poses_true)
    tc, td = tgt["color"].astype(np.float32), tgt["depth"].astype(np.float32)
    g, poses = dev_scene(s)
    t = lambda a: torch.tensor(np.asarray(a, np.float32), device="cuda")
    st = gs.MappingStep(ctx, g, s.cams, poses, t(tc), t(td), gs.StepOptions(w_color=1.0, w_depth=0.1, use_graph=True))
    st()
    torch.cuda.synchronize()
    assert st.status()["flags"] == 0
    out = O.render_views(og, s.cams, s.poses)
    Lc, Ld, _, _ = O.loss_and_upstream(s.cams, out, tc, td, 1.0, 0.1)
    loss = st.loss.cpu().numpy().astype(np.float64)
    assert loss.shape == (1 + 4 * s.V,)
    np.testing.assert_allclose(loss[1::4], Lc, rtol=1e-4, atol=1e-7)
    np.testing.assert_allclose(loss[2::4], Ld, rtol=1e-4, atol=1e-7)
    assert abs(loss[0] - float(np.mean(Lc + 0.1 * Ld))) <= 1e-5 * float(np.mean(Lc + 0.1 * Ld)) + 1e-9


def test_binning_multi_tile_sort_ranges(ctx):
    """More keys than 512 sort blocks x 2048 keys: each radix block then walks
    several tiles of its contiguous range, in both the depth sort (2.4M
    visible records) and the bin sort (about 5M pairs); the result must still
    equal the oracle's (tile, depth, record) order bit for bit, ties included."""
    sizes = [(1200, 680), (1200, 680)]
    n = 1_500_000
    rect, depth = scenes.synthetic_binning_records(sizes, n, seed=77, max_ext=8)
    vals_ref, ranges_ref = O.binning(sizes, n, 16, 16, rect, depth)
    visible = int(np.count_nonzero((rect[:, 0] & 0xFFFF) <= (rect[:, 0] >> 16)))
    print(f"[binning-large] visible={visible} pairs={vals_ref.size}", flush=True)
    assert visible > 2 * 512 * 2048 and vals_ref.size > 2 * 512 * 2048
    cams = [scenes.Camera(w, h, 600.0, 600.0, w / 2, h / 2) for w, h in sizes]
    rt = torch.tensor(rect.view(np.int32), device="cuda")
    dt = torch.tensor(depth, device="cuda")
    vals, ranges = ctx.bin_records(cams, n, (16, 16), rt, dt, capacity=int(vals_ref.size) + 7)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(vals.cpu().numpy(), vals_ref.astype(np.int64))
    np.testing.assert_array_equal(ranges.cpu().numpy(), ranges_ref.astype(np.int64))


@pytest.mark.parametrize("use_graph", [False, True])
def test_mapping_step_accumulates_gradients(ctx, use_graph):
    """With accumulate_grads the step adds its Gaussian gradient to what the
    buffers hold (for Gaussians no view sees too, which keep their content);
    without it the buffers are overwritten whatever they held."""
    import paper_2405_19614_amd as gs
    s = scenes.c3(n=20000, views=4, width=96, height=64, seed=17)
    og = O.Gaussians.from_scene(s)
    tgt = O.render_views(og, s.cams, s.poses_true)
    g, poses = dev_scene(s)
    t = lambda a: torch.tensor(np.asarray(a, np.float32), device="cuda")
    tc, td = t(tgt["color"]), t(tgt["depth"])
    opts = dict(w_color=1.0, w_depth=0.1, use_graph=use_graph)
    st = gs.MappingStep(ctx, g, s.cams, poses, tc, td, gs.StepOptions(**opts))
    for nm in GRAD_NAMES:
        getattr(st.grads, nm).fill_(7.0)
    st()
    torch.cuda.synchronize()
    base = {nm: getattr(st.grads, nm).clone() for nm in GRAD_NAMES}
    assert all(bool(torch.all(base[nm] != 7.0)) for nm in GRAD_NAMES)   # overwritten everywhere
    gen = torch.Generator().manual_seed(5)
    pre = {nm: torch.randn(base[nm].shape, generator=gen).to("cuda") for nm in GRAD_NAMES}
    for nm in GRAD_NAMES:
        getattr(st.grads, nm).copy_(pre[nm])
    st.set_options(gs.StepOptions(accumulate_grads=True, **opts))
    for rep in range(2):
        st()
        torch.cuda.synchronize()
        for nm in GRAD_NAMES:
            want = pre[nm] + (rep + 1) * base[nm]
            got = getattr(st.grads, nm)
            assert torch.allclose(got, want, rtol=1e-4, atol=1e-6 * float(base[nm].abs().max()) + 1e-12), (nm, rep)
    visible = torch.zeros(s.n, dtype=torch.bool)
    for nm in GRAD_NAMES:
        visible |= (base[nm].reshape(s.n, -1) != 0).any(dim=1).cpu()
    print(f"[accumulate] graph={use_graph} Gaussians with a gradient: {int(visible.sum())} of {s.n}", flush=True)
    assert 0 < int(visible.sum()) < s.n


def test_misaligned_state_is_rejected(ctx):
    """The record lines need a 256-byte aligned state buffer: a state pointer
    16 bytes past an aligned one is refused on the host (GS_EINVAL) before any
    launch; the aligned one works."""
    import ctypes
    from paper_2405_19614_amd import _abi as A
    from paper_2405_19614_amd.binding import _p, _stream, cam_array
    s = scenes.c1(n=300, width=32, height=24, seed=3)
    g, poses = dev_scene(s)
    cap = 1 << 14
    nbytes = ctx.state_bytes(s.cams, s.n, cap)
    buf = torch.empty(nbytes + 512, dtype=torch.uint8, device="cuda")
    assert buf.data_ptr() % 256 == 0
    npix = s.npix
    color = torch.empty(3 * npix, device="cuda")
    depth = torch.empty(npix, device="cuda")
    alpha = torch.empty(npix, device="cuda")
    gst = g.struct()
    for off, want in [(16, A.GS_EINVAL), (256, A.GS_OK)]:
        plan = A.gs_plan(0, 0, 0, 0, cap, 0, 0)
        rc = ctx.lib.gs_render_forward(ctx.h, ctypes.byref(gst), cam_array(s.cams), _p(poses), s.V, _p(color),
                                       _p(depth), _p(alpha), ctypes.c_void_p(buf.data_ptr() + off), nbytes,
                                       ctypes.byref(plan), _stream())
        torch.cuda.synchronize()
        print(f"[alignment] offset {off}: rc {rc}", flush=True)
        assert rc == want, (off, rc, ctx.lib.gs_last_error(ctx.h))


def test_misaligned_sh_colours_are_rejected(ctx):
    """With SH degree 1 or 3 a Gaussian's coefficients are a multiple of four
    floats and the kernels read and write them in 16-byte accesses: colour
    parameters or colour gradients 4 bytes past an aligned address are refused
    on the host (GS_EINVAL) before any launch, the aligned ones work."""
    import ctypes
    import paper_2405_19614_amd as gs
    from paper_2405_19614_amd import _abi as A
    from paper_2405_19614_amd.binding import _p, _stream, cam_array
    s = scenes.c5(n=500, views=1, width=32, height=24, seed=4)
    assert s.sh_degree == 3
    g, poses = dev_scene(s)
    _, _, _, state, plan = ctx.forward(g, s.cams, poses)
    torch.cuda.synchronize()
    # the same coefficients, 4 bytes past an aligned address
    m = g.colors.numel()
    buf = torch.zeros(m + 4, device="cuda")
    shifted = buf[1:1 + m].view_as(g.colors)
    shifted.copy_(g.colors)
    assert shifted.data_ptr() % 16 == 4
    bad = gs.Gaussians(g.means, g.log_scales, g.quats, g.opacity_logits, shifted, g.sh_degree)
    with pytest.raises(gs.GSError, match="colors must be 16-byte aligned"):
        ctx.forward(bad, s.cams, poses)
    npix = s.npix
    dC, dD, dA = (torch.ones(k * npix, device="cuda") for k in (3, 1, 1))
    grads = g.zeros_like()
    dpose = torch.zeros(s.V, 6, device="cuda")
    gst = g.struct()
    for colors, want in [(shifted, A.GS_EINVAL), (grads.colors, A.GS_OK)]:
        gg = A.gs_gaussian_grads(_p(grads.means), _p(grads.log_scales), _p(grads.quats), _p(grads.opacity_logits),
                                 _p(colors))
        rc = ctx.lib.gs_render_backward(ctx.h, ctypes.byref(gst), cam_array(s.cams), _p(poses), s.V, _p(state),
                                        state.numel(), ctypes.byref(plan), _p(dC), _p(dD), _p(dA),
                                        ctypes.byref(gg), _p(dpose), _stream())
        torch.cuda.synchronize()
        print(f"[colour alignment] gradient colours at {colors.data_ptr() % 16} mod 16: rc {rc}", flush=True)
        assert rc == want, ctx.lib.gs_last_error(ctx.h)
