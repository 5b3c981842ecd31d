"""HIP path vs FP64 oracle, through the C ABI (element by element)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from synth import scenes
from tests.gpu_helpers import (GRAD_NAMES, TOL_G, check_forward, check_grad, cotangents, dev_scene, oracle_views,
                               rel)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2405_19614_amd as gs
    torch.cuda.set_device(0)
    return gs.Context(0)


def _small_scenes():
    return {
        "c1": scenes.c1(),
        "c1_ragged": scenes.c1(n=1500, width=70, height=45, seed=21),
        "c2_small": scenes.c2(n=20000, width=160, height=120),
        "c3_small": scenes.c3(n=40000, views=8, width=150, height=85),
        "c5_small": scenes.c5(n=30000, views=3, width=120, height=68),
    }


SCENES = _small_scenes()


@pytest.mark.parametrize("name", list(SCENES))
def test_forward_matches_oracle(ctx, name):
    s = SCENES[name]
    print(f"[forward] {name} n={s.n} V={s.V}", flush=True)
    g, poses = dev_scene(s)
    color, depth, alpha, state, plan = ctx.forward(g, s.cams, poses)
    torch.cuda.synchronize()
    _, ref = oracle_views(s)
    print(f"  pairs={plan.n_pairs} vis={plan.n_visible}")
    check_forward(s, color, depth, alpha, ref, f"forward {name}")


@pytest.mark.parametrize("name", ["c1", "c1_ragged", "c3_small", "c5_small"])
def test_backward_matches_oracle(ctx, name):
    s = SCENES[name]
    print(f"[backward] {name}", flush=True)
    g, poses = dev_scene(s)
    color, depth, alpha, state, plan = ctx.forward(g, s.cams, poses)
    og, ref = oracle_views(s)
    dC, dD, dA = cotangents(s, ref, seed=7)
    t = lambda a: torch.tensor(a, device="cuda")
    grads, dpose = ctx.backward(g, s.cams, poses, state, plan, t(dC), t(dD), t(dA))
    torch.cuda.synchronize()
    rg = O.backward_views(og, s.cams, s.poses, dC, dD, dA)
    for nm in GRAD_NAMES:
        check_grad(f"backward {name}", nm, getattr(grads, nm), rg[nm])
    for v in range(s.V):
        check_grad(f"backward {name}", f"pose[{v}]", dpose[v], rg["pose"][v])


LAUNCH_SHAPES = [(16, 16, 1), (16, 16, 2), (16, 16, 4), (16, 8, 1), (16, 8, 2), (8, 8, 1), (32, 8, 1),
                 (32, 8, 2), (32, 8, 4), (32, 16, 1), (32, 16, 2), (32, 16, 4), (32, 16, 8), (32, 32, 4),
                 (32, 32, 8), (32, 64, 8), (64, 32, 8), (64, 64, 8)]


def test_forward_bit_identical_across_tile_shapes(ctx):
    """Every (tile shape, pixels per thread) launch gives the same image bit for bit."""
    s = SCENES["c3_small"]
    g, poses = dev_scene(s)
    outs = []
    for tw, th, ppt in LAUNCH_SHAPES:
        print(f"[tile] {tw}x{th} ppt={ppt}", flush=True)
        ctx.set_tile(tw, th, ppt)
        c, d, a, _, _ = ctx.forward(g, s.cams, poses, tile=(tw, th))
        outs.append((c.cpu(), d.cpu(), a.cpu()))
    ctx.set_tile(16, 16, 2)
    for o in outs[1:]:
        for x, y in zip(o, outs[0]):
            assert torch.equal(x, y)


def test_forward_bit_identical_across_bin_sizes(ctx):
    """Binning granularity changes which list each tile reads, not the result."""
    s = SCENES["c3_small"]
    g, poses = dev_scene(s)
    outs = []
    for bw, bh in [(16, 16), (32, 32), (64, 64), (128, 64), (128, 128), (256, 256)]:
        print(f"[bin] {bw}x{bh}", flush=True)
        c, d, a, _, plan = ctx.forward(g, s.cams, poses, tile=(16, 16), bin=(bw, bh))
        assert (plan.bin_w, plan.bin_h) == (bw, bh)
        outs.append((c.cpu(), d.cpu(), a.cpu()))
    for o in outs[1:]:
        for x, y in zip(o, outs[0]):
            assert torch.equal(x, y)


@pytest.mark.parametrize("bin_size", [(16, 16), (128, 64)])
def test_backward_bin_sizes(ctx, bin_size):
    s = SCENES["c1_ragged"]
    g, poses = dev_scene(s)
    color, depth, alpha, state, plan = ctx.forward(g, s.cams, poses, tile=(16, 16), bin=bin_size)
    og, ref = oracle_views(s)
    dC, dD, dA = cotangents(s, ref, seed=13)
    t = lambda a: torch.tensor(a, device="cuda")
    grads, dpose = ctx.backward(g, s.cams, poses, state, plan, t(dC), t(dD), t(dA))
    rg = O.backward_views(og, s.cams, s.poses, dC, dD, dA)
    for nm in GRAD_NAMES:
        check_grad(f"backward bins {bin_size}", nm, getattr(grads, nm), rg[nm])


@pytest.mark.parametrize("shape", LAUNCH_SHAPES)
def test_backward_every_launch_shape(ctx, shape):
    tw, th, ppt = shape
    s = SCENES["c3_small"]
    print(f"[backward-shape] {tw}x{th} ppt={ppt}", flush=True)
    g, poses = dev_scene(s)
    ctx.set_tile(tw, th, ppt)
    color, depth, alpha, state, plan = ctx.forward(g, s.cams, poses, tile=(tw, th))
    og, ref = oracle_views(s)
    dC, dD, dA = cotangents(s, ref, seed=11)
    t = lambda a: torch.tensor(a, device="cuda")
    grads, dpose = ctx.backward(g, s.cams, poses, state, plan, t(dC), t(dD), t(dA))
    torch.cuda.synchronize()
    ctx.set_tile(16, 16, 2)
    rg = O.backward_views(og, s.cams, s.poses, dC, dD, dA)
    for nm in GRAD_NAMES:
        check_grad(f"backward shape {tw}x{th}x{ppt}", nm, getattr(grads, nm), rg[nm])
    for v in range(s.V):
        check_grad(f"backward shape {tw}x{th}x{ppt}", f"pose[{v}]", dpose[v], rg["pose"][v])


def test_batched_equals_per_view(ctx):
    s = SCENES["c3_small"]
    g, poses = dev_scene(s)
    c, d, a, st, plan = ctx.forward(g, s.cams, poses)
    off = s.pix_offsets()
    og, ref = oracle_views(s)
    dC, dD, dA = cotangents(s, ref, seed=3)
    t = lambda x: torch.tensor(x, device="cuda")
    gb, pb = ctx.backward(g, s.cams, poses, st, plan, t(dC), t(dD), t(dA))
    acc = {nm: torch.zeros_like(getattr(gb, nm)) for nm in GRAD_NAMES}
    for v in range(s.V):
        print(f"[per-view] {v}", flush=True)
        cv, dv, av, stv, pv = ctx.forward(g, [s.cams[v]], poses[v:v + 1])
        P = s.cams[v].npix
        assert torch.equal(cv.cpu(), c[3 * off[v]:3 * off[v + 1]].cpu())
        assert torch.equal(dv.cpu(), d[off[v]:off[v + 1]].cpu())
        assert torch.equal(av.cpu(), a[off[v]:off[v + 1]].cpu())
        gv, pvv = ctx.backward(g, [s.cams[v]], poses[v:v + 1], stv, pv, t(dC[3 * off[v]:3 * off[v + 1]]),
                               t(dD[off[v]:off[v + 1]]), t(dA[off[v]:off[v + 1]]))
        for nm in GRAD_NAMES:
            acc[nm] += getattr(gv, nm)
        assert rel(pvv[0].cpu().numpy(), pb[v].cpu().numpy()) < 1e-4
    for nm in GRAD_NAMES:
        assert rel(acc[nm].cpu().numpy(), getattr(gb, nm).cpu().numpy()) < 1e-4, nm


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_binning_stage_bit_exact(ctx, tile):
    sizes = [(70, 45), (33, 17), (64, 48), (1, 1)]
    n = 3000
    rect, depth = scenes.synthetic_binning_records(sizes, n, seed=tile[0] * 31 + tile[1])
    vals_ref, ranges_ref = O.binning(sizes, n, tile[0], tile[1], rect, depth)
    cams = [scenes.Camera(w, h, 50.0, 50.0, w / 2, h / 2) for w, h in sizes]
    print(f"[binning] tile={tile} pairs={vals_ref.size}", flush=True)
    rt = torch.tensor(rect.view(np.int32), device="cuda")
    dt = torch.tensor(depth, device="cuda")
    vals, ranges = ctx.bin_records(cams, n, tile, rt, dt, capacity=int(vals_ref.size) + 7)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(vals.cpu().numpy(), vals_ref.astype(np.int64))
    np.testing.assert_array_equal(ranges.cpu().numpy(), ranges_ref.astype(np.int64))


def test_binning_capacity_error_then_retry(ctx):
    import paper_2405_19614_amd as gs
    sizes = [(70, 45)]
    n = 500
    rect, depth = scenes.synthetic_binning_records(sizes, n, seed=5)
    vals_ref, ranges_ref = O.binning(sizes, n, 16, 16, rect, depth)
    cams = [scenes.Camera(70, 45, 50.0, 50.0, 35, 22.5)]
    rt = torch.tensor(rect.view(np.int32), device="cuda")
    dt = torch.tensor(depth, device="cuda")
    with pytest.raises(gs.GSError) as ei:
        ctx.bin_records(cams, n, (16, 16), rt, dt, capacity=int(vals_ref.size) - 1)
    assert ei.value.code == gs._abi.GS_ECAPACITY
    vals, ranges = ctx.bin_records(cams, n, (16, 16), rt, dt, capacity=int(vals_ref.size))
    np.testing.assert_array_equal(vals.cpu().numpy(), vals_ref.astype(np.int64))


def test_reproj_matches_oracle(ctx):
    s = scenes.c4(n=20000, views=5, res_scale=0.25, vis_range=(500, 20000), matches=(100, 300), seed=9)
    print(f"[reproj] V={s.V} M={s.points.shape[0]}", flush=True)
    _, poses = dev_scene(s)
    t = lambda a: torch.tensor(a, device="cuda")
    res, loss, dpose = ctx.reproj(s.cams, poses, t(s.points), t(s.uv), t(s.view_idx), 2.0, weight=0.5)
    torch.cuda.synchronize()
    r = O.reproj(s.cams, s.poses, s.points, s.uv, s.view_idx, 2.0)
    np.testing.assert_allclose(res.cpu().numpy(), r["residual"], atol=2e-3)
    np.testing.assert_allclose(loss.cpu().numpy(), r["loss"], rtol=1e-4)
    for v in range(s.V):
        assert rel(dpose[v].cpu().numpy(), 0.5 * r["dpose"][v]) < 1e-3
    # the point side of the bundle adjustment (Sec. 3.2 Eq. for:ba)
    _, _, _, dpts = ctx.reproj(s.cams, poses, t(s.points), t(s.uv), t(s.view_idx), 2.0, weight=0.5,
                               point_grads=True)
    torch.cuda.synchronize()
    g_ref = O.reproj_point_grads(s.cams, s.poses, s.points, s.uv, s.view_idx, 2.0, weight=0.5)
    e = rel(dpts.cpu().numpy(), g_ref)
    print(f"  point gradients rel {e:.2e}", flush=True)
    assert e < 1e-3
    assert np.all(dpts.cpu().numpy()[np.all(g_ref == 0, axis=1)] == 0)


def test_empty_and_culled_scenes(ctx):
    import paper_2405_19614_amd as gs
    s = scenes.c1(n=100, seed=3)
    s.means[:, 2] = -1.0     # every Gaussian behind the camera
    g, poses = dev_scene(s)
    c, d, a, st, plan = ctx.forward(g, s.cams, poses)
    assert plan.n_pairs == 0 and plan.n_visible == 0
    assert float(c.abs().max()) == 0 and float(a.abs().max()) == 0
    t = lambda x: torch.ones(x, device="cuda")
    gr, dp = ctx.backward(g, s.cams, poses, st, plan, t(3 * s.npix), t(s.npix), t(s.npix))
    for nm in GRAD_NAMES:
        assert float(getattr(gr, nm).abs().max()) == 0
    assert float(dp.abs().max()) == 0
    # n = 0
    s0 = scenes.c1(n=1, seed=3)
    g0 = gs.Gaussians.from_arrays(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 4)), np.zeros(0),
                                  np.zeros((0, 3)), -1)
    c, d, a, st, plan = ctx.forward(g0, s0.cams, poses)
    assert plan.n_pairs == 0 and float(c.abs().max()) == 0


@pytest.mark.parametrize("fwd,bwd", [((16, 16, 4), (32, 32, 8)), ((32, 32, 4), (8, 8, 1)), ((32, 8, 2), (32, 16, 4)),
                                     ((16, 16, 4), (64, 32, 8))])
def test_backward_with_its_own_tile_shape(ctx, fwd, bwd):
    """The backward on a different tiling than the forward (ordered by the
    forward's per-tile work) gives the oracle's gradients."""
    s = SCENES["c3_small"]
    print(f"[split-shape] forward {fwd} backward {bwd}", flush=True)
    g, poses = dev_scene(s)
    ctx.set_tile(fwd[0], fwd[1], fwd[2])
    ctx.set_bwd_shape(*bwd)
    color, depth, alpha, state, plan = ctx.forward(g, s.cams, poses, tile=fwd[:2])
    assert (plan.bwd_tile_w, plan.bwd_tile_h) == bwd[:2]
    og, ref = oracle_views(s)
    dC, dD, dA = cotangents(s, ref, seed=17)
    t = lambda a: torch.tensor(a, device="cuda")
    grads, dpose = ctx.backward(g, s.cams, poses, state, plan, t(dC), t(dD), t(dA))
    torch.cuda.synchronize()
    ctx.set_bwd_shape(0, 0, 0)
    ctx.set_tile(16, 16, 2)
    rg = O.backward_views(og, s.cams, s.poses, dC, dD, dA)
    for nm in GRAD_NAMES:
        check_grad(f"backward split {fwd}/{bwd}", nm, getattr(grads, nm), rg[nm])
    for v in range(s.V):
        check_grad(f"backward split {fwd}/{bwd}", f"pose[{v}]", dpose[v], rg["pose"][v])

