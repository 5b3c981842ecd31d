"""Pruning and densification (Sec. 3.4) on the GPU against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from synth import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2405_19614_amd as gs
    torch.cuda.set_device(0)
    return gs.Context(0)


def _params(n, seed, sh=-1):
    rng = np.random.default_rng(seed)
    K = 1 if sh < 0 else (sh + 1) ** 2
    return {"means": rng.standard_normal((n, 3)).astype(np.float32),
            "log_scales": (rng.standard_normal((n, 3)) - 3).astype(np.float32),
            "quats": rng.standard_normal((n, 4)).astype(np.float32),
            "opacity_logits": (rng.standard_normal(n) * 3).astype(np.float32),
            "colors": (rng.random((n, 3)) if sh < 0 else rng.standard_normal((n, K, 3))).astype(np.float32)}


def _dev(p, sh):
    import paper_2405_19614_amd as gs
    return gs.Gaussians.from_arrays(p["means"], p["log_scales"], p["quats"], p["opacity_logits"], p["colors"], sh)


@pytest.mark.parametrize("sh", [-1, 3])
def test_prune_matches_oracle_bit_exact(ctx, sh):
    n, V = 100_000, 3
    print(f"[prune] n={n} sh={sh}", flush=True)
    p = _params(n, 1, sh)
    K = 1 if sh < 0 else (sh + 1) ** 2
    rng = np.random.default_rng(2)
    m = rng.standard_normal(n * (11 + 3 * K) + 6 * V).astype(np.float32)
    v = rng.random(m.shape).astype(np.float32)
    t = lambda a: torch.tensor(a, device="cuda")
    step = torch.tensor([7, 2], dtype=torch.int32, device="cuda")
    out, (m2, v2, _) = ctx.prune(_dev(p, sh), 0.3, adam=(t(m), t(v), step), V=V)
    kept, idx = O.prune(p, 0.3)
    assert out.n == len(idx)
    for k, name in [("means", "means"), ("log_scales", "log_scales"), ("quats", "quats"),
                    ("opacity_logits", "opacity_logits"), ("colors", "colors")]:
        np.testing.assert_array_equal(getattr(out, name).cpu().numpy().reshape(kept[k].shape), kept[k])
    np.testing.assert_array_equal(m2.cpu().numpy(), O.adam_relayout(m, n, sh, V, idx, len(idx)).astype(np.float32))
    np.testing.assert_array_equal(v2.cpu().numpy(), O.adam_relayout(v, n, sh, V, idx, len(idx)).astype(np.float32))


def test_prune_limits(ctx):
    p = _params(1000, 3)
    g = _dev(p, -1)
    assert ctx.prune(g, 0.0)[0].n == 1000
    assert ctx.prune(g, 1.5)[0].n == 0
    empty = _dev(_params(0, 4), -1)
    assert ctx.prune(empty, 0.5)[0].n == 0


def _rgbd(sizes, seed):
    rng = np.random.default_rng(seed)
    P = sum(w * h for w, h in sizes)
    depth = rng.uniform(0.5, 4.0, P).astype(np.float32)
    depth[rng.random(P) < 0.1] = 0.0
    return rng.random(3 * P).astype(np.float32), depth, rng.random(P).astype(np.float32)


SIZES = [(33, 17), (1, 1), (64, 48)]


@pytest.mark.parametrize("sh,all_px", [(-1, False), (-1, True), (2, False)])
def test_densify_matches_oracle(ctx, sh, all_px):
    import paper_2405_19614_amd as gs
    cams = [gs.Camera(w, h, 50.0 + w, 45.0 + h, w / 2 - 0.3, h / 2 + 0.2) for w, h in SIZES]
    poses = [O.se3_exp([0.1 * v, -0.2, 0.05, 0.1, 0.02 * v, -0.2]) for v in range(len(SIZES))]
    col, dep, alpha = _rgbd(SIZES, 5)
    p = _params(500, 6, sh)
    t = lambda a: torch.tensor(np.asarray(a, np.float32), device="cuda")
    P = torch.stack([t(T.reshape(-1)) for T in poses])
    new, where = O.densify(cams, [T.astype(np.float32).astype(np.float64) for T in poses], alpha, col, dep, 0.5,
                           all_px, sh_degree=sh)
    K = 1 if sh < 0 else (sh + 1) ** 2
    rng = np.random.default_rng(7)
    m = rng.standard_normal(500 * (11 + 3 * K) + 6 * 3).astype(np.float32)
    step = torch.tensor([3, 1], dtype=torch.int32, device="cuda")
    cap = 500 + len(where) + 10
    out, (held, asked), (m2, _, _) = ctx.densify(_dev(p, sh), cap, cams, P, t(alpha), t(col), t(dep), gamma=0.5,
                                                 all_pixels=all_px, adam=(t(m), t(m), step))
    print(f"  new {len(where)} held {held} asked {asked}", flush=True)
    assert held == asked == 500 + len(where)
    # existing Gaussians untouched, new ones as the oracle's
    np.testing.assert_array_equal(out.means[:500].cpu().numpy(), p["means"])
    gm = out.means[500:].cpu().numpy().astype(np.float64)
    assert np.abs(gm - new["means"]).max() <= 1e-5 * (1.0 + np.abs(new["means"]).max())
    assert np.abs(out.log_scales[500:].cpu().numpy() - new["log_scales"]).max() < 1e-5
    np.testing.assert_array_equal(out.quats[500:].cpu().numpy(), new["quats"])
    np.testing.assert_array_equal(out.opacity_logits[500:].cpu().numpy(), new["opacity_logits"])
    np.testing.assert_allclose(out.colors[500:].cpu().numpy().reshape(new["colors"].shape), new["colors"],
                               rtol=1e-6, atol=1e-6)
    src = np.concatenate([np.arange(500), -np.ones(len(where), np.int64)])
    np.testing.assert_array_equal(m2.cpu().numpy(), O.adam_relayout(m, 500, sh, 3, src, held).astype(np.float32))


def test_densify_capacity_limit(ctx):
    import paper_2405_19614_amd as gs
    cams = [gs.Camera(w, h, 60.0, 60.0, w / 2, h / 2) for w, h in SIZES]
    poses = torch.eye(4, device="cuda").reshape(1, 16).repeat(3, 1).contiguous()
    col, dep, alpha = _rgbd(SIZES, 8)
    t = lambda a: torch.tensor(a, device="cuda")
    new, where = O.densify(cams, [np.eye(4)] * 3, alpha, col, dep, 0.99, True)
    cap = 20 + len(where) // 2
    out, (held, asked), _ = ctx.densify(_dev(_params(20, 9), -1), cap, cams, poses, t(alpha), t(col), t(dep),
                                        all_pixels=True)
    assert held == cap and asked == 20 + len(where)
    gm = out.means[20:].cpu().numpy().astype(np.float64)
    assert np.abs(gm - new["means"][:cap - 20]).max() <= 1e-5 * (1.0 + np.abs(new["means"]).max())


def test_first_frame_densify_then_mapping(ctx):
    """A map grown from one RGB-D frame (every pixel) and refined with the
    paper's mapping loss: the loss falls; pruning then keeps a consistent map."""
    import paper_2405_19614_amd as gs
    s = scenes.c3(n=40000, views=2, width=120, height=68)
    og = O.Gaussians.from_scene(s)
    ref = O.render_views(og, s.cams, s.poses_true)
    tc = torch.tensor(ref["color"].astype(np.float32), device="cuda")
    td = torch.tensor(ref["depth"].astype(np.float32), device="cuda")
    poses = torch.tensor(np.asarray(s.poses_true, np.float32), device="cuda").reshape(s.V, 16).contiguous()
    empty = gs.Gaussians(torch.empty(0, 3, device="cuda"), torch.empty(0, 3, device="cuda"),
                         torch.empty(0, 4, device="cuda"), torch.empty(0, device="cuda"),
                         torch.empty(0, 3, device="cuda"), -1)
    alpha = torch.zeros(s.npix, device="cuda")
    g, (held, asked), _ = ctx.densify(empty, s.npix, s.cams[:1], poses[:1], alpha[:s.cams[0].npix],
                                      tc[:3 * s.cams[0].npix], td[:s.cams[0].npix], all_pixels=True)
    assert held == asked == int((ref["depth"][:s.cams[0].npix] > 0).sum())
    g = gs.Gaussians(*(x.contiguous() for x in g.tensors()), -1)
    opts = dict(gs.PAPER_MAPPING)
    opts.update(use_graph=True, lr_means=1e-4, lr_colors=5e-3)
    st = gs.MappingStep(ctx, g, s.cams[:1], poses[:1].clone(), tc[:3 * s.cams[0].npix], td[:s.cams[0].npix],
                        gs.StepOptions(**opts))
    st()
    torch.cuda.synchronize()
    l0 = float(st.loss[0].item())
    for _ in range(30):
        st()
    torch.cuda.synchronize()
    l1 = float(st.loss[0].item())
    print(f"  first-frame map: {held} Gaussians, loss {l0:.5f} -> {l1:.5f}", flush=True)
    assert st.status()["flags"] == 0
    assert l1 < 0.8 * l0
    pruned, _ = ctx.prune(st.g, 0.005)
    o = torch.sigmoid(st.g.opacity_logits).cpu().numpy()
    assert pruned.n == int((~(o < 0.005)).sum())


@pytest.mark.parametrize("tau", [0.005, 0.3, 0.7, 0.99, 1e-7])
def test_prune_threshold_exact_at_the_boundary(ctx, tau):
    """FP32 logits on both sides of logit(tau) (the floats next to it, and a
    few ulps further): the GPU keeps exactly the Gaussians whose FP64 opacity
    is >= tau (the paper's tau = 0.005 among the thresholds)."""
    lt = np.log(tau) - np.log1p(-tau)
    f = np.float32(lt)
    cand = [f]
    up, dn = f, f
    for _ in range(3):
        up = np.nextafter(up, np.float32(np.inf))
        dn = np.nextafter(dn, np.float32(-np.inf))
        cand += [up, dn]
    logits = np.array(cand, np.float32)
    n = len(logits)
    p = _params(n, 9)
    p["opacity_logits"] = logits
    out, _ = ctx.prune(_dev(p, -1), tau)
    kept, idx = O.prune(p, tau)
    print(f"[prune boundary tau={tau}] logit(tau)={lt:.9g} kept {len(idx)}/{n}", flush=True)
    assert 0 < len(idx) < n
    np.testing.assert_array_equal(out.opacity_logits.cpu().numpy(), logits[idx])


@pytest.mark.parametrize("gamma", [0.99, 0.5, 0.3])
def test_densify_threshold_exact_at_the_boundary(ctx, gamma):
    """Rendered alphas at float(gamma) and the floats next to it: a pixel is
    densified exactly when its FP32 alpha is <= gamma in FP64."""
    import paper_2405_19614_amd as gs
    f = np.float32(gamma)
    vals = [f]
    up, dn = f, f
    for _ in range(3):
        up = np.nextafter(up, np.float32(np.inf))
        dn = np.nextafter(dn, np.float32(-np.inf))
        vals += [up, dn]
    W = len(vals)
    cams = [gs.Camera(W, 1, 50.0, 50.0, W / 2, 0.5)]
    alpha = np.array(vals, np.float32)
    col = np.full(3 * W, 0.5, np.float32)
    dep = np.full(W, 2.0, np.float32)
    T = np.eye(4)
    t = lambda a: torch.tensor(np.asarray(a, np.float32), device="cuda")
    p = _params(4, 10)
    new, where = O.densify(cams, [T], alpha, col, dep, gamma, False)
    out, (held, asked), _ = ctx.densify(_dev(p, -1), 4 + W, cams, t(T.reshape(1, 16)), t(alpha), t(col), t(dep),
                                        gamma=gamma)
    print(f"[densify boundary gamma={gamma}] oracle new {len(where)} gpu new {held - 4}", flush=True)
    assert 0 < len(where) < W
    assert held == asked == 4 + len(where)
    np.testing.assert_allclose(out.means[4:].cpu().numpy(), new["means"], rtol=1e-6, atol=1e-6)
