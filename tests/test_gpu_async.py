"""The forward pass without host synchronisation (gs_render_forward_async).

* It runs the same kernels as the synchronous forward: identical images, and
  the state's status block holds the pair and visible counts.
* A too small pair capacity is flagged in the state (the render is then
  empty and the backward gives zero gradients); so is a non-finite parameter.
* It can be captured into a graph: every replay, with eager work between the
  replays, equals an eager synchronous forward of the current parameters.
* The autograd path with sync=False gives the synchronous path's image bit
  for bit and its gradients up to the order of the backward's atomic sums.
"""
import numpy as np
import pytest
import torch

from synth import scenes
from tests.gpu_helpers import dev_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2405_19614_amd as gs
    torch.cuda.set_device(0)
    return gs.Context(0)


def _scene():
    return scenes.c3(n=40000, views=4, width=150, height=85, seed=51)


def test_async_forward_equals_sync(ctx):
    s = _scene()
    print(f"[async forward] n={s.n} V={s.V}", flush=True)
    g, poses = dev_scene(s)
    c1, d1, a1, _, plan = ctx.forward(g, s.cams, poses)
    c2, d2, a2, state, plan2 = ctx.forward(g, s.cams, poses, capacity=plan.n_pairs + 10, sync=False)
    assert plan2.n_pairs == -1 and plan2.n_visible == -1
    st = ctx.state_status(state)
    print(f"  sync pairs {plan.n_pairs}, async status {st}", flush=True)
    assert st == {"flags": 0, "n_pairs": plan.n_pairs, "n_visible": plan.n_visible}
    for x, y in ((c1, c2), (d1, d2), (a1, a2)):
        assert torch.equal(x, y)


def test_async_overflow_is_flagged_and_renders_nothing(ctx):
    s = _scene()
    g, poses = dev_scene(s)
    _, _, _, _, plan = ctx.forward(g, s.cams, poses)
    c, d, a, state, plan2 = ctx.forward(g, s.cams, poses, capacity=plan.n_pairs // 2, sync=False)
    st = ctx.state_status(state)
    print(f"[async overflow] needed {plan.n_pairs}, capacity {plan.n_pairs // 2}: {st}", flush=True)
    assert st["flags"] & 1 and st["n_pairs"] == plan.n_pairs
    assert float(c.abs().max()) == 0.0 and float(d.abs().max()) == 0.0 and float(a.abs().max()) == 0.0
    grads, dpose = ctx.backward(g, s.cams, poses, state, plan2, torch.ones_like(c), torch.ones_like(d),
                                torch.ones_like(a))
    torch.cuda.synchronize()
    for t in grads.tensors():
        assert float(t.abs().max()) == 0.0
    assert float(dpose.abs().max()) == 0.0


def test_async_nonfinite_is_flagged(ctx):
    s = _scene()
    g, poses = dev_scene(s)
    g.means[5, 1] = float("nan")
    _, _, _, state, _ = ctx.forward(g, s.cams, poses, capacity=1 << 20, sync=False)
    st = ctx.state_status(state)
    print(f"[async non-finite] {st}", flush=True)
    assert st["flags"] & 4


def test_async_forward_graph_replays(ctx):
    """Capture the asynchronous forward in a graph; between replays the means
    move (eagerly, in place) and each replay must equal a synchronous forward
    of the moved means."""
    s = _scene()
    g, poses = dev_scene(s)
    _, _, _, _, plan = ctx.forward(g, s.cams, poses)
    cap = plan.n_pairs * 2
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ctx.forward(g, s.cams, poses, capacity=cap, sync=False)   # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        outs = ctx.forward(g, s.cams, poses, capacity=cap, sync=False)
    rng = np.random.default_rng(52)
    for k in range(3):
        with torch.no_grad():
            g.means.add_(torch.tensor(rng.normal(0, 0.01, (s.n, 3)).astype(np.float32), device="cuda"))
        graph.replay()
        ref = ctx.forward(g, s.cams, poses)
        torch.cuda.synchronize()
        st = ctx.state_status(outs[3])
        print(f"[graph replay {k}] status {st}, eager pairs {ref[4].n_pairs}", flush=True)
        assert st["flags"] == 0 and st["n_pairs"] == ref[4].n_pairs
        for x, y in zip(outs[:3], ref[:3]):
            assert torch.equal(x, y)


def test_async_autograd_matches_sync(ctx):
    import paper_2405_19614_amd as gs
    s = _scene()
    rng = np.random.default_rng(53)
    t = lambda a: torch.tensor(np.asarray(a, np.float32), device="cuda", requires_grad=True)
    poses = torch.tensor(np.asarray(s.poses, np.float32), device="cuda").reshape(s.V, 16)
    res = []
    for sync in (True, False):
        g = gs.Gaussians(t(s.means), t(s.log_scales), t(s.quats), t(s.opacity_logits), t(s.colors), s.sh_degree)
        xi = torch.zeros(s.V, 6, device="cuda", requires_grad=True)
        C, D, A = gs.render(g, s.cams, poses, pose_tangent=xi, ctx=ctx, sync=sync)
        w = torch.tensor(rng.standard_normal(C.numel()).astype(np.float32), device="cuda") if not res else res[0][0]
        (C * w).sum().add(D.sum() * 0.1).add(A.sum()).backward()
        if not sync:
            assert ctx.check_async()["flags"] == 0
        res.append((w, C.detach(), [x.grad.clone() for x in g.tensors()], xi.grad.clone()))
    assert torch.equal(res[0][1], res[1][1])   # the forward is bit for bit the same
    # the backward's atomic sums may add in another order: the parity
    # protocol's gradient criterion, with a far smaller bound on the L2 error
    for a, b in list(zip(res[0][2], res[1][2])) + [(res[0][3], res[1][3])]:
        a, b = a.double().reshape(-1), b.double().reshape(-1)
        rel = float((a - b).norm() / b.norm())
        rms = float(b.pow(2).mean().sqrt())
        viol = float(((a - b).abs() > 1e-3 * (b.abs() + rms)).double().mean())
        print(f"  sync vs async gradient: rel {rel:.2e}, violations {viol:.2e}", flush=True)
        assert rel < 1e-5 and viol <= 1e-3
