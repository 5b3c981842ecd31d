"""Failure paths of the mapping step, forced from the host.

* Too small a pair capacity: the step flags the overflow on the device,
  renders empty lists, and leaves the parameters, poses, Adam moments and
  step counters as they were; a step re-planned with a large
  enough capacity then succeeds.
* A non-finite parameter written by the host: the step flags it and skips
  its updates; the status word is sticky, so a later good step does not hide
  it, and reading the status clears it.
* The forward pass alone reports a non-finite parameter as an error.
"""
import math

import numpy as np
import pytest
import torch

from synth import scenes
from tests.gpu_helpers import dev_scene

pytestmark = pytest.mark.gpu

FLAG_CAPACITY, FLAG_NONFINITE = 1, 4


@pytest.fixture(scope="module")
def ctx():
    import paper_2405_19614_amd as gs
    torch.cuda.set_device(0)
    return gs.Context(0)


def _scene():
    return scenes.c3(n=30000, views=3, width=160, height=96, seed=31)


def _targets(ctx, s, g):
    pt = torch.tensor(np.asarray(s.poses_true, np.float32), device="cuda").reshape(s.V, 16).contiguous()
    tc, td, _, _, _ = ctx.forward(g, s.cams, pt)
    return tc, td


def _snapshot(st):
    return ([t.clone() for t in st.g.tensors()], st.poses.clone(), st.adam_m.clone(), st.adam_v.clone(),
            st.adam_step.clone())


def _same_bits(a, b):
    """Bit-identical (torch.equal is false wherever both hold a NaN)."""
    return torch.equal(a.contiguous().view(torch.int32), b.contiguous().view(torch.int32))


def _assert_unchanged(st, snap):
    for a, b in zip(st.g.tensors(), snap[0]):
        assert _same_bits(a, b)
    assert _same_bits(st.poses, snap[1])
    assert _same_bits(st.adam_m, snap[2]) and _same_bits(st.adam_v, snap[3])
    assert torch.equal(st.adam_step, snap[4])


@pytest.mark.parametrize("graph", [False, True])
def test_pair_overflow_skips_updates_and_replan_succeeds(ctx, graph):
    import paper_2405_19614_amd as gs
    s = _scene()
    print(f"[overflow] graph={graph} n={s.n} V={s.V}", flush=True)
    g, poses = dev_scene(s)
    tc, td = _targets(ctx, s, g)
    opts = gs.StepOptions(w_color=1.0, w_depth=0.1, update_gaussians=True, update_poses=True, use_graph=graph)
    cap = 256
    st = gs.MappingStep(ctx, g, s.cams, poses, tc, td, opts, capacity=cap)
    snap = _snapshot(st)
    for _ in range(3):
        st()
    torch.cuda.synchronize()
    stat = st.status()
    print(f"  status {stat}", flush=True)
    assert stat["flags"] & FLAG_CAPACITY
    assert stat["n_pairs"] > cap
    _assert_unchanged(st, snap)
    # the overflowing step composited empty lists: a finite, empty render
    assert torch.isfinite(st.loss).all() and float(st.alpha.abs().max()) == 0.0
    # a step sized from a counting pass succeeds and updates
    st2 = gs.MappingStep(ctx, g, s.cams, poses, tc, td, opts)
    st2()
    torch.cuda.synchronize()
    stat2 = st2.status()
    assert stat2["flags"] == 0 and stat2["n_pairs"] == stat["n_pairs"]
    assert st2.adam_step.tolist() == [1, 1]
    assert not torch.equal(st2.g.means, snap[0][0])


def test_nonfinite_parameter_flag_is_sticky(ctx):
    import paper_2405_19614_amd as gs
    s = _scene()
    g, poses = dev_scene(s)
    tc, td = _targets(ctx, s, g)
    opts = gs.StepOptions(w_color=1.0, w_depth=0.1, update_gaussians=True, use_graph=True)
    st = gs.MappingStep(ctx, g, s.cams, poses, tc, td, opts)
    st()
    torch.cuda.synchronize()
    assert st.status()["flags"] == 0
    assert st.adam_step.tolist() == [1, 0]
    for name, idx in [("opacity_logits", (7,)), ("means", (11, 2)), ("quats", (3, 1)), ("log_scales", (5, 0))]:
        t = getattr(st.g, name)
        old = t[idx].item()
        t[idx] = float("nan")
        snap = _snapshot(st)
        st()                      # reads the NaN: flagged, no update
        torch.cuda.synchronize()
        _assert_unchanged(st, snap)
        t[idx] = old
        st()                      # a good step: updates again, the flag stays
        torch.cuda.synchronize()
        step_before = int(snap[4][0].item())
        assert int(st.adam_step[0].item()) == step_before + 1
        stat = st.status()        # read and clear
        print(f"  [{name}] status {stat}", flush=True)
        assert stat["flags"] & FLAG_NONFINITE
        assert st.status()["flags"] == 0


def test_forward_rejects_nonfinite_parameters(ctx):
    import paper_2405_19614_amd as gs
    s = _scene()
    g, poses = dev_scene(s)
    g.opacity_logits[3] = float("inf")
    with pytest.raises(gs.GSError) as ei:
        ctx.forward(g, s.cams, poses)
    assert ei.value.code == gs._abi.GS_EINVAL
    assert "finite" in str(ei.value)


def test_joint_refinement_raises_on_overflow(ctx):
    import paper_2405_19614_amd as gs
    s = _scene()
    g, poses = dev_scene(s)
    tc, td = _targets(ctx, s, g)
    st = gs.MappingStep(ctx, g, s.cams, poses, tc, td, gs.StepOptions(w_color=1.0, w_depth=0.1), capacity=256)
    jr = gs.JointRefinement(st)
    with pytest.raises(gs.GSError) as ei:
        jr(2, 2)
    assert ei.value.code == gs._abi.GS_ECAPACITY
    assert math.isfinite(float(st.loss[0].item()))
