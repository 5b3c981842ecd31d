"""Every SH degree through the forward projection's colour paths, against
the FP64 oracle (forward images and every gradient).

The projection copies the coefficient rows of up to 80 Gaussians per block
and round into LDS and reads the others from the parameter array: the dense
scenes (almost every Gaussian of a block visible in every view) take both
paths in one launch, the sparse ones mostly the staged one.  Degrees 1 and 3
move coefficients in 16-byte accesses, degree 2 (27 floats) one at a time.
"""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import oracle as O
from synth import scenes
from tests.gpu_helpers import GRAD_NAMES, check_forward, check_grad, cotangents, dev_scene, oracle_views

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2405_19614_amd as gs
    torch.cuda.set_device(0)
    return gs.Context(0)


def _sh_scene(deg, dense, seed):
    if dense:
        # the unit box in front of one camera, seen from three nearby poses
        base = scenes.c1(n=3000, width=96, height=72, seed=seed)
        rng = np.random.default_rng(seed)
        T0 = base.poses[0].astype(np.float64)
        poses = np.stack([T0] + [scenes.perturb_pose(T0, rng, 0.05, 0.05) for _ in range(2)]).astype(np.float32)
        cams = [base.cams[0]] * 3
    else:
        base = scenes.c5(n=20000, views=3, width=120, height=68, seed=seed)
        poses, cams = base.poses, base.cams
    K = (deg + 1) ** 2
    rng = np.random.default_rng(seed + 1)
    col = rng.normal(0.0, 0.1, (base.n, K, 3)).astype(np.float32)
    col[:, 0, :] = rng.uniform(0.0, 1.0, (base.n, 3))
    return dataclasses.replace(base, colors=col, sh_degree=deg, cams=cams, poses=poses, poses_true=poses.copy(),
                               target_color=None, target_depth=None)


@pytest.mark.parametrize("dense", [True, False], ids=["dense", "sparse"])
@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_sh_degree_matches_oracle(ctx, deg, dense):
    s = _sh_scene(deg, dense, seed=60 + deg)
    g, poses = dev_scene(s)
    color, depth, alpha, state, plan = ctx.forward(g, s.cams, poses)
    frac = plan.n_visible / (s.n * s.V)
    print(f"[sh degree {deg} {'dense' if dense else 'sparse'}] n={s.n} V={s.V} visible {frac:.2f} of the records, "
          f"pairs {plan.n_pairs}", flush=True)
    if dense:
        assert frac > 0.5   # more than 80 visible Gaussians in a full block: both colour paths run
    og, ref = oracle_views(s)
    label = f"sh{deg} {'dense' if dense else 'sparse'}"
    check_forward(s, color, depth, alpha, ref, label)
    dC, dD, dA = cotangents(s, ref, seed=70 + deg)
    t = lambda a: torch.tensor(a, device="cuda")
    grads, dpose = ctx.backward(g, s.cams, poses, state, plan, t(dC), t(dD), t(dA))
    torch.cuda.synchronize()
    rg = O.backward_views(og, s.cams, s.poses, dC, dD, dA)
    for nm in GRAD_NAMES:
        check_grad(label, nm, getattr(grads, nm), rg[nm])
    for v in range(s.V):
        if np.linalg.norm(rg["pose"][v]) > 0:
            check_grad(label, f"pose[{v}]", dpose[v], rg["pose"][v])
