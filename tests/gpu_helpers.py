"""Shared helpers of the GPU parity tests (HIP path vs FP64 oracle).

Forward protocol, per view:
* pixels where a 1/255 skip or the 1e-4 stop sits within FP32 reach of its
  threshold (oracle flags AMB_UNBOUNDED) are excluded and counted; their
  share of a view's pixels (of at least 100) must stay below MAX_EXCLUDED;
* pixels whose only ambiguity is the blend order of near-tied depths
  (AMB_ORDER, AMB_ORDER_STOP) are checked against the oracle's bound on what
  reordering can change (order_bound), plus the tolerance, plus n 2^-24
  times the value for the n blended terms an FP32 sum may now add in
  another order;
* every other pixel: colour and alpha within 1e-5, depth within 1e-5
  absolute.
Gradients, per tensor: relative L2 error <= 1e-3, and the element-wise
criterion |g - r| <= 1e-3 (|r| + rms(r)) violated by at most 0.1 % of the
elements.  Every measurement is appended (JSON lines) to the file named by
the GS_PARITY_REPORT environment variable, when it is set.
"""
import json
import os

import numpy as np
import torch

from oracle import oracle as O
from synth import scenes

TOL_C = 1e-5
TOL_A = 1e-5
TOL_D = 1e-5
# gradients: relative L2 error per tensor, and the element-wise criterion
TOL_G = 1e-3
MAX_VIOLATION = 1e-3
MAX_EXCLUDED = 0.05


def dev_scene(s, device="cuda"):
    import paper_2405_19614_amd as gs
    g = gs.Gaussians.from_scene(s, device)
    poses = torch.tensor(np.asarray(s.poses, np.float32), device=device).reshape(s.V, 16).contiguous()
    return g, poses


def oracle_views(s, poses=None, bands=O.SMALL_BANDS):
    og = O.Gaussians.from_scene(s)
    poses = s.poses if poses is None else poses
    return og, O.render_views(og, s.cams, poses, bands=bands)


def report(**rec):
    path = os.environ.get("GS_PARITY_REPORT")
    if not path:
        return
    with open(path, "a") as f:
        f.write(json.dumps(rec) + "\n")


def _np(x):
    return x.detach().cpu().numpy().astype(np.float64) if torch.is_tensor(x) else np.asarray(x, np.float64)


def check_forward_view(label, c, d, a, r, view=None):
    """One view (or a pixel sample of it): c [3,P], d [P], a [P] against the
    oracle's render r (same pixels).  Asserts the protocol above and returns
    the per-output statistics."""
    c, d, a = _np(c).reshape(3, -1), _np(d).reshape(-1), _np(a).reshape(-1)
    rc, rd, ra = r["color"].reshape(3, -1), r["depth"].reshape(-1), r["alpha"].reshape(-1)
    amb = r["ambiguous"].reshape(-1)
    bnd = r["order_bound"].reshape(5, -1)
    excl = (amb & O.AMB_UNBOUNDED) != 0
    bounded = ~excl & ((amb & (O.AMB_ORDER | O.AMB_ORDER_STOP)) != 0)
    strict = ~excl & ~bounded
    n = amb.size
    ec, ed, ea = np.abs(c - rc), np.abs(d - rd), np.abs(a - ra)
    stats = {}
    for name, e, ref, tol in (("C", ec, rc, TOL_C), ("D", ed, rd, TOL_D), ("A", ea, ra, TOL_A)):
        es = e[..., strict]
        refs = ref[..., strict]
        st = {"max_abs": float(es.max(initial=0.0)), "rms": float(np.sqrt(np.mean(es ** 2))) if es.size else 0.0,
              "rel_l2": float(np.linalg.norm(es) / max(np.linalg.norm(refs), 1e-30)), "tol": tol}
        stats[name] = st
    # order-ambiguous pixels: within the reordering bound, plus the tolerance
    # and the rounding a different FP32 summation order of the pixel's n
    # blended terms can produce (n 2^-24 times the sum of the non-negative
    # terms, i.e. of the value itself)
    nb = r["nblend"].reshape(-1).astype(np.float64)
    reassoc = nb * 2.0 ** -24
    over_c = (ec[:, bounded] - bnd[:3, bounded] - TOL_C - reassoc[bounded] * np.abs(rc[:, bounded])).max(initial=-1.0)
    over_d = (ed[bounded] - bnd[3, bounded] - TOL_D - reassoc[bounded] * np.abs(rd[bounded])).max(initial=-1.0)
    over_a = (ea[bounded] - bnd[4, bounded] - TOL_A - reassoc[bounded]).max(initial=-1.0)
    share = float(excl.sum()) / max(n, 1)
    out = {"config": label, "view": view, "pixels": int(n), "strict": int(strict.sum()),
           "order_bounded": int(bounded.sum()), "excluded": int(excl.sum()), "excluded_share": share,
           "bounded_max_excess": [float(over_c), float(over_d), float(over_a)] if bounded.any() else None,
           "bounded_max_abs": [float(ec[:, bounded].max(initial=0.0)), float(ed[bounded].max(initial=0.0)),
                               float(ea[bounded].max(initial=0.0))] if bounded.any() else None,
           **{k: v for k, v in stats.items()}}
    report(kind="forward", **out)
    for name, st in stats.items():
        assert st["max_abs"] <= st["tol"], (label, view, name, st)
    assert over_c <= 0 and over_d <= 0 and over_a <= 0, (label, view, over_c, over_d, over_a)
    if n >= 100:   # a share of a handful of pixels says nothing
        assert share <= MAX_EXCLUDED, (label, view, share)
    return out


def check_forward(s, color, depth, alpha, ref, label):
    """Every view of a concatenated render against render_views' output."""
    color, depth, alpha = _np(color), _np(depth), _np(alpha)
    off = s.pix_offsets()
    res = []
    for v, cam in enumerate(s.cams):
        P = cam.npix
        sl = slice(int(off[v]), int(off[v]) + P)
        r = {"color": ref["color"][3 * int(off[v]):3 * int(off[v]) + 3 * P], "depth": ref["depth"][sl],
             "alpha": ref["alpha"][sl], "ambiguous": ref["ambiguous"][sl], "order_bound": ref["order_bound"][:, sl],
             "nblend": ref["nblend"][sl]}
        res.append(check_forward_view(label, color[3 * int(off[v]):3 * int(off[v]) + 3 * P], depth[sl], alpha[sl], r,
                                      view=v))
    worst = {k: max(x[k]["max_abs"] for x in res) for k in ("C", "D", "A")}
    excl = sum(x["excluded"] for x in res)
    bounded = sum(x["order_bounded"] for x in res)
    print(f"  [{label}] forward max |err| C={worst['C']:.2e} D={worst['D']:.2e} A={worst['A']:.2e}; "
          f"order-bounded {bounded}, excluded {excl} of {s.npix}", flush=True)
    return res


def check_grad(label, name, g, r, tol=TOL_G, viol_max=MAX_VIOLATION):
    """Relative L2 error and the element-wise criterion of one gradient."""
    g = _np(g).reshape(-1)
    r = np.asarray(r, np.float64).reshape(-1)
    e = np.abs(g - r)
    nr = np.linalg.norm(r)
    rl = float(np.linalg.norm(g - r) / nr) if nr > 0 else float(np.linalg.norm(g))
    rms = float(np.sqrt(np.mean(r * r))) if r.size else 0.0
    viol = float(np.mean(e > 1e-3 * (np.abs(r) + rms))) if r.size else 0.0
    report(kind="gradient", config=label, output=name, rel_l2=rl, violation_fraction=viol,
           max_abs=float(e.max(initial=0.0)), rms_ref=rms, elements=int(r.size))
    print(f"  [{label}] {name}: rel {rl:.2e}, element-wise violations {viol:.2e}", flush=True)
    assert rl < tol and viol <= viol_max, (label, name, rl, viol)
    return rl, viol


def zmax(s):
    return float(np.abs(s.means).max()) * 3.0 + 10.0


def rel(a, r):
    a = np.asarray(a, np.float64).reshape(-1)
    r = np.asarray(r, np.float64).reshape(-1)
    n = np.linalg.norm(r)
    return float(np.linalg.norm(a - r) / n) if n > 0 else float(np.linalg.norm(a))


def cotangents(s, ref, seed, scale=1.0):
    """Random upstream gradients, zero at pixels the oracle flags ambiguous
    (including the 0.99 clamp, which changes gradients)."""
    dC, dD, dA = scenes.random_cotangents(s, seed, scale)
    ok = (ref["ambiguous"] == 0).astype(np.float32)
    okc = np.concatenate([np.tile(ok[o:o + cm.npix], 3) for cm, o in zip(s.cams, s.pix_offsets()[:-1])])
    return dC * okc, dD * ok, dA * ok


GRAD_NAMES = ["means", "log_scales", "quats", "opacity_logits", "colors"]
