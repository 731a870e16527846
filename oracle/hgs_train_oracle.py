"""FP64 CPU oracle of the optimisation step that follows the rasterizer's
backward pass in 3D-HGS training: Adam on the raw parameters with the 3D-GS
schedule and the half-Gaussian changes, the densification statistics, and
densify / prune / opacity reset with the half-Gaussian thresholds.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this module: only ``tests/`` use it.  It shares no code with the HIP
library and does not import the rasterizer oracle's arithmetic; inputs come
from seeded draws.

Paper passages: Sec. 4 (implementation: the normal is the three unused
normal parameters of 3D-GS, one opacity per half, 3D-GS's training settings
otherwise, normal learning rate 0.003), Supp. training settings (opacity and
normal learning rates divided by 1.4 every 5000 iterations; pruning opacity
threshold 0.01; opacity reset to 0.02).  Everything else is the published
3D-GS recipe the paper adopts (Kerbl et al. 2023, Sec. 5 and 7):

* raw parameters: means, log-scales, quaternions, normals, opacity logits
  (one per half), SH coefficients; the rasterizer sees exp(log-scale) and
  sigmoid(logit);
* Adam (Kingma and Ba), beta = (0.9, 0.999), eps = 1e-15, one step counter;
* learning rates: means 1.6e-4 * extent decaying log-linearly to
  1.6e-6 * extent over 30000 iterations; SH degree-0 coefficients 0.0025,
  higher ones 0.0025 / 20; opacities 0.05; log-scales 0.005; quaternions
  0.001; normals 0.003;
* densification statistics: per view in which a kernel is visible (its
  pixel rect is not empty), the norm of the loss gradient with respect to
  its projected centre in normalised device coordinates (pixel gradient
  times W/2 and H/2) is summed and the view counted; the largest 3-sigma
  screen radius is kept;
* densify: average gradient >= 0.0002 -> clone if the largest scale is
  <= 0.01 * extent, else split into two children drawn from the kernel's
  own Gaussian with scales divided by 0.8 * 2; prune kernels whose opacity
  is below the threshold, and (when enabled) those with screen radius > 20
  px or largest scale > 0.1 * extent; new kernels start with zero Adam
  moments and zero screen radius.

Readings (listed in the design notes): a half-Gaussian is pruned when BOTH
halves are below the opacity threshold; the reset takes each half to
min(opacity, 0.02); the decay factor is 1.4 ** -floor(t / 5000) at
iteration t (1-based, the learning rate of the step being taken); scale and
opacity thresholds are compared on the raw parameters against the logarithm
or logit of the threshold (the activations are monotone), the average
gradient as accum >= threshold * count with count > 0, all in float64, so that the two
implementations take every decision on the same numbers; a child's
log-scale is the parent's minus log(0.8 * 2), rounded to float32; the
screen radius is ceil(3 sqrt(lambda_max)) of the dilated screen covariance,
from the float32 conic; output order: surviving originals, then clones, then
first children, then second children, each in kernel order.
"""
from __future__ import annotations

import math

import numpy as np

PLANES = ("means", "scales", "quats", "normals", "opac1", "opac2", "sh")
WIDTH = dict(means=3, scales=3, quats=4, normals=3, opac1=1, opac2=1)

BETA1, BETA2, EPS = 0.9, 0.999, 1e-15


def sh_planes(sh_degree: int) -> int:
    return 3 * (sh_degree + 1) ** 2


def learning_rates(t: int, extent: float, normal_lr: float = 0.003) -> dict:
    """Per-group learning rate of iteration t (1-based).  Means: 3D-GS's
    log-linear decay over 30000 iterations; opacities and normals: the
    paper's division by 1.4 every 5000 iterations (Supp. training
    settings); normal base rate 0.003 (Sec. 4)."""
    r = min(max(t / 30000.0, 0.0), 1.0)
    lr0, lr1 = 1.6e-4 * extent, 1.6e-6 * extent
    means = math.exp((1.0 - r) * math.log(lr0) + r * math.log(lr1))
    decay = 1.4 ** -(t // 5000)
    return dict(means=means, scales=0.005, quats=0.001, normals=normal_lr * decay,
                opac=0.05 * decay, sh_dc=0.0025, sh_rest=0.0025 / 20.0)


def _plane_lr(name: str, k: int, lrs: dict) -> float:
    if name in ("opac1", "opac2"):
        return lrs["opac"]
    if name == "sh":
        return lrs["sh_dc"] if k < 3 else lrs["sh_rest"]
    return lrs[name]


def activate(raw: dict) -> dict:
    """The rasterizer's inputs from the raw parameters."""
    out = {k: np.asarray(v, np.float64).copy() for k, v in raw.items()}
    out["scales"] = np.exp(out["scales"])
    out["opac1"] = 1.0 / (1.0 + np.exp(-out["opac1"]))
    out["opac2"] = 1.0 / (1.0 + np.exp(-out["opac2"]))
    return out


def raw_gradients(raw: dict, grad_act: dict) -> dict:
    """Chain rule from the gradient with respect to the activated values to
    the raw ones: d exp(x)/dx = exp(x), d sigmoid(x)/dx = s (1 - s)."""
    g = {k: np.asarray(v, np.float64).copy() for k, v in grad_act.items()}
    g["scales"] = g["scales"] * np.exp(np.asarray(raw["scales"], np.float64))
    for k in ("opac1", "opac2"):
        s = 1.0 / (1.0 + np.exp(-np.asarray(raw[k], np.float64)))
        g[k] = g[k] * s * (1.0 - s)
    return g


def adam_step(raw: dict, grad_act: dict, m: dict, v: dict, t: int, lrs: dict,
              betas=(BETA1, BETA2), eps: float = EPS):
    """One Adam step (t = the step number, 1-based) on every raw plane with
    its group's learning rate.  Arrays are [planes, n]; returns new
    (raw, m, v, activated).  ``betas`` and ``eps`` default to 3D-GS's."""
    b1, b2 = betas
    g = raw_gradients(raw, grad_act)
    c1, c2 = 1.0 - b1 ** t, 1.0 - b2 ** t
    raw2, m2, v2 = {}, {}, {}
    for name in PLANES:
        p = np.asarray(raw[name], np.float64)
        mm = b1 * np.asarray(m[name], np.float64) + (1.0 - b1) * g[name]
        vv = b2 * np.asarray(v[name], np.float64) + (1.0 - b2) * g[name] ** 2
        lr = np.array([_plane_lr(name, k, lrs) for k in range(p.shape[0])])[:, None]
        raw2[name] = p - lr * (mm / c1) / (np.sqrt(vv / c2) + eps)
        m2[name], v2[name] = mm, vv
    return raw2, m2, v2, activate(raw2)


def screen_radius(conic: np.ndarray, kappa: float = 3.0) -> np.ndarray:
    """ceil(kappa sqrt(lambda_max)) of the screen covariance whose inverse
    is the conic [[a, b], [b, c]] (float32 values, evaluated in float64)."""
    a, b, c = (np.asarray(conic[:, i], np.float32).astype(np.float64) for i in range(3))
    mid = 0.5 * (a + c)
    lam_min = mid - np.sqrt(np.maximum(0.25 * (a - c) ** 2 + b * b, 0.0))
    return np.ceil(kappa * np.sqrt(1.0 / lam_min))


def densify_stats(n: int, views: list, accum=None, count=None, max_radii=None):
    """Accumulate the densification statistics over views.  Each view is a
    dict with the camera width/height, the visible kernels ``idx``, their
    pixel-space centre gradients ``g_mean`` [V, 2] and float32 ``conic``
    [V, 3].  Returns (accum float64, count int, max_radii float64)."""
    accum = np.zeros(n) if accum is None else np.asarray(accum, np.float64).copy()
    count = np.zeros(n, np.int64) if count is None else np.asarray(count, np.int64).copy()
    max_radii = np.zeros(n) if max_radii is None else np.asarray(max_radii, np.float64).copy()
    for vw in views:
        idx = np.asarray(vw["idx"])
        g = np.asarray(vw["g_mean"], np.float64)
        gx = g[:, 0] * (0.5 * vw["width"])
        gy = g[:, 1] * (0.5 * vw["height"])
        accum[idx] += np.sqrt(gx * gx + gy * gy)
        count[idx] += 1
        max_radii[idx] = np.maximum(max_radii[idx], screen_radius(vw["conic"]))
    return accum, count, max_radii


def _logit(p: float) -> float:
    return math.log(p / (1.0 - p))


def densify_and_prune(raw: dict, m: dict, v: dict, accum, count, max_radii, samples, *,
                      extent: float, grad_threshold: float = 0.0002, percent_dense: float = 0.01,
                      min_opacity: float = 0.01, max_screen_radius: float = 0.0,
                      max_world_scale: float = 0.0):
    """Clone, split and prune (3D-GS densification with the half-Gaussian
    pruning threshold).  ``samples`` [2, 3, n]: standard normal draws of the
    two children of every kernel (used only where it splits).  Thresholds of
    0 disable the screen-radius and world-scale prunes; max_world_scale is a
    fraction of the extent.  Returns (raw, m, v, dict of index arrays)."""
    n = np.asarray(raw["means"]).shape[1]
    ls = np.asarray(raw["scales"], np.float32).astype(np.float64)
    smax = ls.max(0)
    acc = np.asarray(accum, np.float32).astype(np.float64)
    cnt = np.asarray(count, np.float64)
    big_grad = (cnt > 0) & (acc >= float(np.float32(grad_threshold)) * cnt)
    small = smax <= math.log(percent_dense * extent)
    clone = big_grad & small
    split = big_grad & ~small

    def pruned(omax, lsmax, radii):
        p = omax < _logit(min_opacity)
        if max_screen_radius > 0.0:
            p |= radii > max_screen_radius
        if max_world_scale > 0.0:
            p |= lsmax > math.log(max_world_scale * extent)
        return p

    o1 = np.asarray(raw["opac1"], np.float32).astype(np.float64)[0]
    o2 = np.asarray(raw["opac2"], np.float32).astype(np.float64)[0]
    omax = np.maximum(o1, o2)
    radii = np.asarray(max_radii, np.float64)
    shrink = np.float32(math.log(0.8 * 2))
    child_ls = (np.asarray(raw["scales"], np.float32) - shrink).astype(np.float64)
    keep = ~split & ~pruned(omax, smax, radii)
    clone_keep = clone & ~pruned(omax, smax, np.zeros(n))
    child_keep = split & ~pruned(omax, child_ls.max(0), np.zeros(n))

    # children: mean + R(q) (scale * z), R from the normalised quaternion
    q = np.asarray(raw["quats"], np.float64)
    qn = np.linalg.norm(q, axis=0)
    q = np.where(qn > 0, q / np.where(qn > 0, qn, 1.0), np.array([[1.0], [0.0], [0.0], [0.0]]))
    w, x, y, z = q
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    s = np.exp(ls)
    mu = np.asarray(raw["means"], np.float64)
    zs = np.asarray(samples, np.float64)
    child_mu = [mu + np.einsum("ijn,jn->in", R, s * zs[c]) for c in range(2)]

    src_keep = np.nonzero(keep)[0]
    src_clone = np.nonzero(clone_keep)[0]
    src_child = np.nonzero(child_keep)[0]
    out_raw, out_m, out_v = {}, {}, {}
    for name in PLANES:
        a = np.asarray(raw[name], np.float64)
        parts = [a[:, src_keep], a[:, src_clone], a[:, src_child], a[:, src_child]]
        if name == "means":
            parts[2], parts[3] = child_mu[0][:, src_child], child_mu[1][:, src_child]
        if name == "scales":
            parts[2] = parts[3] = child_ls[:, src_child]
        out_raw[name] = np.concatenate(parts, 1)
        for dst, src in ((out_m, m), (out_v, v)):
            b = np.asarray(src[name], np.float64)
            new = len(src_clone) + 2 * len(src_child)
            dst[name] = np.concatenate([b[:, src_keep], np.zeros((b.shape[0], new))], 1)
    info = dict(keep=src_keep, clone=src_clone, child=src_child, clone_mask=clone, split_mask=split)
    return out_raw, out_m, out_v, info


def reset_opacity(raw: dict, m: dict, v: dict, value: float = 0.02):
    """Opacity reset of the half-Gaussian recipe (Supp. training settings):
    each half's opacity becomes min(opacity, value); its Adam moments are
    cleared.  Returns new (raw, m, v)."""
    raw2 = {k: np.asarray(a, np.float64).copy() for k, a in raw.items()}
    m2 = {k: np.asarray(a, np.float64).copy() for k, a in m.items()}
    v2 = {k: np.asarray(a, np.float64).copy() for k, a in v.items()}
    cap = _logit(value)
    for k in ("opac1", "opac2"):
        raw2[k] = np.minimum(raw2[k], cap)
        m2[k][:] = 0.0
        v2[k][:] = 0.0
    return raw2, m2, v2
