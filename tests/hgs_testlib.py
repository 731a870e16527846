"""Shared helpers of the GPU tests: run the HIP pipeline through the C ABI
and view its buffers as numpy arrays, run the oracle on the same inputs."""
from __future__ import annotations

import numpy as np
import torch

from oracle import hgs_oracle as O
from paper_2406_02720_amd import binding as B
from paper_2406_02720_amd import raster as R

# Relative distances to a decision threshold below which a pixel's discrete
# choices may differ between the FP32 raster and the FP64 oracle, per kind of
# decision (the columns of the oracle's margin): alpha vs alpha_min (alpha
# carries ~1e-6 relative error from the float32 quadratic form, exp and
# erfc), transmittance vs t_min (a product of up to ~10^3 rounded float32
# factors), power vs 0 (the float32 quadratic form is exact to a few ulp of
# the sum of its absolute terms, so its sign can only flip when |power| is
# that small relative to them); then alpha and transmittance per unit of
# the terms of the quadratic form: the float32 exponent is off by up to
# about 3 ulp of those terms (2e-7 per unit: a pair 2000 pixels from the
# centre of a thin kernel has terms ~1e4, where alpha is only good to
# ~1e-3), and each blended factor passes its alpha error on to the
# transmittance, weighted by alpha / (1 - alpha).  Such pixels are excluded
# from exact-count and image checks.
BANDS = np.array([2e-5, 1e-4, 4e-6, 2e-7, 2e-7])


def ambiguous(margin) -> np.ndarray:
    """Pixels with any decision inside its band (margin: [..., 5])."""
    m = margin.numpy() if hasattr(margin, "numpy") else np.asarray(margin)
    return (m < BANDS).any(-1)

OPT_KEYS = ("tile", "batch", "lowpass", "kappa", "alpha_min", "alpha_max", "t_min", "fov_clamp", "bg",
            "full_box", "sort_full_keys", "mip2d")


def split_opts(kw):
    gpu = {k: v for k, v in kw.items() if k in OPT_KEYS}
    orc = {k: v for k, v in kw.items() if k in OPT_KEYS and k not in ("batch", "sort_full_keys")}
    return gpu, O.options(**orc)


def gpu_forward(scene, cams, capacity=None, persistent=True, render=True, **kw):
    gkw, _ = split_opts(kw)
    soa = R.scene_to_soa(scene)
    f3 = scene.get("filter3d")
    f3 = None if f3 is None else torch.as_tensor(np.asarray(f3, np.float32)).cuda()
    fr = R.forward_pass(soa, scene["means"].shape[0], scene["sh_degree"], B.make_cameras(cams),
                        B.default_options(**gkw), capacity=capacity, persistent=persistent, filter3d=f3,
                        render=render)
    torch.cuda.synchronize()
    return fr


def oracle_pre(scene, cams, **kw):
    _, o = split_opts(kw)
    sc = O.scene_to_torch(scene)
    with torch.no_grad():
        return [O.preprocess(sc, O.camera_to_torch(c), o) for c in cams]


def records_np(fr):
    raw = fr.records.cpu().numpy()
    return raw.view(np.float32).reshape(-1, 16), raw.view(np.uint32).reshape(-1, 16)


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def u64(t):
    return t.cpu().numpy().view(np.uint64)


def sorted_entries(fr):
    n = int(fr.n_dup.item())
    return u64(fr.keys)[:n], u32(fr.values)[:n], u32(fr.ranges)[:2 * B.hgs_tiles_total(fr.cams, fr.opts)].reshape(-1, 2)


def kernel_terms(pre, pixels, chunk: int = 64, min_power: float = -5.6) -> np.ndarray:
    """Per kernel, the largest sum of absolute terms of the quadratic form
    (0.5 (|a| dx^2 + |c| dy^2) + |b dx dy|, float32 record values, FP64)
    over the given pixels inside its rect where its exponent can still give
    alpha >= alpha_min (power >= min_power); 0 where there are none.  The
    float32 exponent of such a pair is off by up to ~3 ulp of this sum, so a
    large value marks a kernel whose blend, and therefore its gradient, is
    evaluated with a correspondingly larger rounding error."""
    recs = O.raster_records(pre, "rec")
    rect = recs["rect"]
    ids = recs["id"]
    out = torch.zeros(pre["N"], dtype=torch.float64)
    pix = torch.as_tensor(np.asarray(pixels), dtype=torch.int64)
    for s in range(0, pix.shape[0], chunk):
        px, py = pix[s:s + chunk, 0], pix[s:s + chunk, 1]
        hit = ((rect[:, 0] <= px.max()) & (rect[:, 1] >= px.min()) & (rect[:, 2] <= py.max()) & (rect[:, 3] >= py.min()))
        cand = torch.nonzero(hit).squeeze(-1)
        if cand.numel() == 0:
            continue
        r = rect[cand]
        inside = ((px[:, None] >= r[None, :, 0]) & (px[:, None] <= r[None, :, 1]) &
                  (py[:, None] >= r[None, :, 2]) & (py[:, None] <= r[None, :, 3]))
        dx = (px[:, None] - r[None, :, 0]).double() + 0.5 - recs["mu_rel"][cand][None, :, 0]
        dy = (py[:, None] - r[None, :, 2]).double() + 0.5 - recs["mu_rel"][cand][None, :, 1]
        a_, b_, c_ = recs["conic"][cand].unbind(-1)
        power = -0.5 * (a_ * dx * dx + c_ * dy * dy) - b_ * dx * dy
        terms = 0.5 * (a_.abs() * dx * dx + c_.abs() * dy * dy) + (b_ * dx * dy).abs()
        terms = torch.where(inside & (power >= min_power), terms, torch.zeros_like(terms)).max(0).values
        k = ids[cand]
        out[k] = torch.maximum(out[k], terms)
    return out.numpy()


# Gradient bar (per element): |got - ref| <= 1e-3 |ref| + 1e-5 max |ref|, and
# per tensor a relative L2 error <= 1e-3.  Elements outside the bar are
# allowed only on kernels whose exponent is ill-conditioned in float32 (the
# sum of the absolute terms of its quadratic form above ILL_TERMS at some
# pair that can blend, see kernel_terms), at most OUTLIER_FRACTION of the
# tensor (and at least 2 elements' worth), each within OUTLIER_RATIO times
# the bar; every such element is printed.  The ratio covers the worst case
# seen: a needle-shaped kernel 0.45 units in front of the camera, covering
# the whole 1080p image with terms ~1.2e4 (its float32 alpha is good to
# ~2e-3 per pixel), whose scale gradient sums contributions of both signs;
# builds that only regroup the float32 accumulation gave 0.512 and 0.539
# against the FP64 0.520 (ratios 4.6 and 10.8, on both sides of it).
ILL_TERMS = 1000.0
OUTLIER_RATIO = 20.0
OUTLIER_FRACTION = 1e-5


def check_gradients(got: dict, ref: dict, terms=None, label: str = "") -> dict:
    """got, ref: {parameter: [N, ...] arrays}; terms: kernel_terms per kernel
    (None: no outlier allowed).  Returns {parameter: worst |d| / bar}."""
    worst = {}
    for k, r in ref.items():
        g = np.asarray(got[k], np.float64).reshape(r.shape)
        assert np.abs(r).max() > 0, k
        rel_l2 = np.linalg.norm(g - r) / np.linalg.norm(r)
        bar = 1e-3 * np.abs(r) + 1e-5 * np.abs(r).max()
        ratio = np.abs(g - r) / bar
        out = np.argwhere(ratio > 1.0)
        worst[k] = float(ratio.max())
        print(f"[grad{label}] {k}: rel_l2 {rel_l2:.2e} out-of-bar {len(out)}/{ratio.size} "
              f"worst |d|/bar {worst[k]:.3g}", flush=True)
        for idx in out[:20]:
            t = None if terms is None else float(terms[idx[0]])
            print(f"    {k}{tuple(int(i) for i in idx)}: got {g[tuple(idx)]:.7g} ref {r[tuple(idx)]:.7g} "
                  f"|d|/bar {ratio[tuple(idx)]:.3g} kernel terms {t}", flush=True)
        assert rel_l2 <= 1e-3, (k, rel_l2)
        if len(out):
            assert terms is not None, (k, "elements outside the bar", len(out))
            assert len(out) <= max(2, OUTLIER_FRACTION * ratio.size), (k, len(out))
            assert all(terms[i[0]] > ILL_TERMS for i in out), (k, "outlier on a well-conditioned kernel")
            assert worst[k] <= OUTLIER_RATIO, (k, worst[k])
    return worst
