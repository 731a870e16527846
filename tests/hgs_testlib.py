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
# decision: alpha vs alpha_min (alpha carries ~1e-6 relative error from the
# float32 quadratic form, exp and erfc), transmittance vs t_min (a product of
# up to ~10^3 rounded float32 factors), and power vs 0 (the float32 quadratic
# form is exact to a few ulp of the sum of its absolute terms, so its sign can
# only flip when |power| is that small relative to them).  Such pixels are
# excluded from exact-count and image checks.
BANDS = np.array([2e-5, 1e-4, 4e-6])


def ambiguous(margin) -> np.ndarray:
    """Pixels with any decision inside its band (margin: [..., 3])."""
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
