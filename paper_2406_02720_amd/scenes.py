"""Seeded synthetic scenes and cameras for the half-Gaussian rasterizer.

This module only draws inputs.  It holds none of the rasterizer's arithmetic:
both the FP64 oracle and the HIP path are fed from here, so it must stay free
of projection, compositing or sorting code.

Every scene is a dict of float32 numpy arrays in natural (row-per-kernel)
layout:

    means   [N,3]   world-space centres
    scales  [N,3]   activated (linear, > 0) axis lengths
    quats   [N,4]   rotation quaternions, (w, x, y, z), normalised
    normals [N,3]   splitting-plane normals, unit length
    opac1   [N]     opacity of the half on the +normal side, in [0,1]
    opac2   [N]     opacity of the half on the -normal side, in [0,1]
    sh      [N,K,3] spherical-harmonic colour coefficients, K = (D+1)^2
    sh_degree int   D

Cameras are dicts with a world->camera rotation ``R`` (3x3, rows = camera
x-right, y-down, z-forward axes in world coordinates), translation ``t``,
pinhole intrinsics in pixels and the image size.

The workloads mirror the paper's setting (scenes of one to three million
kernels rendered at camera resolutions; Table 2 and the rendering-speed
ablation in Supp. C) with synthetic distributions, because the paper's
datasets and trained models are not available.
"""
from __future__ import annotations

import math

import numpy as np

HFOV_DEG = 60.0
ZNEAR = 0.2


# --------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------
def pinhole(width: int, height: int, R, t, hfov_deg: float = HFOV_DEG, znear: float = ZNEAR) -> dict:
    """Pinhole camera with horizontal field of view ``hfov_deg``, square pixels
    and the principal point at the image centre."""
    f = (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    return dict(R=np.asarray(R, np.float32).reshape(3, 3), t=np.asarray(t, np.float32).reshape(3),
                fx=np.float32(f), fy=np.float32(f), cx=np.float32(width / 2.0), cy=np.float32(height / 2.0),
                width=int(width), height=int(height), znear=np.float32(znear))


def look_at(position, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)):
    """World->camera (R, t) for a camera at ``position`` looking at ``target``
    with OpenCV axes (x right, y down, z forward)."""
    p = np.asarray(position, np.float64)
    fwd = np.asarray(target, np.float64) - p
    fwd /= np.linalg.norm(fwd)
    upv = np.asarray(up, np.float64)
    if abs(float(np.dot(fwd, upv))) > 0.999:
        upv = np.array([0.0, 1.0, 0.0]) if abs(fwd[1]) < 0.9 else np.array([1.0, 0.0, 0.0])
    right = np.cross(fwd, upv)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    t = -R @ p
    return R, t


def axis_camera(width: int, height: int, distance: float = 4.0) -> dict:
    """Camera on the world -z axis at ``distance`` looking along +z (R = I)."""
    return pinhole(width, height, np.eye(3), (0.0, 0.0, distance))


# --------------------------------------------------------------------------
# kernels
# --------------------------------------------------------------------------
def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _unit_rows(x):
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def _draw_kernels(rng, n, means, log_scale_mu, log_scale_sd, sh_degree, sh_sd=0.2,
                  dc_colour=False, big_frac=0.0, big_mu=-1.0, big_sd=0.5):
    """Draw the per-kernel parameters after the means, in the fixed order
    log-scales, quaternions, normals, opacity-1 logits, opacity-2 logits, SH."""
    log_s = rng.normal(log_scale_mu, log_scale_sd, size=(n, 3))
    if big_frac > 0.0:
        big = rng.random(n) < big_frac
        log_s[big] = rng.normal(big_mu, big_sd, size=(int(big.sum()), 3))
    quats = _unit_rows(rng.normal(size=(n, 4)))
    normals = _unit_rows(rng.normal(size=(n, 3)))
    opac1 = _sigmoid(rng.normal(size=n))
    opac2 = _sigmoid(rng.normal(size=n))
    k = (sh_degree + 1) ** 2
    if dc_colour:
        # degree-0 colour drawn directly: the coefficient is chosen so that the
        # constant basis function (value 1 / (2 sqrt(pi))) plus the 0.5 offset
        # reproduces the drawn colour.
        colour = rng.random((n, 3))
        sh = np.zeros((n, k, 3))
        sh[:, 0, :] = (colour - 0.5) * (2.0 * math.sqrt(math.pi))
    else:
        sh = rng.normal(0.0, sh_sd, size=(n, k, 3))
    return dict(means=means.astype(np.float32), scales=np.exp(log_s).astype(np.float32),
                quats=quats.astype(np.float32), normals=normals.astype(np.float32),
                opac1=opac1.astype(np.float32), opac2=opac2.astype(np.float32),
                sh=sh.astype(np.float32), sh_degree=int(sh_degree))


def _shell_mixture(rng, n, shell_frac=0.7, shell_sd=0.05, box=3.0):
    n_shell = int(round(shell_frac * n))
    d = _unit_rows(rng.normal(size=(n_shell, 3)))
    r = 1.0 + rng.normal(0.0, shell_sd, size=(n_shell, 1))
    shell = d * r
    rest = rng.uniform(-box, box, size=(n - n_shell, 3))
    pts = np.concatenate([shell, rest])
    return pts[rng.permutation(n)]


RESOLUTIONS_CFG4 = ((640, 480), (1024, 768), (1297, 840), (1600, 1064))


def make_config(cfg: int, seed: int | None = None, n: int | None = None, n_cams: int | None = None,
                width: int | None = None, height: int | None = None):
    """Scene and cameras of workload ``cfg`` (1..5); ``n``, ``n_cams`` and the
    image size may be shrunk for tests.  Returns (scene, cameras)."""
    rng = np.random.Generator(np.random.PCG64(cfg if seed is None else seed))
    if cfg == 1:
        n = 1000 if n is None else n
        means = rng.uniform(-1.0, 1.0, size=(n, 3))
        scene = _draw_kernels(rng, n, means, -3.0, 0.5, 0, dc_colour=True)
        cams = [axis_camera(width or 128, height or 128)]
    elif cfg == 2:
        n = 100_000 if n is None else n
        means = rng.uniform(-1.0, 1.0, size=(n, 3))
        scene = _draw_kernels(rng, n, means, -3.0, 0.5, 3)
        cams = [axis_camera(width or 1280, height or 720)]
    elif cfg == 3:
        n = 1_000_000 if n is None else n
        means = _shell_mixture(rng, n)
        scene = _draw_kernels(rng, n, means, -4.0, 1.0, 3)
        R, t = look_at(4.0 * np.ones(3) / math.sqrt(3.0))
        cams = [pinhole(width or 1920, height or 1080, R, t)]
    elif cfg == 4:
        n = 500_000 if n is None else n
        means = _shell_mixture(rng, n)
        scene = _draw_kernels(rng, n, means, -4.0, 1.0, 3)
        nc = 16 if n_cams is None else n_cams
        dirs = _unit_rows(rng.normal(size=(nc, 3)))
        res = rng.integers(0, len(RESOLUTIONS_CFG4), size=nc)
        cams = []
        for i in range(nc):
            R, t = look_at(4.0 * dirs[i])
            w, h = RESOLUTIONS_CFG4[int(res[i])]
            if width is not None:
                w, h = width, height
            cams.append(pinhole(w, h, R, t))
    elif cfg == 5:
        n = 3_000_000 if n is None else n
        means = np.stack([rng.uniform(-10, 10, n), rng.uniform(-10, 10, n), rng.uniform(-2.5, 2.5, n)], 1)
        scene = _draw_kernels(rng, n, means, -3.0, 0.5, 3, big_frac=0.05)
        nc = 8 if n_cams is None else n_cams
        az = 2.0 * math.pi * (np.arange(nc) + rng.uniform(-0.1, 0.1, nc)) / nc
        cams = []
        for i in range(nc):
            pos = (14.0 * math.cos(az[i]), 14.0 * math.sin(az[i]), 4.0)
            R, t = look_at(pos)
            cams.append(pinhole(width or 3840, height or 2160, R, t))
    else:
        raise ValueError(f"unknown workload {cfg}")
    return scene, cams


# --------------------------------------------------------------------------
# variants used by tests
# --------------------------------------------------------------------------
def with_transparent_halves(scene: dict, frac: float = 0.5, seed: int = 7) -> dict:
    """Copy of ``scene`` where a seeded ``frac`` of the kernels get one half of
    opacity 0 (which half is drawn too): the trained-scene regime in which the
    paper's efficient splatting pays off."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = scene["opac1"].shape[0]
    pick = rng.random(n) < frac
    side = rng.random(n) < 0.5
    out = dict(scene)
    o1, o2 = scene["opac1"].copy(), scene["opac2"].copy()
    o1[pick & side] = 0.0
    o2[pick & ~side] = 0.0
    out["opac1"], out["opac2"] = o1, o2
    return out


def with_equal_opacities(scene: dict) -> dict:
    """Copy of ``scene`` with opacity-2 set equal to opacity-1 (a standard
    Gaussian per kernel)."""
    out = dict(scene)
    out["opac2"] = scene["opac1"].copy()
    return out


def subset(scene: dict, idx) -> dict:
    out = {k: (v[idx] if isinstance(v, np.ndarray) else v) for k, v in scene.items()}
    return out


def target_image(cameras, seed: int = 102):
    """Seeded U[0,1] target images, one [3,H,W] float32 array per camera."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [rng.random((3, c["height"], c["width"])).astype(np.float32) for c in cameras]


def sample_pixels(camera: dict, count: int, seed: int = 11):
    """Seeded distinct pixel coordinates (px, py) of one camera."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w, h = camera["width"], camera["height"]
    count = min(count, w * h)
    flat = rng.choice(w * h, size=count, replace=False)
    return np.stack([flat % w, flat // w], 1).astype(np.int64)


def sample_pixel_blocks(camera: dict, blocks: int, side: int = 8, seed: int = 11):
    """Seeded pixels of `blocks` distinct side x side squares of one camera
    (squares on a grid of that pitch, clipped at the image border), each
    square's pixels consecutive: a sample whose consecutive pixels share
    their neighbourhood."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w, h = camera["width"], camera["height"]
    gx, gy = (w + side - 1) // side, (h + side - 1) // side
    picks = rng.choice(gx * gy, size=min(blocks, gx * gy), replace=False)
    out = []
    for b in picks:
        x0, y0 = (b % gx) * side, (b // gx) * side
        yy, xx = np.meshgrid(np.arange(y0, min(y0 + side, h)), np.arange(x0, min(x0 + side, w)), indexing="ij")
        out.append(np.stack([xx.ravel(), yy.ravel()], 1))
    return np.concatenate(out).astype(np.int64)


def depth_maps(cameras, seed: int = 7):
    """Seeded blended-depth and transmittance maps, one [H,W] float32 pair
    per camera: a tilted wavy surface at depth ~3 seen through a random
    coverage 1 - T in [0.7, 1], with ~3% empty pixels (T = 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ds, Ts = [], []
    for c in cameras:
        H, W = c["height"], c["width"]
        yy, xx = np.mgrid[0:H, 0:W]
        z = 3.0 + 0.01 * xx + 0.004 * yy + 0.05 * np.sin(xx / 7.0) * np.cos(yy / 5.0)
        T = rng.uniform(0.0, 0.3, (H, W))
        T[rng.uniform(size=(H, W)) < 0.03] = 1.0
        Ds.append((z * (1.0 - T)).astype(np.float32))
        Ts.append(T.astype(np.float32))
    return Ds, Ts


def train_state(n: int, sh_degree: int, extent: float = 2.0, seed: int = 21):
    """Seeded optimiser state of n half-Gaussians in the raw layout
    (float32 [planes, n] arrays: means, log-scales, quaternions, normals,
    opacity logits, SH), activated-space gradients, Adam moments, and
    densification statistics spread around the 3D-GS thresholds (largest
    scale around 0.01 * extent, opacities around 0.01, average NDC gradient
    around 0.0002, screen radii 0..40 px), plus the standard normal draws of
    two children per kernel ([2, 3, n])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    K = 3 * (sh_degree + 1) ** 2
    f32 = np.float32
    raw = dict(
        means=rng.normal(0.0, extent, (3, n)).astype(f32),
        scales=(np.log(0.01 * extent) + rng.normal(0.0, 1.0, (3, n))).astype(f32),
        quats=rng.normal(0.0, 1.0, (4, n)).astype(f32),
        normals=rng.normal(0.0, 1.0, (3, n)).astype(f32),
        opac1=(np.log(0.01 / 0.99) + rng.normal(0.0, 2.0, (1, n))).astype(f32),
        opac2=(np.log(0.01 / 0.99) + rng.normal(0.0, 2.0, (1, n))).astype(f32),
        sh=rng.normal(0.0, 0.3, (K, n)).astype(f32),
    )
    grads = {k: (rng.normal(0.0, 1e-2, v.shape) * (rng.random(v.shape) < 0.9)).astype(f32) for k, v in raw.items()}
    m = {k: rng.normal(0.0, 1e-3, v.shape).astype(f32) for k, v in raw.items()}
    v2 = {k: (rng.random(v.shape) * 1e-4).astype(f32) for k, v in raw.items()}
    count = rng.integers(0, 6, n).astype(np.int32)
    accum = (count * rng.lognormal(np.log(0.0002), 0.7, n)).astype(f32)
    radii = np.floor(rng.random(n) * 40.0).astype(f32)
    samples = rng.normal(0.0, 1.0, (2, 3, n)).astype(f32)
    return dict(raw=raw, grads=grads, m=m, v=v2, accum=accum, count=count, radii=radii, samples=samples)


def with_filter3d(scene: dict, seed: int = 13, scale: float = 0.5) -> dict:
    """Copy of ``scene`` with a seeded Mip-Splatting 3-D filter variance per
    kernel: (scale * smallest axis)^2 times a log-uniform factor in
    [0.1, 10], so that the filter ranges from negligible to dominant."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = dict(scene)
    smin = np.asarray(scene["scales"], np.float64).min(1)
    fac = np.exp(rng.uniform(np.log(0.1), np.log(10.0), smin.shape[0]))
    out["filter3d"] = ((scale * smin) ** 2 * fac).astype(np.float32)
    return out
