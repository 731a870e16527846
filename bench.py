#!/usr/bin/env python3
"""Benchmark of the half-Gaussian tile rasterizer on one GPU.

One step = one forward + backward pass of the whole rasterizer over the
workload's views: hgs_preprocess, hgs_bin_sort, hgs_render_fwd, the L1 loss
gradient against a seeded target, then the two halves of hgs_render_bwd
(hgs_raster_bwd, hgs_preprocess_bwd) so that each is timed on its own.
Inputs (parameters, target) are resident in HBM before timing starts;
buffers are allocated once.

Default workload: 1M half-Gaussians, one 1920x1080 camera, SH degree 3,
FP32 (shell + box mixture, log-scales N(-4, 1)).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VECTOR_PEAK_TF = 157.3    # MI355X FP32 vector (256 CU x 2.4 GHz)
# the same without packed FP32 (compiled with packed-fp32-ops off): one wave64 FP32
# instruction per SIMD every 4 cycles, 256 CUs x 4 SIMDs x 16 lanes x 2 x 2.4 GHz
FP32_UNPACKED_PEAK_TF = 78.6

WORKLOADS = {
    3: "1M half-Gaussians, 1920x1080, SH deg 3, fwd+bwd (shell+box mixture)",
    2: "100k half-Gaussians, 1280x720, SH deg 3, fwd+bwd",
    1: "1k half-Gaussians, 128x128, SH deg 0, fwd+bwd",
    4: "500k half-Gaussians, 16 views of uneven size, SH deg 3, fwd+bwd",
    5: "3M half-Gaussians (5% large splats), 8 views of 3840x2160, SH deg 3, fwd+bwd",
}


PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "hbm_traffic_1M_1080p.txt")
TRAFFIC_SOURCES = ("include/hgs.h", "paper_2406_02720_amd/csrc/hgs_internal.h",
                   "paper_2406_02720_amd/csrc/geometry.h", "paper_2406_02720_amd/csrc/preprocess.hip",
                   "paper_2406_02720_amd/csrc/sort.hip", "paper_2406_02720_amd/csrc/render.hip",
                   "paper_2406_02720_amd/csrc/train.hip", "paper_2406_02720_amd/build.py")


def sources_digest() -> str:
    """sha256 over the kernel sources and build flags: the HBM counters in
    profiles/ belong to the build whose digest they record."""
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(kernel_prefix: str):
    """HBM bytes per launch of the kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, scaled by the copy-kernel factors it
    records; None when the summary is missing or was taken on other sources."""
    try:
        lines = open(PROFILE_TRAFFIC).read().splitlines()
    except OSError:
        return None
    digest = next((l.split(":", 1)[1].strip() for l in lines if l.startswith("sources_sha256:")), None)
    if digest != sources_digest():
        return None
    for l in lines:
        if l.startswith("kernel ") and kernel_prefix in l:
            fields = dict(kv.split("=") for kv in l.split()[1:] if "=" in kv)
            return int(float(fields["traffic_bytes"]))
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--tile", type=int, default=0,
                    help="tile edge in pixels (8, 16, 32); 0: raster.default_tile for the workload's views")
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--cpu-pixels", type=int, default=1024, help="pixels of the oracle CPU sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stages", action="store_true", help="print per-stage timings to stderr")
    ap.add_argument("--no-pair-counts", action="store_true",
                    help="skip counting the raster's pixel-entry pairs (its FLOP roofline then reads zero)")
    ap.add_argument("--full-keys", action="store_true", help="sort the 64-bit keys over all bits")
    ap.add_argument("--persistent", action="store_true",
                    help="persistent raster grid taking tiles longest list first (default: one workgroup per "
                         "tile, in tile order, which keeps neighbouring tiles' records together in the caches)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES, 5 times (counter calibration)")
    ap.add_argument("--no-multiview", action="store_true",
                    help="skip the multi-view comparison (batched graph step against a per-view loop, autotuned)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the efficient-rasterizer ablation, the equal-opacity run and the stress workload")
    ap.add_argument("--no-stress", action="store_true", help="skip the 3M-kernel 8 x 4K stress workload")
    ap.add_argument("--multiview-steps", type=int, default=10)
    ap.add_argument("--train", action="store_true",
                    help="add the training step after the backward pass (Adam, densification statistics, "
                         "densify) on the same 1M kernels")
    ap.add_argument("--no-autograd", action="store_true",
                    help="skip timing the torch.autograd path (Rasterizer forward + torch L1 loss + backward)")
    ap.add_argument("--autotune", metavar="JSON", default="",
                    help="autotune cache for the multi-view workload (JSON; default: tune every run, no cache)")
    ap.add_argument("--no-autotune", action="store_true", help="multi-view at --tile / --batch, not autotuned")
    return ap.parse_args()


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Read + write GB/s of a plain device-to-device copy (torch's copy of a
    resident float32 buffer): the measured reference beside the 8 TB/s
    specification for the HBM-bound stages."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def copy_probe(nbytes: int):
    """A plain device-to-device copy of known size: the reference for scaling
    the HBM byte counters of the rasterizer's kernels."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(5):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / 5
    print(json.dumps({"copy_bytes": nbytes, "ms": round(ms, 4),
                      "GBps_read_plus_write": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}), flush=True)


class PipelineStep:
    """One fwd + bwd step of the rasterizer over fixed buffers: hgs_preprocess,
    hgs_bin_sort, hgs_render_fwd, the L1 loss gradient against a seeded
    target, hgs_raster_bwd, hgs_preprocess_bwd, all on the current stream.
    Inputs are resident on the device; the entry buffers are sized by one
    untimed forward pass of this fixed scene."""

    STAGES = ["preprocess", "bin_sort", "render_fwd", "loss_grad", "raster_bwd", "preprocess_bwd"]

    def __init__(self, scene, cams, tile, batch, persistent, full_keys, dev, flags=0):
        import torch

        from paper_2406_02720_amd import binding as B
        from paper_2406_02720_amd import raster as R
        from paper_2406_02720_amd import scenes

        self.B, self.torch = B, torch
        n = scene["means"].shape[0]
        deg = scene["sh_degree"]
        self.n, self.deg, self.cameras = n, deg, cams
        self.soa = R.scene_to_soa(scene, dev)
        self.cams = ca = B.make_cameras(cams)
        self.tile = tile = tile or R.default_tile(cams)
        self.opts = opts = B.default_options(tile=tile, batch=batch, sort_full_keys=full_keys)
        self.opts.flags |= flags
        self.target = torch.cat([torch.as_tensor(t).reshape(-1) for t in scenes.target_image(cams, seed=102)]).to(dev)
        # sizing pass (not timed): entry count of this fixed scene
        fr = R.forward_pass(self.soa, n, deg, ca, opts, keys=False, render=False)
        torch.cuda.synchronize()
        self.n_dup = cap = int(fr.n_dup.item())
        del fr
        self.n_rec = n_rec = n * len(cams)
        self.tiles_total = tiles_total = B.hgs_tiles_total(ca, opts)
        npix = B.hgs_pixels_total(ca)

        self.params = B.params_struct(self.soa, n, n, deg)
        self.grads = torch.zeros_like(self.soa)
        self.gstruct = B.grads_struct(self.grads, n)
        u8, i32, i64, f32 = torch.uint8, torch.int32, torch.int64, torch.float32
        # every buffer of the step in one allocation (raster.Arena: buffers
        # the raster uses together do not compete for the same sets of the
        # address-translation caches); zeroed once, so the record gradients
        # start cleared
        a = R.Arena(dev, [
            ("records", n_rec * 64, u8), ("tiles", n_rec, i32),
            ("offsets", n_rec, i64) if full_keys else None, ("ndup", 1, i64),
            ("ws_pre", B.hgs_workspace_bytes(B.HGS_WS_PREPROCESS, n_rec, ca, opts), u8),
            ("keys", cap, i64) if full_keys else None, ("values", cap, i32),
            ("ranges", 2 * tiles_total, i32), ("order", tiles_total, i32) if persistent else None,
            ("overflow", 1, i32), ("ws_sort", B.hgs_workspace_bytes(B.HGS_WS_BIN_SORT, n_rec, ca, opts, cap), u8),
            ("images", 3 * npix, f32), ("T_final", npix, f32), ("last_idx", npix, i32), ("n_contrib", npix, i32),
            ("ws_r", B.hgs_workspace_bytes(B.HGS_WS_RENDER, n_rec, ca, opts, cap), u8),
            ("rgrad", n_rec * B.HGS_RECORD_GRAD_FLOATS, f32), ("dL", 3 * npix, f32)], zero=True)
        self.arena = a
        for name in ("records", "tiles", "ndup", "ws_pre", "values", "ranges", "overflow", "ws_sort", "images",
                     "T_final", "last_idx", "n_contrib", "ws_r", "rgrad", "dL"):
            setattr(self, name, a[name])
        self.offsets = a["offsets"] if full_keys else None
        self.keys = a["keys"] if full_keys else None
        self.order = a["order"] if persistent else None
        self.cap = cap
        self.pixels = sum(c["width"] * c["height"] for c in cams)

    def step(self, ev=None, upto=None):
        B = self.B
        stream = self.torch.cuda.current_stream().cuda_stream
        ca, opts = self.cams, self.opts

        def mark(i):
            if ev is not None:
                ev[i].record()
        mark(0)
        B.hgs_preprocess(self.params, ca, opts, self.records, self.tiles, self.offsets, self.ndup, self.ws_pre,
                         stream)
        mark(1)
        B.hgs_bin_sort(self.records, self.tiles, self.offsets, self.ndup, self.n_rec, ca, opts, self.keys,
                       self.values, self.cap, self.ranges, self.order, self.overflow, self.ws_sort, stream)
        mark(2)
        B.hgs_render_fwd(self.records, self.values, self.ranges, self.order, ca, opts, self.images, self.T_final,
                         self.last_idx, self.n_contrib, self.ws_r, stream)
        mark(3)
        B.hgs_l1_loss_grad(self.images, self.target, self.dL, stream)
        mark(4)
        # record gradients start cleared (hgs_preprocess_bwd clears them after use)
        B.hgs_raster_bwd(self.records, self.values, self.ranges, self.order, ca, opts, self.T_final,
                         self.last_idx, self.dL, self.rgrad, self.ws_r, stream)
        mark(5)
        if upto == "raster_bwd":
            return
        B.hgs_preprocess_bwd(self.params, ca, opts, self.records, self.rgrad, self.gstruct, stream)
        mark(6)

    def nonzero_gradients(self):
        """(records, kernels) with a nonzero record gradient in one step: the
        backward preprocess reads the parameters, and clears the record
        gradients, of these only.  One untimed step, looked at before its
        backward preprocess (which then runs and clears them)."""
        torch = self.torch
        self.step(upto="raster_bwd")
        nz = (self.rgrad.view(self.n_rec, -1) != 0).any(1)
        records = int(nz.sum().item())
        kernels = int(nz.view(len(self.cameras), self.n).any(0).sum().item())
        self.B.hgs_preprocess_bwd(self.params, self.cams, self.opts, self.records, self.rgrad, self.gstruct,
                                  torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        return records, kernels

    def time(self, steps, warmup):
        """(ms per whole step, {stage: ms}): whole steps back to back with
        nothing else in the stream, then a separate run with events between
        the stage calls."""
        import numpy as np
        torch = self.torch
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        assert int(self.overflow.item()) == 0
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(steps):
            self.step()
        t1.record()
        torch.cuda.synchronize()
        ms_step = t0.elapsed_time(t1) / steps
        ns = len(self.STAGES)
        stage_ms = np.zeros(ns)
        for _ in range(steps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(ns + 1)]
            self.step(ev)
            torch.cuda.synchronize()
            for i in range(ns):
                stage_ms[i] += ev[i].elapsed_time(ev[i + 1])
        stage_ms /= steps
        return ms_step, {k: float(v) for k, v in zip(self.STAGES, stage_ms)}

    def pair_counts(self, chunk: int = 32768):
        """(pairs, tested, listed, blended): `pairs` are the pixel-entry pairs
        the raster must evaluate -- for every pixel, the entries of its tile
        list up to its last blended one whose record's pixel rect contains
        the pixel (the rect test is the raster's first, per wavefront; pixels
        outside it are never evaluated); `tested` those of them whose
        Gaussian exponent passes the bound below which alpha_min cannot be
        reached (the raster's second test; only these go on to exp, the half
        factor and Eq. 10); `listed` counts every entry up to the last
        blended one, rect or not; `blended` the blended pairs.  Counted on
        the device from the step's own buffers, tile by tile (the exponent
        in float32 as the raster forms it, so a pair on the bound may
        count either way)."""
        torch = self.torch
        listed = int((self.last_idx.to(torch.int64) + 1).sum().item())
        blended = int(self.n_contrib.to(torch.int64).sum().item())
        T = int(self.opts.tile)
        dev = self.last_idx.device
        rec = self.records.view(torch.int32).view(-1, 16)
        recf = self.records.view(torch.float32).view(-1, 16)
        xr, yr = rec[:, 12].to(torch.int64), rec[:, 13].to(torch.int64)
        log2e = 1.4426950408889634
        l2amin = math.log2(float(self.opts.alpha_min))
        tested = 0
        ranges = self.ranges.view(-1, 2).to(torch.int64)
        vals = self.values.to(torch.int64)
        lin = torch.arange(T, device=dev)
        pairs = 0
        tile_off = pix_off = 0
        for cam in self.cameras:
            W, H = int(cam["width"]), int(cam["height"])
            tx, ty = (W + T - 1) // T, (H + T - 1) // T
            nt = tx * ty
            pad = torch.full((ty * T, tx * T), -1, dtype=torch.int32, device=dev)
            pad[:H, :W] = self.last_idx[pix_off:pix_off + W * H].view(H, W)
            lt = pad.view(ty, T, tx, T).permute(0, 2, 1, 3).reshape(nt, T, T)   # [tile][row][col]
            r = ranges[tile_off:tile_off + nt]
            cnt = r[:, 1] - r[:, 0]
            ends = torch.cumsum(cnt, 0)
            first = ends - cnt
            total = int(ends[-1].item()) if nt else 0
            linf = lin.to(torch.float32) + 0.5
            # entries in chunks of the camera's concatenated tile lists (no
            # array over all of its entries: a 4K view holds ~10^8)
            for a in range(0, total, chunk):
                k = torch.arange(a, min(a + chunk, total), device=dev)
                tid = torch.searchsorted(ends, k, right=True)
                pos = k - first[tid]
                rid = vals[r[tid, 0] + pos]
                ox, oy = (tid % tx) * T, (tid // tx) * T
                x0, x1 = (xr[rid] & 0xffff) - ox, (xr[rid] >> 16) - ox
                y0, y1 = (yr[rid] & 0xffff) - oy, (yr[rid] >> 16) - oy
                colm = (lin[None, :] >= x0[:, None]) & (lin[None, :] <= x1[:, None])
                rowm = (lin[None, :] >= y0[:, None]) & (lin[None, :] <= y1[:, None])
                live = lt[tid] >= pos[:, None, None].to(torch.int32)
                inr = live & rowm[:, :, None] & colm[:, None, :]
                pairs = pairs + inr.sum()
                f = recf[rid]
                hb = torch.maximum(f[:, 7], f[:, 7] + 2.0 * f[:, 11])
                p2min = (l2amin - torch.log2(hb)) - 2.0 ** -10
                dx = (linf[None, :] - x0[:, None].to(torch.float32)) - f[:, 0:1]        # [E, col]
                dy = (linf[None, :] - y0[:, None].to(torch.float32)) - f[:, 1:2]        # [E, row]
                p2a = f[:, 4:5] * (dx * dx * (-0.5 * log2e))
                p2b = f[:, 5:6] * (dx * -log2e)
                p2c = f[:, 6:7] * (-0.5 * log2e)
                p2 = (p2c[:, :, None] * dy[:, :, None] + p2b[:, None, :]) * dy[:, :, None] + p2a[:, None, :]
                ok = (p2 <= 0.0) & (p2 >= p2min[:, None, None])
                tested = tested + (inr & ok).sum()
            tile_off += nt
            pix_off += W * H
        return int(pairs), int(tested), listed, blended

    def summary(self, steps, warmup):
        ms, st = self.time(steps, warmup)
        fwd = st["preprocess"] + st["bin_sort"] + st["render_fwd"]
        bwd = st["raster_bwd"] + st["preprocess_bwd"]
        return {"entries": self.n_dup, "ms_per_step": round(ms, 4),
                "Mpix_s": round(self.pixels / (ms * 1e-3) / 1e6, 2),
                "fwd_bwd_over_fwd": round((fwd + bwd) / fwd, 3),
                "stage_ms": {k: round(v, 4) for k, v in st.items()}}


def extra_workloads(args, dev):
    """The other measurements the method's workloads call for, each a
    PipelineStep on its own scene (freed before the next):
      - efficient_rasterizer: the 1M-kernel 1080p scene with one half of
        half the kernels transparent, with the half-aware valid region
        against both halves splatted with the full box (the paper's
        rendering-speed ablation of its efficient rasterizer);
      - equal_opacities: the headline scene with alpha2 := alpha1 (standard
        Gaussians: the raster skips the half factor);
      - stress: 3M kernels (5 % large splats) over 8 views at 3840x2160 in one
        batched call per stage (persistent raster), per-stage times, and the
        same through the autograd Rasterizer."""
    import torch

    from paper_2406_02720_amd import binding as B
    from paper_2406_02720_amd import raster as R
    from paper_2406_02720_amd import scenes

    out = {}
    scene, cams = scenes.make_config(3)
    clear = scenes.with_transparent_halves(scene)
    half = PipelineStep(clear, cams, args.tile, args.batch, args.persistent, False, dev)
    a = half.summary(args.steps, args.warmup)
    del half
    full = PipelineStep(clear, cams, args.tile, args.batch, args.persistent, False, dev, flags=B.HGS_FLAG_FULL_BOX)
    b = full.summary(args.steps, args.warmup)
    del full
    out["efficient_rasterizer"] = {
        "workload": "1M half-Gaussians, 1920x1080, half of the kernels with one transparent half",
        "half_aware": a, "full_box": b,
        "speedup": round(b["ms_per_step"] / a["ms_per_step"], 3),
        "entries_ratio": round(b["entries"] / max(a["entries"], 1), 3)}
    eq = PipelineStep(scenes.with_equal_opacities(scene), cams, args.tile, args.batch, args.persistent, False, dev)
    out["equal_opacities"] = dict(workload="1M Gaussians (alpha2 = alpha1), 1920x1080",
                                  **eq.summary(args.steps, args.warmup))
    del eq, scene, clear
    torch.cuda.empty_cache()
    if not args.no_stress:
        scene, cams = scenes.make_config(5)
        st = PipelineStep(scene, cams, args.tile, args.batch, True, False, dev)
        k = max(3, args.steps // 4)
        r = st.summary(k, 2)
        planes = st.soa.clone().requires_grad_(True)
        target = st.target
        del st
        torch.cuda.empty_cache()
        rast = R.Rasterizer(cams, scene["sh_degree"], tile=args.tile or None, batch=args.batch, persistent=True)

        def auto_step():
            planes.grad = None
            loss = (rast(planes) - target).abs().mean()
            loss.backward()

        auto_step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            auto_step()
        e1.record()
        torch.cuda.synchronize()
        r["autograd_ms_per_step"] = round(e0.elapsed_time(e1) / k, 4)
        out["stress"] = dict(workload="3M half-Gaussians (5% large splats), 8 views of 3840x2160, persistent raster",
                             views=len(cams), pixels=sum(c["width"] * c["height"] for c in cams), steps=k, **r)
        del planes, rast, scene
        torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(views would shard across GPUs with one gradient all-reduce; not built).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2406_02720_amd import binding as B
    from paper_2406_02720_amd import raster as R
    from paper_2406_02720_amd import scenes

    B.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    scene, cams = scenes.make_config(args.config)
    n = scene["means"].shape[0]
    deg = scene["sh_degree"]
    run = PipelineStep(scene, cams, args.tile, args.batch, args.persistent, args.full_keys, dev)
    tile = run.tile
    soa, target, ca, opts = run.soa, run.target, run.cams, run.opts
    n_dup, n_rec, tiles_total = run.n_dup, run.n_rec, run.tiles_total
    ms_step, st = run.time(args.steps, args.warmup)
    stage_names = PipelineStep.STAGES
    if args.no_pair_counts:     # (profiler runs: the count launches thousands of small kernels)
        pairs = tested = listed = blended = 0
    else:
        pairs, tested, listed, blended = run.pair_counts()
    ns = len(stage_names)

    fwd_ms = st["preprocess"] + st["bin_sort"] + st["render_fwd"]
    bwd_ms = st["raster_bwd"] + st["preprocess_bwd"]
    W = sum(c["width"] * c["height"] for c in cams)
    value = W / (ms_step * 1e-3) / 1e6

    # ---- algorithmic work per stage
    sh_floats = 3 * (deg + 1) ** 2
    param_bytes = 4 * (15 + sh_floats)
    tb = max(0, math.ceil(math.log2(max(tiles_total, 1))))
    bytes_pre = n * param_bytes + n_rec * (64 + 4) + n_rec * (4 + 4 + 8)
    if args.full_keys:
        passes = (32 + tb + 7) // 8
        bytes_sort = (n_rec * 28 + n_dup * 12 + passes * n_dup * 24 + n_dup * 8 + tiles_total * 8)
    else:
        # placement: what it must move at least -- depth keys (16 B) and four
        # record passes (16 B each) per record, each record's tile rectangle
        # read once (16 B), 4 B written per entry, the ranges (8 B per tile)
        passes = 0
        bytes_sort = n_rec * (16 + 4 * 16 + 16) + 4 * n_dup + 8 * tiles_total
    # backward preprocess: every kernel's parameter gradients written, every
    # record's 48 B of gradients and every kernel's 15 geometry parameters
    # read; the SH coefficients read, and the record gradients cleared, only
    # where some record gradient is nonzero (the kernel skips the rest:
    # culled records and those no pixel blended)
    nz_rec, nz_kernels = run.nonzero_gradients()
    bytes_pbwd = (n * param_bytes + n_rec * 48 + n * 4 * 15 + nz_kernels * 4 * sh_floats + nz_rec * 48)
    # FP32 operations of one pair, written out (fma = 2): the exponent test
    # of every pair in a record's rect (row offset, the quadratic in it, two
    # comparisons), the rest of the evaluation for the pairs past it (exp,
    # the alpha_min bound, half factor, Eq. 10 opacity, clamp) and, for a
    # blended pair, compositing.  The backward must replay only the blended
    # pairs (which pairs blended is known from the forward pass), each in
    # full, and adds the gradient formulas.
    F_TEST, F_EVAL, F_BLEND, F_GRAD = 8.0, 34.0, 9.0, 75.0
    flops_fwd = pairs * F_TEST + tested * F_EVAL + blended * F_BLEND
    flops_bwd = blended * (F_TEST + F_EVAL + F_BLEND + F_GRAD)
    roof = {}
    copy_gbs = copy_bandwidth()

    def add(name, bound, amount):
        ms = float(st[name])
        if bound == "hbm":
            a = amount / (ms * 1e-3) / 1e9
            roof[name] = dict(bound="hbm", achieved=round(a, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                              frac=round(a / HBM_PEAK_GBS, 4), frac_of_copy=round(a / copy_gbs, 4),
                              bytes=int(amount), ms=round(ms, 4))
        else:
            a = amount / (ms * 1e-3) / 1e12
            roof[name] = dict(bound="alu", achieved=round(a, 2), peak=FP32_VECTOR_PEAK_TF, unit="TFLOP/s",
                              frac=round(a / FP32_VECTOR_PEAK_TF, 4),
                              frac_of_unpacked=round(a / FP32_UNPACKED_PEAK_TF, 4),
                              flops=float(amount), ms=round(ms, 4))
    add("preprocess", "hbm", bytes_pre)
    add("bin_sort", "hbm", bytes_sort)
    add("render_fwd", "alu", flops_fwd)
    add("raster_bwd", "alu", flops_bwd)
    add("preprocess_bwd", "hbm", bytes_pbwd)
    # the dominant kernel: the longest single-kernel stage
    dominant = max(("render_fwd", "raster_bwd", "preprocess_bwd"), key=lambda k: st[k])
    roofline = {k: v for k, v in roof[dominant].items() if k not in ("ms", "bytes", "flops")}
    roofline["kernel"] = dominant
    kname = {"render_fwd": "render_fwd", "raster_bwd": "render_bwd", "preprocess_bwd": "preprocess_bwd"}[dominant]
    if dominant in ("render_fwd", "raster_bwd"):
        kname += f"_persistent_kernel<{tile},{args.batch // 64}>" if args.persistent else \
            f"_kernel<{tile},{args.batch // 64}>"
    roofline["traffic"] = measured_traffic(kname)

    if args.stages:
        for name in stage_names:
            print(f"{name:15s} {st[name]:8.3f} ms", file=sys.stderr)
        print(f"n_dup {n_dup}  entry passes {passes}  pairs {pairs} (tested {tested}, listed {listed})  "
              f"blended {blended}  "
              f"step {ms_step:.3f} ms", file=sys.stderr)
        print(json.dumps(roof), file=sys.stderr)

    auto = None
    if not args.no_autograd:
        auto = autograd_bench(args, soa, deg, cams, target, ms_step)
    train = None
    if args.train:
        train = train_bench(args, n, deg, run.records, run.rgrad, ca, opts, cams)
    del run, soa, target
    torch.cuda.empty_cache()
    multi = None if args.no_multiview else multiview(args)
    extra = None if args.no_extra else extra_workloads(args, dev)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(scene, cams, args.cpu_pixels)

    out = {
        "metric": "fwd+bwd Mpixel/s at 1M half-Gaussians 1080p; bwd/fwd time ratio; % HBM roof",
        "value": round(value, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS.get(args.config, str(args.config)), "n_kernels": n,
                   "views": len(cams), "pixels": W, "tile": tile, "batch": args.batch,
                   "entries": n_dup, "sort": "full_keys" if args.full_keys else "placement",
                   "raster": "persistent" if args.persistent else "per_tile"},
        "bwd_over_fwd": round(bwd_ms / fwd_ms, 3),
        "fwd_bwd_over_fwd": round((fwd_ms + bwd_ms) / fwd_ms, 3),
        "stage_ms": {k: round(float(v), 4) for k, v in st.items()},
        "roofline": roofline,
        "roofline_stages": roof,
        "work": {"pairs_in_rect": pairs, "pairs_past_exponent_test": tested, "pairs_listed": listed,
                 "blended": blended, "records_with_gradient": nz_rec, "kernels_with_gradient": nz_kernels},
        "copy_GBps": round(copy_gbs, 1),
        "cpu_baseline": cpu,
        "autograd": auto,
        "multiview": multi,
        "workloads": extra,
    }
    if train is not None:
        out["train"] = train
    print(json.dumps(out), flush=True)


def autograd_bench(args, soa, deg, cams, target, ms_step):
    """The same fwd + bwd through torch.autograd, as a training loop calls
    it: a Rasterizer over the parameter planes (requires_grad), the L1 loss
    written with torch operations, loss.backward().  Includes the
    Rasterizer's end-of-forward overflow check (one small read-back) and
    torch's loss kernels."""
    import torch

    from paper_2406_02720_amd import raster as R

    planes = soa.clone().requires_grad_(True)
    rast = R.Rasterizer(cams, deg, tile=args.tile or None, batch=args.batch, persistent=args.persistent)

    def step():
        planes.grad = None
        img = rast(planes)
        loss = (img - target).abs().mean()
        loss.backward()

    for _ in range(max(args.warmup, 2)):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    del planes
    return {"ms_per_step": round(ms, 4), "over_native_step": round(ms / ms_step, 3),
            "overflow_reruns": rast.overflows, "entry_capacity": rast.capacity,
            "what": "Rasterizer(planes) + torch L1 loss + loss.backward(), same workload and launch configuration"}


def train_bench(args, n, deg, records, rgrad, ca, opts, cams):
    """The step after the backward pass on the bench's kernels: one fused
    Adam step over every raw plane (HBM-bound: per kernel and plane 16 B
    read, 12 B written, plus 4 B for each of the 5 activated planes), the
    densification statistics of one view, and one densify / prune call."""
    import numpy as np
    import torch

    from paper_2406_02720_amd import binding as B
    from paper_2406_02720_amd import scenes
    from paper_2406_02720_amd import train as TR

    dev = torch.device("cuda:0")
    st = scenes.train_state(n, deg, extent=2.0, seed=77)
    planes = np.concatenate([st["raw"][k] for k in ("means", "scales", "quats", "normals", "opac1", "opac2", "sh")])
    grads = np.concatenate([st["grads"][k] for k in ("means", "scales", "quats", "normals", "opac1", "opac2", "sh")])
    state = TR.TrainState(torch.from_numpy(planes).to(dev), n, deg, extent=2.0)
    g = torch.from_numpy(grads).to(dev)
    del planes, grads
    P = g.shape[0]
    reps = max(args.steps, 5)
    for _ in range(3):
        state.adam_step(g)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        state.adam_step(g)
    e1.record()
    torch.cuda.synchronize()
    adam_ms = e0.elapsed_time(e1) / reps
    adam_bytes = n * (P * 28 + 5 * 4)
    stream = torch.cuda.current_stream().cuda_stream
    e0.record()
    for _ in range(reps):
        B.hgs_densify_stats(records, rgrad, ca, opts, n, state.grad_accum, state.grad_count, state.max_radii,
                            stream)
    e1.record()
    torch.cuda.synchronize()
    stats_ms = e0.elapsed_time(e1) / reps
    state.grad_accum.copy_(torch.from_numpy(st["accum"]).to(dev))
    state.grad_count.copy_(torch.from_numpy(st["count"]).to(dev))
    state.max_radii.copy_(torch.from_numpy(st["radii"]).to(dev))
    smp = torch.from_numpy(np.ascontiguousarray(st["samples"])).to(dev)
    torch.cuda.synchronize()
    e0.record()
    n_new = state.densify(samples=smp)
    e1.record()
    torch.cuda.synchronize()
    dens_ms = e0.elapsed_time(e1)
    a = adam_bytes / (adam_ms * 1e-3) / 1e9
    return {"n_kernels": n, "planes": P, "adam_ms": round(adam_ms, 4),
            "adam_roofline": {"bound": "hbm", "achieved": round(a, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(a / HBM_PEAK_GBS, 4), "bytes": adam_bytes},
            "densify_stats_ms": round(stats_ms, 4), "densify_ms_incl_readback": round(dens_ms, 4),
            "densify_n_out": n_new}


def multiview(args):
    """500k half-Gaussians, SH degree 3, 16 orbit views of uneven size: the
    whole fwd + loss + bwd step over all views as one HIP-graph replay (one
    launch per stage, in the launch configuration the autotuner picks)
    against a loop over the views (one call chain per view, gradients summed
    over views), both eager and with one captured graph per view, in either
    raster schedule (the faster is the baseline).  Returns the timings and
    the ratios."""
    import torch

    from paper_2406_02720_amd import batch as BT
    from paper_2406_02720_amd import binding as B
    from paper_2406_02720_amd import raster as R
    from paper_2406_02720_amd import scenes

    dev = torch.device("cuda:0")
    scene, cams = scenes.make_config(4)
    n = scene["means"].shape[0]
    deg = scene["sh_degree"]
    soa = R.scene_to_soa(scene, dev)
    tgt = [torch.as_tensor(t).reshape(-1).to(dev) for t in scenes.target_image(cams, seed=102)]
    target = torch.cat(tgt)
    W = sum(c["width"] * c["height"] for c in cams)
    tile, batch, persistent, tuned, tune_s = args.tile or R.default_tile(cams), args.batch, True, None, None
    if not args.no_autotune:
        t0 = time.perf_counter()
        tile, batch, persistent, tuned = BT.autotune(soa, n, deg, cams, target, cache_path=args.autotune or None)
        tune_s = time.perf_counter() - t0
        tuned = {k: round(v, 4) for k, v in tuned.items()}
    K = args.multiview_steps

    br = BT.BatchedRasterizer(soa, n, deg, cams, tile=tile, batch=batch, persistent=persistent)
    loss = BT.l1_loss_grad(target)
    br.capture(loss)
    assert not br.replay()
    ms_batched = BT.time_steps(lambda: br.graph.replay(), K, 3)
    ms_batched_eager = BT.time_steps(lambda: br.step(loss), K, 3)
    torch.cuda.synchronize()
    img_batched = br.images.clone()
    grads_batched = br.grads.clone()
    del br
    torch.cuda.empty_cache()

    # per-view loop; the L1 gradient scale is that of the whole batch so that
    # the summed gradients are the batched ones
    inv = 1.0 / float(target.numel())

    def view_loss(t):
        def fn(images, dL):
            B.hgs_l1_loss_grad(images, t, dL, torch.cuda.current_stream().cuda_stream, scale=inv)
        return fn

    losses = [view_loss(t) for t in tgt]
    total = torch.zeros_like(soa)
    loop = {}
    img_diff = grad_diff = 0.0
    gscale = float(grads_batched.abs().max().item())
    # the loop in both raster schedules, at the batched call's tuned tile
    # size and at 16 pixels (one view alone has 16x fewer tiles to balance);
    # the fastest is the baseline
    for tl, sched in [(t_, p_) for t_ in sorted({tile, 16}) for p_ in (True, False)]:
        views = [BT.BatchedRasterizer(soa, n, deg, [c], tile=tl, batch=batch, persistent=sched) for c in cams]

        def loop_eager():
            total.zero_()
            for v, lf in zip(views, losses):
                v.step(lf)
                total.add_(v.grads)

        ms_eager = BT.time_steps(loop_eager, K, 3)
        img_loop = torch.cat([v.images for v in views])
        img_diff = max(img_diff, float((img_loop - img_batched).abs().max().item()))
        grad_diff = max(grad_diff, float((total - grads_batched).abs().max().item()) / max(gscale, 1e-30))
        for v, lf in zip(views, losses):
            v.capture(lf)

        def loop_graph():
            total.zero_()
            for v in views:
                v.graph.replay()
                total.add_(v.grads)

        ms_graph = BT.time_steps(loop_graph, K, 3)
        loop[BT._config_name(tl, batch, sched)] = {"eager_ms": round(ms_eager, 4), "graph_ms": round(ms_graph, 4)}
        del views, img_loop
        torch.cuda.empty_cache()
    ms_loop = min(v["eager_ms"] for v in loop.values())
    ms_loop_graph = min(v["graph_ms"] for v in loop.values())
    return {
        "workload": "500k half-Gaussians, SH deg 3, 16 orbit views {640x480,1024x768,1297x840,1600x1064}",
        "pixels": W, "tile": tile, "batch": batch, "raster": "persistent" if persistent else "per_tile",
        "autotune_ms": tuned, "autotune_s": None if tune_s is None else round(tune_s, 2),
        "batched_graph_ms": round(ms_batched, 4), "batched_eager_ms": round(ms_batched_eager, 4),
        "loop_eager_ms": round(ms_loop, 4), "loop_graph_ms": round(ms_loop_graph, 4), "loop_by_config": loop,
        "batched_Mpix_s": round(W / (ms_batched * 1e-3) / 1e6, 2),
        "speedup_vs_loop_eager": round(ms_loop / ms_batched, 3),
        "speedup_vs_loop_graph": round(ms_loop_graph / ms_batched, 3),
        "image_max_diff_vs_loop": img_diff, "grad_max_rel_diff_vs_loop": grad_diff,
    }


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(scene, cams, n_pix):
    """The FP64 oracle, as it stands, on a bounded sample of the same
    workload: forward and backward (autograd) of seeded pixels of view 0
    over all kernels, run for n_pix / 4 and for n_pix pixels.  The
    difference of the two runs is the per-pixel cost; the rest of the small
    run is the per-frame cost (projection of every kernel, forward and
    backward), so a full frame is extrapolated as per-frame + per-pixel x
    W x H.  Per-pixel work is independent, so the extrapolation is linear."""
    import numpy as np
    import torch

    from oracle import hgs_oracle as O
    from paper_2406_02720_amd import scenes

    o = O.options()
    cam = cams[0]
    small = max(n_pix // 4, 1)
    pix = scenes.sample_pixels(cam, n_pix, seed=5)
    w = np.random.default_rng(1).normal(size=(n_pix, 3))
    t0 = time.perf_counter()
    O.render_grad(scene, [cam], [w[:small]], o, pixels=[pix[:small]])
    t_small = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.render_grad(scene, [cam], [w], o, pixels=[pix])
    t_big = time.perf_counter() - t0
    per_pix = max(t_big - t_small, 1e-9) / (n_pix - small)
    per_frame = max(t_small - per_pix * small, 0.0)
    npx = cam["width"] * cam["height"]
    full = per_frame + per_pix * npx
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {"value": round(npx / full / 1e6, 9), "unit": "Mpixel/s",
            "cores": torch.get_num_threads(), "kind": "oracle",
            "cpu_model": _cpu_model(), "affinity_cores": affinity,
            "per_frame_s": round(per_frame, 2), "per_pixel_ms": round(per_pix * 1e3, 3),
            "sample": f"fwd+bwd of {small} and of {n_pix} seeded pixels of view 0 over all kernels "
                      f"({t_small:.1f} s + {t_big:.1f} s measured); full frame extrapolated as per-frame "
                      f"{per_frame:.1f} s + {npx} px x {per_pix * 1e3:.2f} ms = {full:.0f} s"}


if __name__ == "__main__":
    main()
