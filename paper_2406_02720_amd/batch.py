"""Multi-view training step of the half-Gaussian rasterizer: all views in one
call per stage, the persistent tile scheduler, HIP-graph capture of the whole
forward + loss + backward step, and an autotuner for the tile size, the
raster schedule and the batch depth.

Every view shares one preprocess launch (parameters read once), one sort (one
global tile numbering) and one raster launch per direction.  A captured step
replays with no host work at all; the entry capacity is fixed at capture, and
an overflow (more entries than capacity, reported on the device) is detected
after replay and answered by re-capturing with more room.
"""
from __future__ import annotations

import json
import math
import os
import time

import torch

from . import binding as B
from . import raster as R


def _bytes(n, dev):
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device=dev)


class BatchedRasterizer:
    """Forward + backward of one scene over many views with fixed buffers.

    ``soa`` is the structure-of-arrays parameter tensor (see
    ``raster.soa_from_natural``); ``cameras`` a list of camera dicts (at most
    HGS_MAX_CAMERAS).  ``capacity`` bounds the number of (tile, kernel)
    entries; by default it is measured once and given ``headroom``."""

    def __init__(self, soa, n, sh_degree, cameras, tile=16, batch=256, capacity=None, headroom=1.25,
                 persistent=True, full_keys=False):
        self.dev = soa.device
        self.soa, self.n, self.deg = soa, n, sh_degree
        self.cameras = list(cameras)
        self.cams = B.make_cameras(self.cameras)
        self.opts = B.default_options(tile=tile, batch=batch, sort_full_keys=full_keys)
        self.persistent = persistent
        nc = len(self.cameras)
        self.n_rec = n * nc
        self.tiles_total = B.hgs_tiles_total(self.cams, self.opts)
        self.npix = B.hgs_pixels_total(self.cams)
        dev = self.dev
        self.params = B.params_struct(soa, n, soa.shape[1], sh_degree)
        self.grads = torch.zeros_like(soa)
        self.gstruct = B.grads_struct(self.grads, soa.shape[1])
        self.graph = None
        if capacity is None:    # one preprocess into throw-away buffers sizes the entries
            records = _bytes(self.n_rec * B.HGS_RECORD_BYTES, dev)
            tiles = torch.empty(max(self.n_rec, 1), dtype=torch.int32, device=dev)
            n_dup = torch.zeros(1, dtype=torch.int64, device=dev)
            ws = _bytes(B.hgs_workspace_bytes(B.HGS_WS_PREPROCESS, self.n_rec, self.cams, self.opts), dev)
            B.hgs_preprocess(self.params, self.cams, self.opts, records, tiles, None, n_dup, ws, self._stream())
            capacity = max(1, int(math.ceil(int(n_dup.item()) * headroom)))
            del records, tiles, n_dup, ws
        self._alloc(capacity)

    @staticmethod
    def _stream():
        return torch.cuda.current_stream().cuda_stream

    def _alloc(self, capacity):
        """Every buffer of the step, for ``capacity`` entries, carved from one
        zeroed allocation (raster.Arena); the per-record gradients start
        cleared and every backward pass leaves them cleared."""
        self.capacity = int(capacity)
        full = bool(self.opts.flags & B.HGS_FLAG_SORT_FULL_KEYS)
        u8, i32, i64, f32 = torch.uint8, torch.int32, torch.int64, torch.float32
        n_rec, npix, nt, cams, opts = self.n_rec, self.npix, max(self.tiles_total, 1), self.cams, self.opts
        a = R.Arena(self.dev, [
            ("records", n_rec * B.HGS_RECORD_BYTES, u8), ("tiles", n_rec, i32),
            ("offsets", n_rec, i64) if full else None, ("n_dup", 1, i64),
            ("ws_pre", B.hgs_workspace_bytes(B.HGS_WS_PREPROCESS, n_rec, cams, opts), u8),
            ("keys", self.capacity, i64) if full else None, ("values", self.capacity, i32),
            ("ranges", 2 * nt, i32), ("order", nt, i32) if self.persistent else None, ("overflow", 1, i32),
            ("ws_sort", B.hgs_workspace_bytes(B.HGS_WS_BIN_SORT, n_rec, cams, opts, self.capacity), u8),
            ("images", 3 * npix, f32), ("T_final", npix, f32), ("last_idx", npix, i32),
            ("n_contrib", npix, i32), ("ws_r", B.hgs_workspace_bytes(B.HGS_WS_RENDER, n_rec, cams, opts, capacity), u8),
            ("rgrad", max(n_rec, 1) * B.HGS_RECORD_GRAD_FLOATS, f32), ("dL", 3 * npix, f32)], zero=True)
        self.arena = a
        for name in ("records", "tiles", "n_dup", "ws_pre", "values", "ranges", "overflow", "ws_sort", "images",
                     "T_final", "last_idx", "n_contrib", "ws_r", "rgrad", "dL"):
            setattr(self, name, a[name])
        self.offsets = a["offsets"] if full else None
        self.keys = a["keys"] if full else None
        self.order = a["order"] if self.persistent else None

    # -- stages ------------------------------------------------------------
    def forward(self):
        st = self._stream()
        B.hgs_preprocess(self.params, self.cams, self.opts, self.records, self.tiles, self.offsets, self.n_dup,
                         self.ws_pre, st)
        B.hgs_bin_sort(self.records, self.tiles, self.offsets, self.n_dup, self.n_rec, self.cams, self.opts,
                       self.keys, self.values, self.capacity, self.ranges, self.order, self.overflow,
                       self.ws_sort, st)
        B.hgs_render_fwd(self.records, self.values, self.ranges, self.order, self.cams, self.opts, self.images,
                         self.T_final, self.last_idx, self.n_contrib, self.ws_r, st)

    def backward(self):
        st = self._stream()
        B.hgs_raster_bwd(self.records, self.values, self.ranges, self.order, self.cams, self.opts, self.T_final,
                         self.last_idx, self.dL, self.rgrad, self.ws_r, st)
        B.hgs_preprocess_bwd(self.params, self.cams, self.opts, self.records, self.rgrad, self.gstruct, st)

    def step(self, loss_grad):
        """forward; loss_grad(images, dL) writes dL/dimages into dL; backward."""
        self.forward()
        loss_grad(self.images, self.dL)
        self.backward()

    # -- graph ---------------------------------------------------------------
    def capture(self, loss_grad):
        """Capture step(loss_grad) in a HIP graph (after two eager warm-ups on
        a side stream)."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(2):
                self.step(loss_grad)
        torch.cuda.current_stream().wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step(loss_grad)
        self.graph = g
        self._loss_grad = loss_grad
        return g

    def replay(self, check=True):
        """Replay the captured step; with ``check``, read the overflow flag and
        re-capture with twice the capacity when the entries did not fit (the
        step is then run again)."""
        self.graph.replay()
        if check and int(self.overflow.item()) != 0:
            need = int(self.n_dup.item())
            self._alloc(max(2 * self.capacity, int(need * 1.25)))
            self.capture(self._loss_grad)
            self.graph.replay()
            return True
        return False

    # -- views ---------------------------------------------------------------
    def image(self, c):
        off = sum(self.cameras[i]["width"] * self.cameras[i]["height"] for i in range(c))
        w, h = self.cameras[c]["width"], self.cameras[c]["height"]
        return self.images[3 * off:3 * (off + w * h)].view(3, h, w)


def l1_loss_grad(target):
    """dL/dimages of the mean L1 loss against ``target`` (packed like
    images), by the library's hgs_l1_loss_grad on the current stream."""

    def fn(images, dL):
        B.hgs_l1_loss_grad(images, target, dL, torch.cuda.current_stream().cuda_stream)
    return fn


def time_steps(run, steps=10, warmup=3):
    """Average milliseconds of run() over ``steps`` after ``warmup``."""
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        run()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


# ---------------------------------------------------------------------------
# autotuner
# ---------------------------------------------------------------------------
TILES = (8, 16, 32)
BATCHES = (128, 256, 512)
SCHEDULES = (True, False)      # persistent longest-first grid, one workgroup per tile


def shape_class(n, cameras):
    """Cache key: kernel count and pixel count rounded to powers of two, and
    the number of views (outputs never depend on the choice, only speed)."""
    pix = sum(c["width"] * c["height"] for c in cameras)
    return f"n{2 ** round(math.log2(max(n, 1)))}_p{2 ** round(math.log2(max(pix, 1)))}_v{len(cameras)}"


def _config_name(tile, batch, persistent):
    return f"{tile}x{batch}{'p' if persistent else 'g'}"


def autotune(soa, n, sh_degree, cameras, target, cache_path=None, steps=5, warmup=2, tiles=TILES,
             batches=BATCHES, schedules=SCHEDULES):
    """Time the graph-captured step and pick the fastest launch
    configuration: first every (tile size, raster schedule) at the default
    batch depth, then every batch depth at the best of those (the batch depth
    -- entry ids a raster wavefront fetches per round -- matters least).
    Returns (tile, batch, persistent, {config: ms}), config names
    "<tile>x<batch>p" (persistent grid) or "...g" (one workgroup per tile);
    results are cached per shape class in ``cache_path`` (JSON)."""
    key = shape_class(n, cameras)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            e = cache[key]
            return e["tile"], e["batch"], e["persistent"], e["ms"]
    loss = l1_loss_grad(target)
    ms = {}

    def run(t, b, p):
        name = _config_name(t, b, p)
        if name not in ms:
            br = BatchedRasterizer(soa, n, sh_degree, cameras, tile=t, batch=b, persistent=p)
            br.capture(loss)
            ms[name] = time_steps(lambda: br.graph.replay(), steps, warmup)
            del br
        return ms[name]

    b0 = 256 if 256 in batches else batches[0]
    t, p = min(((t, p) for t in tiles for p in schedules), key=lambda tp: run(tp[0], b0, tp[1]))
    b = min(batches, key=lambda bb: run(t, bb, p))
    if cache_path:
        cache[key] = {"tile": t, "batch": b, "persistent": p, "ms": ms}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return t, b, p, ms
