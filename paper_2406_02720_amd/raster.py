"""Rasterizer pipeline over libhgs with torch-owned device memory, and its
``torch.autograd.Function``.

Forward: hgs_preprocess -> (read the entry count) -> hgs_bin_sort ->
hgs_render_fwd.  The state kept for backward is the records, the sorted
values, the tile ranges, and per pixel the final transmittance and the
position of the last blended entry -- no per-pair blend history.
Backward: hgs_render_bwd.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import binding as B

BASE_PLANES = 15  # means 3, scales 3, quats 4, normals 3, opac1, opac2


def sh_planes(sh_degree: int) -> int:
    return 3 * (sh_degree + 1) ** 2


def soa_from_natural(means, scales, quats, normals, opac1, opac2, sh) -> torch.Tensor:
    """Pack natural-layout tensors ([N,3], [N,4], [N], [N,K,3]) into one
    float32 structure-of-arrays tensor of planes, stride N."""
    n = means.shape[0]
    planes = [means.T, scales.T, quats.T, normals.T, opac1.reshape(1, n), opac2.reshape(1, n),
              sh.reshape(n, sh.shape[1] * sh.shape[2]).T]
    return torch.cat(planes, 0).to(torch.float32).contiguous()


def natural_from_soa(soa: torch.Tensor, K: int):
    n = soa.shape[1]
    return (soa[0:3].T, soa[3:6].T, soa[6:10].T, soa[10:13].T, soa[13], soa[14],
            soa[15:15 + 3 * K].T.reshape(n, K, 3))


def scene_to_soa(scene: dict, device="cuda") -> torch.Tensor:
    t = {k: torch.as_tensor(np.asarray(scene[k], np.float32)) for k in
         ("means", "scales", "quats", "normals", "opac1", "opac2", "sh")}
    return soa_from_natural(t["means"], t["scales"], t["quats"], t["normals"], t["opac1"], t["opac2"],
                            t["sh"]).to(device)


def _stream():
    return torch.cuda.current_stream().cuda_stream


@dataclass
class Frame:
    """Device buffers of one forward pass (all views)."""
    soa: torch.Tensor
    n: int
    sh_degree: int
    cams: object
    opts: object
    records: torch.Tensor
    tiles: torch.Tensor
    offsets: torch.Tensor
    n_dup: torch.Tensor
    keys: torch.Tensor
    values: torch.Tensor
    ranges: torch.Tensor
    overflow: torch.Tensor
    images: torch.Tensor
    T_final: torch.Tensor
    last_idx: torch.Tensor
    n_contrib: torch.Tensor
    capacity: int
    ws_render: torch.Tensor
    tile_order: torch.Tensor | None = None
    depth: torch.Tensor | None = None
    params: object | None = None      # the hgs_params the frame was rendered with
    filter3d: torch.Tensor | None = None
    record_grads: torch.Tensor | None = None   # cleared per-record gradient buffer for the backward pass

    def image(self, c: int) -> torch.Tensor:
        """[3,H,W] view of camera c's image."""
        off = 0
        for i in range(c):
            off += self.cams[i].width * self.cams[i].height
        w, h = self.cams[c].width, self.cams[c].height
        return self.images[3 * off:3 * off + 3 * w * h].view(3, h, w)

    def per_pixel(self, t: torch.Tensor, c: int) -> torch.Tensor:
        off = 0
        for i in range(c):
            off += self.cams[i].width * self.cams[i].height
        w, h = self.cams[c].width, self.cams[c].height
        return t[off:off + w * h].view(h, w)


def _bytes(n: int, device) -> torch.Tensor:
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device=device)


def default_tile(cameras, min_tiles: int = 1024) -> int:
    """Tile edge for views of these sizes: 32 pixels while the 32-pixel tiles
    still number at least `min_tiles` (four workgroups per compute unit),
    otherwise 16.  Larger tiles have fewer entries (a third at 1080p: the
    sort and the per-entry raster work shrink), but below about four tiles
    per CU the raster leaves the chip underfilled (1M kernels at 1920x1080,
    2040 tiles: 1.60 ms per fwd + bwd step at 32 pixels against about
    1.9 ms at 16; 100k kernels at 1280x720, 920 tiles: 1.21 ms at 32, 0.97 ms
    at 16)."""
    n32 = sum(((int(c["width"]) + 31) // 32) * ((int(c["height"]) + 31) // 32) for c in cameras)
    return 32 if n32 >= min_tiles else 16


class Arena:
    """Device buffers carved from one allocation, back to back at 256-byte
    alignment.  Separate large allocations start at equally aligned virtual
    addresses, and buffers a kernel uses together then compete for the same
    sets of the compute units' address-translation caches; carved from one
    allocation their pages follow one another (measured on the backward
    raster, 1M kernels at 1080p: 6.5x fewer translation misses, 0.69 ->
    0.62 ms).  ``specs``: (name, element count, dtype) triples, None entries
    skipped; ``zero`` clears the whole allocation."""

    def __init__(self, device, specs, zero: bool = False):
        specs = [sp for sp in specs if sp is not None]
        offs, off = [], 0
        for _, numel, dt in specs:
            nbytes = max(int(numel), 1) * torch.empty((), dtype=dt).element_size()
            offs.append((off, nbytes))
            off += (nbytes + 255) // 256 * 256
        make = torch.zeros if zero else torch.empty
        self.base = make(max(off, 1), dtype=torch.uint8, device=device)
        self.views = {name: self.base[o:o + nb].view(dt) for (name, _, dt), (o, nb) in zip(specs, offs)}

    def __getitem__(self, name):
        return self.views[name]


def forward_pass(soa: torch.Tensor, n: int, sh_degree: int, cams, opts, capacity: int | None = None,
                 persistent: bool = True, keys: bool = True, depth: bool = False, params=None,
                 filter3d: torch.Tensor | None = None, render: bool = True) -> Frame:
    """Run the forward rasterizer.  ``cams`` is a C camera array from
    ``binding.make_cameras``; ``opts`` an ``hgs_options``.  With
    ``capacity`` None the entry count is read back (one synchronisation) and
    the key buffers are sized exactly; otherwise they have ``capacity``
    entries and an overflow is reported in ``frame.overflow``.  With
    ``persistent`` the raster takes tiles longest-list first from a
    persistent grid; ``keys`` False skips the 64-bit sort keys (the raster
    does not need them); ``depth`` adds the blended depth per pixel;
    ``params`` (an hgs_params) overrides the parameter planes taken from
    ``soa`` (which then only gives the device and the gradient layout);
    ``filter3d`` (float32 [n] on the device) is the Mip-Splatting 3-D
    filter variance per kernel; ``render`` False stops after the sort (the
    per-pixel outputs are left unwritten)."""
    dev = soa.device
    nc = len(cams)
    n_rec = n * nc
    stream = _stream()
    if params is None:
        params = B.params_struct(soa, n, soa.shape[1], sh_degree)
    if filter3d is not None:
        params.filter3d = filter3d.data_ptr()
    records = _bytes(n_rec * B.HGS_RECORD_BYTES, dev)
    tiles = torch.empty(max(n_rec, 1), dtype=torch.int32, device=dev)
    full = bool(opts.flags & B.HGS_FLAG_SORT_FULL_KEYS)
    # per-record entry offsets: only the full-key sort reads them
    offsets = torch.empty(max(n_rec, 1), dtype=torch.int64, device=dev) if full else None
    n_dup = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = _bytes(B.hgs_workspace_bytes(B.HGS_WS_PREPROCESS, n_rec, cams, opts), dev)
    B.hgs_preprocess(params, cams, opts, records, tiles, offsets, n_dup, ws, stream)
    if capacity is None:
        capacity = int(n_dup.item())
    tiles_total = B.hgs_tiles_total(cams, opts)
    keys_t = torch.empty(max(capacity, 1), dtype=torch.int64, device=dev) if (keys or full) else None
    values = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
    ranges = torch.empty(max(2 * tiles_total, 1), dtype=torch.int32, device=dev)
    order = torch.empty(max(tiles_total, 1), dtype=torch.int32, device=dev) if persistent else None
    overflow = torch.zeros(1, dtype=torch.int32, device=dev)
    ws_sort = _bytes(B.hgs_workspace_bytes(B.HGS_WS_BIN_SORT, n_rec, cams, opts, capacity), dev)
    B.hgs_bin_sort(records, tiles, offsets, n_dup, n_rec, cams, opts, keys_t, values, capacity, ranges,
                   order, overflow, ws_sort, stream)
    npix = B.hgs_pixels_total(cams)
    images = torch.empty(3 * npix, dtype=torch.float32, device=dev)
    T_final = torch.empty(npix, dtype=torch.float32, device=dev)
    last_idx = torch.empty(npix, dtype=torch.int32, device=dev)
    n_contrib = torch.empty(npix, dtype=torch.int32, device=dev)
    depth_t = torch.empty(npix, dtype=torch.float32, device=dev) if depth else None
    ws_r = _bytes(B.hgs_workspace_bytes(B.HGS_WS_RENDER, n_rec, cams, opts, capacity), dev)
    if render:
        B.hgs_render_fwd(records, values, ranges, order, cams, opts, images, T_final, last_idx, n_contrib, ws_r,
                         stream, depth=depth_t)
    return Frame(soa, n, sh_degree, cams, opts, records, tiles, offsets, n_dup, keys_t, values, ranges,
                 overflow, images, T_final, last_idx, n_contrib, capacity, ws_r, order, depth_t, params,
                 filter3d)


def depth_normals(fr: Frame) -> torch.Tensor:
    """Normals estimated from the frame's depth (forward_pass(depth=True)),
    packed like the images: [3][H][W] per camera."""
    if fr.depth is None:
        raise ValueError("the frame was rendered without depth")
    out = torch.empty(3 * fr.T_final.numel(), dtype=torch.float32, device=fr.T_final.device)
    B.hgs_depth_normals(fr.depth, fr.T_final, fr.cams, out, _stream())
    return out


def backward_pass(fr: Frame, dL_dimages: torch.Tensor, record_grads: torch.Tensor | None = None,
                  grads: torch.Tensor | None = None, stats=None):
    """Gradients of every parameter plane (same SoA layout as ``fr.soa``) and
    the per-record gradients.  ``stats`` = (grad_accum, grad_count,
    max_radii) runs the two halves of the backward pass separately and
    accumulates the densification statistics between them."""
    dev = fr.soa.device
    n_rec = fr.n * len(fr.cams)
    if record_grads is None:
        record_grads = torch.empty(max(n_rec, 1) * B.HGS_RECORD_GRAD_FLOATS, dtype=torch.float32, device=dev)
    if grads is None:
        grads = torch.zeros_like(fr.soa)
    params = fr.params if fr.params is not None else B.params_struct(fr.soa, fr.n, fr.soa.shape[1], fr.sh_degree)
    gs = B.grads_struct(grads, fr.soa.shape[1])
    if stats is None:
        B.hgs_render_bwd(params, fr.cams, fr.opts, fr.records, fr.values, fr.ranges, fr.tile_order, fr.T_final,
                         fr.last_idx, dL_dimages, record_grads, gs, fr.ws_render, _stream())
    else:
        accum, count, radii = stats
        record_grads.zero_()
        B.hgs_raster_bwd(fr.records, fr.values, fr.ranges, fr.tile_order, fr.cams, fr.opts, fr.T_final,
                         fr.last_idx, dL_dimages, record_grads, fr.ws_render, _stream())
        B.hgs_densify_stats(fr.records, record_grads, fr.cams, fr.opts, fr.n, accum, count, radii, _stream())
        B.hgs_preprocess_bwd(params, fr.cams, fr.opts, fr.records, record_grads, gs, _stream())
    return grads, record_grads


class Rasterizer:
    """Differentiable rasterization of fixed cameras with fixed options, the
    parameters given as one float32 structure-of-arrays tensor of planes
    ([means 3 | scales 3 | quats 4 | normals 3 | opac1 | opac2 | sh 3(D+1)^2]
    x N, activated values; see ``soa_from_natural``).  Its gradient comes
    back in the same layout, so no repacking happens on either pass.

    A call enqueues preprocess, sort and raster back to back: the sort runs
    in capacity mode, with entry buffers sized from earlier calls with
    ``headroom``.  The entry count is copied to pinned host memory right after
    the preprocess, and the host waits for that copy only once sort and
    raster are already queued behind it, so the device never idles for the
    check; if the entries did not fit, the entry buffers grow and the sort and
    raster are queued again.  Workspaces are kept between calls; the state
    saved for the backward pass (records, tile lists, per-pixel results, the
    per-record gradient buffer) is carved from one allocation per call (see
    Arena), the images are a second; both come from torch's caching
    allocator (no device allocation after the first call of a size)."""

    def __init__(self, cameras, sh_degree: int, tile: int | None = None, persistent: bool | None = None,
                 headroom: float = 1.25, **options):
        self.cameras = list(cameras)
        self.cams = B.make_cameras(self.cameras)
        self.opts = B.default_options(tile=default_tile(self.cameras) if tile is None else tile, **options)
        self.sh_degree = int(sh_degree)
        # one view: one workgroup per tile in tile order (neighbouring tiles
        # share records in the caches); several views: the persistent grid
        self.persistent = len(self.cameras) > 1 if persistent is None else bool(persistent)
        self.headroom = float(headroom)
        self.capacity = 0
        self._ws = {}
        self._count = None
        self.tiles_total = B.hgs_tiles_total(self.cams, self.opts)
        self.npix = B.hgs_pixels_total(self.cams)
        self.overflows = 0          # re-runs after an entry overflow (for tests and logs)

    def _workspace(self, which: str, nbytes: int, dev) -> torch.Tensor:
        t = self._ws.get(which)
        if t is None or t.numel() < nbytes or t.device != dev:
            t = _bytes(nbytes, dev)
            self._ws[which] = t
        return t

    def forward_frame(self, planes: torch.Tensor) -> Frame:
        n = planes.shape[1]
        dev = planes.device
        cams, opts = self.cams, self.opts
        n_rec = n * len(self.cameras)
        stream = _stream()
        params = B.params_struct(planes, n, planes.shape[1], self.sh_degree)
        if self.capacity == 0:      # first call: size the entry buffers from this scene
            self.capacity = self._first_capacity(params, n_rec, dev)
        npix, nt = self.npix, max(self.tiles_total, 1)
        a = Arena(dev, [("records", n_rec * B.HGS_RECORD_BYTES, torch.uint8),
                        ("tiles", n_rec, torch.int32), ("n_dup", 1, torch.int64), ("overflow", 1, torch.int32),
                        ("values", self.capacity, torch.int32), ("ranges", 2 * nt, torch.int32),
                        ("order", nt, torch.int32) if self.persistent else None,
                        ("T_final", npix, torch.float32), ("last_idx", npix, torch.int32),
                        ("n_contrib", npix, torch.int32),
                        ("record_grads", max(n_rec, 1) * B.HGS_RECORD_GRAD_FLOATS, torch.float32)])
        a["record_grads"].zero_()
        records, tiles, n_dup, overflow = a["records"], a["tiles"], a["n_dup"], a["overflow"]
        ranges, T_final, last_idx, n_contrib = a["ranges"], a["T_final"], a["last_idx"], a["n_contrib"]
        order = a["order"] if self.persistent else None
        values = a["values"]
        # the output the caller keeps: a separate allocation, so that holding
        # it does not hold the rest
        images = torch.empty(3 * npix, dtype=torch.float32, device=dev)
        ws_pre = self._workspace("pre", B.hgs_workspace_bytes(B.HGS_WS_PREPROCESS, n_rec, cams, opts), dev)
        B.hgs_preprocess(params, cams, opts, records, tiles, None, n_dup, ws_pre, stream)
        if self._count is None:
            self._count = torch.empty(1, dtype=torch.int64, pin_memory=True)
        self._count.copy_(n_dup, non_blocking=True)
        copied = torch.cuda.Event()
        copied.record()
        while True:
            if values.numel() < self.capacity:      # after an overflow: more room, outside the arena
                values = torch.empty(self.capacity, dtype=torch.int32, device=dev)
            ws_sort = self._workspace("sort", B.hgs_workspace_bytes(B.HGS_WS_BIN_SORT, n_rec, cams, opts,
                                                                    self.capacity), dev)
            ws_r = self._workspace("render", B.hgs_workspace_bytes(B.HGS_WS_RENDER, n_rec, cams, opts,
                                                                   self.capacity), dev)
            B.hgs_bin_sort(records, tiles, None, n_dup, n_rec, cams, opts, None, values, self.capacity, ranges,
                           order, overflow, ws_sort, stream)
            B.hgs_render_fwd(records, values, ranges, order, cams, opts, images, T_final, last_idx, n_contrib,
                             ws_r, stream)
            copied.synchronize()        # the entry count, long before the raster ends
            entries = int(self._count.item())
            if entries <= self.capacity:
                break
            self.overflows += 1
            self.capacity = int(math.ceil(entries * self.headroom))
        return Frame(planes, n, self.sh_degree, cams, opts, records, tiles, None, n_dup, None, values, ranges,
                     overflow, images, T_final, last_idx, n_contrib, self.capacity, ws_r, order, None, params,
                     record_grads=a["record_grads"])

    def _first_capacity(self, params, n_rec: int, dev) -> int:
        """Entry capacity from one preprocess of the first scene (one
        synchronisation, first call only)."""
        cams, opts = self.cams, self.opts
        records = _bytes(n_rec * B.HGS_RECORD_BYTES, dev)
        tiles = torch.empty(max(n_rec, 1), dtype=torch.int32, device=dev)
        n_dup = torch.empty(1, dtype=torch.int64, device=dev)
        ws_pre = self._workspace("pre", B.hgs_workspace_bytes(B.HGS_WS_PREPROCESS, n_rec, cams, opts), dev)
        B.hgs_preprocess(params, cams, opts, records, tiles, None, n_dup, ws_pre, _stream())
        return max(1, int(math.ceil(int(n_dup.item()) * self.headroom)))

    def backward_frame(self, fr: Frame, d_images: torch.Tensor) -> torch.Tensor:
        """Parameter gradients (plane layout) of a frame from this rasterizer."""
        grads = torch.empty_like(fr.soa)      # hgs_preprocess_bwd overwrites every plane
        rgrad = fr.record_grads               # cleared in the forward pass
        st = _stream()
        B.hgs_raster_bwd(fr.records, fr.values, fr.ranges, fr.tile_order, fr.cams, fr.opts, fr.T_final,
                         fr.last_idx, d_images, rgrad, fr.ws_render, st)
        B.hgs_preprocess_bwd(fr.params, fr.cams, fr.opts, fr.records, rgrad, B.grads_struct(grads, fr.soa.shape[1]),
                             st)
        return grads

    def __call__(self, planes: torch.Tensor) -> torch.Tensor:
        """Packed images of all cameras (camera c's [3,H,W] image follows
        those of cameras 0..c-1), differentiable with respect to planes."""
        return _RasterizePlanes.apply(planes, self)

    def images(self, packed: torch.Tensor) -> list:
        """[3,H,W] views of the packed images, one per camera."""
        out, off = [], 0
        for c in self.cameras:
            w, h = int(c["width"]), int(c["height"])
            out.append(packed[3 * off:3 * off + 3 * w * h].view(3, h, w))
            off += w * h
        return out


class _RasterizePlanes(torch.autograd.Function):
    @staticmethod
    def forward(ctx, planes, rasterizer):
        fr = rasterizer.forward_frame(planes.detach())
        ctx.fr, ctx.rast = fr, rasterizer
        return fr.images

    @staticmethod
    def backward(ctx, d_images):
        grads = ctx.rast.backward_frame(ctx.fr, d_images.contiguous().to(torch.float32))
        ctx.fr = None
        return grads, None


class HGSRasterize(torch.autograd.Function):
    """Differentiable half-Gaussian rasterization of one or more views from
    natural-layout CUDA tensors (activated values): packs them into planes
    (one copy per call) and runs a ``Rasterizer``; the gradients are
    unpacked back.  Training loops that keep their parameters as planes call
    a ``Rasterizer`` directly and skip both copies."""

    @staticmethod
    def forward(ctx, means, scales, quats, normals, opac1, opac2, sh, rasterizer):
        K = sh.shape[1]
        soa = soa_from_natural(means.detach(), scales.detach(), quats.detach(), normals.detach(),
                               opac1.detach(), opac2.detach(), sh.detach())
        fr = rasterizer.forward_frame(soa)
        ctx.fr, ctx.rast = fr, rasterizer
        ctx.K = K
        return fr.images

    @staticmethod
    def backward(ctx, d_images):
        grads = ctx.rast.backward_frame(ctx.fr, d_images.contiguous().to(torch.float32))
        ctx.fr = None
        m, s, q, nrm, o1, o2, sh = natural_from_soa(grads, ctx.K)
        return m, s, q, nrm, o1, o2, sh, None


def rasterize(means, scales, quats, normals, opac1, opac2, sh, cameras, **options):
    """Render ``cameras`` (list of camera dicts); returns a list of [3,H,W]
    images, differentiable with respect to every parameter."""
    K = sh.shape[1]
    rast = Rasterizer(cameras, int(round(K ** 0.5)) - 1, **options)
    packed = HGSRasterize.apply(means, scales, quats, normals, opac1, opac2, sh, rast)
    return rast.images(packed)
