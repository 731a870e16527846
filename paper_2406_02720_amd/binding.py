"""ctypes binding of libhgs.so: the C structs and entry points of include/hgs.h
with the same names.  Arguments are marshalled only -- every step of the
rasterizer runs in the library's HIP kernels.  Device buffers are torch
tensors (torch is used for device memory and streams).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhgs.so")

HGS_OK, HGS_EINVAL, HGS_ECAPACITY, HGS_EHIP = 0, 1, 2, 3
HGS_MAX_CAMERAS = 32
HGS_RECORD_BYTES = 64
HGS_RECORD_GRAD_FLOATS = 12
HGS_FLAG_FULL_BOX = 1
HGS_FLAG_SORT_FULL_KEYS = 2
HGS_FLAG_MIP_2D = 4
HGS_WS_PREPROCESS, HGS_WS_BIN_SORT, HGS_WS_RENDER = 0, 1, 2
HGS_NOALLOC_MAX_RECORDS = 134217728

EXPORTS = ("hgs_default_options", "hgs_workspace_bytes", "hgs_tiles_total", "hgs_pixels_total",
           "hgs_preprocess", "hgs_preprocess_noalloc", "hgs_bin_sort", "hgs_render_fwd", "hgs_render_bwd",
           "hgs_raster_bwd", "hgs_preprocess_bwd", "hgs_depth_normals", "hgs_mip_filter3d",
           "hgs_l1_loss_grad", "hgs_adam_schedule", "hgs_adam_step",
           "hgs_activate", "hgs_densify_stats", "hgs_densify_default", "hgs_densify_workspace_bytes",
           "hgs_densify", "hgs_reset_opacity", "hgs_strerror", "hgs_last_error")


class hgs_camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32),
                ("znear", C.c_float), ("reserved", C.c_int32)]


class hgs_params(C.Structure):
    _fields_ = [("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("normals", C.c_void_p), ("opac1", C.c_void_p), ("opac2", C.c_void_p),
                ("sh", C.c_void_p), ("n", C.c_int64), ("stride", C.c_int64),
                ("sh_degree", C.c_int32), ("reserved", C.c_int32), ("filter3d", C.c_void_p)]


class hgs_param_grads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("normals", C.c_void_p), ("opac1", C.c_void_p), ("opac2", C.c_void_p),
                ("sh", C.c_void_p)]


class hgs_options(C.Structure):
    _fields_ = [("tile", C.c_int32), ("batch", C.c_int32), ("lowpass", C.c_float),
                ("kappa", C.c_float), ("alpha_min", C.c_float), ("alpha_max", C.c_float),
                ("t_min", C.c_float), ("fov_clamp", C.c_float), ("bg", C.c_float * 3),
                ("flags", C.c_uint32)]


class hgs_adam_config(C.Structure):
    _fields_ = [("lr_means", C.c_float), ("lr_scales", C.c_float), ("lr_quats", C.c_float),
                ("lr_normals", C.c_float), ("lr_opacity", C.c_float), ("lr_sh_dc", C.c_float),
                ("lr_sh_rest", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("step", C.c_int32), ("reserved", C.c_int32)]


class hgs_densify_config(C.Structure):
    _fields_ = [("extent", C.c_float), ("grad_threshold", C.c_float), ("percent_dense", C.c_float),
                ("min_opacity", C.c_float), ("max_screen_radius", C.c_float), ("max_world_scale", C.c_float)]


class HGSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hgs error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libhgs.so (raises if it has not been built: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libhgs.so not found at {path}; build it with "
                           "`python -m paper_2406_02720_amd.build` (there is no CPU fallback)")
    # torch's HIP runtime first: the library's dependency on the HIP runtime
    # is then resolved to the copy already loaded, and the process holds one
    # runtime.  Loaded the other way round, torch brings a second copy, and
    # the two contend for the device (the library's launches then fail with
    # "no ROCm-capable device").
    import torch  # noqa: F401
    lib = C.CDLL(path)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    P = C.POINTER
    lib.hgs_default_options.argtypes = [P(hgs_options)]
    lib.hgs_default_options.restype = None
    lib.hgs_workspace_bytes.argtypes = [i32, i64, P(hgs_camera), i32, P(hgs_options), i64]
    lib.hgs_workspace_bytes.restype = sz
    lib.hgs_tiles_total.argtypes = [P(hgs_camera), i32, P(hgs_options)]
    lib.hgs_tiles_total.restype = i64
    lib.hgs_pixels_total.argtypes = [P(hgs_camera), i32]
    lib.hgs_pixels_total.restype = i64
    lib.hgs_preprocess.argtypes = [P(hgs_params), P(hgs_camera), i32, P(hgs_options), vp, vp, vp, vp,
                                   vp, sz, vp]
    lib.hgs_preprocess.restype = C.c_int
    lib.hgs_preprocess_noalloc.argtypes = [P(hgs_params), P(hgs_camera), i32, P(hgs_options), vp, vp, vp, vp,
                                           vp]
    lib.hgs_preprocess_noalloc.restype = C.c_int
    lib.hgs_bin_sort.argtypes = [vp, vp, vp, vp, i64, P(hgs_camera), i32, P(hgs_options), vp, vp, i64,
                                 vp, vp, vp, vp, sz, vp]
    lib.hgs_bin_sort.restype = C.c_int
    lib.hgs_render_fwd.argtypes = [vp, vp, vp, vp, P(hgs_camera), i32, P(hgs_options), vp, vp, vp, vp, vp,
                                   vp, sz, vp]
    lib.hgs_render_fwd.restype = C.c_int
    lib.hgs_depth_normals.argtypes = [vp, vp, P(hgs_camera), i32, vp, vp]
    lib.hgs_depth_normals.restype = C.c_int
    lib.hgs_render_bwd.argtypes = [P(hgs_params), P(hgs_camera), i32, P(hgs_options), vp, vp, vp, vp,
                                   vp, vp, vp, vp, P(hgs_param_grads), vp, sz, vp]
    lib.hgs_render_bwd.restype = C.c_int
    lib.hgs_raster_bwd.argtypes = [vp, vp, vp, vp, P(hgs_camera), i32, P(hgs_options), vp, vp, vp, vp,
                                   vp, sz, vp]
    lib.hgs_raster_bwd.restype = C.c_int
    lib.hgs_preprocess_bwd.argtypes = [P(hgs_params), P(hgs_camera), i32, P(hgs_options), vp, vp,
                                       P(hgs_param_grads), vp]
    lib.hgs_preprocess_bwd.restype = C.c_int
    lib.hgs_mip_filter3d.argtypes = [vp, i64, i64, P(hgs_camera), i32, C.c_float, C.c_float, vp, vp, vp]
    lib.hgs_mip_filter3d.restype = C.c_int
    lib.hgs_l1_loss_grad.argtypes = [vp, vp, i64, C.c_float, vp, vp, vp]
    lib.hgs_l1_loss_grad.restype = C.c_int
    PG = P(hgs_param_grads)
    lib.hgs_adam_schedule.argtypes = [i32, C.c_float, C.c_float, P(hgs_adam_config)]
    lib.hgs_adam_schedule.restype = C.c_int
    lib.hgs_adam_step.argtypes = [P(hgs_adam_config), i64, i64, i32, PG, PG, PG, PG, PG, vp]
    lib.hgs_adam_step.restype = C.c_int
    lib.hgs_activate.argtypes = [i64, i64, i32, PG, PG, vp]
    lib.hgs_activate.restype = C.c_int
    lib.hgs_densify_stats.argtypes = [vp, vp, P(hgs_camera), i32, P(hgs_options), i64, vp, vp, vp, vp]
    lib.hgs_densify_stats.restype = C.c_int
    lib.hgs_densify_default.argtypes = [C.c_float, P(hgs_densify_config)]
    lib.hgs_densify_default.restype = None
    lib.hgs_densify_workspace_bytes.argtypes = [i64]
    lib.hgs_densify_workspace_bytes.restype = sz
    lib.hgs_densify.argtypes = [P(hgs_densify_config), i64, i64, i32, PG, PG, PG, vp, vp, vp, vp, i64, i64,
                                PG, PG, PG, vp, vp, vp, sz, vp]
    lib.hgs_densify.restype = C.c_int
    lib.hgs_reset_opacity.argtypes = [C.c_float, i64, PG, PG, PG, PG, vp]
    lib.hgs_reset_opacity.restype = C.c_int
    lib.hgs_strerror.argtypes = [C.c_int]
    lib.hgs_strerror.restype = C.c_char_p
    lib.hgs_last_error.argtypes = []
    lib.hgs_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def check(rc: int):
    if rc != HGS_OK:
        raise HGSError(rc, load().hgs_last_error().decode())


def default_options(**kw) -> hgs_options:
    o = hgs_options()
    load().hgs_default_options(C.byref(o))
    for k, v in kw.items():
        if k == "bg":
            o.bg[:] = [float(x) for x in v]
        elif k == "full_box":
            o.flags = (o.flags | HGS_FLAG_FULL_BOX) if v else (o.flags & ~HGS_FLAG_FULL_BOX)
        elif k == "sort_full_keys":
            o.flags = (o.flags | HGS_FLAG_SORT_FULL_KEYS) if v else (o.flags & ~HGS_FLAG_SORT_FULL_KEYS)
        elif k == "mip2d":
            o.flags = (o.flags | HGS_FLAG_MIP_2D) if v else (o.flags & ~HGS_FLAG_MIP_2D)
        else:
            setattr(o, k, v)
    return o


def make_cameras(cams) -> C.Array:
    """Camera dicts (R, t, fx, fy, cx, cy, width, height, znear) -> C array."""
    arr = (hgs_camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i].R[:] = [float(x) for x in np.asarray(c["R"], np.float32).ravel()]
        arr[i].t[:] = [float(x) for x in np.asarray(c["t"], np.float32).ravel()]
        arr[i].fx, arr[i].fy = float(c["fx"]), float(c["fy"])
        arr[i].cx, arr[i].cy = float(c["cx"]), float(c["cy"])
        arr[i].width, arr[i].height = int(c["width"]), int(c["height"])
        arr[i].znear = float(c["znear"])
    return arr


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def params_struct(soa, n: int, stride: int, sh_degree: int) -> hgs_params:
    """hgs_params over one float32 structure-of-arrays tensor of planes
    [means 3 | scales 3 | quats 4 | normals 3 | opac1 | opac2 | sh 3(D+1)^2]."""
    base = soa.data_ptr()
    f = 4 * stride
    p = hgs_params()
    p.means, p.scales, p.quats = base, base + 3 * f, base + 6 * f
    p.normals, p.opac1, p.opac2, p.sh = base + 10 * f, base + 13 * f, base + 14 * f, base + 15 * f
    p.n, p.stride, p.sh_degree = n, stride, sh_degree
    return p


def grads_struct(soa, stride: int) -> hgs_param_grads:
    base = soa.data_ptr()
    f = 4 * stride
    g = hgs_param_grads()
    g.means, g.scales, g.quats = base, base + 3 * f, base + 6 * f
    g.normals, g.opac1, g.opac2, g.sh = base + 10 * f, base + 13 * f, base + 14 * f, base + 15 * f
    return g


# -- entry points with the C names -------------------------------------------
def hgs_workspace_bytes(which, n_rec, cams, opts, capacity=0) -> int:
    return int(load().hgs_workspace_bytes(which, n_rec, cams, len(cams), C.byref(opts), capacity))


def hgs_tiles_total(cams, opts) -> int:
    return int(load().hgs_tiles_total(cams, len(cams), C.byref(opts)))


def hgs_pixels_total(cams) -> int:
    return int(load().hgs_pixels_total(cams, len(cams)))


def hgs_preprocess(params, cams, opts, records, tiles, offsets, n_dup, ws, stream):
    check(load().hgs_preprocess(C.byref(params), cams, len(cams), C.byref(opts), _ptr(records), _ptr(tiles),
                                _ptr(offsets), _ptr(n_dup), _ptr(ws), ws.numel() * ws.element_size(), stream))


def hgs_preprocess_noalloc(params, cams, opts, records, tiles, offsets, n_dup, stream):
    check(load().hgs_preprocess_noalloc(C.byref(params), cams, len(cams), C.byref(opts), _ptr(records),
                                        _ptr(tiles), _ptr(offsets), _ptr(n_dup), stream))


def hgs_bin_sort(records, tiles, offsets, n_dup, n_rec, cams, opts, keys, values, capacity, ranges,
                 tile_order, overflow, ws, stream):
    check(load().hgs_bin_sort(_ptr(records), _ptr(tiles), _ptr(offsets), _ptr(n_dup), n_rec, cams, len(cams),
                              C.byref(opts), _ptr(keys), _ptr(values), capacity, _ptr(ranges), _ptr(tile_order),
                              _ptr(overflow), _ptr(ws), ws.numel() * ws.element_size(), stream))


def hgs_render_fwd(records, values, ranges, tile_order, cams, opts, images, T_final, last_idx, n_contrib, ws,
                   stream, depth=None):
    check(load().hgs_render_fwd(_ptr(records), _ptr(values), _ptr(ranges), _ptr(tile_order), cams, len(cams),
                                C.byref(opts),
                                _ptr(images), _ptr(T_final), _ptr(last_idx), _ptr(n_contrib), _ptr(depth),
                                _ptr(ws), ws.numel() * ws.element_size(), stream))


def hgs_depth_normals(depth, T_final, cams, normals, stream):
    check(load().hgs_depth_normals(_ptr(depth), _ptr(T_final), cams, len(cams), _ptr(normals), stream))


def hgs_render_bwd(params, cams, opts, records, values, ranges, tile_order, T_final, last_idx, dL_dimages,
                   record_grads, grads, ws, stream):
    check(load().hgs_render_bwd(C.byref(params), cams, len(cams), C.byref(opts), _ptr(records), _ptr(values),
                                _ptr(ranges), _ptr(tile_order), _ptr(T_final), _ptr(last_idx), _ptr(dL_dimages),
                                _ptr(record_grads), C.byref(grads), _ptr(ws), ws.numel() * ws.element_size(),
                                stream))


def hgs_raster_bwd(records, values, ranges, tile_order, cams, opts, T_final, last_idx, dL_dimages, record_grads,
                   ws, stream):
    check(load().hgs_raster_bwd(_ptr(records), _ptr(values), _ptr(ranges), _ptr(tile_order), cams, len(cams),
                                C.byref(opts), _ptr(T_final), _ptr(last_idx), _ptr(dL_dimages),
                                _ptr(record_grads), _ptr(ws), ws.numel() * ws.element_size(), stream))


def hgs_preprocess_bwd(params, cams, opts, records, record_grads, grads, stream):
    check(load().hgs_preprocess_bwd(C.byref(params), cams, len(cams), C.byref(opts), _ptr(records),
                                    _ptr(record_grads), C.byref(grads), stream))


def hgs_mip_filter3d(means, n, stride, cams, s, margin, filter3d, ws, stream):
    check(load().hgs_mip_filter3d(_ptr(means), n, stride, cams, len(cams), s, margin, _ptr(filter3d), _ptr(ws),
                                  stream))


def hgs_l1_loss_grad(images, target, dL, stream, loss=None, scale=None):
    n = images.numel()
    s = 1.0 / max(n, 1) if scale is None else float(scale)
    check(load().hgs_l1_loss_grad(_ptr(images), _ptr(target), n, s, _ptr(dL), _ptr(loss), stream))


def hgs_adam_schedule(step: int, extent: float, normal_lr: float = 0.003) -> hgs_adam_config:
    cfg = hgs_adam_config()
    check(load().hgs_adam_schedule(step, extent, normal_lr, C.byref(cfg)))
    return cfg


def hgs_adam_step(cfg, n, stride, sh_degree, raw, grads, m, v, act, stream):
    check(load().hgs_adam_step(C.byref(cfg), n, stride, sh_degree, C.byref(raw), C.byref(grads), C.byref(m),
                               C.byref(v), C.byref(act), stream))


def hgs_activate(n, stride, sh_degree, raw, act, stream):
    check(load().hgs_activate(n, stride, sh_degree, C.byref(raw), C.byref(act), stream))


def hgs_densify_stats(records, record_grads, cams, opts, n, accum, count, max_radii, stream):
    check(load().hgs_densify_stats(_ptr(records), _ptr(record_grads), cams, len(cams), C.byref(opts), n,
                                   _ptr(accum), _ptr(count), _ptr(max_radii), stream))


def hgs_densify_default(extent: float) -> hgs_densify_config:
    cfg = hgs_densify_config()
    load().hgs_densify_default(extent, C.byref(cfg))
    return cfg


def hgs_densify_workspace_bytes(n: int) -> int:
    return int(load().hgs_densify_workspace_bytes(n))


def hgs_densify(cfg, n, stride, sh_degree, raw, m, v, accum, count, max_radii, samples, capacity, stride_out,
                raw_out, m_out, v_out, n_out, overflow, ws, stream):
    check(load().hgs_densify(C.byref(cfg), n, stride, sh_degree, C.byref(raw), C.byref(m), C.byref(v),
                             _ptr(accum), _ptr(count), _ptr(max_radii), _ptr(samples), capacity, stride_out,
                             C.byref(raw_out), C.byref(m_out), C.byref(v_out), _ptr(n_out), _ptr(overflow),
                             _ptr(ws), ws.numel() * ws.element_size(), stream))


def hgs_reset_opacity(value, n, raw, m, v, act, stream):
    check(load().hgs_reset_opacity(value, n, C.byref(raw), C.byref(m), C.byref(v),
                                   None if act is None else C.byref(act), stream))
