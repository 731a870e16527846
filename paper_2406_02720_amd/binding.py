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
HGS_WS_PREPROCESS, HGS_WS_BIN_SORT, HGS_WS_RENDER = 0, 1, 2

EXPORTS = ("hgs_default_options", "hgs_workspace_bytes", "hgs_tiles_total", "hgs_pixels_total",
           "hgs_preprocess", "hgs_bin_sort", "hgs_render_fwd", "hgs_render_bwd",
           "hgs_raster_bwd", "hgs_preprocess_bwd", "hgs_depth_normals", "hgs_strerror", "hgs_last_error")


class hgs_camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32),
                ("znear", C.c_float), ("reserved", C.c_int32)]


class hgs_params(C.Structure):
    _fields_ = [("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("normals", C.c_void_p), ("opac1", C.c_void_p), ("opac2", C.c_void_p),
                ("sh", C.c_void_p), ("n", C.c_int64), ("stride", C.c_int64),
                ("sh_degree", C.c_int32), ("reserved", C.c_int32)]


class hgs_param_grads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("normals", C.c_void_p), ("opac1", C.c_void_p), ("opac2", C.c_void_p),
                ("sh", C.c_void_p)]


class hgs_options(C.Structure):
    _fields_ = [("tile", C.c_int32), ("batch", C.c_int32), ("lowpass", C.c_float),
                ("kappa", C.c_float), ("alpha_min", C.c_float), ("alpha_max", C.c_float),
                ("t_min", C.c_float), ("fov_clamp", C.c_float), ("bg", C.c_float * 3),
                ("flags", C.c_uint32)]


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
