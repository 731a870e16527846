"""Host-side checks of the C ABI (no GPU needed): the shared library loads,
exports every function the public header declares, and its host-only entry
points validate arguments."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2406_02720_amd import binding as B
from paper_2406_02720_amd import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hgs.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hgs_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_four_stages():
    names = _declared_functions()
    for stage in ("hgs_preprocess", "hgs_bin_sort", "hgs_render_fwd", "hgs_render_bwd"):
        assert stage in names
    assert set(names) == set(B.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libhgs.so not built")
    lib = C.CDLL(B.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_struct_sizes_match_header():
    assert C.sizeof(B.hgs_camera) == 80
    assert C.sizeof(B.hgs_options) == 48
    assert C.sizeof(B.hgs_params) == 7 * 8 + 8 + 8 + 8 + 8
    assert C.sizeof(B.hgs_param_grads) == 7 * 8


@pytest.mark.skipif(not os.path.exists(B.LIB_PATH), reason="libhgs.so not built")
def test_host_side_validation_and_sizes():
    o = B.default_options()
    assert (o.tile, o.batch) == (16, 256)
    assert o.alpha_min == float(np.float32(1 / 255)) and o.t_min == float(np.float32(1e-4))
    _, cams = scenes.make_config(3, n=10)
    ca = B.make_cameras(cams)
    assert B.hgs_tiles_total(ca, o) == 120 * 68
    assert B.hgs_pixels_total(ca) == 1920 * 1080
    for tile, tiles in ((8, 240 * 135), (32, 60 * 34)):
        assert B.hgs_tiles_total(ca, B.default_options(tile=tile)) == tiles
    assert B.hgs_tiles_total(ca, B.default_options(tile=12)) == -1
    assert B.hgs_tiles_total(ca, B.default_options(batch=100)) == -1
    assert B.hgs_workspace_bytes(B.HGS_WS_BIN_SORT, 100, ca, o, 1000) > 12 * 1000
    assert B.hgs_workspace_bytes(B.HGS_WS_BIN_SORT, 100, ca, B.default_options(tile=12), 1000) == 0
    # calls with invalid arguments fail before touching the GPU
    lib = B.load()
    rc = lib.hgs_preprocess(None, ca, 1, C.byref(o), None, None, None, None, None, 0, None)
    assert rc == B.HGS_EINVAL and b"params" in lib.hgs_last_error()
    p = B.hgs_params()
    p.n, p.stride, p.sh_degree = 10, 10, 4
    rc = lib.hgs_preprocess(C.byref(p), ca, 1, C.byref(o), None, None, None, None, None, 0, None)
    assert rc == B.HGS_EINVAL and b"sh_degree" in lib.hgs_last_error()
    p.sh_degree = 0
    rc = lib.hgs_preprocess(C.byref(p), ca, 0, C.byref(o), None, None, None, None, None, 0, None)
    assert rc == B.HGS_EINVAL
    big = (B.hgs_camera * 1)()
    big[0].width, big[0].height, big[0].fx, big[0].fy = 70000, 10, 1.0, 1.0
    assert B.hgs_tiles_total(big, o) == -1
    assert lib.hgs_strerror(B.HGS_ECAPACITY) == b"buffer too small"


@pytest.mark.skipif(not os.path.exists(B.LIB_PATH), reason="libhgs.so not built")
def test_render_workspace_holds_the_strip_marks():
    """The render workspace is 256 bytes of head plus one strip-mark byte
    per entry of the capacity and forward wavefront of a tile (four at
    32-pixel tiles, one at 16 and 8), rounded up to 256 bytes; capacity 0
    gives the head alone (a valid workspace, without marks)."""
    _, cams = scenes.make_config(1)
    ca = B.make_cameras(cams)
    for tile, planes in ((32, 4), (16, 1), (8, 1)):
        o = B.default_options(tile=tile)
        assert B.hgs_workspace_bytes(B.HGS_WS_RENDER, 100, ca, o, 0) == 256
        for cap in (1, 1000, 123457):
            want = 256 + (planes * cap + 255) // 256 * 256
            assert B.hgs_workspace_bytes(B.HGS_WS_RENDER, 100, ca, o, cap) == want
    assert B.hgs_workspace_bytes(B.HGS_WS_RENDER, 100, ca, B.default_options(tile=12), 1000) == 0


def test_near_plane_must_be_positive_and_finite():
    """A near plane at or behind the camera (or not a number) is rejected:
    with znear < 0, kernels with camera z in (znear, 0) would pass the cull,
    project mirrored, and their negative depth bits would sort after every
    positive depth."""
    o = B.default_options()
    _, cams = scenes.make_config(1, n=10)
    assert B.hgs_tiles_total(B.make_cameras(cams), o) == 64
    lib = B.load()
    p = B.hgs_params()
    p.n, p.stride, p.sh_degree = 0, 0, 0
    for zn in (0.0, -0.5, float("nan"), float("inf")):
        bad = [dict(cams[0], znear=np.float32(zn))]
        ca = B.make_cameras(bad)
        assert B.hgs_tiles_total(ca, o) == -1, zn
        assert B.hgs_workspace_bytes(B.HGS_WS_BIN_SORT, 10, ca, o, 100) == 0
        rc = lib.hgs_preprocess(C.byref(p), ca, 1, C.byref(o), None, None, None, None, None, 0, None)
        assert rc == B.HGS_EINVAL and b"znear" in lib.hgs_last_error(), zn


def test_autotune_shape_class_is_stable():
    from paper_2406_02720_amd import batch
    _, cams = scenes.make_config(4, n=10, n_cams=3)
    a = batch.shape_class(500_000, cams)
    assert a == batch.shape_class(510_000, cams) and a.endswith("_v3")
    assert a != batch.shape_class(500_000, cams[:2])


def test_raster_erfc_approximation_error_bound():
    """The half factor's erfc in the raster kernels is exp2 of a fitted
    polynomial in |x| (clamped at 3.9): its coefficients, read from the
    kernel source and evaluated in float32 Horner arithmetic, stay within
    1e-7 of erfc over the whole real line (the sign by erfc(-z) = 2 - erfc(z))."""
    import re
    from scipy.special import erfc
    src = open(os.path.join(ROOT, "paper_2406_02720_amd", "csrc", "render.hip")).read()
    body = src[src.index("float erfc_fast(float x)"):]
    body = body[:body.index("}")]
    zmax = float(re.search(r"fmed3f\(fabsf\(x\), 0\.0f, ([0-9.]+)f\)", body).group(1))
    lead = float(re.search(r"float p = ([-0-9.e]+)f;", body).group(1))
    rest = [float(c) for c in re.findall(r"p = fmaf\(p, z, ([-0-9.e]+)f\);", body)]
    x = np.linspace(-8.0, 8.0, 400001).astype(np.float32)
    z = np.minimum(np.abs(x), np.float32(zmax))
    p = np.full_like(z, np.float32(lead))
    for c in rest:
        p = (p * z + np.float32(c)).astype(np.float32)   # fma rounds once; this rounds twice
    e = np.exp2(p.astype(np.float64))
    approx = np.where(x >= 0, e, 2.0 - e)
    assert np.abs(approx - erfc(x.astype(np.float64))).max() < 1e-7


def test_adam_schedule_host_call_matches_oracle():
    """hgs_adam_schedule is host code: its rates are the oracle's schedule
    rounded to float32, and it rejects bad arguments."""
    import numpy as np
    from oracle import hgs_train_oracle as T
    for t in (1, 2, 4999, 5000, 12345, 30000, 45000):
        for ext in (0.5, 3.7):
            cfg = B.hgs_adam_schedule(t, ext)
            want = T.learning_rates(t, float(np.float32(ext)))
            got = dict(means=cfg.lr_means, scales=cfg.lr_scales, quats=cfg.lr_quats, normals=cfg.lr_normals,
                       opac=cfg.lr_opacity, sh_dc=cfg.lr_sh_dc, sh_rest=cfg.lr_sh_rest)
            for k, v in want.items():
                assert got[k] == np.float32(v), (t, ext, k, got[k], v)
            assert (cfg.beta1, cfg.beta2, cfg.step) == (np.float32(0.9), np.float32(0.999), t)
            assert cfg.eps == np.float32(1e-15)
    lib = B.load()
    c = B.hgs_adam_config()
    assert lib.hgs_adam_schedule(0, 1.0, 0.003, C.byref(c)) == B.HGS_EINVAL
    assert lib.hgs_adam_schedule(1, 0.0, 0.003, C.byref(c)) == B.HGS_EINVAL
    d = B.hgs_densify_default(2.0)
    assert (d.grad_threshold, d.percent_dense, d.min_opacity) == (np.float32(0.0002), np.float32(0.01),
                                                                  np.float32(0.01))
    assert B.hgs_densify_workspace_bytes(1000) > 3 * 4 * 1000 + 3 * 8 * 1000
    assert B.hgs_densify_workspace_bytes(-1) == 0


@pytest.mark.skipif(not os.path.exists(B.LIB_PATH), reason="libhgs.so not built")
def test_noalloc_preprocess_rejects_more_records_than_its_array_holds():
    """hgs_preprocess_noalloc returns HGS_ECAPACITY for more records than its
    device array serves, before it touches the GPU (the pointers below are
    never dereferenced)."""
    lib = B.load()
    o = B.default_options()
    _, cams = scenes.make_config(1, n=10)
    ca = B.make_cameras(cams * 3)
    p = B.hgs_params()
    fake = 1 << 40
    p.means = p.scales = p.quats = p.normals = p.opac1 = p.opac2 = p.sh = fake
    p.n = B.HGS_NOALLOC_MAX_RECORDS // 3 + 1          # three views: one record over the limit
    p.stride, p.sh_degree = p.n, 0
    rc = lib.hgs_preprocess_noalloc(C.byref(p), ca, 3, C.byref(o), fake, fake, None, fake, None)
    assert rc == B.HGS_ECAPACITY and b"no-alloc limit" in lib.hgs_last_error()
    # null outputs are still EINVAL
    rc = lib.hgs_preprocess_noalloc(C.byref(p), ca, 3, C.byref(o), None, None, None, fake, None)
    assert rc == B.HGS_EINVAL


def test_default_tile_keeps_four_workgroups_per_cu():
    """32-pixel tiles while their count stays at 1024 or more, else 16."""
    from paper_2406_02720_amd import raster as R
    cam = lambda w, h: dict(width=w, height=h)  # noqa: E731
    assert R.default_tile([cam(1920, 1080)]) == 32          # 60 x 34 = 2040 tiles
    assert R.default_tile([cam(1280, 720)]) == 16           # 40 x 23 = 920
    assert R.default_tile([cam(1280, 720)] * 2) == 32       # 1840 over two views
    assert R.default_tile([cam(1024, 1024)]) == 32          # exactly 1024
    assert R.default_tile([cam(1023, 1024)]) == 32
    assert R.default_tile([cam(992, 1024)]) == 16           # 31 x 32 = 992
