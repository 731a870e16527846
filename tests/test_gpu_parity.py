"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Bars: records' integer fields (pixel rect, tiles touched, fp32 depth bits),
sort keys, values and tile ranges bit-exact; record floats to float32
rounding; per-pixel contributor counts and last contributors exact and images
within 1e-4 on pixels with no decision within a relative 2e-4 of its
threshold (REC mode: the oracle blends the float32 record values in FP64);
gradients within 1e-3 relative (per-tensor L2 and elementwise with a floor)
against FP64 autograd of the end-to-end oracle.
"""
import math

import numpy as np
import pytest
import torch

from oracle import hgs_oracle as O
from paper_2406_02720_amd import binding as B
from paper_2406_02720_amd import raster as R
from paper_2406_02720_amd import scenes

from hgs_testlib import (ambiguous, check_gradients, gpu_forward, kernel_terms, oracle_pre, records_np,
                         sorted_entries, split_opts, u32)

pytestmark = pytest.mark.gpu


def _cases():
    s1, c1 = scenes.make_config(1)
    s2, c2 = scenes.make_config(2, n=20000, width=320, height=180)
    s4, c4 = scenes.make_config(4, n=6000, n_cams=3)
    c4 = [scenes.pinhole(w, h, c["R"], c["t"]) for c, (w, h) in zip(c4, ((200, 150), (129, 84), (160, 106)))]
    s3, c3 = scenes.make_config(3, n=30000, width=330, height=190)
    return {
        "cfg1": (s1, c1),
        "cfg2_small": (s2, c2),
        "cfg2_halfclear": (scenes.with_transparent_halves(s2), c2),
        "cfg4_three_views": (s4, c4),
        "cfg3_small": (s3, c3),
    }


CASES = _cases()


def _check_records(scene, cams, fr, pres):
    f, u = records_np(fr)
    n = scene["means"].shape[0]
    for c, pre in enumerate(pres):
        fs, us = f[c * n:(c + 1) * n], u[c * n:(c + 1) * n]
        valid = pre["valid"].numpy()
        # integer decisions: an FP64 edge within 1e-9 of an integer could round
        # either way on the two sides; none is expected
        e = pre["edges"].numpy()[valid]
        amb = (np.abs(e - np.round(e)) < 1e-9).any(1)
        assert amb.sum() == 0
        np.testing.assert_array_equal(us[:, 15] > 0, valid)
        np.testing.assert_array_equal(us[:, 15], pre["tiles_touched"].numpy().astype(np.uint32))
        r = pre["rect"].numpy()[valid]
        np.testing.assert_array_equal(us[valid, 12] & 0xffff, r[:, 0])
        np.testing.assert_array_equal(us[valid, 12] >> 16, r[:, 1])
        np.testing.assert_array_equal(us[valid, 13] & 0xffff, r[:, 2])
        np.testing.assert_array_equal(us[valid, 13] >> 16, r[:, 3])
        np.testing.assert_array_equal(us[valid, 14], pre["depth_bits"][valid])
        g = pre["rec"]
        corner = np.stack([r[:, 0], r[:, 2]], 1)
        ref = np.concatenate([g["mean2d"].numpy() - corner, g["k"].numpy(), g["conic"].numpy(),
                              g["alpha2"].numpy()[:, None], g["colour"].numpy(), g["d_o"].numpy()[:, None]], 1)
        got = fs[valid][:, [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11]]
        # fields: mx my kx ky qa qb qc alpha2 r g b d_o
        scale = np.maximum(np.abs(ref), 1e-30)
        rel = np.abs(got - ref.astype(np.float32).astype(np.float64)) / scale
        assert rel.max() < 1e-6, rel.max()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("tile,full_keys", [(16, False), (8, False), (32, False), (16, True), (8, True)])
def test_preprocess_and_sort_match_oracle(name, tile, full_keys):
    scene, cams = CASES[name]
    print(f"[case] preprocess+sort {name} tile={tile} full_keys={full_keys}", flush=True)
    fr = gpu_forward(scene, cams, tile=tile, sort_full_keys=full_keys)
    pres = oracle_pre(scene, cams, tile=tile)
    _check_records(scene, cams, fr, pres)
    bs = O.bin_sort(pres)
    keys, vals, ranges = sorted_entries(fr)
    assert int(fr.overflow.item()) == 0
    assert keys.size == bs["keys"].size
    np.testing.assert_array_equal(keys, bs["keys"])
    np.testing.assert_array_equal(vals, bs["vals"])
    np.testing.assert_array_equal(ranges, bs["ranges"])


def _check_render(scene, cams, fr, pres, mode="rec"):
    n = scene["means"].shape[0]
    vals = u32(fr.values)
    flagged_total = pix_total = 0
    for c, pre in enumerate(pres):
        ref = O.render(pre, mode)
        img = fr.image(c).cpu().numpy()
        T = fr.per_pixel(fr.T_final, c).cpu().numpy()
        cnt = fr.per_pixel(fr.n_contrib, c).cpu().numpy()
        last = fr.per_pixel(fr.last_idx, c).cpu().numpy()
        ok = ~ambiguous(ref["margin"])
        flagged_total += int((~ok).sum())
        pix_total += ok.size
        ref_img = ref["image"].numpy()
        err = np.abs(img - ref_img).max(0)
        assert err[ok].max() <= 1e-4, err[ok].max()
        np.testing.assert_array_equal(cnt[ok], ref["n_contrib"].numpy()[ok])
        assert np.abs(T - ref["T_final"].numpy())[ok].max() <= 1e-4
        starts = u32(fr.ranges).reshape(-1, 2)[:, 0].astype(np.int64)
        T = fr.opts.tile
        cam = cams[c]
        toff = sum(((cc["width"] + T - 1) // T) * ((cc["height"] + T - 1) // T) for cc in cams[:c])
        ys, xs = np.meshgrid(np.arange(cam["height"]) // T, np.arange(cam["width"]) // T, indexing="ij")
        tstart = starts[toff + ys * ((cam["width"] + T - 1) // T) + xs]
        last_id = np.where(last >= 0, vals[np.maximum(tstart + last, 0)].astype(np.int64) - c * n, -1)
        np.testing.assert_array_equal(last_id[ok], ref["last_id"].numpy()[ok])
    print(f"[flagged] {flagged_total}/{pix_total} = {flagged_total / max(pix_total, 1):.4%}", flush=True)
    assert flagged_total < 0.01 * pix_total, (flagged_total, pix_total)
    return flagged_total, pix_total


@pytest.mark.parametrize("name", list(CASES))
def test_render_fwd_matches_oracle(name):
    scene, cams = CASES[name]
    print(f"[case] render_fwd {name}", flush=True)
    fr = gpu_forward(scene, cams)
    pres = oracle_pre(scene, cams)
    flagged, total = _check_render(scene, cams, fr, pres)
    print(f"flagged {flagged}/{total}", flush=True)


def test_render_fwd_end_to_end_fp64():
    scene, cams = CASES["cfg2_small"]
    fr = gpu_forward(scene, cams)
    _check_render(scene, cams, fr, oracle_pre(scene, cams), mode="e2e")


def test_outputs_identical_across_tile_batch_and_runs():
    scene, cams = CASES["cfg4_three_views"]
    ref = gpu_forward(scene, cams)
    base = ref.images.cpu()
    for tile in (8, 16, 32):
        for batch in (128, 256, 512):
            fr = gpu_forward(scene, cams, tile=tile, batch=batch)
            assert torch.equal(fr.images.cpu(), base), (tile, batch)
            assert torch.equal(fr.n_contrib.cpu(), ref.n_contrib.cpu())
            assert torch.equal(fr.T_final.cpu(), ref.T_final.cpu())
    again = gpu_forward(scene, cams)
    assert torch.equal(again.images.cpu(), base)
    # one workgroup per tile instead of the persistent grid
    plain = gpu_forward(scene, cams, persistent=False)
    assert torch.equal(plain.images.cpu(), base) and torch.equal(plain.last_idx.cpu(), ref.last_idx.cpu())
    # the batched multi-view call equals one call per view
    for c, cam in enumerate(cams):
        single = gpu_forward(scene, [cam])
        assert torch.equal(single.image(0).cpu(), ref.image(c).cpu())


def test_tile_order_is_longest_list_first():
    scene, cams = CASES["cfg4_three_views"]
    fr = gpu_forward(scene, cams)
    order = fr.tile_order.cpu().numpy().astype(np.int64)
    r = u32(fr.ranges).reshape(-1, 2).astype(np.int64)
    lengths = r[:, 1] - r[:, 0]
    assert sorted(order.tolist()) == list(range(lengths.size))
    # log-scale buckets of the list length, 16 per doubling, longest first
    v = (lengths + 1).astype(np.uint64)
    msb = np.floor(np.log2(v.astype(np.float64))).astype(np.int64)
    frac = ((v << (32 - msb).astype(np.uint64)) >> np.uint64(28)).astype(np.int64) & 15
    key = 255 - np.minimum(255, 16 * msb + frac)
    np.testing.assert_array_equal(order, np.lexsort((np.arange(lengths.size), key)))
    # a later tile is never longer than an earlier one by more than one bucket
    lo = (lengths[order] + 1).astype(np.float64)
    assert np.all(lo[1:] < np.maximum.accumulate(lo)[:-1] * (17 / 16) + 1e-9)


@pytest.mark.parametrize("tile", [16, 32, 8])
def test_persistent_backward_equals_per_tile_backward(tile):
    """Three views with odd tile counts (13x10, 9x6, 10x7 tiles at 16; 7x5,
    5x3, 5x4 at 32): the per-tile backward grid, whose launch slots take the
    tiles in XCD-grouped 2x2 block order, covers every tile once, like the
    persistent one."""
    scene, cams = CASES["cfg4_three_views"]
    a = gpu_forward(scene, cams, persistent=True, tile=tile)
    b = gpu_forward(scene, cams, persistent=False, tile=tile)
    dl = torch.randn(a.images.numel(), device="cuda")
    ga, _ = R.backward_pass(a, dl)
    gb, _ = R.backward_pass(b, dl)
    torch.cuda.synchronize()
    # same per-entry sums; only the order of the float atomics differs
    # between the two schedules, so compare each parameter plane by norm
    # (float32 sums of many signed terms per kernel: at 8-pixel tiles a
    # kernel takes several times more atomics, and the scale planes, whose
    # terms cancel, differ by ~1e-5 of their norm)
    diff = (ga - gb).norm(dim=1)
    scale = ga.norm(dim=1).clamp_min(1e-30)
    assert float((diff / scale).max()) <= 1e-4


@pytest.mark.parametrize("name,tile", [("cfg4_three_views", 32), ("cfg4_three_views", 16),
                                       ("cfg4_three_views", 8), ("cfg3_small", 32)])
def test_per_tile_backward_covers_every_tile_once(name, tile):
    """With dL/dimage = 1 each record's colour gradient is a sum of
    non-negative terms (alpha T), so the float-atomic order moves it by a few
    ulps only, while a tile that a schedule skipped or took twice changes it
    outright: the per-tile grid (XCD-grouped block order) and the persistent
    queue give the same sums record by record."""
    scene, cams = CASES[name]
    a = gpu_forward(scene, cams, persistent=False, tile=tile)
    b = gpu_forward(scene, cams, persistent=True, tile=tile)
    one = torch.ones(a.images.numel(), device="cuda")
    sums = []
    for fr in (a, b):
        rg = torch.zeros(fr.n * len(fr.cams) * B.HGS_RECORD_GRAD_FLOATS, device="cuda")
        B.hgs_raster_bwd(fr.records, fr.values, fr.ranges, fr.tile_order, fr.cams, fr.opts, fr.T_final,
                         fr.last_idx, one, rg, fr.ws_render, torch.cuda.current_stream().cuda_stream)
        sums.append(rg.view(-1, B.HGS_RECORD_GRAD_FLOATS)[:, 9:12])
    torch.cuda.synchronize()
    ga, gb = sums
    assert bool((gb >= 0).all()) and float(gb.max()) > 0
    tol = 1e-4 * gb.abs() + 1e-7 * float(gb.abs().max())
    assert int(((ga - gb).abs() > tol).sum()) == 0


@pytest.mark.parametrize("name,tile,persistent", [("cfg4_three_views", 32, False), ("cfg4_three_views", 32, True),
                                                  ("cfg4_three_views", 16, False), ("cfg4_three_views", 8, True),
                                                  ("cfg3_small", 32, False)])
def test_backward_strip_marks_skip_nothing(name, tile, persistent):
    """hgs_raster_bwd skips entries and pixel strips that the forward pass
    marked as blending nothing; replayed in full (a workspace without marks,
    or marks whose tag does not match) it gives the same record gradients:
    with dL/dimage = 1 the colour sums (non-negative terms, only the atomic
    order differs) within a few ulps record by record, with a seeded dL/dimage
    all twelve within 1e-4 of each record's gradient norm."""
    scene, cams = CASES[name]
    fr = gpu_forward(scene, cams, persistent=persistent, tile=tile)
    _marked_backward_equals_full_replay(fr)


@pytest.mark.parametrize("persistent", [False, True])
def test_backward_strip_marks_past_the_staged_rounds(persistent):
    """A forward walk longer than the rounds whose marks are staged in LDS
    (2048 list positions) marks the rest in full: 4000 faint kernels that all
    cover a 64x64 view keep its pixels open past position 2048, and the
    backward still equals a full replay."""
    scene, _ = scenes.make_config(1, n=4000)
    n = scene["means"].shape[0]
    scene = dict(scene, scales=np.full((n, 3), 2.0, np.float32),
                 opac1=np.full(n, 0.007, np.float32), opac2=np.full(n, 0.005, np.float32))
    cam = scenes.axis_camera(64, 64)
    fr = gpu_forward(scene, [cam], persistent=persistent, tile=32)
    torch.cuda.synchronize()
    assert int(fr.last_idx.max()) >= 2048
    _marked_backward_equals_full_replay(fr)


def _marked_backward_equals_full_replay(fr):
    assert fr.ws_render.numel() > 256            # room for the marks
    st = torch.cuda.current_stream().cuda_stream
    bare = torch.zeros(256, dtype=torch.uint8, device="cuda")
    untagged = fr.ws_render.clone()
    untagged[64:72] = 0
    n_rec = fr.n * len(fr.cams)
    for dl in (torch.ones(fr.images.numel(), device="cuda"),
               torch.randn(fr.images.numel(), device="cuda", generator=torch.Generator("cuda").manual_seed(5))):
        out = []
        for ws in (fr.ws_render, bare, untagged):
            rg = torch.zeros(n_rec * B.HGS_RECORD_GRAD_FLOATS, device="cuda")
            B.hgs_raster_bwd(fr.records, fr.values, fr.ranges, fr.tile_order, fr.cams, fr.opts, fr.T_final,
                             fr.last_idx, dl, rg, ws, st)
            out.append(rg.view(n_rec, B.HGS_RECORD_GRAD_FLOATS))
        torch.cuda.synchronize()
        marked = out[0]
        assert float(marked.abs().max()) > 0
        for full in out[1:]:
            if bool((dl == 1).all()):
                a, b = marked[:, 9:12], full[:, 9:12]
                tol = 1e-4 * b.abs() + 1e-7 * float(b.abs().max())
            else:
                a, b = marked, full
                tol = 1e-4 * b.norm(dim=1, keepdim=True) + 1e-7 * float(b.abs().max())
            assert int(((a - b).abs() > tol).sum()) == 0


def test_gpu_matches_golden_fixture():
    """The stored oracle fixture of the 1000-kernel 128x128 workload
    (tests/golden/cfg1_oracle.json, 16-pixel tiles): every tile's list length
    exactly, and at its 256 pixels the colour within 1e-4 and the blended
    count exactly, away from ambiguous decisions."""
    import json
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    want = json.load(open(os.path.join(here, "cfg1_oracle.json")))
    scene, cams = scenes.make_config(1)
    fr = gpu_forward(scene, cams, tile=16)
    _, _, ranges = sorted_entries(fr)
    np.testing.assert_array_equal(ranges[:, 1] - ranges[:, 0], np.asarray(want["list_lengths"]))
    assert int(fr.n_dup.item()) == want["entries"]
    pix = np.asarray(want["pixels"])
    img = fr.image(0).cpu().numpy()[:, pix[:, 1], pix[:, 0]].T
    cnt = fr.per_pixel(fr.n_contrib, 0).cpu().numpy()[pix[:, 1], pix[:, 0]]
    ok = ~ambiguous(np.asarray(want["margin"]))
    assert ok.mean() > 0.99
    assert np.abs(img - np.asarray(want["values"]))[ok].max() <= 1e-4
    np.testing.assert_array_equal(cnt[ok], np.asarray(want["n_contrib"])[ok])


def test_flipped_normals_swap_halves():
    scene, cams = CASES["cfg2_halfclear"]
    flipped = dict(scene, normals=-scene["normals"], opac1=scene["opac2"], opac2=scene["opac1"])
    a = gpu_forward(scene, cams)
    b = gpu_forward(flipped, cams)
    ka, va, ra = sorted_entries(a)
    kb, vb, rb = sorted_entries(b)
    np.testing.assert_array_equal(ka, kb)
    np.testing.assert_array_equal(va, vb)
    assert (a.images - b.images).abs().max().item() < 1e-5


def test_equal_opacities_take_the_standard_gaussian_path():
    scene, cams = CASES["cfg2_small"]
    eq = scenes.with_equal_opacities(scene)
    fr = gpu_forward(eq, cams)
    f, _ = records_np(fr)
    assert np.all(f[:, 11] == 0.0)   # delta opacity exactly zero -> no half factor
    _check_render(eq, cams, fr, oracle_pre(eq, cams))


def test_full_box_mode_matches_oracle():
    scene, cams = CASES["cfg2_halfclear"]
    fr = gpu_forward(scene, cams, full_box=True)
    pres = oracle_pre(scene, cams, full_box=True)
    _check_records(scene, cams, fr, pres)
    _check_render(scene, cams, fr, pres)
    half = gpu_forward(scene, cams)
    assert int(half.n_dup.item()) < int(fr.n_dup.item())


# ---------------------------------------------------------------------------
# gradients
# ---------------------------------------------------------------------------
def _grad_case(scene, cams, seed=5, **kw):
    fr = gpu_forward(scene, cams, **kw)
    pres = oracle_pre(scene, cams, **kw)
    rng = np.random.default_rng(seed)
    dls = []
    for c, (cam, pre) in enumerate(zip(cams, pres)):
        ref = O.render(pre, "e2e")
        w = rng.normal(size=(3, cam["height"], cam["width"]))
        w[:, ambiguous(ref["margin"])] = 0.0        # no gradient through ambiguous pixels
        dls.append(w)
    packed = torch.cat([torch.as_tensor(w, dtype=torch.float32).reshape(-1) for w in dls]).cuda()
    grads, _ = R.backward_pass(fr, packed)
    torch.cuda.synchronize()
    _, o = split_opts(kw)
    ref = O.render_grad(scene, cams, dls, o)
    K = scene["sh"].shape[1]
    got = dict(zip(O.PARAM_KEYS, [t.cpu().numpy() for t in R.natural_from_soa(grads, K)]))
    check_gradients(got, ref)


def test_gradients_match_oracle_small():
    scene, _ = scenes.make_config(2, n=64)
    cams = [scenes.axis_camera(32, 32, distance=2.5)]
    _grad_case(scene, cams)


def test_gradients_match_oracle_degree3_ragged():
    scene, _ = scenes.make_config(2, n=1500)
    cams = [scenes.axis_camera(150, 110, distance=3.0)]
    _grad_case(scene, cams)


def test_gradients_match_oracle_half_clear_multiview():
    scene, cams = scenes.make_config(4, n=1200, n_cams=2)
    cams = [scenes.pinhole(96, 72, c["R"], c["t"]) for c in cams]
    scene = scenes.with_transparent_halves(scene)
    _grad_case(scene, cams, seed=9, tile=8, batch=128)


def test_raster_bwd_record_gradients_match_oracle():
    """hgs_raster_bwd alone: the 12 per-record gradients against FP64
    autograd of the blend with the record fields as leaves; then
    hgs_preprocess_bwd on them equals hgs_render_bwd and clears them."""
    scene, _ = scenes.make_config(2, n=1500)
    scene = scenes.with_transparent_halves(scene)
    cam = scenes.axis_camera(150, 110, distance=3.0)
    fr = gpu_forward(scene, [cam])
    pre = oracle_pre(scene, [cam])[0]
    ref_amb = O.render(pre, "e2e")
    w = np.random.default_rng(4).normal(size=(3, 110, 150))
    w[:, ambiguous(ref_amb["margin"])] = 0.0
    dl = torch.as_tensor(w, dtype=torch.float32).reshape(-1).cuda()
    n_rec = fr.n
    rg = torch.zeros(n_rec * B.HGS_RECORD_GRAD_FLOATS, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    B.hgs_raster_bwd(fr.records, fr.values, fr.ranges, fr.tile_order, fr.cams, fr.opts, fr.T_final, fr.last_idx,
                     dl, rg, fr.ws_render, st)
    torch.cuda.synchronize()
    got = rg.cpu().numpy().reshape(n_rec, B.HGS_RECORD_GRAD_FLOATS).astype(np.float64)
    idx, ref = O.record_grads(scene, cam, w)
    refm = np.concatenate([ref["mu_rel"], ref["conic"], ref["k"], ref["alpha2"][:, None],
                           ref["d_o"][:, None], ref["colour"]], 1)
    gotm = got[idx]
    assert np.all(got[np.setdiff1d(np.arange(n_rec), idx)] == 0)
    for q in range(B.HGS_RECORD_GRAD_FLOATS):
        g, r = gotm[:, q], refm[:, q]
        rel = np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-30)
        assert rel <= 1e-3, (q, rel)
    # the chain rule half equals the full call and clears the buffer
    grads = torch.zeros_like(fr.soa)
    params = B.params_struct(fr.soa, fr.n, fr.soa.shape[1], fr.sh_degree)
    B.hgs_preprocess_bwd(params, fr.cams, fr.opts, fr.records, rg, B.grads_struct(grads, fr.soa.shape[1]), st)
    g_ref, _ = R.backward_pass(fr, dl)
    torch.cuda.synchronize()
    assert (rg == 0).all()
    assert torch.allclose(grads, g_ref, rtol=1e-4, atol=1e-7)


def test_autograd_function_matches_backward_pass():
    scene, _ = scenes.make_config(2, n=500)
    cams = [scenes.axis_camera(64, 48, distance=3.0)]
    t = {k: torch.tensor(scene[k], device="cuda", requires_grad=True)
         for k in ("means", "scales", "quats", "normals", "opac1", "opac2", "sh")}
    imgs = R.rasterize(t["means"], t["scales"], t["quats"], t["normals"], t["opac1"], t["opac2"], t["sh"], cams)
    target = torch.rand_like(imgs[0])
    loss = (imgs[0] - target).abs().mean()
    loss.backward()
    fr = gpu_forward(scene, cams)
    dl = (torch.sign(fr.image(0) - target) / target.numel()).reshape(-1)
    grads, _ = R.backward_pass(fr, dl.contiguous())
    ref = R.natural_from_soa(grads, scene["sh"].shape[1])
    for k, r in zip(("means", "scales", "quats", "normals", "opac1", "opac2", "sh"), ref):
        assert torch.allclose(t[k].grad, r.reshape(t[k].shape), rtol=1e-5, atol=1e-9), k


def test_rasterizer_planes_match_the_pipeline_and_rerun_on_overflow():
    """The autograd Rasterizer over a structure-of-arrays parameter tensor:
    images bit-identical to the stage-by-stage pipeline, gradients (returned
    in the same plane layout) equal to backward_pass up to the order of the
    float atomics; a call whose entries overflow the capacity kept from the
    previous call grows it and runs the sort and raster again."""
    scene, cams = CASES["cfg4_three_views"]
    n, K = scene["means"].shape[0], scene["sh"].shape[1]
    soa = R.scene_to_soa(scene)
    planes = soa.clone().requires_grad_(True)
    rast = R.Rasterizer(cams, scene["sh_degree"], tile=16)
    img = rast(planes)
    fr = gpu_forward(scene, cams, tile=16)
    assert torch.equal(img.detach(), fr.images)
    dl = torch.randn_like(img)
    img.backward(dl)
    g_ref, _ = R.backward_pass(fr, dl)
    torch.cuda.synchronize()

    def same_grads(g):
        # per plane, up to the order of the float atomics, which differs
        # between any two runs: repeated runs of this case differ by
        # 2.5e-7 to 3.8e-6 per plane, dominated by single kernels whose
        # gradient cancels (one element off by 4e-4 of itself), and once
        # by more than 1e-5
        return float(((g - g_ref).norm(dim=1) / g_ref.norm(dim=1).clamp_min(1e-30)).max()) <= 1e-4

    assert same_grads(planes.grad)
    assert rast.overflows == 0
    # a scene with more entries than the capacity sized on the first call
    rast.capacity = max(1, int(fr.n_dup.item()) // 3)
    planes.grad = None
    img2 = rast(planes)
    assert rast.overflows == 1 and rast.capacity >= int(fr.n_dup.item())
    assert torch.equal(img2.detach(), fr.images)
    img2.backward(dl)
    torch.cuda.synchronize()
    assert same_grads(planes.grad)


@pytest.mark.parametrize("tile", [32, 16])
def test_backward_after_a_forward_of_other_lists(tile):
    """The strip marks of an earlier forward pass over other lists stay in
    the workspace wherever the current pass marked nothing; the backward of
    the current pass still equals a fresh forward + backward of its scene
    (a stale mark only costs a full evaluation of a strip)."""
    scene, cams = CASES["cfg4_three_views"]
    other = dict(scene, means=(scene["means"] + np.random.default_rng(3).normal(
        scale=0.05, size=scene["means"].shape)).astype(np.float32))
    rast = R.Rasterizer(cams, scene["sh_degree"], tile=tile)
    with torch.no_grad():
        rast(R.scene_to_soa(other))
    planes = R.scene_to_soa(scene).clone().requires_grad_(True)
    img = rast(planes)
    dl = torch.randn(img.shape, device="cuda", generator=torch.Generator("cuda").manual_seed(8))
    img.backward(dl)
    fr = gpu_forward(scene, cams, tile=tile)
    assert torch.equal(img.detach(), fr.images)
    g_ref, _ = R.backward_pass(fr, dl)
    torch.cuda.synchronize()
    rel = (planes.grad - g_ref).norm(dim=1) / g_ref.norm(dim=1).clamp_min(1e-30)
    assert float(rel.max()) <= 1e-4


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------
def test_empty_scene_and_all_culled():
    scene, cams = scenes.make_config(1, n=0)
    fr = gpu_forward(scene, cams)
    assert int(fr.n_dup.item()) == 0
    assert fr.images.abs().max().item() == 0.0 and fr.T_final.min().item() == 1.0
    scene, cams = scenes.make_config(1, n=200)
    behind = dict(scene, means=(scene["means"] - np.float32([0, 0, 10])).astype(np.float32))
    fr = gpu_forward(behind, cams)
    assert int(fr.n_dup.item()) == 0 and (fr.n_contrib.cpu() == 0).all()


def test_one_pixel_and_ragged_images():
    scene, _ = scenes.make_config(1, n=300)
    for w, h in ((1, 1), (17, 5), (33, 47)):
        cams = [scenes.axis_camera(w, h, distance=1.5)]
        fr = gpu_forward(scene, cams, tile=16)
        pres = oracle_pre(scene, cams)
        keys, vals, ranges = sorted_entries(fr)
        bs = O.bin_sort(pres)
        np.testing.assert_array_equal(keys, bs["keys"])
        _check_render(scene, cams, fr, pres)


def test_capacity_overflow_is_flagged_and_safe():
    scene, cams = CASES["cfg1"]
    fr = gpu_forward(scene, cams, capacity=100)
    assert int(fr.n_dup.item()) > 100
    assert int(fr.overflow.item()) == 1
    ranges = u32(fr.ranges)
    assert (ranges == 0).all()
    assert fr.images.abs().max().item() == 0.0


def test_non_finite_and_degenerate_parameters_are_culled_or_defined():
    scene, cams = scenes.make_config(1, n=50)
    bad = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in scene.items()}
    bad["means"][0, 0] = np.nan
    bad["scales"][1, 2] = np.inf
    bad["quats"][2] = 0.0            # identity rotation
    bad["normals"][3] = 0.0          # no preferred side: half factor 1
    bad["opac1"][4] = np.nan
    fr = gpu_forward(bad, cams)
    _, u = records_np(fr)
    assert u[0, 15] == 0 and u[1, 15] == 0 and u[4, 15] == 0
    pres = oracle_pre(bad, cams)
    valid = pres[0]["valid"].numpy()
    np.testing.assert_array_equal(u[:, 15] > 0, valid)
    f, _ = records_np(fr)
    assert f[3, 2] == 0.0 and f[3, 3] == 0.0


def test_maximum_camera_count_matches_oracle():
    """HGS_MAX_CAMERAS (32) views of uneven small sizes in one call: records,
    sorted lists (global tile ids across all 32 views) and every pixel
    against the oracle; one camera more is rejected."""
    scene, cams = scenes.make_config(4, n=2000, n_cams=B.HGS_MAX_CAMERAS)
    sizes = [(33 + 7 * (c % 5), 21 + 5 * (c % 7)) for c in range(len(cams))]
    cams = [scenes.pinhole(w, h, c["R"], c["t"]) for c, (w, h) in zip(cams, sizes)]
    print(f"[case] {len(cams)} cameras", flush=True)
    fr = gpu_forward(scene, cams, tile=16)
    pres = oracle_pre(scene, cams, tile=16)
    _check_records(scene, cams, fr, pres)
    bs = O.bin_sort(pres)
    _, vals, ranges = sorted_entries(fr)
    np.testing.assert_array_equal(vals, bs["vals"])
    np.testing.assert_array_equal(ranges, bs["ranges"])
    _check_render(scene, cams, fr, pres)
    with pytest.raises(B.HGSError) as e:
        gpu_forward(scene, cams + cams[:1], tile=16)
    assert e.value.code == B.HGS_EINVAL


def test_invalid_arguments_return_einval():
    scene, cams = scenes.make_config(1, n=10)
    with pytest.raises(B.HGSError) as e:
        gpu_forward(scene, cams, tile=12)
    assert e.value.code == B.HGS_EINVAL
    with pytest.raises(B.HGSError):
        gpu_forward(scene, cams, batch=64)


# ---------------------------------------------------------------------------
# full-size workload, sampled
# ---------------------------------------------------------------------------
@pytest.mark.slow
@pytest.mark.parametrize("tile,persistent", [(32, False), (16, True)])
def test_full_size_1080p_one_million_sampled(tile, persistent):
    """1M half-Gaussians at 1920x1080 (the benchmark workload, first in the
    benchmark's launch configuration: 32-pixel tiles, one workgroup per
    tile): every record's integer fields, the sorted lists of 64 sampled
    tiles and 1024 sampled pixels against the oracle."""
    scene, cams = scenes.make_config(3)
    print(f"[case] full-size 1080p 1M tile={tile} persistent={persistent}", flush=True)
    fr = gpu_forward(scene, cams, tile=tile, persistent=persistent)
    pres = oracle_pre(scene, cams, tile=tile)
    pre = pres[0]
    f, u = records_np(fr)
    valid = pre["valid"].numpy()
    np.testing.assert_array_equal(u[:, 15], pre["tiles_touched"].numpy().astype(np.uint32))
    np.testing.assert_array_equal(u[valid, 14], pre["depth_bits"][valid])
    r = pre["rect"].numpy()[valid]
    np.testing.assert_array_equal(u[valid, 12], (r[:, 0] | (r[:, 1] << 16)).astype(np.uint32))
    np.testing.assert_array_equal(u[valid, 13], (r[:, 2] | (r[:, 3] << 16)).astype(np.uint32))
    keys, vals, ranges = sorted_entries(fr)
    assert keys.size == int(pre["tiles_touched"].sum())
    assert np.all(keys[:-1] <= keys[1:])
    # sampled tiles: list = records covering the tile, by (depth, id)
    tr = pre["trect"].numpy()
    rng = np.random.default_rng(0)
    tx_n = pre["tiles_x"]
    for t in rng.choice(ranges.shape[0], 64, replace=False):
        ty, tx = divmod(int(t), tx_n)
        cover = np.nonzero(valid & (tr[:, 0] <= tx) & (tr[:, 1] >= tx) & (tr[:, 2] <= ty) & (tr[:, 3] >= ty))[0]
        order = np.lexsort((cover, pre["depth_bits"][cover]))
        s, e = ranges[t]
        np.testing.assert_array_equal(vals[s:e], cover[order].astype(np.uint32))
    # sampled pixels in REC mode
    pix = scenes.sample_pixels(cams[0], 1024, seed=3)
    ref = O.render(pre, "rec", pixels=pix)
    img = fr.image(0).cpu().numpy()[:, pix[:, 1], pix[:, 0]].T
    cnt = fr.per_pixel(fr.n_contrib, 0).cpu().numpy()[pix[:, 1], pix[:, 0]]
    ok = ~ambiguous(ref["margin"])
    print(f"[flagged-full] {int((~ok).sum())}/{ok.size}", flush=True)
    assert ok.mean() > 0.99
    assert np.abs(img - ref["values"].numpy())[ok].max() <= 1e-4
    np.testing.assert_array_equal(cnt[ok], ref["n_contrib"].numpy()[ok])


@pytest.mark.slow
def test_full_size_1080p_gradients_sampled():
    """Parameter gradients of all 1M kernels at 1920x1080 in the benchmark's
    launch configuration, with dL/dimage nonzero only at 512 seeded pixels
    (zero at ambiguous ones), against FP64 autograd of the oracle rendering
    just those pixels: per tensor relative L2 <= 1e-3 and elementwise
    |d| <= 1e-3 |ref| + 1e-5 max |ref|."""
    scene, cams = scenes.make_config(3)
    cam = cams[0]
    print("[case] full-size 1080p 1M gradients, 512 pixels", flush=True)
    fr = gpu_forward(scene, cams, tile=32, persistent=False)
    pre = oracle_pre(scene, cams, tile=32)[0]
    pix = scenes.sample_pixels(cam, 512, seed=21)
    amb = ambiguous(O.render(pre, "e2e", pixels=pix)["margin"])
    print(f"[flagged-full-grad] {int(amb.sum())}/{amb.size}", flush=True)
    assert amb.mean() < 0.01
    w = np.random.default_rng(4).normal(size=(pix.shape[0], 3))
    w[amb] = 0.0
    dl = np.zeros((3, cam["height"], cam["width"]), np.float32)
    dl[:, pix[:, 1], pix[:, 0]] = w.T
    grads, _ = R.backward_pass(fr, torch.as_tensor(dl).reshape(-1).cuda())
    torch.cuda.synchronize()
    ref = O.render_grad(scene, [cam], [w], O.options(tile=32), pixels=[pix])
    K = scene["sh"].shape[1]
    got = dict(zip(O.PARAM_KEYS, [t.cpu().numpy() for t in R.natural_from_soa(grads, K)]))
    check_gradients(got, ref, terms=kernel_terms(pre, pix), label="-1080p")


@pytest.mark.slow
def test_placement_equals_full_key_sort_at_4k_tile8():
    """Two 3840x2160 views with 8-pixel tiles (259k tiles, 127 bands) and
    150k kernels (300k records, blocks of ~4.6k records, far above the
    minimum): the entries placed by counting are the entries of the full
    64-bit radix sort, bit for bit, and so are the ranges and the tile
    order."""
    scene, cams = scenes.make_config(5, n=150_000, n_cams=2)
    print("[case] 4k tile-8 placement vs full keys", flush=True)
    a = gpu_forward(scene, cams, tile=8)
    b = gpu_forward(scene, cams, tile=8, sort_full_keys=True)
    n = int(a.n_dup.item())
    assert n == int(b.n_dup.item()) and n > 0
    ka, va, ra = sorted_entries(a)
    kb, vb, rb = sorted_entries(b)
    np.testing.assert_array_equal(ra, rb)
    np.testing.assert_array_equal(va, vb)
    np.testing.assert_array_equal(ka, kb)
    np.testing.assert_array_equal(u32(a.tile_order), u32(b.tile_order))


def test_placement_of_a_very_wide_image_matches_oracle():
    """A 4200 x 40 image at 8-pixel tiles: 525 tiles per row, a band wider
    than the 32-bit cursor layout takes (packed 16-bit cursors, entry-wise
    counting), sorted lists and ranges equal to the oracle's."""
    scene, _ = scenes.make_config(2, n=3000)
    cam = scenes.pinhole(4200, 40, np.eye(3), (0.0, 0.0, 3.0), hfov_deg=120.0)
    print("[case] wide image 4200x40 tile 8", flush=True)
    fr = gpu_forward(scene, [cam], tile=8)
    pres = oracle_pre(scene, [cam], tile=8)
    bs = O.bin_sort(pres)
    keys, vals, ranges = sorted_entries(fr)
    assert int(fr.overflow.item()) == 0
    assert vals.size == bs["vals"].size > 0
    np.testing.assert_array_equal(vals, bs["vals"])
    np.testing.assert_array_equal(ranges, bs["ranges"])


def test_blended_depth_matches_oracle():
    """The optional depth output of hgs_render_fwd against the oracle's
    blended depth (REC mode), relative to the depth scale, on the pixels
    whose decisions are not ambiguous; no depth requested gives the same
    image."""
    scene, cams = CASES["cfg2_small"]
    fr = gpu_forward(scene, cams)
    frd = R.forward_pass(R.scene_to_soa(scene), scene["means"].shape[0], scene["sh_degree"],
                         B.make_cameras(cams), B.default_options(), depth=True)
    torch.cuda.synchronize()
    assert torch.equal(fr.images, frd.images)
    pre = oracle_pre(scene, cams)[0]
    ref = O.render(pre, "rec")
    ok = ~ambiguous(ref["margin"])
    D = frd.per_pixel(frd.depth, 0).cpu().numpy()
    Dr = ref["depth"].numpy()
    scale = float(np.abs(Dr).max())
    assert scale > 0
    assert np.abs(D - Dr)[ok].max() <= 1e-4 * scale


def test_depth_normals_match_oracle_on_seeded_maps():
    """hgs_depth_normals against the oracle's estimate on seeded synthetic
    depth and transmittance maps (a tilted wavy surface with empty pixels),
    two cameras of different sizes packed one after the other."""
    _, cams = CASES["cfg4_three_views"]
    cams = cams[:2]
    Ds, Ts = scenes.depth_maps(cams, seed=7)
    depth = torch.from_numpy(np.concatenate([d.ravel() for d in Ds])).cuda()
    T_final = torch.from_numpy(np.concatenate([t.ravel() for t in Ts])).cuda()
    out = torch.empty(3 * depth.numel(), dtype=torch.float32, device="cuda")
    B.hgs_depth_normals(depth, T_final, B.make_cameras(cams), out, R._stream())
    torch.cuda.synchronize()
    off = 0
    for c, cam in enumerate(cams):
        H, W = cam["height"], cam["width"]
        ref = O.depth_normals(Ds[c], Ts[c], cam)
        got = out[3 * off:3 * (off + H * W)].view(3, H, W).cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-5
        assert (np.abs(ref).sum(0) > 0).mean() > 0.5
        off += H * W


def test_depth_normals_of_a_render_match_oracle():
    """End to end: normals from the GPU's depth and transmittance against
    the oracle's from its own (REC mode), on pixels whose 3x3 neighbourhood
    holds no ambiguous decision.  The finite differences divide depth errors
    (~1e-6 relative) by neighbour depth differences, so the bound is loose."""
    scene, cams = CASES["cfg2_small"]
    fr = R.forward_pass(R.scene_to_soa(scene), scene["means"].shape[0], scene["sh_degree"],
                        B.make_cameras(cams), B.default_options(), depth=True)
    nrm = R.depth_normals(fr)
    torch.cuda.synchronize()
    pre = oracle_pre(scene, cams)[0]
    ref = O.render(pre, "rec")
    cam = cams[0]
    H, W = cam["height"], cam["width"]
    want = O.depth_normals(ref["depth"].numpy(), ref["T_final"].numpy(), cam)
    got = nrm[:3 * H * W].view(3, H, W).cpu().numpy()
    amb = ambiguous(ref["margin"])
    near = amb.copy()
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            near |= np.roll(np.roll(amb, dy, 0), dx, 1)
    # the expected depth divides by 1 - T: keep pixels with real coverage
    acc = 1.0 - ref["T_final"].numpy()
    thin = acc < 0.1
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            near |= np.roll(np.roll(thin, dy, 0), dx, 1)
    ok = ~near
    assert ok.mean() > 0.5
    err = np.abs(got - want).max(0)[ok]
    print(f"normals: {ok.sum()} pixels, err q50 {np.median(err):.2e} q99 {np.quantile(err, 0.99):.2e} max {err.max():.2e}")
    assert np.quantile(err, 0.99) <= 1e-3
    assert err.max() <= 5e-2


def test_white_kernels_on_black_image_is_one_minus_transmittance():
    """All colours 1 and a black background: each channel is the total
    blending weight, 1 - T_final (an identity of front-to-back
    compositing)."""
    scene, cams = CASES["cfg4_three_views"]
    scene = dict(scene)
    sh = np.zeros_like(np.asarray(scene["sh"], np.float32))
    sh[:, 0, :] = np.float32(0.5 / 0.28209479177387814)     # 0.5 + Y00 c = 1
    scene["sh"] = sh
    fr = gpu_forward(scene, cams)
    for c in range(len(cams)):
        img = fr.image(c).cpu().numpy().astype(np.float64)
        T = fr.per_pixel(fr.T_final, c).cpu().numpy().astype(np.float64)
        assert np.abs(img - (1.0 - T)[None]).max() <= 1e-5
        assert (T < 1.0).mean() > 0.2 and np.all((T >= 0.0) & (T <= 1.0))
