"""The sort alone (no raster): hgs_preprocess + hgs_bin_sort against the
oracle's sorted lists, over tile sizes, camera mixes and band widths
(including a band wider than the 32-bit cursor layout).  Collected before
the other GPU tests so that a placement error shows here, before any raster
consumes the lists."""
import numpy as np
import pytest

from oracle import hgs_oracle as O
from paper_2406_02720_amd import scenes

from hgs_testlib import gpu_forward, oracle_pre, sorted_entries

pytestmark = pytest.mark.gpu


def _cases():
    s2, _ = scenes.make_config(2, n=20000)
    c2 = [scenes.pinhole(320, 180, np.eye(3), (0.0, 0.0, 3.0))]
    s4, c4 = scenes.make_config(4, n=6000, n_cams=3)
    c4 = [scenes.pinhole(w, h, c["R"], c["t"]) for c, (w, h) in zip(c4, ((200, 150), (129, 84), (160, 106)))]
    sw, _ = scenes.make_config(2, n=3000)
    cw = [scenes.pinhole(4200, 40, np.eye(3), (0.0, 0.0, 3.0), hfov_deg=120.0)]
    return {"single": (s2, c2), "three_views": (s4, c4), "wide": (sw, cw)}


CASES = _cases()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("tile", [8, 16, 32])
def test_sorted_lists_match_oracle_without_raster(name, tile):
    scene, cams = CASES[name]
    print(f"[case] placement only {name} tile={tile}", flush=True)
    fr = gpu_forward(scene, cams, tile=tile, render=False)
    pres = oracle_pre(scene, cams, tile=tile)
    bs = O.bin_sort(pres)
    keys, vals, ranges = sorted_entries(fr)
    assert int(fr.overflow.item()) == 0
    assert vals.size == bs["vals"].size
    np.testing.assert_array_equal(vals, bs["vals"])
    np.testing.assert_array_equal(keys, bs["keys"])
    np.testing.assert_array_equal(ranges, bs["ranges"])


def _check(scene, cams, tile):
    fr = gpu_forward(scene, cams, tile=tile, render=False)
    pres = oracle_pre(scene, cams, tile=tile)
    bs = O.bin_sort(pres)
    keys, vals, ranges = sorted_entries(fr)
    assert int(fr.overflow.item()) == 0
    assert vals.size == bs["vals"].size
    np.testing.assert_array_equal(vals, bs["vals"])
    np.testing.assert_array_equal(keys, bs["keys"])
    np.testing.assert_array_equal(ranges, bs["ranges"])
    return vals.size


@pytest.mark.parametrize("tile", [8, 32])
def test_all_equal_depths_order_by_record_id(tile):
    """Every kernel at the same camera depth: each list is in record id
    order (the tie rule), across two cameras at the same distance."""
    scene, _ = scenes.make_config(2, n=5000)
    scene = dict(scene)
    m = np.asarray(scene["means"], np.float32).copy()
    m[:, 2] = np.float32(0.0)
    scene["means"] = m
    cams = [scenes.pinhole(160, 120, np.eye(3), (0.0, 0.0, 3.0)),
            scenes.pinhole(96, 64, np.eye(3), (0.1, 0.0, 3.0))]
    assert _check(scene, cams, tile) > 1000


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_single_tile_image_and_a_single_entry(tile):
    scene, _ = scenes.make_config(2, n=3000)
    cams = [scenes.pinhole(8, 8, np.eye(3), (0.0, 0.0, 3.0))]
    assert _check(scene, cams, tile) > 0
    one = scenes.subset(scene, np.array([0]))
    one = dict(one)
    one["means"] = np.zeros((1, 3), np.float32)
    one["scales"] = np.full((1, 3), 0.002, np.float32)
    assert _check(one, [scenes.pinhole(8, 8, np.eye(3), (0.0, 0.0, 3.0))], tile) == 1
