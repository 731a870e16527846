"""hgs_preprocess_noalloc (the preprocess entry point for callers that cannot
allocate) against hgs_preprocess with a caller workspace, through the C ABI:
records, tiles touched, entry offsets and the entry total bit for bit, on two
calls in a row, the second with a smaller input (its scan partials must not
depend on what the first call left in the library's device array)."""
import numpy as np
import pytest
import torch

from paper_2406_02720_amd import binding as B
from paper_2406_02720_amd import raster as R
from paper_2406_02720_amd import scenes

pytestmark = pytest.mark.gpu


def _run(scene, cams, no_alloc, with_offsets=True):
    n = scene["means"].shape[0]
    soa = R.scene_to_soa(scene)
    ca = B.make_cameras(cams)
    opts = B.default_options(tile=16)
    params = B.params_struct(soa, n, soa.shape[1], scene["sh_degree"])
    n_rec = n * len(cams)
    records = torch.full((max(n_rec, 1) * B.HGS_RECORD_BYTES,), 0xA5, dtype=torch.uint8, device="cuda")
    tiles = torch.full((max(n_rec, 1),), -1, dtype=torch.int32, device="cuda")
    offsets = torch.full((max(n_rec, 1),), -1, dtype=torch.int64, device="cuda") if with_offsets else None
    n_dup = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    if no_alloc:
        B.hgs_preprocess_noalloc(params, ca, opts, records, tiles, offsets, n_dup, st)
    else:
        ws = torch.empty(max(B.hgs_workspace_bytes(B.HGS_WS_PREPROCESS, n_rec, ca, opts), 1), dtype=torch.uint8,
                         device="cuda")
        B.hgs_preprocess(params, ca, opts, records, tiles, offsets, n_dup, ws, st)
    torch.cuda.synchronize()
    out = [records.cpu(), tiles.cpu(), n_dup.cpu()]
    if with_offsets:
        out.append(offsets.cpu())
    return out


def _same(a, b):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_noalloc_preprocess_equals_workspace_preprocess():
    # first call: 3 views x 30k kernels = 90k records (22 scan partials);
    # second: 2 views x 5k kernels = 10k records (3 partials, still above the
    # single-block scan), then 2 x 700 records (the single-block scan), each
    # with and without per-record offsets
    big, cams_big = scenes.make_config(4, n=30000, n_cams=3)
    cams_big = [scenes.pinhole(w, h, c["R"], c["t"]) for c, (w, h) in zip(cams_big, ((320, 200), (257, 130), (160, 90)))]
    small, cams_small = scenes.make_config(4, n=5000, n_cams=2)
    cams_small = [scenes.pinhole(w, h, c["R"], c["t"]) for c, (w, h) in zip(cams_small, ((200, 150), (129, 84)))]
    tiny, _ = scenes.make_config(4, n=350, n_cams=2)
    for name, scene, cams in (("90k records", big, cams_big), ("10k records", small, cams_small),
                              ("700 records", tiny, cams_small)):
        for with_offsets in (True, False):
            print(f"[case] no-alloc preprocess {name} offsets={with_offsets}", flush=True)
            ref = _run(scene, cams, False, with_offsets)
            got = _run(scene, cams, True, with_offsets)
            _same(got, ref)
            assert int(ref[2].item()) > 0
            if with_offsets:
                t = ref[1].numpy().astype(np.int64)
                np.testing.assert_array_equal(ref[3].numpy(), np.concatenate([[0], np.cumsum(t)[:-1]]))
