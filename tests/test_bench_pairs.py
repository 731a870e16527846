"""bench.PipelineStep.pair_counts (the raster's work count behind the FLOP
roofline) against a per-pixel brute force on CPU tensors: pairs inside a
record's rect up to the pixel's last blended entry, and those past the
exponent bound."""
import math
import types

import numpy as np
import torch

import bench


def _brute(recs, lists, last, cams, T):
    L2E = 1.4426950408889634
    pairs = tested = 0
    pix_off = t0 = 0
    for W, H in cams:
        tx = (W + T - 1) // T
        for py in range(H):
            for px in range(W):
                t = t0 + (py // T) * tx + px // T
                L = last[pix_off + py * W + px]
                for pos, r in enumerate(lists[t]):
                    if pos > L:
                        break
                    x0, x1 = recs[r, 12] & 0xffff, recs[r, 12] >> 16
                    y0, y1 = recs[r, 13] & 0xffff, recs[r, 13] >> 16
                    if not (x0 <= px <= x1 and y0 <= py <= y1):
                        continue
                    pairs += 1
                    f = recs[r].view(np.float32).astype(np.float64)
                    dx, dy = px + 0.5 - x0 - f[0], py + 0.5 - y0 - f[1]
                    p2 = -0.5 * L2E * (f[4] * dx * dx + f[6] * dy * dy) - L2E * f[5] * dx * dy
                    hb = max(f[7], f[7] + 2 * f[11])
                    tested += p2 <= 0 and p2 >= math.log2(1 / 255) - math.log2(hb) - 2 ** -10
        pix_off += W * H
        t0 += tx * ((H + T - 1) // T)
    return pairs, tested


def test_pair_counts_match_brute_force():
    rng = np.random.default_rng(3)
    T = 8
    cams = [(37, 21), (16, 9)]
    n_rec = 50
    recs = np.zeros((n_rec, 16), np.int32)
    for i in range(n_rec):
        W, H = cams[0] if i < 25 else cams[1]
        x0 = rng.integers(0, W); x1 = rng.integers(x0, W)
        y0 = rng.integers(0, H); y1 = rng.integers(y0, H)
        recs[i, 12] = x0 | (x1 << 16)
        recs[i, 13] = y0 | (y1 << 16)
        fl = np.array([rng.uniform(0, x1 - x0 + 1), rng.uniform(0, y1 - y0 + 1), 0, 0, rng.uniform(0.05, 1),
                       rng.uniform(-0.02, 0.02), rng.uniform(0.05, 1), rng.uniform(0.1, 0.9)], np.float32)
        recs[i, 0:8] = fl.view(np.int32)
        recs[i, 11] = np.float32(rng.uniform(-0.05, 0.05)).view(np.int32)
    nt = sum(((W + T - 1) // T) * ((H + T - 1) // T) for W, H in cams)
    lists = [rng.choice(n_rec, size=rng.integers(0, 12), replace=False) for _ in range(nt)]
    vals = np.concatenate(lists).astype(np.int32)
    ranges = np.zeros((nt, 2), np.int32)
    o = 0
    for t, lst in enumerate(lists):
        ranges[t] = (o, o + len(lst)) if len(lst) else (0, 0)    # empty tiles read [0, 0)
        o += len(lst)
    npix = sum(W * H for W, H in cams)
    last = rng.integers(-1, 12, size=npix).astype(np.int32)
    step = types.SimpleNamespace(
        torch=torch, records=torch.from_numpy(recs.view(np.uint8).reshape(-1)),
        ranges=torch.from_numpy(ranges.reshape(-1)), values=torch.from_numpy(vals),
        last_idx=torch.from_numpy(last), n_contrib=torch.zeros(npix, dtype=torch.int32),
        opts=types.SimpleNamespace(tile=T, alpha_min=1 / 255),
        cameras=[dict(width=W, height=H) for W, H in cams])
    pairs, tested, listed, blended = bench.PipelineStep.pair_counts(step, chunk=7)
    assert (pairs, tested) == _brute(recs, lists, last, cams, T)
    assert listed == int((last + 1).sum()) and blended == 0
    assert 0 < tested < pairs < listed
