"""Writes cfg1_oracle.json beside this script: a regression fixture of the
FP64 oracle on the 1000-kernel 128x128 workload (SH degree 0, 16-pixel
tiles): the length of every tile's sorted list and, at 256 seeded pixels,
the REC-mode colour, final transmittance, blended count and decision margins.

It calls only the oracle and the seeded input generator.  The paper prints no
worked numerical example, so no value here comes from the paper; the fixture
records what the oracle computes for this input, so that a later change to
the oracle's arithmetic shows up as a diff of this file.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import hgs_oracle as O            # noqa: E402
from paper_2406_02720_amd import scenes       # noqa: E402

PATH = os.path.join(HERE, "cfg1_oracle.json")


def compute() -> dict:
    scene, cams = scenes.make_config(1)
    o = O.options(tile=16)
    with torch.no_grad():
        pre = O.preprocess(O.scene_to_torch(scene), O.camera_to_torch(cams[0]), o)
    bs = O.bin_sort([pre])
    ranges = np.asarray(bs["ranges"], np.int64).reshape(-1, 2)
    pix = scenes.sample_pixels(cams[0], 256, seed=17)
    ref = O.render(pre, "rec", pixels=pix)
    return {
        "workload": "1000 half-Gaussians, 128x128, SH degree 0, 16-pixel tiles (scenes.make_config(1))",
        "generator": "tests/golden/make_golden.py (oracle only)",
        "entries": int(pre["tiles_touched"].sum()),
        "list_lengths": (ranges[:, 1] - ranges[:, 0]).tolist(),
        "pixels": pix.tolist(),
        "values": ref["values"].numpy().tolist(),
        "T_final": ref["T_final"].numpy().tolist(),
        "n_contrib": ref["n_contrib"].numpy().astype(int).tolist(),
        "margin": ref["margin"].numpy().tolist(),
    }


if __name__ == "__main__":
    with open(PATH, "w") as f:
        json.dump(compute(), f, indent=0)
        f.write("\n")
    print("wrote", PATH)
