"""Pins of the training-step oracle (Adam with the 3D-GS / half-Gaussian
schedule, densification statistics, densify / prune / reset) against values
fixed independently of its code: closed forms of the schedule, torch's own
Adam and autograd, eigenvalues, and hand-built cases whose outcome is known."""
import math

import numpy as np
import pytest
import torch

from oracle import hgs_train_oracle as T


def test_learning_rate_schedule_closed_forms():
    ext = 2.5
    a, b = 1.6e-4 * ext, 1.6e-6 * ext
    assert T.learning_rates(0, ext)["means"] == pytest.approx(a, rel=1e-14)
    assert T.learning_rates(30000, ext)["means"] == pytest.approx(b, rel=1e-14)
    assert T.learning_rates(60000, ext)["means"] == pytest.approx(b, rel=1e-14)
    assert T.learning_rates(15000, ext)["means"] == pytest.approx(math.sqrt(a * b), rel=1e-12)
    # the half-Gaussian rates: normal 0.003, opacity and normal / 1.4 every 5000
    for t, k in ((1, 0), (4999, 0), (5000, 1), (9999, 1), (10000, 2), (29999, 5)):
        lr = T.learning_rates(t, ext)
        assert lr["normals"] == pytest.approx(0.003 / 1.4 ** k, rel=1e-14)
        assert lr["opac"] == pytest.approx(0.05 / 1.4 ** k, rel=1e-14)
        assert lr["scales"] == 0.005 and lr["quats"] == 0.001
        assert lr["sh_dc"] == 0.0025 and lr["sh_rest"] == pytest.approx(0.000125, rel=1e-15)


def _random_state(n, sh_degree, seed):
    rng = np.random.default_rng(seed)
    raw = {k: rng.normal(size=(w, n)) for k, w in T.WIDTH.items()}
    raw["sh"] = rng.normal(size=(T.sh_planes(sh_degree), n))
    g = {k: rng.normal(scale=1e-2, size=a.shape) for k, a in raw.items()}
    return raw, g


def test_activation_chain_rule_is_autograd():
    raw, g = _random_state(50, 1, 1)
    got = T.raw_gradients(raw, g)
    for k in T.PLANES:
        x = torch.tensor(raw[k], dtype=torch.float64, requires_grad=True)
        y = torch.exp(x) if k == "scales" else torch.sigmoid(x) if k.startswith("opac") else x * 1.0
        (y * torch.tensor(g[k])).sum().backward()
        np.testing.assert_allclose(got[k], x.grad.numpy(), rtol=1e-14, atol=0)


def test_adam_step_is_torch_adam_with_group_rates():
    """Three steps of the oracle against torch.optim.Adam (float64) with one
    parameter group per learning-rate group, eps 1e-15."""
    n, D = 40, 3
    raw, _ = _random_state(n, D, 2)
    rng = np.random.default_rng(3)
    lrs_of = lambda t: T.learning_rates(t, 3.0)  # noqa: E731
    # torch side: one tensor per (plane-group) so each gets its own rate
    groups = dict(means=("means", slice(None)), scales=("scales", slice(None)), quats=("quats", slice(None)),
                  normals=("normals", slice(None)), opac1=("opac1", slice(None)), opac2=("opac2", slice(None)),
                  sh_dc=("sh", slice(0, 3)), sh_rest=("sh", slice(3, None)))
    tens = {g: torch.tensor(raw[k][s], dtype=torch.float64, requires_grad=True) for g, (k, s) in groups.items()}

    def lr_of(g, lrs):
        return lrs["opac"] if g.startswith("opac") else lrs[g]

    opt = torch.optim.Adam([{"params": [tens[g]], "lr": lr_of(g, lrs_of(1)), "name": g} for g in groups],
                           betas=(T.BETA1, T.BETA2), eps=T.EPS)
    m = {k: np.zeros_like(a) for k, a in raw.items()}
    v = {k: np.zeros_like(a) for k, a in raw.items()}
    cur = raw
    for t in (1, 2, 3):
        g_act = {k: rng.normal(scale=1e-2, size=a.shape) for k, a in raw.items()}
        lrs = lrs_of(t)
        cur, m, v, act = T.adam_step(cur, g_act, m, v, t, lrs)
        # torch: gradient of <g_act, activation(raw)>
        opt.zero_grad()
        for g, (k, s) in groups.items():
            x = tens[g]
            y = torch.exp(x) if k == "scales" else torch.sigmoid(x) if k.startswith("opac") else x
            (y * torch.tensor(g_act[k][s])).sum().backward()
        for pg in opt.param_groups:
            pg["lr"] = lr_of(pg["name"], lrs)
        opt.step()
        for g, (k, s) in groups.items():
            np.testing.assert_allclose(cur[k][s], tens[g].detach().numpy(), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(act["scales"], np.exp(cur["scales"]), rtol=1e-15)


def test_screen_radius_is_three_sigma_of_the_largest_axis():
    rng = np.random.default_rng(4)
    covs = []
    for _ in range(200):
        A = rng.normal(size=(2, 2)) * rng.uniform(0.5, 20.0)
        covs.append(A @ A.T + 0.3 * np.eye(2))
    covs = np.array(covs)
    inv = np.linalg.inv(covs)
    conic = np.stack([inv[:, 0, 0], inv[:, 0, 1], inv[:, 1, 1]], 1).astype(np.float32)
    lam = np.linalg.eigvalsh(np.linalg.inv(np.stack([conic[:, [0, 1]], conic[:, [1, 2]]], 1).astype(np.float64)))
    want = np.ceil(3.0 * np.sqrt(lam[:, -1]))
    got = T.screen_radius(conic)
    frac = 3.0 * np.sqrt(lam[:, -1])
    clear = np.abs(frac - np.round(frac)) > 1e-9
    np.testing.assert_array_equal(got[clear], want[clear])
    # axis-aligned: sigma_x = 4 -> radius 12
    assert T.screen_radius(np.array([[1 / 16.0, 0.0, 1 / 4.0]], np.float32))[0] == 12.0


def test_densify_stats_hand_case():
    """Two views of three kernels; kernel 1 unseen in the second view."""
    v1 = dict(width=100, height=50, idx=[0, 1], g_mean=[[1.0, 0.0], [0.0, 2.0]],
              conic=np.array([[1 / 4.0, 0.0, 1 / 4.0], [1.0, 0.0, 1.0]], np.float32))
    v2 = dict(width=200, height=100, idx=[0, 2], g_mean=[[0.3, 0.4], [0.0, 0.0]],
              conic=np.array([[1 / 64.0, 0.0, 1 / 16.0], [1.0, 0.0, 1.0]], np.float32))
    acc, cnt, rad = T.densify_stats(3, [v1, v2])
    np.testing.assert_allclose(acc, [50.0 + math.hypot(30.0, 20.0), 50.0, 0.0], rtol=1e-15)
    np.testing.assert_array_equal(cnt, [2, 1, 1])
    np.testing.assert_array_equal(rad, [24.0, 3.0, 3.0])


def _hand_state():
    """Six kernels: 0 keep, 1 clone (small, big gradient), 2 split (large,
    big gradient), 3 prune (both halves below 0.01), 4 kept (one half
    opaque), 5 split whose children are pruned by the world-scale rule."""
    ext = 1.0
    n = 6
    raw = {k: np.zeros((w, n)) for k, w in T.WIDTH.items()}
    raw["sh"] = np.arange(3 * n, dtype=np.float64).reshape(3, n)
    raw["means"] = np.arange(3 * n, dtype=np.float64).reshape(3, n)
    raw["quats"][0] = 1.0
    small, large = math.log(0.005), math.log(0.05)
    raw["scales"][:] = small
    raw["scales"][0, 2] = large
    raw["scales"][1, 5] = math.log(0.5)
    raw["opac1"][:] = 0.0
    raw["opac2"][:] = 0.0
    raw["opac1"][0, 3] = raw["opac2"][0, 3] = T._logit(0.005)
    raw["opac1"][0, 4] = T._logit(0.005)
    raw["opac2"][0, 4] = T._logit(0.9)
    raw = {k: a.astype(np.float32).astype(np.float64) for k, a in raw.items()}
    m = {k: np.full_like(a, 0.25) for k, a in raw.items()}
    v = {k: np.full_like(a, 0.5) for k, a in raw.items()}
    accum = np.array([1e-5, 3e-3, 3e-3, 0.0, 0.0, 3e-3])
    count = np.array([1, 2, 2, 1, 0, 1])
    radii = np.zeros(n)
    z = np.zeros((2, 3, n))
    z[0, 0, :] = 1.0
    z[1, 1, :] = -2.0
    return raw, m, v, accum, count, radii, z, ext


def test_densify_and_prune_hand_case():
    raw, m, v, accum, count, radii, z, ext = _hand_state()
    out, om, ov, info = T.densify_and_prune(raw, m, v, accum, count, radii, z, extent=ext,
                                            max_world_scale=0.1)
    np.testing.assert_array_equal(info["keep"], [0, 1, 4])
    np.testing.assert_array_equal(info["clone"], [1])
    np.testing.assert_array_equal(info["child"], [2])
    assert out["means"].shape[1] == 3 + 1 + 2
    # order: kept 0, 1, 4; clone of 1; first child of 2; second child of 2
    np.testing.assert_array_equal(out["sh"][0], raw["sh"][0][[0, 1, 4, 1, 2, 2]])
    # children: mean + R (s * z) with identity rotation
    s = np.exp(raw["scales"][:, 2])
    np.testing.assert_allclose(out["means"][:, 4], raw["means"][:, 2] + s * np.array([1.0, 0.0, 0.0]), rtol=1e-12)
    np.testing.assert_allclose(out["means"][:, 5], raw["means"][:, 2] + s * np.array([0.0, -2.0, 0.0]), rtol=1e-12)
    np.testing.assert_allclose(np.exp(out["scales"][:, 4]), s / 1.6, rtol=1e-6)
    # moments: kept ones carried, new ones zero
    np.testing.assert_array_equal(om["means"][:, :3], 0.25)
    np.testing.assert_array_equal(om["means"][:, 3:], 0.0)
    np.testing.assert_array_equal(ov["opac1"][:, 3:], 0.0)


def test_densify_rotation_of_children_is_the_kernel_axes():
    """A child drawn with z = e_k lands at scale_k along the k-th column of
    R(q): check against scipy's rotation of the same quaternion."""
    from scipy.spatial.transform import Rotation
    raw, m, v, accum, count, radii, z, ext = _hand_state()
    q = np.array([0.8, 0.3, -0.2, 0.4])
    raw["quats"][:, 2] = 2.0 * q                  # any length
    out, _, _, info = T.densify_and_prune(raw, m, v, accum, count, radii, z, extent=ext)
    Rm = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    s = np.exp(raw["scales"][:, 2])
    k = list(info["child"]).index(2)
    nk = len(info["keep"]) + len(info["clone"])
    nc = len(info["child"])
    np.testing.assert_allclose(out["means"][:, nk + k], raw["means"][:, 2] + Rm[:, 0] * s[0], rtol=1e-12)
    np.testing.assert_allclose(out["means"][:, nk + nc + k], raw["means"][:, 2] - 2.0 * Rm[:, 1] * s[1],
                               rtol=1e-12)


def test_prune_needs_both_halves_transparent():
    raw, m, v, accum, count, radii, z, ext = _hand_state()
    accum[:] = 0.0
    out, _, _, info = T.densify_and_prune(raw, m, v, accum, count, radii, z, extent=ext)
    np.testing.assert_array_equal(info["keep"], [0, 1, 2, 4, 5])
    radii[0] = 25.0
    out, _, _, info = T.densify_and_prune(raw, m, v, accum, count, radii, z, extent=ext, max_screen_radius=20.0)
    np.testing.assert_array_equal(info["keep"], [1, 2, 4, 5])


def test_opacity_reset_caps_each_half():
    raw, m, v, *_ = _hand_state()
    r2, m2, v2 = T.reset_opacity(raw, m, v, 0.02)
    for k in ("opac1", "opac2"):
        sig = 1.0 / (1.0 + np.exp(-raw[k]))
        np.testing.assert_allclose(1.0 / (1.0 + np.exp(-r2[k])), np.minimum(sig, 0.02), rtol=1e-12)
        assert (m2[k] == 0).all() and (v2[k] == 0).all()
    np.testing.assert_array_equal(m2["means"], m["means"])
