"""Pins of the oracle's convolution and lifting transform (CPU only)."""
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
from wvgen import get_config, make_weights, gradient_noise_image, sinusoid_1f_planes

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))


def test_conv_matches_direct_loops():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((2, 5, 6, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    np.testing.assert_allclose(O.conv3x3(x, w, b), O.conv3x3_direct(x, w, b), rtol=0, atol=1e-12)


def test_conv_matches_torch_conv2d_float64():
    rng = np.random.default_rng(8)
    x = rng.standard_normal((3, 9, 7, 5))
    w = rng.standard_normal((6, 5, 3, 3))
    b = rng.standard_normal(6)
    ref = torch.nn.functional.conv2d(torch.from_numpy(x).permute(0, 3, 1, 2), torch.from_numpy(w),
                                     torch.from_numpy(b), padding=1).permute(0, 2, 3, 1).numpy()
    np.testing.assert_allclose(O.conv3x3(x, w, b), ref, rtol=0, atol=1e-11)


def _zero_residual(cfg):
    w = make_weights(cfg)
    L = cfg["lift_layers"]
    for nm in O.LIFT_NAMES:
        w[f"lift.{nm}.{L - 1}.w"][...] = 0
        w[f"lift.{nm}.{L - 1}.b"][...] = 0
    return w


def test_layout_counts_match_paper():
    cfg = get_config("ycbcr512x768")
    lay, n = O.subband_layout(cfg, 512, 768)
    assert len(lay) == GOLD["subbands"]["value"] == 3 * GOLD["levels"]["value"] + 1
    assert [s["name"] for s in lay] == GOLD["coding_order_names"]["value"]
    fh, fw = GOLD["ll_fraction"]["value"]
    assert (lay[0]["h"], lay[0]["w"]) == (512 // fh, 768 // fw)
    assert n == 512 * 768
    with pytest.raises(ValueError):
        O.subband_layout(cfg, 520, 768)


def test_haar_special_case_one_level_closed_form():
    # With zero residual networks P(z) = z and U(z) = z/2: the unnormalised Haar.
    cfg = get_config("gray64", levels=1)
    w = _zero_residual(cfg)
    x = np.random.default_rng(3).integers(0, 256, (2, 8, 10)).astype(np.uint8)
    LL, HL, LH, HH = O.analyze(x, cfg, w)
    X = x.astype(np.float64) - 128
    a, b, c, d = X[:, 0::2, 0::2], X[:, 0::2, 1::2], X[:, 1::2, 0::2], X[:, 1::2, 1::2]
    np.testing.assert_array_equal(LL, (a + b + c + d) / 4)
    np.testing.assert_array_equal(LH, (c + d - a - b) / 2)
    np.testing.assert_array_equal(HL, (b - a + d - c) / 2)
    np.testing.assert_array_equal(HH, (d - c) - (b - a))


def test_haar_special_case_ll_is_block_mean():
    cfg = get_config("ycbcr512x768")
    w = _zero_residual(cfg)
    x = np.random.default_rng(4).integers(0, 256, (1, 32, 48)).astype(np.uint8)
    ys = O.analyze(x, cfg, w)
    blk = (x.astype(np.float64) - 128).reshape(1, 2, 16, 3, 16).mean(axis=(2, 4))
    np.testing.assert_allclose(ys[0], blk, rtol=0, atol=1e-12)


def test_perfect_reconstruction_float(cfg_small, weights_small):
    x = gradient_noise_image(64, 64, seed=1)[None]
    ys = O.analyze(x, cfg_small, weights_small)
    xr = O.synthesize(ys, cfg_small, weights_small)
    assert np.max(np.abs(xr - x)) <= 1e-10


def test_perfect_reconstruction_float_four_levels(cfg_big, weights_big):
    x = sinusoid_1f_planes(32, 48, planes=2, seed=9)
    ys = O.analyze(x, cfg_big, weights_big)
    assert len(ys) == 13 and ys[0].shape == (2, 2, 3)
    xr = O.synthesize(ys, cfg_big, weights_big)
    assert np.max(np.abs(xr - x)) <= 1e-10


def test_perfect_reconstruction_integer_lifting_is_exact():
    cfg = get_config("gray64", lift_int=1)
    w = make_weights(cfg)
    x = gradient_noise_image(64, 64, seed=1)[None]
    ys = O.analyze(x, cfg, w)
    assert all(np.array_equal(y, np.rint(y)) for y in ys)
    xr = O.synthesize(ys, cfg, w)
    assert np.array_equal(xr, x.astype(np.float64))


def test_lifting_nonlinear_filters_are_active(cfg_small, weights_small):
    # Guards against a filter that silently collapses to Haar (e.g. a dropped residual).
    cfg = cfg_small
    x = gradient_noise_image(64, 64, seed=1)[None]
    ys = O.analyze(x, cfg, weights_small)
    yh = O.analyze(x, cfg, _zero_residual(cfg))
    assert max(np.max(np.abs(a - b)) for a, b in zip(ys, yh)) > 1e-2


def test_quantize_rounds_half_even_and_clamps(cfg_small):
    cfg = dict(cfg_small, step=1.0)
    ys = [np.array([[[0.5, 1.5, -2.5, 100.0, -100.0, 2.49]]])]
    qs, clips = O.quantize(ys, cfg)
    assert qs[0].tolist() == [[[0, 2, -2, 64, -64, 2]]]
    assert clips == 2


def test_temporal_haar_closed_forms_and_inverse():
    rng = np.random.default_rng(5)
    f = rng.standard_normal((8, 3, 4))
    s = O.temporal_haar_forward(f, 3)
    np.testing.assert_allclose(s[0], f.mean(axis=0), atol=1e-12)          # L_3 = GOP mean
    np.testing.assert_allclose(s[4:], f[1::2] - f[0::2], atol=1e-12)       # H_1 = odd - even
    np.testing.assert_allclose(O.temporal_haar_inverse(s, 3), f, atol=1e-12)


def _haar_basis(name, size=16):
    """Closed-form synthesis basis of the unnormalised Haar lifting for a 1-valued
    coefficient at (0, 0) of subband `name` (e.g. "HL2") on a size x size grid."""
    t, j = name[:2], int(name[2:])
    B = 1 << j
    out = np.zeros((size, size))
    lo = np.ones(B)
    hi = np.concatenate([-0.5 * np.ones(B // 2), 0.5 * np.ones(B // 2)])
    rows = hi if t[1] == "H" else lo   # second letter: vertical (column) band
    cols = hi if t[0] == "H" else lo   # first letter: horizontal (row) band
    out[:B, :B] = np.outer(rows, cols)
    return out


def test_subband_impulse_response_of_haar_is_haar_basis():
    cfg = get_config("ycbcr512x768")
    w = _zero_residual(cfg)
    lay, _ = O.subband_layout(cfg, 32, 32)
    # One-hot subbands at (0,0) with value 3 (quantised), step 4 -> amplitude 12.
    qs = []
    for s in lay:
        q = np.zeros((1, s["h"], s["w"]), np.int64)
        q[0, 0, 0] = 3
        qs.append(q)
    sir = O.subband_impulse_responses(qs, cfg, w, size=16)
    assert sir.shape == (13, 16, 16)
    names = [s["name"] for s in lay]
    for i, nm in enumerate(names):
        np.testing.assert_allclose(sir[i], 12.0 * _haar_basis(nm), atol=1e-12, err_msg=nm)
