"""Pins of the oracle's context model: groups, ConvLSTM, causality, head (CPU only)."""
import json
import os

import numpy as np
import scipy.special
import torch

import oracle as O
from wvgen import gradient_noise_image

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))


def test_group_fractions_and_neighbour_counts_match_paper():
    g = O.group_map(10, 12)
    for k in range(4):
        assert np.mean(g == k) == GOLD["fraction_per_step"]["value"]
    # Brute force: coded 3x3 neighbours of an interior position of each step.
    counts = []
    for k in range(4):
        rr, cc = np.nonzero(g == k)
        sel = [(r, c) for r, c in zip(rr, cc) if 0 < r < 9 and 0 < c < 11]
        r, c = sel[0]
        win = g[r - 1:r + 2, c - 1:c + 2].copy()
        win[1, 1] = 99
        n = int(np.sum(win < k))
        assert all(int(np.sum(np.where(np.arange(9).reshape(3, 3) == 4, 99,
                                       g[a - 1:a + 2, b - 1:b + 2]) < k)) == n for a, b in sel)
        counts.append(n)
    assert counts == GOLD["neighbours_per_step"]["value"]
    assert np.mean(counts) == GOLD["mean_neighbours"]["value"]


def test_convlstm_centre_tap_equals_torch_lstmcell():
    # With only the centre tap non-zero the ConvLSTM is a per-pixel LSTM cell.
    rng = np.random.default_rng(11)
    C = 5
    w = rng.standard_normal((4 * C, 1 + C, 3, 3))
    w[:, :, [0, 0, 0, 1, 1, 2, 2, 2], [0, 1, 2, 0, 2, 0, 1, 2]] = 0
    b = rng.standard_normal(4 * C)
    x = rng.standard_normal((2, 4, 3, 1))
    h = rng.standard_normal((2, 4, 3, C))
    c = rng.standard_normal((2, 4, 3, C))
    hn, cn = O.lstm_cell(O.conv3x3(np.concatenate([x, h], -1), w, b), c)
    cell = torch.nn.LSTMCell(1, C).double()
    with torch.no_grad():
        cell.weight_ih.copy_(torch.from_numpy(w[:, :1, 1, 1]))
        cell.weight_hh.copy_(torch.from_numpy(w[:, 1:, 1, 1]))
        cell.bias_ih.copy_(torch.from_numpy(b))
        cell.bias_hh.zero_()
        ht, ct = cell(torch.from_numpy(x.reshape(-1, 1)),
                      (torch.from_numpy(h.reshape(-1, C)), torch.from_numpy(c.reshape(-1, C))))
    np.testing.assert_allclose(hn.reshape(-1, C), ht.numpy(), atol=1e-13)
    np.testing.assert_allclose(cn.reshape(-1, C), ct.numpy(), atol=1e-13)


def test_head_formulas_match_library_routines(cfg_small):
    rng = np.random.default_rng(12)
    r = 5 * rng.standard_normal((50, 9))
    p = O.mixture_head(r, cfg_small)
    np.testing.assert_allclose(p[:, :3], scipy.special.softmax(r[:, :3], axis=1), atol=1e-15)
    np.testing.assert_array_equal(p[:, 3:6], r[:, 3:6])
    sp = torch.nn.functional.softplus(torch.from_numpy(r[:, 6:])).numpy()
    np.testing.assert_allclose(p[:, 6:], np.maximum(sp, 0.11), atol=1e-14)
    assert np.all(p[:, 6:] >= 0.11)
    np.testing.assert_allclose(p[:, :3].sum(1), 1.0, atol=1e-15)


def _cfg1_q(cfg, w):
    x = gradient_noise_image(64, 64, seed=1)[None]
    qs, _ = O.quantize(O.analyze(x, cfg, w), cfg)
    return qs


def test_causality_of_steps_and_subbands(cfg_small, weights_small):
    cfg, w = cfg_small, weights_small
    qs = _cfg1_q(cfg, w)
    ref = O.context_params_all(qs, cfg, w)
    rng = np.random.default_rng(13)
    i = 4                                   # HL1 .. any subband after the first
    ls = O.long_context(qs, cfg, w)
    t = O.subband_layout(cfg, 64, 64)[0][i]["type"]
    for g in range(4):
        # Perturb the current subband at steps >= g and every later subband.
        pert = [q.copy() for q in qs]
        gm = O.group_map(*qs[i].shape[1:])
        noise = rng.integers(-20, 21, qs[i].shape)
        pert[i] = np.where(gm[None] >= g, np.clip(qs[i] + noise, -64, 64), qs[i])
        for k in range(i + 1, len(qs)):
            pert[k] = np.clip(qs[k] + rng.integers(-20, 21, qs[k].shape), -64, 64)
        lp = O.long_context(pert, cfg, w, upto=i + 1)
        got = O.step_params(pert[i], lp[i], t, g, cfg, w)
        assert np.array_equal(got, ref[i][g]), g
        np.testing.assert_array_equal(lp[i], ls[i])
    # Step 0 does not read the current subband at all; step 1 does.
    anything = np.full_like(qs[i], 17)
    assert np.array_equal(O.step_params(anything, ls[i], t, 0, cfg, w), ref[i][0])
    assert not np.array_equal(O.step_params(anything, ls[i], t, 1, cfg, w), ref[i][1])
    # The long context of subband i reads subband i-1.
    pert = [q.copy() for q in qs]
    pert[i - 1] = np.clip(qs[i - 1] + 5, -64, 64)
    assert not np.array_equal(O.long_context(pert, cfg, w, upto=i + 1)[i], ls[i])


def test_params_shapes_and_counts(cfg_small, weights_small):
    qs = _cfg1_q(cfg_small, weights_small)
    prm = O.context_params_all(qs, cfg_small, weights_small)
    assert len(prm) == 7
    for i, row in enumerate(prm):
        assert len(row) == GOLD["steps_per_subband"]["value"]
        assert sum(p.shape[1] for p in row) == qs[i].shape[1] * qs[i].shape[2]
        for p in row:
            assert p.shape[2] == 9 and np.all(np.isfinite(p))


def test_long_context_sequence_equals_per_pixel_lstm_with_replicated_state():
    # Centre-tap-only gate conv: the long context over all subbands must equal a
    # per-pixel torch LSTMCell whose state is replicated (nearest x2) whenever the
    # resolution doubles and whose input is the previously coded subband.
    from wvgen import get_config, make_weights
    cfg = get_config("gray64", levels=2, ctx_ch=4)
    w = make_weights(cfg)
    C = 4
    wl = w["lstm.w"].astype(np.float64)
    wl[:, :, [0, 0, 0, 1, 1, 2, 2, 2], [0, 1, 2, 0, 2, 0, 1, 2]] = 0
    w = dict(w, **{"lstm.w": wl.astype(np.float32)})
    lay, _ = O.subband_layout(cfg, 16, 16)
    rng = np.random.default_rng(14)
    qs = [rng.integers(-5, 6, (2, s["h"], s["w"])) for s in lay]
    ls = O.long_context(qs, cfg, w)
    cell = torch.nn.LSTMCell(1, C).double()
    W64 = torch.from_numpy(w["lstm.w"].astype(np.float64))
    with torch.no_grad():
        cell.weight_ih.copy_(W64[:, :1, 1, 1])
        cell.weight_hh.copy_(W64[:, 1:, 1, 1])
        cell.bias_ih.copy_(torch.from_numpy(w["lstm.b"].astype(np.float64)))
        cell.bias_hh.zero_()
        h = torch.zeros(2, lay[0]["h"], lay[0]["w"], C, dtype=torch.float64)
        c = torch.zeros_like(h)
        for i, s in enumerate(lay):
            if h.shape[1] != s["h"]:
                h = h.repeat_interleave(2, 1).repeat_interleave(2, 2)
                c = c.repeat_interleave(2, 1).repeat_interleave(2, 2)
            u = torch.zeros(2, s["h"], s["w"], dtype=torch.float64) if i == 0 else \
                torch.from_numpy(qs[i - 1].astype(np.float64))
            if u.shape[1] != s["h"]:
                u = u.repeat_interleave(2, 1).repeat_interleave(2, 2)
            hn, cn = cell(u.reshape(-1, 1), (h.reshape(-1, C), c.reshape(-1, C)))
            h, c = hn.reshape(h.shape), cn.reshape(c.shape)
            np.testing.assert_allclose(ls[i], h.numpy(), atol=1e-13, err_msg=s["name"])


def test_upsample_is_nearest_replication():
    a = np.arange(6.0).reshape(1, 2, 3)
    u = O.upsample2(a)
    assert u.shape == (1, 4, 6)
    np.testing.assert_array_equal(u[:, 0::2, 0::2], a)
    np.testing.assert_array_equal(u[:, 1::2, 1::2], a)
    np.testing.assert_array_equal(u[:, 0::2, 1::2], a)
    np.testing.assert_array_equal(u[:, 1::2, 0::2], a)


def test_block_architecture_pieces_match_torch():
    # Depth-wise conv = torch conv2d with one group per channel; 1x1 conv = a linear map.
    rng = np.random.default_rng(15)
    x = rng.standard_normal((2, 5, 6, 8))
    w = rng.standard_normal((8, 1, 3, 3))
    b = rng.standard_normal(8)
    ref = torch.nn.functional.conv2d(torch.from_numpy(x).permute(0, 3, 1, 2), torch.from_numpy(w),
                                     torch.from_numpy(b), padding=1, groups=8).permute(0, 2, 3, 1)
    np.testing.assert_allclose(O.dwconv3x3(x, w, b), ref.numpy(), atol=1e-12)
    w1 = rng.standard_normal((4, 8, 1, 1))
    ref1 = torch.nn.functional.conv2d(torch.from_numpy(x).permute(0, 3, 1, 2), torch.from_numpy(w1),
                                      torch.from_numpy(b[:4])).permute(0, 2, 3, 1)
    np.testing.assert_allclose(O.conv1x1(x, w1, b[:4]), ref1.numpy(), atol=1e-12)


def test_block_architecture_residual_paths_and_causality():
    from wvgen import get_config, make_weights
    cfg = get_config("gray64", ctx_arch="blocks")
    w = make_weights(cfg)
    x = np.random.default_rng(16).standard_normal((1, 6, 7, cfg["ctx_ch"]))
    # Zero second convs leave only the skip paths: both blocks become the identity.
    z = dict(w)
    for k in ("p1b", "p2b"):
        z[f"ctx.LL.0.{k}.w"] = np.zeros_like(w[f"ctx.LL.0.{k}.w"])
        z[f"ctx.LL.0.{k}.b"] = np.zeros_like(w[f"ctx.LL.0.{k}.b"])
    z["ctx.LL.1.rb.w"] = np.zeros_like(w["ctx.LL.1.rb.w"])
    z["ctx.LL.1.rb.b"] = np.zeros_like(w["ctx.LL.1.rb.b"])
    np.testing.assert_array_equal(O.depth_conv_block(x, z, "ctx.LL.0"), x)
    np.testing.assert_array_equal(O.residual_block(x, z, "ctx.LL.1"), x)
    assert not np.allclose(O.depth_conv_block(x, w, "ctx.LL.0"), x)
    # Causality holds for the block stacks too.
    xim = gradient_noise_image(64, 64, seed=1)[None]
    qs, _ = O.quantize(O.analyze(xim, cfg, w), cfg)
    ref = O.context_params_all(qs, cfg, w)
    i, g = 4, 2
    pert = [q.copy() for q in qs]
    gm = O.group_map(*qs[i].shape[1:])
    pert[i] = np.where(gm[None] >= g, np.clip(qs[i] + 9, -64, 64), qs[i])
    got = O.step_params(pert[i], O.long_context(pert, cfg, w, upto=i + 1)[i], 1, g, cfg, w)
    assert np.array_equal(got, ref[i][g])


def test_ar_ll_model_causal_taps_and_brute_force():
    from wvgen import get_config, make_weights
    cfg = get_config("gray64", ll_ar=1)
    w = make_weights(cfg)
    assert len(O.AR_TAPS) == 12
    assert all(dy < 0 or (dy == 0 and dx < 0) for dy, dx in O.AR_TAPS)     # strictly causal
    rng = np.random.default_rng(17)
    q = rng.integers(-6, 7, (1, 5, 7))
    p = O.ar_params(q, cfg, w)
    # Brute force: one position's parameters from an explicit loop over its neighbours.
    r, c = 3, 4
    W0, b0 = w["ar.0.w"].astype(np.float64), w["ar.0.b"].astype(np.float64)
    a = b0.copy()
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            if (dy, dx) in O.AR_TAPS and 0 <= r + dy < 5 and 0 <= c + dx < 7:
                a += W0[:, 0, dy + 2, dx + 2] * q[0, r + dy, c + dx]
    a = np.maximum(a, 0)
    a = np.maximum(w["ar.1.w"][:, :, 0, 0].astype(np.float64) @ a + w["ar.1.b"], 0)
    raw = w["ar.2.w"][:, :, 0, 0].astype(np.float64) @ a + w["ar.2.b"]
    np.testing.assert_allclose(p[0, r * 7 + c], O.mixture_head(raw[None], cfg)[0], atol=1e-12)
    # Causality: changing the symbol at raster position k only affects positions after k.
    k = 17
    q2 = q.copy()
    q2.reshape(-1)[k] += 5
    p2 = O.ar_params(q2, cfg, w)
    assert np.array_equal(p2[0, :k + 1], p[0, :k + 1])
    assert not np.array_equal(p2[0, k + 1:], p[0, k + 1:])


def test_ar_ll_oracle_roundtrip(cfg_small):
    from wvgen import get_config, make_weights
    cfg = get_config("gray64", ll_ar=1)
    w = make_weights(cfg)
    x = gradient_noise_image(64, 64, seed=1)[None]
    streams, qs, _ = O.encode(x, cfg, w)
    assert streams[0][0][1:] == [b"", b"", b""]
    xr, qd = O.decode(streams, cfg, w, 64, 64, 1)
    for a, b in zip(qs, qd):
        assert np.array_equal(a, b)
