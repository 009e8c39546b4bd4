"""Pins of the oracle's network compositions against independent torch modules (CPU only).

The lifting filters (Sec. 3.1: residual CNN modules as predict and update
filters), the plain step stacks and the block step stacks (Sec. 3.2) are
rebuilt here as float64 ``torch.nn`` module chains (NCHW ``Conv2d`` with zero
padding, ``Tanh``/``ReLU`` modules) from the same weights, and compared with the
oracle's NHWC im2col evaluation.  Closed-form special cases pin where the
activations sit: a chain whose last conv has zero weights returns that conv's
bias exactly, so an activation after the last conv (a tanh on a bias of 3, a
ReLU on a bias of -2) fails.  The impulse-response placement (Sec. 3.4) is
pinned against a brute-force max-pool written with loops.
"""
import numpy as np
import pytest
import torch

import oracle as O
from wvgen import get_config, make_weights, gradient_noise_image


def _conv_module(w, b, groups=1):
    w = torch.from_numpy(np.asarray(w, np.float64))
    k = w.shape[-1]
    m = torch.nn.Conv2d(w.shape[1] * groups, w.shape[0], k, padding=k // 2, groups=groups,
                        dtype=torch.float64)
    with torch.no_grad():
        m.weight.copy_(w)
        m.bias.copy_(torch.from_numpy(np.asarray(b, np.float64)))
    return m


def _chain(convs, act):
    mods = []
    for l, (w, b) in enumerate(convs):
        mods.append(_conv_module(w, b))
        if l + 1 < len(convs):
            mods.append(act())
    return torch.nn.Sequential(*mods)


def _nhwc(t):
    return t.permute(0, 2, 3, 1).detach().numpy()


def _nchw(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float64))).permute(0, 3, 1, 2)


def _lift_convs(cfg, w, nm):
    return [(w[f"lift.{nm}.{l}.w"], w[f"lift.{nm}.{l}.b"]) for l in range(cfg["lift_layers"])]


def _ctx_convs(cfg, w, t, g):
    return [(w[f"ctx.{t}.{g}.{l}.w"], w[f"ctx.{t}.{g}.{l}.b"]) for l in range(cfg["ctx_layers"])]


@pytest.mark.parametrize("name", ["gray64", "ycbcr512x768"])
def test_lift_residual_equals_torch_conv_tanh_chain(name):
    cfg = get_config(name)
    w = make_weights(cfg)
    z = np.random.default_rng(21).standard_normal((2, 9, 11)) * 20.0
    for nm in O.LIFT_NAMES:
        convs = _lift_convs(cfg, w, nm)
        net = _chain(convs, torch.nn.Tanh)
        ref = net(torch.from_numpy(z)[:, None])[:, 0].detach().numpy()
        np.testing.assert_allclose(O.lift_residual(z, convs), ref, rtol=0, atol=1e-12, err_msg=nm)
        # P(z) = z + N_P(z), U(z) = z/2 + N_U(z) (the residual structure read from Sec. 3.1).
        np.testing.assert_allclose(O.predict(z, convs), z + ref, rtol=0, atol=1e-12)
        np.testing.assert_allclose(O.update(z, convs), 0.5 * z + ref, rtol=0, atol=1e-12)


def test_lift_residual_last_conv_is_linear():
    # Zero weights in the last conv: N(z) is that conv's bias at every position,
    # whatever the earlier layers do (no activation follows the last conv).
    cfg = get_config("gray64")
    w = make_weights(cfg)
    convs = [(np.asarray(a, np.float64).copy(), np.asarray(b, np.float64).copy())
             for a, b in _lift_convs(cfg, w, "P_row")]
    convs[-1][0][...] = 0.0
    convs[-1][1][...] = 3.0
    z = np.random.default_rng(22).standard_normal((1, 6, 8)) * 50.0
    assert np.array_equal(O.lift_residual(z, convs), np.full_like(z, 3.0))
    # One-hot centre taps (every layer a per-pixel scalar map) reduce the filter
    # to a*tanh(c*tanh(e*z + f) + d) + b, with z entering once and tanh between layers.
    convs = [(np.zeros_like(a), np.zeros_like(b)) for a, b in convs]
    convs[0][0][0, 0, 1, 1], convs[0][1][0] = 0.7, 0.2
    convs[1][0][0, 0, 1, 1], convs[1][1][0] = -1.3, 0.1
    convs[2][0][0, 0, 1, 1], convs[2][1][0] = 2.5, -0.4
    want = 2.5 * np.tanh(-1.3 * np.tanh(0.7 * z + 0.2) + 0.1) - 0.4
    np.testing.assert_allclose(O.lift_residual(z, convs), want, rtol=0, atol=1e-13)


@pytest.mark.parametrize("name", ["gray64", "ycbcr512x768"])
def test_step_stack_equals_torch_conv_relu_chain(name):
    cfg = get_config(name)
    w = make_weights(cfg)
    C = cfg["ctx_ch"]
    rng = np.random.default_rng(23)
    for t in O.TYPE_NAMES:
        for g in range(4):
            cin = C if g == 0 else C + 1
            z = rng.standard_normal((1, 7, 9, cin))
            convs = _ctx_convs(cfg, w, t, g)
            ref = _nhwc(_chain(convs, torch.nn.ReLU)(_nchw(z)))
            np.testing.assert_allclose(O.step_stack(z, convs), ref, rtol=0, atol=1e-11,
                                       err_msg=f"{t}{g}")


def test_step_stack_head_conv_is_linear():
    # Zero weights and a negative bias in the head conv: the raw outputs are that
    # bias (negative), so no ReLU follows the last conv.
    cfg = get_config("gray64")
    w = make_weights(cfg)
    convs = [(np.asarray(a, np.float64).copy(), np.asarray(b, np.float64).copy())
             for a, b in _ctx_convs(cfg, w, "HL", 2)]
    convs[-1][0][...] = 0.0
    convs[-1][1][...] = -2.0
    z = np.random.default_rng(24).standard_normal((1, 5, 6, cfg["ctx_ch"] + 1))
    out = O.step_stack(z, convs)
    assert np.array_equal(out, np.full(out.shape, -2.0))
    # ReLU between layers: with every inner layer's bias at -1e3 and zero weights,
    # the next layer sees zeros, so the output is the head's bias plus nothing.
    convs = [(np.asarray(a, np.float64).copy(), np.asarray(b, np.float64).copy())
             for a, b in _ctx_convs(cfg, w, "HL", 2)]
    for l in range(len(convs) - 1):
        convs[l][0][...] = 0.0
        convs[l][1][...] = -1e3
    out = O.step_stack(z, convs)
    np.testing.assert_array_equal(out, np.broadcast_to(convs[-1][1], out.shape))


def test_step_params_equal_torch_stack_at_group_positions():
    # The whole of a step: input assembly (symbols of earlier steps, zero elsewhere,
    # ahead of l_i), the conv/ReLU chain, selection of the step's positions in raster
    # order, and the head, against torch modules and torch's softmax/softplus.
    cfg = get_config("gray64")
    w = make_weights(cfg)
    C, K = cfg["ctx_ch"], cfg["mix_k"]
    rng = np.random.default_rng(25)
    q = rng.integers(-9, 10, (1, 6, 7))
    l_i = np.tanh(rng.standard_normal((1, 6, 7, C)))
    for t in range(4):
        for g in range(4):
            got = O.step_params(q, l_i, t, g, cfg, w)
            mask = torch.tensor([[2 * (r % 2) + (c % 2) < g for c in range(7)] for r in range(6)])
            sym = torch.from_numpy(q.astype(np.float64))[:, None] * mask
            lt = _nchw(l_i)
            z = lt if g == 0 else torch.cat([sym, lt], dim=1)
            raw = _chain(_ctx_convs(cfg, w, O.TYPE_NAMES[t], g), torch.nn.ReLU)(z)[0]
            pos = [(r, c) for r in range(6) for c in range(7) if 2 * (r % 2) + (c % 2) == g]
            rv = torch.stack([raw[:, r, c] for r, c in pos])
            want = torch.cat([torch.softmax(rv[:, :K], -1), rv[:, K:2 * K],
                              torch.clamp(torch.nn.functional.softplus(rv[:, 2 * K:]),
                                          min=cfg["sigma_min"])], -1)
            np.testing.assert_allclose(got[0], want.detach().numpy(), rtol=0, atol=1e-12,
                                       err_msg=f"t{t} g{g}")


class _DepthConvBlock(torch.nn.Module):
    """x + 1x1(dw3x3(relu(1x1 x))), then x + 1x1(relu(1x1 x)), as torch modules."""

    def __init__(self, w, pre, C):
        super().__init__()
        self.p1a = _conv_module(w[pre + ".p1a.w"], w[pre + ".p1a.b"])
        self.dw = _conv_module(w[pre + ".dw.w"], w[pre + ".dw.b"], groups=C)
        self.p1b = _conv_module(w[pre + ".p1b.w"], w[pre + ".p1b.b"])
        self.p2a = _conv_module(w[pre + ".p2a.w"], w[pre + ".p2a.b"])
        self.p2b = _conv_module(w[pre + ".p2b.w"], w[pre + ".p2b.b"])

    def forward(self, x):
        x = x + self.p1b(self.dw(torch.relu(self.p1a(x))))
        return x + self.p2b(torch.relu(self.p2a(x)))


class _ResidualBlock(torch.nn.Module):
    def __init__(self, w, pre):
        super().__init__()
        self.ra = _conv_module(w[pre + ".ra.w"], w[pre + ".ra.b"])
        self.rb = _conv_module(w[pre + ".rb.w"], w[pre + ".rb.b"])

    def forward(self, x):
        return x + self.rb(torch.relu(self.ra(x)))


def test_step_stack_blocks_equal_torch_modules():
    cfg = get_config("gray64", ctx_arch="blocks")
    w = make_weights(cfg)
    C = cfg["ctx_ch"]
    rng = np.random.default_rng(26)
    for t in O.TYPE_NAMES:
        for g in range(4):
            pre = f"ctx.{t}.{g}"
            blk = _DepthConvBlock(w, pre, C) if g == 0 else _ResidualBlock(w, pre)
            net = torch.nn.Sequential(_conv_module(w[pre + ".in.w"], w[pre + ".in.b"]),
                                      torch.nn.ReLU(), blk,
                                      _conv_module(w[pre + ".out.w"], w[pre + ".out.b"]))
            z = rng.standard_normal((1, 6, 8, C if g == 0 else C + 1))
            ref = _nhwc(net(_nchw(z)))
            np.testing.assert_allclose(O.step_stack_blocks(z, w, pre, g), ref, rtol=0, atol=1e-11,
                                       err_msg=pre)


def test_step_stack_blocks_out_conv_is_linear():
    cfg = get_config("gray64", ctx_arch="blocks")
    w = {k: np.asarray(v, np.float64).copy() for k, v in make_weights(cfg).items()}
    for g in (0, 3):
        pre = f"ctx.LH.{g}"
        w[pre + ".out.w"][...] = 0.0
        w[pre + ".out.b"][...] = -1.5
        z = np.random.default_rng(27).standard_normal((1, 4, 5, cfg["ctx_ch"] + (g > 0)))
        out = O.step_stack_blocks(z, w, pre, g)
        assert np.array_equal(out, np.full(out.shape, -1.5))


def _pool_argmax_loops(a, sh, sw):
    """Brute force: max over each (h/sh) x (w/sw) window, first maximal cell in raster order."""
    h, w = a.shape
    ph, pw = h // sh, w // sw
    best, cell = -1.0, None
    for r in range(sh):
        for c in range(sw):
            m = max(a[r * ph + i, c * pw + j] for i in range(ph) for j in range(pw))
            if m > best:
                best, cell = m, (r, c)
    return cell, best


def test_impulse_response_places_pooled_maximum_off_origin():
    # Sec. 3.4: the largest |q_i| goes into subband i of a 16x16 pyramid at the cell
    # whose pooled window holds it.  Planted maxima away from (0, 0), one of them a
    # tie between two cells (the first in raster order wins), checked against a loop
    # max-pool and against the synthesis of the expected one-hot pyramid.
    cfg = get_config("gray64", levels=2)
    w = make_weights(cfg)
    H = W = 64
    lay, _ = O.subband_layout(cfg, H, W)
    rng = np.random.default_rng(28)
    qs = [rng.integers(-3, 4, (1, s["h"], s["w"])) for s in lay]
    plant = {0: [(13, 9, 40)], 2: [(5, 11, -33)], 4: [(30, 2, 25), (17, 20, -25)],
             6: [(31, 31, 60)]}
    for i, pts in plant.items():
        for r, c, v in pts:
            qs[i][0, r, c] = v
    sir = O.subband_impulse_responses(qs, cfg, w, size=16)
    small, _ = O.subband_layout(cfg, 16, 16)
    for i, s in enumerate(small):
        a = np.abs(qs[i][0]).astype(np.float64)
        cell, best = _pool_argmax_loops(a, s["h"], s["w"])
        if i in plant:
            assert best == max(abs(v) for _, _, v in plant[i])
        pyr = [np.zeros((1, t["h"], t["w"])) for t in small]
        pyr[i][0][cell] = best
        want = O.synthesize(O.dequantize(pyr, cfg), cfg, w, add_offset=False)[0]
        np.testing.assert_allclose(sir[i], want, rtol=0, atol=1e-12, err_msg=s["name"])
    # The planted cells themselves: (13, 9) in a 16x16 LL pooled to 4x4 -> (3, 2);
    # the tie in subband 4 (32x32 pooled to 8x8): (17, 20) -> (4, 5) precedes (30, 2) -> (7, 0).
    assert _pool_argmax_loops(np.abs(qs[0][0]).astype(float), 4, 4)[0] == (3, 2)
    assert _pool_argmax_loops(np.abs(qs[4][0]).astype(float), 8, 8)[0] == (4, 5)
    assert _pool_argmax_loops(np.abs(qs[6][0]).astype(float), 8, 8)[0] == (7, 7)
