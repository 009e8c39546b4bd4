"""Random-init weight blob and its manifest.

The blob is a flat little-endian float32 array: the tensors of `manifest(cfg)`
concatenated in manifest order, each conv as weight [Cout][Cin][3][3] followed
by bias [Cout].  Every conv is drawn from one numpy Generator seeded with
cfg["seed_weights"], weight then bias, uniform on +-1/sqrt(9*Cin).

Manifest order:
  1. four lifting filters P_row, U_row, P_col, U_col, each `lift_layers` convs:
     1 -> lift_ch, (lift_ch -> lift_ch) x (lift_layers - 2), lift_ch -> 1;
  2. the ConvLSTM gate conv, (1 + ctx_ch) -> 4*ctx_ch, gate blocks in the order
     input, forget, cell, output; input channels [previous subband, hidden];
  3. sixteen step stacks, subband type t in (LL, HL, LH, HH) outer, coding step
     g in 0..3 inner, each `ctx_layers` convs: Cin_g -> ctx_ch,
     (ctx_ch -> ctx_ch) x (ctx_layers - 2), ctx_ch -> 3*mix_k, where Cin_0 =
     ctx_ch and Cin_g = 1 + ctx_ch for g >= 1 with channel 0 the symbol channel.
     With ctx_arch == "blocks" a stack is instead: in (3x3, Cin_g -> C), then
     for g = 0 a DepthConvBlock p1a (1x1), dw (depth-wise 3x3, weight
     [C][1][3][3]), p1b (1x1), p2a (1x1), p2b (1x1), for g >= 1 a Residual
     Block ra, rb (3x3), then out (3x3, C -> 3K).
  4. with ll_ar: the autoregressive LL model ar.0 (5x5, 1 -> ar_ch, of which
     only the 12 causal taps are used), ar.1 (1x1, ar_ch -> ar_ch), ar.2
     (1x1, ar_ch -> 3*mix_k).
"""
import numpy as np

LIFT_NAMES = ("P_row", "U_row", "P_col", "U_col")
TYPE_NAMES = ("LL", "HL", "LH", "HH")


def _lift_chain(cfg):
    C, L = cfg["lift_ch"], cfg["lift_layers"]
    return [1] + [C] * (L - 1) + [1]


def _ctx_chain(cfg, g):
    C, L, K = cfg["ctx_ch"], cfg["ctx_layers"], cfg["mix_k"]
    cin = C if g == 0 else C + 1
    return [cin] + [C] * (L - 1) + [3 * K]


def manifest(cfg):
    """List of (name, shape) in blob order."""
    out = []

    def conv(prefix, cin, cout, k=3):
        out.append((prefix + ".w", (cout, cin, k, k)))
        out.append((prefix + ".b", (cout,)))

    for nm in LIFT_NAMES:
        ch = _lift_chain(cfg)
        for l in range(len(ch) - 1):
            conv(f"lift.{nm}.{l}", ch[l], ch[l + 1])
    C = cfg["ctx_ch"]
    conv("lstm", 1 + C, 4 * C)
    blocks = cfg.get("ctx_arch", "plain") == "blocks"
    for t in TYPE_NAMES:
        for g in range(4):
            if not blocks:
                ch = _ctx_chain(cfg, g)
                for l in range(len(ch) - 1):
                    conv(f"ctx.{t}.{g}.{l}", ch[l], ch[l + 1])
                continue
            pre = f"ctx.{t}.{g}"
            conv(pre + ".in", C if g == 0 else C + 1, C)
            if g == 0:   # DepthConvBlock: 1x1, depth-wise 3x3, 1x1 | 1x1, 1x1
                conv(pre + ".p1a", C, C, 1)
                out.append((pre + ".dw.w", (C, 1, 3, 3)))
                out.append((pre + ".dw.b", (C,)))
                conv(pre + ".p1b", C, C, 1)
                conv(pre + ".p2a", C, C, 1)
                conv(pre + ".p2b", C, C, 1)
            else:        # Residual Block: 3x3, 3x3
                conv(pre + ".ra", C, C)
                conv(pre + ".rb", C, C)
            conv(pre + ".out", C, 3 * cfg["mix_k"])
    if cfg.get("ll_ar", 0):
        A = cfg.get("ar_ch", 32)
        conv("ar.0", 1, A, 5)                 # masked 5x5: only the 12 causal taps are used
        conv("ar.1", A, A, 1)
        conv("ar.2", A, 3 * cfg["mix_k"], 1)
    return out


def make_weights(cfg):
    """Dict name -> float32 array, drawn in manifest order."""
    rng = np.random.default_rng(cfg["seed_weights"])
    out = {}
    pending_bound = None
    for name, shape in manifest(cfg):
        if name.endswith(".w"):
            pending_bound = 1.0 / np.sqrt(float(shape[1] * shape[2] * shape[3]))
        out[name] = rng.uniform(-pending_bound, pending_bound, shape).astype(np.float32)
    return out


def pack_weights(cfg, weights):
    """Flat float32 blob in manifest order."""
    return np.concatenate([np.ascontiguousarray(weights[n], np.float32).ravel()
                           for n, _ in manifest(cfg)])


def weights_nbytes(cfg):
    return 4 * sum(int(np.prod(s)) for _, s in manifest(cfg))
