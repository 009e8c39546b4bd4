"""Plain FP64 reference of the pWave++ four-step path (test infrastructure only).

Paper: A. Meyer, S. Prativadibhayankaram, A. Kaup, "Efficient Learned Wavelet
Image and Video Coding", ICIP 2024 (arXiv 2405.12631).  Each function names
the passage it follows.  Where the paper is silent the function states the
reading it takes; the same readings are listed in the design notes.

Conventions
-----------
* Planes are float64 arrays [N][h][w]; feature maps are NHWC [N][h][w][C].
* Every conv is a 3x3 cross-correlation, stride 1, zero padding 1, with bias,
  weight [Cout][Cin][3][3] (the weight blob's layout).
* Subband coding order (Sec. 3.1, Fig. 1; Fig. 11 caption): LL_J, then
  HL_j, LH_j, HH_j for j = J .. 1.  Type codes: LL 0, HL 1, LH 2, HH 3.
* Symbols are integers in [sym_min, sym_max]; the entropy coder codes the
  index symbol - sym_min.
"""
import numpy as np
from scipy.special import erfc as _erfc

TYPE_NAMES = ("LL", "HL", "LH", "HH")
LIFT_NAMES = ("P_row", "U_row", "P_col", "U_col")


# ----------------------------------------------------------------------------
# Convolution (definition, and a brute-force loop version for pins)
# ----------------------------------------------------------------------------
def conv3x3(x, w, b):
    """out[n,r,c,o] = b[o] + sum_{i,dy,dx} w[o,i,dy,dx] * x[n, r+dy-1, c+dx-1, i].

    Zero padding outside the plane.  The sum over the nine taps is written out
    tap by tap; each tap is one matrix product over input channels.
    """
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    N, H, W, Cin = x.shape
    Cout = w.shape[0]
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = np.empty((N * H * W, Cout), np.float64)
    out[...] = np.asarray(b, np.float64)
    for dy in range(3):
        for dx in range(3):
            tap = np.ascontiguousarray(xp[:, dy:dy + H, dx:dx + W, :]).reshape(-1, Cin)
            out += tap @ np.ascontiguousarray(w[:, :, dy, dx].T)
    return out.reshape(N, H, W, Cout)


def conv3x3_direct(x, w, b):
    """Same definition as conv3x3, evaluated with explicit loops (tiny inputs only)."""
    x = np.asarray(x, np.float64)
    N, H, W, Cin = x.shape
    Cout = w.shape[0]
    out = np.zeros((N, H, W, Cout))
    for n in range(N):
        for r in range(H):
            for c in range(W):
                for o in range(Cout):
                    s = float(b[o])
                    for dy in range(3):
                        for dx in range(3):
                            rr, cc = r + dy - 1, c + dx - 1
                            if 0 <= rr < H and 0 <= cc < W:
                                for i in range(Cin):
                                    s += float(w[o, i, dy, dx]) * x[n, rr, cc, i]
                    out[n, r, c, o] = s
    return out


def _convs(weights, prefix, count):
    return [(np.asarray(weights[f"{prefix}.{l}.w"], np.float64),
             np.asarray(weights[f"{prefix}.{l}.b"], np.float64)) for l in range(count)]


# ----------------------------------------------------------------------------
# Lifting (Sec. 3.1 and Fig. 2)
# ----------------------------------------------------------------------------
def lift_residual(z, convs):
    """Residual CNN of a predict/update filter: conv, tanh, ..., conv (Sec. 3.1).

    The paper only says residual CNN modules act as predict and update filters;
    the depth and width come from the workload (3 convs, tanh between them).
    z: [N][h][w] -> [N][h][w].
    """
    a = z[..., None]
    for l, (w, b) in enumerate(convs):
        a = conv3x3(a, w, b)
        if l + 1 < len(convs):
            a = np.tanh(a)
    return a[..., 0]


def predict(z, convs, lift_int=False):
    """P(z) = z + N_P(z); rounded to an integer in the lossless mode (Fig. 2)."""
    p = z + lift_residual(z, convs)
    return np.rint(p) if lift_int else p


def update(z, convs, lift_int=False):
    """U(z) = z/2 + N_U(z); rounded to an integer in the lossless mode (Fig. 2)."""
    u = 0.5 * z + lift_residual(z, convs)
    return np.rint(u) if lift_int else u


def _lift_convs(cfg, weights):
    L = cfg["lift_layers"]
    return {nm: _convs(weights, f"lift.{nm}", L) for nm in LIFT_NAMES}


def lift_forward_1d(x, axis, P, U, lift_int=False):
    """1-D lifting along `axis` (1 = columns of a row, i.e. row-wise; 2-D planes [N][h][w]).

    Sec. 3.1: split into even and odd samples, HP = odd - P(even),
    LP = even + U(HP).  Indices are 0-based: even = x[2m], odd = x[2m+1].
    The filters act on the whole 2-D array of even (resp. HP) samples.
    Returns (LP, HP).
    """
    if axis == 2:
        e, o = x[:, :, 0::2], x[:, :, 1::2]
    else:
        e, o = x[:, 0::2, :], x[:, 1::2, :]
    hp = o - predict(e, P, lift_int)
    lp = e + update(hp, U, lift_int)
    return lp, hp


def lift_inverse_1d(lp, hp, axis, P, U, lift_int=False):
    """Inverse of lift_forward_1d: even = LP - U(HP), odd = HP + P(even), interleave."""
    e = lp - update(hp, U, lift_int)
    o = hp + predict(e, P, lift_int)
    N, h, w = e.shape
    if axis == 2:
        x = np.empty((N, h, 2 * w))
        x[:, :, 0::2], x[:, :, 1::2] = e, o
    else:
        x = np.empty((N, 2 * h, w))
        x[:, 0::2, :], x[:, 1::2, :] = e, o
    return x


def subband_layout(cfg, H, W):
    """Coding-order list of dicts {name, level, type, h, w, offset} and coefficients per plane.

    J levels give 3J+1 subbands; level-j subbands are H/2^j x W/2^j (Sec. 3.1,
    Sec. 3.2: LL is H/16 x W/16 for four levels).  HL is high-pass along rows
    (horizontal) and low-pass along columns.
    """
    J = cfg["levels"]
    if H % (1 << J) or W % (1 << J):
        raise ValueError("H and W must be divisible by 2^levels")
    out, off = [], 0

    def add(name, lev, t):
        nonlocal off
        h, w = H >> lev, W >> lev
        out.append(dict(name=name, level=lev, type=t, h=h, w=w, offset=off))
        off += h * w

    add(f"LL{J}", J, 0)
    for j in range(J, 0, -1):
        add(f"HL{j}", j, 1)
        add(f"LH{j}", j, 2)
        add(f"HH{j}", j, 3)
    return out, off


def analyze(x, cfg, weights):
    """Forward transform of planes x [N][H][W] (uint8 or float) -> subbands y in coding order.

    Sec. 3.1: the input is centred (x - 128, a reading: the paper does not state
    the offset); each level applies 1-D lifting row-wise then column-wise and
    recurses on LL.  Returns a list of float64 arrays [N][h][w].
    """
    X = np.asarray(x, np.float64)
    if np.asarray(x).dtype == np.uint8:
        X = X - 128.0
    f = _lift_convs(cfg, weights)
    li = bool(cfg.get("lift_int", 0))
    J = cfg["levels"]
    details = {}
    for j in range(1, J + 1):
        l, h = lift_forward_1d(X, 2, f["P_row"], f["U_row"], li)
        LL, LH = lift_forward_1d(l, 1, f["P_col"], f["U_col"], li)
        HL, HH = lift_forward_1d(h, 1, f["P_col"], f["U_col"], li)
        details[j] = (HL, LH, HH)
        X = LL
    ys = [X]
    for j in range(J, 0, -1):
        ys.extend(details[j])
    return ys


def synthesize(ys, cfg, weights, add_offset=True):
    """Inverse transform (Sec. 3.1): subbands in coding order -> planes [N][H][W] (float64).

    Level j = J..1: inverse column step on (LL, LH) and on (HL, HH), then the
    inverse row step; finally the +128 offset of the forward transform.
    """
    f = _lift_convs(cfg, weights)
    li = bool(cfg.get("lift_int", 0))
    J = cfg["levels"]
    X = np.asarray(ys[0], np.float64)
    k = 1
    for j in range(J, 0, -1):
        HL, LH, HH = (np.asarray(a, np.float64) for a in ys[k:k + 3])
        k += 3
        l = lift_inverse_1d(X, LH, 1, f["P_col"], f["U_col"], li)
        h = lift_inverse_1d(HL, HH, 1, f["P_col"], f["U_col"], li)
        X = lift_inverse_1d(l, h, 2, f["P_row"], f["U_row"], li)
    return X + 128.0 if add_offset else X


# ----------------------------------------------------------------------------
# Quantisation (Sec. 3.1)
# ----------------------------------------------------------------------------
def deltas(cfg):
    """(Delta_L, Delta_H): the paper trains one step for LL and one for the rest;
    here both are 1/step of the workload."""
    d = 1.0 / float(cfg["step"])
    return d, d


def quantize(ys, cfg):
    """q = clamp(round_half_even(y * Delta), sym_min, sym_max) per subband (Sec. 3.1).

    Returns (list of int64 arrays, number of clamped coefficients).
    """
    dL, dH = deltas(cfg)
    qs, clips = [], 0
    for i, y in enumerate(ys):
        v = np.rint(np.asarray(y, np.float64) * (dL if i == 0 else dH))
        clips += int(np.count_nonzero((v < cfg["sym_min"]) | (v > cfg["sym_max"])))
        qs.append(np.clip(v, cfg["sym_min"], cfg["sym_max"]).astype(np.int64))
    return qs, clips


def dequantize(qs, cfg):
    """y_hat = q / Delta (Sec. 3.1)."""
    dL, dH = deltas(cfg)
    return [np.asarray(q, np.float64) / (dL if i == 0 else dH) for i, q in enumerate(qs)]


def pack(qs):
    """Concatenate subbands (coding order, each row-major) -> [N][coefs]."""
    return np.concatenate([q.reshape(q.shape[0], -1) for q in qs], axis=1)


def unpack(flat, cfg, H, W):
    lay, _ = subband_layout(cfg, H, W)
    flat = np.asarray(flat)
    return [flat[:, s["offset"]:s["offset"] + s["h"] * s["w"]].reshape(-1, s["h"], s["w"])
            for s in lay]


# ----------------------------------------------------------------------------
# Context model (Sec. 3.2, Figs. 3 and 4)
# ----------------------------------------------------------------------------
def group_map(h, w):
    """Coding step of each position: 2*(r mod 2) + (c mod 2).

    Sec. 3.2: four steps each code a quarter of the positions; a 3x3 kernel
    then sees 0, 2, 6 and 8 already coded neighbours.  This lattice order is
    one of the orders with that property (pinned by the neighbour-count test).
    """
    r = np.arange(h)[:, None] % 2
    c = np.arange(w)[None, :] % 2
    return 2 * r + c


def sigmoid(v):
    return 1.0 / (1.0 + np.exp(-v))


def lstm_cell(gates, c_prev):
    """LSTM cell update from pre-activation gates [.., 4C] in order input, forget, cell, output."""
    C = gates.shape[-1] // 4
    gi, gf, gg, go = (gates[..., k * C:(k + 1) * C] for k in range(4))
    c = sigmoid(gf) * c_prev + sigmoid(gi) * np.tanh(gg)
    h = sigmoid(go) * np.tanh(c)
    return h, c


def upsample2(a):
    """Nearest-neighbour x2 along the two spatial axes of [N][h][w](...)."""
    return np.repeat(np.repeat(a, 2, axis=1), 2, axis=2)


def long_context(qs, cfg, weights, upto=None):
    """Long-term context l_i of every subband (Sec. 3.2: hidden state of a ConvLSTM).

    Reading: state (h, c) starts at zero at the LL resolution; before subband i
    the previously coded subband q_{i-1} (zero for i = 0) is the input; when the
    resolution doubles, h, c and the input are upsampled (nearest, x2); the
    gates come from one 3x3 conv over [input, h].  Returns a list of l_i
    [N][h_i][w_i][C].
    """
    C = cfg["ctx_ch"]
    w = np.asarray(weights["lstm.w"], np.float64)
    b = np.asarray(weights["lstm.b"], np.float64)
    n = len(qs) if upto is None else upto
    N, h0, w0 = qs[0].shape
    hs = np.zeros((N, h0, w0, C))
    cs = np.zeros((N, h0, w0, C))
    out = []
    for i in range(n):
        hi, wi = qs[i].shape[1:]
        u = np.zeros((N, hi, wi)) if i == 0 else np.asarray(qs[i - 1], np.float64)
        if hs.shape[1] != hi:
            hs, cs = upsample2(hs), upsample2(cs)
        if u.shape[1] != hi:
            u = upsample2(u)
        gates = conv3x3(np.concatenate([u[..., None], hs], axis=-1), w, b)
        hs, cs = lstm_cell(gates, cs)
        out.append(hs)
    return out


def step_input(q_i, l_i, g):
    """Input of coding step g: l_i alone for g = 0; otherwise [q_i at steps < g (else 0), l_i]."""
    if g == 0:
        return l_i
    hi, wi = q_i.shape[1:]
    s = np.where(group_map(hi, wi)[None] < g, np.asarray(q_i, np.float64), 0.0)
    return np.concatenate([s[..., None], l_i], axis=-1)


def step_stack(z, convs):
    """Plain conv stack of one (subband type, step): conv, ReLU, ..., conv (no activation last)."""
    a = z
    for l, (w, b) in enumerate(convs):
        a = conv3x3(a, w, b)
        if l + 1 < len(convs):
            a = np.maximum(a, 0.0)
    return a


def conv1x1(x, w, b):
    """Pointwise conv: out[..., o] = b[o] + sum_i w[o, i, 0, 0] x[..., i]."""
    return np.asarray(x, np.float64) @ np.asarray(w, np.float64)[:, :, 0, 0].T + np.asarray(b, np.float64)


def dwconv3x3(x, w, b):
    """Depth-wise 3x3 conv, one group per channel (Sec. 3.2: each input channel is
    convolved with its own kernel): out[n,r,c,ch] = b[ch] + sum_tap w[ch,0,tap] x[n,r+dy-1,c+dx-1,ch]."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    N, H, W, C = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = np.empty_like(x)
    out[...] = np.asarray(b, np.float64)
    for dy in range(3):
        for dx in range(3):
            out += xp[:, dy:dy + H, dx:dx + W, :] * w[:, 0, dy, dx]
    return out


def _wb(weights, name):
    return np.asarray(weights[name + ".w"], np.float64), np.asarray(weights[name + ".b"], np.float64)


def depth_conv_block(x, weights, pre):
    """DepthConvBlock (Sec. 3.2, Fig. 5): a two-part residual block whose first part holds a
    depth-wise conv.  Reading (the figure is not in the text): part 1
    x + 1x1(dw3x3(relu(1x1(x)))), part 2 x + 1x1(relu(1x1(x)))."""
    t = np.maximum(conv1x1(x, *_wb(weights, pre + ".p1a")), 0.0)
    t = dwconv3x3(t, *_wb(weights, pre + ".dw"))
    x = x + conv1x1(t, *_wb(weights, pre + ".p1b"))
    t = np.maximum(conv1x1(x, *_wb(weights, pre + ".p2a")), 0.0)
    return x + conv1x1(t, *_wb(weights, pre + ".p2b"))


def residual_block(x, weights, pre):
    """Two-layer Residual Block (Sec. 3.2): x + conv3x3(relu(conv3x3(x)))."""
    t = np.maximum(conv3x3(x, *_wb(weights, pre + ".ra")), 0.0)
    return x + conv3x3(t, *_wb(weights, pre + ".rb"))


def step_stack_blocks(z, weights, pre, g):
    """Step stack of the block architecture: conv3x3 in, ReLU, the step's block
    (DepthConvBlock for step 0, Residual Block otherwise, Sec. 3.2), conv3x3 out."""
    a = np.maximum(conv3x3(z, *_wb(weights, pre + ".in")), 0.0)
    a = depth_conv_block(a, weights, pre) if g == 0 else residual_block(a, weights, pre)
    return conv3x3(a, *_wb(weights, pre + ".out"))


def softplus(v):
    return np.log1p(np.exp(-np.abs(v))) + np.maximum(v, 0.0)


def softmax(v):
    m = v.max(axis=-1, keepdims=True)
    e = np.exp(v - m)
    return e / e.sum(axis=-1, keepdims=True)


def mixture_head(r, cfg):
    """Raw 3K outputs -> (w, mu, sigma) per coefficient (reading: the paper's model is a
    Laplacian with mu, sigma; the workload asks for a K-component Gaussian mixture).

    w = softmax(r[0:K]), mu = r[K:2K], sigma = max(softplus(r[2K:3K]), sigma_min).
    """
    K = cfg["mix_k"]
    w = softmax(r[..., :K])
    mu = r[..., K:2 * K]
    sg = np.maximum(softplus(r[..., 2 * K:3 * K]), cfg["sigma_min"])
    return np.concatenate([w, mu, sg], axis=-1)


def group_positions(h, w, g):
    """Raster-order (r, c) of the positions coded at step g."""
    m = group_map(h, w) == g
    return np.nonzero(m)


def step_params(q_i, l_i, t, g, cfg, weights):
    """Entropy parameters [N][n_g][3K] of coding step g of a subband of type t (Sec. 3.2)."""
    pre = f"ctx.{TYPE_NAMES[t]}.{g}"
    if cfg.get("ctx_arch", "plain") == "blocks":
        r = step_stack_blocks(step_input(q_i, l_i, g), weights, pre, g)
    else:
        r = step_stack(step_input(q_i, l_i, g), _convs(weights, pre, cfg["ctx_layers"]))
    rr, cc = group_positions(q_i.shape[1], q_i.shape[2], g)
    return mixture_head(r[:, rr, cc, :], cfg)


# Causal 5x5 neighbourhood of the autoregressive LL model (raster order): the two
# rows above and the two positions to the left.
AR_TAPS = tuple((dy, dx) for dy in (-2, -1) for dx in (-2, -1, 0, 1, 2)) + ((0, -2), (0, -1))


def ar_params(q_ll, cfg, weights):
    """Autoregressive context model of the LL subband (Sec. 3.2, Fig. 4a: LL is coded
    from its own causal spatial context only).  Reading: a 5x5 masked conv over the 12
    already-coded neighbours (zero outside the subband), ReLU, 1x1 conv, ReLU, 1x1 conv
    to 3K, the same mixture head.  q_ll [N][h][w] -> params [N][h*w][3K], raster order."""
    q = np.asarray(q_ll, np.float64)
    N, h, w = q.shape
    qp = np.pad(q, ((0, 0), (2, 2), (2, 2)))
    W0, b0 = _wb(weights, "ar.0")
    a = np.empty((N, h, w, W0.shape[0]))
    a[...] = b0
    for dy, dx in AR_TAPS:
        a += qp[:, 2 + dy:2 + dy + h, 2 + dx:2 + dx + w, None] * W0[:, 0, dy + 2, dx + 2]
    a = np.maximum(a, 0.0)
    a = np.maximum(conv1x1(a, *_wb(weights, "ar.1")), 0.0)
    r = conv1x1(a, *_wb(weights, "ar.2"))
    return mixture_head(r.reshape(N, h * w, -1), cfg)


def context_params_all(qs, cfg, weights):
    """Parameters of every (subband, step) in coding order, from the complete q.

    Because step g only reads q at earlier steps and earlier subbands, this
    teacher-forced evaluation equals what the decoder computes from the
    symbols it has decoded so far.  Returns params[i][g] = [N][n_g][3K].
    """
    ls = long_context(qs, cfg, weights)
    lay = [s["type"] for s in subband_layout(cfg, *_image_hw(qs, cfg))[0]]
    out = [[step_params(qs[i], ls[i], lay[i], g, cfg, weights) for g in range(4)]
           for i in range(len(qs))]
    if cfg.get("ll_ar", 0):
        out[0] = [ar_params(qs[0], cfg, weights)]   # one raster-order step
    return out


def _image_hw(qs, cfg):
    J = cfg["levels"]
    return qs[0].shape[1] << J, qs[0].shape[2] << J


# ----------------------------------------------------------------------------
# CDF tables
# ----------------------------------------------------------------------------
def _phi(z):
    """Standard normal CDF, 0.5 * erfc(-z / sqrt 2), accurate in the lower tail."""
    return 0.5 * _erfc(-z / np.sqrt(2.0))


def _laplace_cdf(z):
    """Standard Laplace CDF: exp(z)/2 for z < 0, 1 - exp(-z)/2 otherwise (Sec. 3.1 uses a
    Laplacian with a mean and a scale per coefficient)."""
    return np.where(z < 0, 0.5 * np.exp(np.minimum(z, 0.0)), 1.0 - 0.5 * np.exp(-np.maximum(z, 0.0)))


def cdf_tables(params, cfg):
    """Integer CDF rows [n][N_s + 1] of the discretised mixture (Gaussian components, or
    Laplacian components when cfg["dist"] == "laplace").

    The paper only says the symbols are arithmetic coded with the estimated
    distribution (Sec. 3.1).  Reading (a 16-bit table over the alphabet):
      T = 2^cdf_bits, N_s = sym_max - sym_min + 1 symbols, F_max = T - N_s;
      C_j = sum_k w_k Phi((b_j - mu_k) / sigma_k) / sum_k w_k (Phi the standard
      normal or standard Laplace CDF, sigma the Laplace scale) at the interior
      boundaries b_j = sym_min + j - 0.5, j = 1 .. N_s - 1 (the weights are
      renormalised because a stored softmax sums to 1 only up to rounding);
      F_j = floor(F_max * C_j), F_0 = 0, F_{N_s} = F_max;
      F made non-decreasing by a running maximum (the identity in exact
      arithmetic); cdf[j] = j + F_j.  Every symbol gets freq >= 1 and the
      table sums to T.
    The value is evaluated as in exact arithmetic: where C_j > 1/2 it is
    computed from the upper tail, F_j = F_max - ceil(F_max * (1 - C_j)), and
    since 1 - C_j > 0 for both families the ceiling is at least 1.
    Entry N_s (= T) is stored as T mod 2^16 = 0 in the uint16 tables.
    """
    K = cfg["mix_k"]
    Ns = cfg["sym_max"] - cfg["sym_min"] + 1
    T = 1 << cfg["cdf_bits"]
    Fmax = T - Ns
    cdf1 = _laplace_cdf if cfg.get("dist", "gauss") == "laplace" else _phi
    p = np.asarray(params, np.float64).reshape(-1, 3 * K)
    w, mu, sg = p[:, :K], p[:, K:2 * K], p[:, 2 * K:]
    j = np.arange(1, Ns)
    b = cfg["sym_min"] + j - 0.5
    z = (b[None, :, None] - mu[:, None, :]) / sg[:, None, :]      # [n][Ns-1][K]
    wsum = w.sum(-1, keepdims=True)
    lower = (w[:, None, :] * cdf1(z)).sum(-1) / wsum
    upper = (w[:, None, :] * cdf1(-z)).sum(-1) / wsum
    F_lo = np.floor(Fmax * lower)
    F_hi = Fmax - np.maximum(1.0, np.ceil(Fmax * upper))
    F = np.where(lower <= upper, F_lo, F_hi)
    F = np.maximum.accumulate(F, axis=1)
    n = p.shape[0]
    out = np.zeros((n, Ns + 1), np.int64)
    out[:, 1:Ns] = j[None, :] + F
    out[:, Ns] = T
    return out


def cdf_to_u16(cdf):
    """Store rows as uint16 (the final entry T wraps to 0)."""
    return (np.asarray(cdf, np.int64) % 65536).astype(np.uint16)


def cdf_trim(cdf):
    """Lossless trim of integer CDF rows [n][N_s + 1] (entry N_s = T), written from the
    table definition of cdf_tables: F_j = cdf[j] - j is 0 below each row's mass window
    and F_max - 1 above it (the upper-tail ceiling is at least 1), so a row is
    (lo, len, F_lo .. F_{lo+len-1}) with lo = 1 + the number of j in 1 .. N_s-1 with
    F_j = 0 and len = the number with 0 < F_j < F_max - 1.
    Returns (lolen int [n][2], packed int [sum len])."""
    cdf = np.asarray(cdf, np.int64)
    n, E = cdf.shape
    ns = E - 1
    T = int(cdf[0, -1]) if n else 65536
    fmax = T - ns
    lolen = np.zeros((n, 2), np.int64)
    parts = []
    for r in range(n):
        F = [int(cdf[r, j]) - j for j in range(1, ns)]
        zeros = sum(1 for v in F if v == 0)
        mid = [v for v in F if 0 < v < fmax - 1]
        lolen[r] = (1 + zeros, len(mid))
        parts.append(np.asarray(mid, np.int64))
    packed = np.concatenate(parts) if parts else np.zeros(0, np.int64)
    return lolen, packed


def cdf_untrim(lolen, packed, n_sym, T=65536):
    """Inverse of cdf_trim: rows [n][n_sym + 1] with entry n_sym = T."""
    lolen = np.asarray(lolen, np.int64)
    out = np.zeros((len(lolen), n_sym + 1), np.int64)
    off = 0
    for r, (lo, ln) in enumerate(lolen):
        for j in range(n_sym):
            F = 0 if j < lo else int(packed[off + j - lo]) if j < lo + ln else T - n_sym - 1
            out[r, j] = j + F
        out[r, n_sym] = T
        off += ln
    return out


def ideal_bits(cdf, idx):
    """sum -log2(freq / T) of symbol indices idx under rows cdf (int, entry N_s = T)."""
    cdf = np.asarray(cdf, np.int64)
    n = cdf.shape[0]
    f = cdf[np.arange(n), idx + 1] - cdf[np.arange(n), idx]
    T = cdf[0, -1]
    return float(-np.log2(f / T).sum())


# ----------------------------------------------------------------------------
# Whole-image encode / decode with the reference coder
# ----------------------------------------------------------------------------
def encode(x, cfg, weights):
    """Planes -> (streams[plane][i][g] bytes, q list, clip count) with the reference rANS."""
    from .rans_ref import rans_encode_ref
    ys = analyze(x, cfg, weights)
    qs, clips = quantize(ys, cfg)
    prm = context_params_all(qs, cfg, weights)
    N = qs[0].shape[0]
    streams = [[[None] * 4 for _ in qs] for _ in range(N)]
    for i, q in enumerate(qs):
        if i == 0 and cfg.get("ll_ar", 0):
            for n in range(N):
                streams[n][0] = [rans_encode_ref(cdf_tables(prm[0][0][n], cfg),
                                                 q[n].ravel() - cfg["sym_min"]), b"", b"", b""]
            continue
        for g in range(4):
            rr, cc = group_positions(q.shape[1], q.shape[2], g)
            for n in range(N):
                cdf = cdf_tables(prm[i][g][n], cfg)
                streams[n][i][g] = rans_encode_ref(cdf, q[n][rr, cc] - cfg["sym_min"])
    return streams, qs, clips


def decode_symbols(streams, cfg, weights, H, W, N):
    """Decode q group by group using only symbols already decoded (Sec. 3.2)."""
    from .rans_ref import rans_decode_ref
    lay, _ = subband_layout(cfg, H, W)
    qs = [np.zeros((N, s["h"], s["w"]), np.int64) for s in lay]
    C = cfg["ctx_ch"]
    wl = np.asarray(weights["lstm.w"], np.float64)
    bl = np.asarray(weights["lstm.b"], np.float64)
    hs = np.zeros((N, lay[0]["h"], lay[0]["w"], C))
    cs = np.zeros_like(hs)
    for i, s in enumerate(lay):
        u = np.zeros((N, s["h"], s["w"])) if i == 0 else qs[i - 1].astype(np.float64)
        if hs.shape[1] != s["h"]:
            hs, cs = upsample2(hs), upsample2(cs)
        if u.shape[1] != s["h"]:
            u = upsample2(u)
        hs, cs = lstm_cell(conv3x3(np.concatenate([u[..., None], hs], -1), wl, bl), cs)
        if i == 0 and cfg.get("ll_ar", 0):
            # Raster order, one symbol at a time, from the symbols decoded so far.
            from .rans_ref import RansDecoderRef
            for n in range(N):
                dec = RansDecoderRef(streams[n][0][0])
                for p in range(s["h"] * s["w"]):
                    r, c = divmod(p, s["w"])
                    prm = ar_params(qs[0][n:n + 1], cfg, weights)[0, p]
                    qs[0][n, r, c] = dec.next(cdf_tables(prm[None], cfg)[0]) + cfg["sym_min"]
                dec.finish()
            continue
        for g in range(4):
            prm = step_params(qs[i], hs, s["type"], g, cfg, weights)
            rr, cc = group_positions(s["h"], s["w"], g)
            for n in range(N):
                idx = rans_decode_ref(cdf_tables(prm[n], cfg), streams[n][i][g], len(rr))
                qs[i][n, rr, cc] = np.asarray(idx) + cfg["sym_min"]
    return qs


def decode(streams, cfg, weights, H, W, N):
    qs = decode_symbols(streams, cfg, weights, H, W, N)
    return synthesize(dequantize(qs, cfg), cfg, weights), qs


def decode_path(qs, cfg, weights):
    """The GPU-timed decode path with symbols supplied (coder elided): the context
    model of every (subband, step), its CDF tables, and synthesis of q.

    Returns (params, cdf tables, reconstruction)."""
    prm = context_params_all(qs, cfg, weights)
    tabs = [[cdf_tables(p, cfg) for p in row] for row in prm]
    xh = synthesize(dequantize(qs, cfg), cfg, weights)
    return prm, tabs, xh


# ----------------------------------------------------------------------------
# Video: temporal Haar lifting
# ----------------------------------------------------------------------------
def temporal_haar_forward(frames, levels=3):
    """Temporal lifting of centred frames [T][...]: H = f_odd - f_even, L = f_even + H/2,
    recursing on the L frames (lifting form of Sec. 3.3 without motion compensation).

    Returns temporal subbands [T][...] ordered L_J, H_J, H_{J-1} (2 frames), ..., H_1.
    """
    f = np.asarray(frames, np.float64)
    highs = []
    for _ in range(levels):
        e, o = f[0::2], f[1::2]
        h = o - e
        f = e + 0.5 * h
        highs.append(h)
    return np.concatenate([f] + highs[::-1], axis=0)


def temporal_haar_inverse(sub, levels=3):
    """Inverse of temporal_haar_forward: f_even = L - H/2, f_odd = H + f_even."""
    s = np.asarray(sub, np.float64)
    n = 1
    f = s[:1]
    k = 1
    for _ in range(levels):
        h = s[k:k + n]
        k += n
        e = f - 0.5 * h
        o = h + e
        f = np.empty((2 * n,) + s.shape[1:])
        f[0::2], f[1::2] = e, o
        n *= 2
    return f


# ----------------------------------------------------------------------------
# Subband impulse response (Sec. 3.4)
# ----------------------------------------------------------------------------
def subband_impulse_responses(qs, cfg, weights, size=16):
    """One response per subband (Sec. 3.4).

    For subband i, the maximum absolute quantised value is placed into the i-th
    subband of an otherwise all-zero `size` x `size` pyramid (level-J subbands
    are 1x1 for size 16 and J = 4).  Its position is the arg-max of |q_i|
    max-pooled down to that subband's size.  The pyramid is dequantised and
    inverse transformed (no +128 offset).  Returns [3J+1][size][size].
    """
    lay, _ = subband_layout(cfg, size, size)
    out = []
    for i, s in enumerate(lay):
        a = np.abs(np.asarray(qs[i][0], np.float64))
        h, w = a.shape
        ph, pw = h // s["h"], w // s["w"]
        pooled = a[:ph * s["h"], :pw * s["w"]].reshape(s["h"], ph, s["w"], pw).max(axis=(1, 3))
        r, c = np.unravel_index(int(np.argmax(pooled)), pooled.shape)
        pyr = [np.zeros((1, t["h"], t["w"])) for t in lay]
        pyr[i][0, r, c] = a.max()
        out.append(synthesize(dequantize(pyr, cfg), cfg, weights, add_offset=False)[0])
    return np.stack(out)
