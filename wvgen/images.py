"""Seeded synthetic images and video.

* gradient_noise_image: a diagonal ramp plus Gaussian noise (small 64x64 case).
* sinusoid_1f_planes: sums of random-phase 2-D sinusoids with a 1/f amplitude
  spectrum plus Gaussian noise, one independent texture per colour plane.  The
  1/f spectrum imitates natural-image statistics; it stands in for the photo
  test sets used in the paper's experiments, matching their shapes only.
* video_gop_420: a group of frames of a 1/f texture moving by a global shift per
  frame, luma at full size and both chroma planes at half size (4:2:0).

All outputs are uint8 arrays.  The sinusoid sums are evaluated exactly through
the identity cos(a + b) = cos a cos b - sin a sin b, which turns the sum over
sinusoids into two small matrix products.
"""
import numpy as np


def _to_u8(v):
    return np.clip(np.rint(v), 0, 255).astype(np.uint8)


def gradient_noise_image(H=64, W=64, seed=1, noise=10.0):
    """Ramp 255*(r+c)/(H+W-2) plus N(0, noise^2), rounded and clipped to uint8."""
    rng = np.random.default_rng(seed)
    r = np.arange(H, dtype=np.float64)[:, None]
    c = np.arange(W, dtype=np.float64)[None, :]
    ramp = 255.0 * (r + c) / float(H + W - 2)
    return _to_u8(ramp + noise * rng.standard_normal((H, W)))


def _sinusoid_params(rng, M, fmin, fmax=0.5):
    f = np.exp(rng.uniform(np.log(fmin), np.log(fmax), M))   # cycles / pixel
    theta = rng.uniform(0.0, np.pi, M)
    phase = rng.uniform(0.0, 2.0 * np.pi, M)
    amp = 1.0 / f
    return 2.0 * np.pi * f * np.cos(theta), 2.0 * np.pi * f * np.sin(theta), phase, amp


def _sinusoid_texture(H, W, params, x0=0.0):
    """sum_m amp_m cos(ax_m (x + x0) + ay_m y + phase_m) on an H x W grid."""
    ax, ay, phase, amp = params
    x = np.arange(W, dtype=np.float64)[:, None] + x0
    y = np.arange(H, dtype=np.float64)[:, None]
    cx = np.cos(x * ax[None, :] + phase[None, :]) * amp[None, :]
    sx = np.sin(x * ax[None, :] + phase[None, :]) * amp[None, :]
    cy = np.cos(y * ay[None, :])
    sy = np.sin(y * ay[None, :])
    return cy @ cx.T - sy @ sx.T


def sinusoid_1f_planes(H, W, planes=3, seed=2, M=256, stds=(40.0, 20.0, 20.0), noise=5.0):
    """`planes` independent 1/f textures (Y, Cb, Cr order), uint8 [planes][H][W].

    Plane p has standard deviation stds[p] around 128 before the N(0, noise^2)
    noise is added.  `seed` is an int or a numpy SeedSequence.
    """
    rng = np.random.default_rng(seed)
    out = np.empty((planes, H, W), np.uint8)
    fmin = 1.0 / max(H, W)
    for p in range(planes):
        tex = _sinusoid_texture(H, W, _sinusoid_params(rng, M, fmin))
        tex = (tex - tex.mean()) * (stds[p % len(stds)] / tex.std())
        out[p] = _to_u8(128.0 + tex + noise * rng.standard_normal((H, W)))
    return out


def video_gop_420(T=8, H=1088, W=1920, seed=5, shift_px=2, M=256, stds=(40.0, 20.0, 20.0),
                  noise=5.0):
    """A GOP of T frames of a texture moving `shift_px` px/frame to the left.

    Returns (luma uint8 [T][H][W], chroma uint8 [T][2][H/2][W/2]).  Chroma moves
    by shift_px/2 px/frame.  The texture scale is fixed by frame 0 so all frames
    share it.
    """
    rng = np.random.default_rng(seed)
    luma = np.empty((T, H, W), np.uint8)
    chroma = np.empty((T, 2, H // 2, W // 2), np.uint8)
    specs = [(luma, None, H, W, shift_px, stds[0]),
             (chroma, 0, H // 2, W // 2, shift_px / 2.0, stds[1]),
             (chroma, 1, H // 2, W // 2, shift_px / 2.0, stds[2])]
    for arr, ch, h, w, sh, sd in specs:
        prm = _sinusoid_params(rng, M, 1.0 / max(h, w))
        base = _sinusoid_texture(h, w, prm)
        mean, scale = base.mean(), sd / base.std()
        for t in range(T):
            tex = base if t == 0 else _sinusoid_texture(h, w, prm, x0=sh * t)
            v = _to_u8(128.0 + (tex - mean) * scale + noise * rng.standard_normal((h, w)))
            if ch is None:
                arr[t] = v
            else:
                arr[t, ch] = v
    return luma, chroma


def batch_sizes(n, sizes, seed=3):
    """n (H, W) pairs drawn uniformly from `sizes`, plus one SeedSequence per image."""
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, len(sizes), n)
    seeds = np.random.SeedSequence(seed).spawn(n)
    return [tuple(sizes[i]) for i in idx], seeds
