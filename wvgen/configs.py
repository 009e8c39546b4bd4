"""Workload parameters of the five synthetic workloads.

Each entry fixes the model hyper-parameters (transform depth, channel counts,
mixture size, quantisation step, alphabet) and the input recipe.  The numbers
are parameters, not results of the method.
"""
import copy

_BASE = dict(
    lift_layers=3,      # conv3x3 layers inside one predict/update filter
    mix_k=3,            # mixture components per coefficient
    dist="gauss",       # component family: "gauss" or "laplace"
    ctx_arch="plain",   # step stacks: "plain" conv stacks or "blocks" (DepthConv / Residual)
    ll_ar=0,            # 1: LL_J coded autoregressively (raster order) instead of in four steps
    ar_ch=32,           # channels of the autoregressive LL model
    sym_min=-64,        # symbol alphabet [sym_min, sym_max]
    sym_max=64,
    cdf_bits=16,        # CDF tables are 16-bit integers summing to 2**cdf_bits
    sigma_min=0.11,     # floor of the mixture scales, in symbol units
    lift_int=0,         # 1: predict/update outputs rounded to integers (lossless lifting)
    seed_weights=0,
)

CONFIGS = {
    # 64x64 grayscale gradient + N(0, 10^2), 2-level lifting with 16-channel
    # filters, 3-layer 32-channel context stacks, step 8.
    "gray64": dict(_BASE, name="gray64", H=64, W=64, planes=1, levels=2,
                   lift_ch=16, ctx_ch=32, ctx_layers=3, step=8.0,
                   image="gradient", seed_image=1),
    # 512x768 YCbCr (three full-resolution planes), 1/f sinusoids + N(0, 5^2),
    # 4-level lifting with 32-channel filters, 4-layer 64-channel context
    # stacks, step 4.
    "ycbcr512x768": dict(_BASE, name="ycbcr512x768", H=512, W=768, planes=3, levels=4,
                         lift_ch=32, ctx_ch=64, ctx_layers=4, step=4.0,
                         image="sinusoid_1f", seed_image=2),
    # Mixed-size batch: 64 images drawn from four sizes, same model as above.
    "batch64_mixed": dict(_BASE, name="batch64_mixed", H=None, W=None, planes=3, levels=4,
                          lift_ch=32, ctx_ch=64, ctx_layers=4, step=4.0,
                          image="sinusoid_1f", seed_image=3, batch=64,
                          sizes=((256, 256), (512, 768), (1024, 1024), (1088, 1920))),
    # Serving mix: Poisson arrivals, 70% stills (sizes above), 30% 8-frame
    # 1088x1920 4:2:0 GOPs.
    "serve_mix": dict(_BASE, name="serve_mix", H=None, W=None, planes=3, levels=4,
                      lift_ch=32, ctx_ch=64, ctx_layers=4, step=4.0,
                      image="sinusoid_1f", seed_image=3, seed_arrivals=4,
                      rate_hz=200.0, duration_s=60.0, frac_video=0.3, gop=8,
                      video_hw=(1088, 1920), shift_px=2,
                      sizes=((256, 256), (512, 768), (1024, 1024), (1088, 1920))),
}


def get_config(name, **overrides):
    """Return a deep copy of a named workload with optional overrides."""
    cfg = copy.deepcopy(CONFIGS[name])
    cfg.update(overrides)
    return cfg


def subband_count(levels):
    """Number of subbands of a `levels`-level 2-D decomposition."""
    return 3 * levels + 1
