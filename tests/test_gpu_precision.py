"""BF16 and FP8 context convs: error against the FP64 oracle, bit-exact GPU round
trip, batch invariance (needs an MI355X)."""
import numpy as np
import pytest
import torch

import oracle as O
from wvgen import get_config, make_weights, pack_weights, sinusoid_1f_planes, gradient_noise_image
from gpu_common import REDUCED_BARS, check_cdf_rows, need_gpu, q_to_device, reduced_errs, say

pytestmark = pytest.mark.gpu

BARS = REDUCED_BARS
_errs = reduced_errs


def _prec(name):
    from paper_2405_12631_amd import WV_BF16, WV_FP8
    return {"bf16": WV_BF16, "fp8": WV_FP8}[name]


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("name,H,W,N", [("gray64", 64, 64, 1), ("ycbcr512x768", 64, 96, 3)])
def test_reduced_precision_params_against_oracle(prec, name, H, W, N):
    need_gpu()
    from paper_2405_12631_amd import codec
    say(prec, "params", name)
    cfg = get_config(name)
    w = make_weights(cfg)
    model = codec.Model(cfg, pack_weights(cfg, w), precision=_prec(prec))
    x = gradient_noise_image(H, W, seed=1)[None] if N == 1 else sinusoid_1f_planes(H, W, planes=N, seed=2)
    qs, _ = O.quantize(O.analyze(x, cfg, w), cfg)
    ws = codec.Workspace(model, N, H, W)
    got = codec.params_all(model, q_to_device(qs), ws)
    ref = O.context_params_all(qs, cfg, w)
    rels, wmax = [], 0.0
    for i in range(len(ref)):
        for g in range(4):
            r, wm = _errs(got[i][g].cpu().numpy(), ref[i][g], cfg["mix_k"])
            rels.append(r.ravel())
            wmax = max(wmax, wm)
    rel = np.concatenate(rels)
    say(f"{prec} {name}: mean rel {rel.mean():.3e} median {np.median(rel):.3e} max {rel.max():.3e} "
        f"max |dw| {wmax:.3e}")
    assert rel.mean() < BARS[prec][0] and wmax < BARS[prec][1]
    for i in (0, len(ref) - 1):
        cdf = codec.cdf_tables(model, got[i][3])
        check_cdf_rows(cdf.cpu().numpy().view(np.uint16), got[i][3].cpu().numpy(), cfg)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_reduced_precision_roundtrip_bit_exact_and_batch_invariant(prec):
    need_gpu()
    from paper_2405_12631_amd import codec
    say(prec, "roundtrip")
    cfg = get_config("ycbcr512x768")
    model = codec.Model(cfg, pack_weights(cfg, make_weights(cfg)), precision=_prec(prec))
    x = sinusoid_1f_planes(64, 96, planes=3, seed=3)
    data, q_enc = codec.encode(model, x)
    _, _, q_dec = codec.decode(model, data)
    assert torch.equal(q_enc, q_dec)
    ws3 = codec.Workspace(model, 3, 64, 96)
    ws1 = codec.Workspace(model, 1, 64, 96)
    p3 = codec.params_all(model, q_enc, ws3)
    p1 = codec.params_all(model, q_enc[2:3].contiguous(), ws1)
    for i in range(13):
        for g in range(4):
            assert torch.equal(p3[i][g][2:3], p1[i][g])
    # A stream written by the FP32 model is refused by the reduced-precision model.
    fp32 = codec.Model(cfg, pack_weights(cfg, make_weights(cfg)))
    d32, _ = codec.encode(fp32, x[:1])
    with pytest.raises(Exception):
        codec.decode(model, d32)
