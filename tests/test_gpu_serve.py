"""Continuous-batching server: each result is the same alone and in the mix (needs an MI355X)."""
import numpy as np
import pytest
import torch

from wvgen import get_config, make_weights, pack_weights, sinusoid_1f_planes, video_gop_420
from gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu


def _alone(model, prep):
    """Decode one prepared input by itself with the single-request calls."""
    from paper_2405_12631_amd import codec
    outs = []
    for H, W, N, q_known, syms, _ in prep.groups:
        ws = codec.Workspace(model, N, H, W)
        q = torch.zeros_like(q_known)
        for i in range(len(ws.lay)):
            for g in range(4):
                prm = codec.context_params(model, q, ws, i, g)
                codec.cdf_tables(model, prm, out=ws.cdf)
                codec.scatter_symbols(model, syms[i][g], q, ws, i, g)
        x, _ = codec.synthesize(model, ws, q=q, offset=128.0 if prep.kind == "image" else 0.0)
        if prep.kind == "gop":
            v = x.view(prep.T, -1)
            codec.temporal_haar(v, inverse=True)
            codec.add_offset(v, 128.0)
        outs.append(x)
    torch.cuda.synchronize()
    return outs


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_served_results_equal_alone_results(prec):
    need_gpu()
    from paper_2405_12631_amd import codec, serve, WV_BF16, WV_FP32, WV_FP8
    say("serve mix", prec)
    cfg = get_config("ycbcr512x768")
    model = codec.Model(cfg, pack_weights(cfg, make_weights(cfg)),
                        precision={"fp32": WV_FP32, "bf16": WV_BF16, "fp8": WV_FP8}[prec])
    luma, chroma = video_gop_420(T=8, H=64, W=64, seed=5)
    preps = {0: serve.Prepared(model, "image", sinusoid_1f_planes(64, 96, 3, seed=1)),
             1: serve.Prepared(model, "image", sinusoid_1f_planes(32, 48, 3, seed=2)),
             2: serve.Prepared(model, "gop", (luma, chroma))}
    # Staggered arrivals on the server's virtual clock (one unit per iteration; a request
    # takes 52 iterations): later requests join while earlier ones are mid-decode.
    reqs = [(0.0, 0), (0.0, 2), (4.0, 1), (8.0, 0), (12.0, 2), (20.0, 1)]
    budget = 3 * max(serve.footprint(model, p) for p in preps.values())     # forces queueing
    seen = {}

    def record(slot, b, i, g, prm):   # parameters of the first request of input 1, as served
        if slot.prep is preps[1] and seen.setdefault("slot", slot) is slot:
            seen[(b, i, g)] = prm.cpu().numpy().copy()

    srv = serve.Server(model, budget, on_params=record if prec == "fp32" else None)
    stats, done = srv.run(reqs, preps, max_seconds=1e9, keep_outputs=True, tick=1.0)
    say(stats)
    assert stats["completed"] == len(reqs) and stats["rejected"] == 0
    # Continuous batching happened: requests were active together, and some joined while
    # another was past its first step.
    assert stats["peak_active"] > 1 and stats["mid_decode_joins"] >= 1, stats
    alone = {pid: _alone(model, p) for pid, p in preps.items()}
    for s in done:
        for b, x in enumerate(s.xhat):
            assert torch.equal(x, alone[s.req["prep"]][b]), (s.req, b)
    # The GOP decodes back to frames close to the input (lossy, step 4).
    g = [s for s in done if s.req["prep"] == 2][0]
    err = (g.xhat[0].cpu().numpy() - luma.astype(np.float32)).std()
    assert err < 8.0, err
    if prec == "fp32":
        # The served FP32 request against the FP64 oracle on the same symbols: every plane's
        # parameters at every (subband, step), and the reconstruction.
        import oracle as O
        from gpu_common import PARAM_RTOL, XHAT_ATOL, param_err
        w = make_weights(cfg)
        H, W, N, q_known, _, _ = preps[1].groups[0]
        qs = O.unpack(q_known.cpu().numpy().astype(np.int64), cfg, H, W)
        ref = O.context_params_all(qs, cfg, w)
        worst = max(param_err(seen[(0, i, g)], ref[i][g], cfg["mix_k"]) for i in range(len(ref)) for g in range(4))
        say("served request vs oracle: worst param rel err", worst)
        assert worst <= PARAM_RTOL
        s1 = [s for s in done if s.req["prep"] == 1][0]
        ref_x = O.synthesize(O.dequantize(qs, cfg), cfg, w)
        assert np.max(np.abs(s1.xhat[0].cpu().numpy() - ref_x)) <= XHAT_ATOL


def test_served_with_host_coder_equals_alone():
    """The coder-inclusive server: every iteration's tables trimmed on the device, copied to
    the host, decoded by the host rANS threads from real GPU-encoded streams, symbols copied
    back.  The decoded symbols and reconstructions equal the coder-elided lone decodes bit
    for bit (FP32 and BF16 context)."""
    need_gpu()
    from paper_2405_12631_amd import codec, serve, WV_BF16
    say("serve with host coder")
    cfg = get_config("ycbcr512x768")
    model = codec.Model(cfg, pack_weights(cfg, make_weights(cfg)), precision=WV_BF16)
    luma, chroma = video_gop_420(T=8, H=64, W=64, seed=7)
    preps = {0: serve.Prepared(model, "image", sinusoid_1f_planes(64, 96, 3, seed=3), coder=True),
             1: serve.Prepared(model, "gop", (luma, chroma), coder=True),
             2: serve.Prepared(model, "image", sinusoid_1f_planes(32, 48, 3, seed=4), coder=True)}
    reqs = [(0.0, 0), (0.0, 1), (3.0, 2), (6.0, 0), (10.0, 1)]
    srv = serve.Server(model, 8 * max(serve.footprint(model, p, coder=True) for p in preps.values()), coder=True)
    stats, done = srv.run(reqs, preps, max_seconds=1e9, keep_outputs=True, tick=1.0)
    say(stats)
    assert stats["completed"] == len(reqs) and stats["mid_decode_joins"] >= 1
    assert stats["table_bytes_to_host"] > 0 and 0 < stats["coder_utilisation"] <= 1.0
    alone = {pid: _alone(model, p) for pid, p in preps.items()}
    for s in done:
        for b, x in enumerate(s.xhat):
            assert torch.equal(x, alone[s.req["prep"]][b]), (s.req, b)
