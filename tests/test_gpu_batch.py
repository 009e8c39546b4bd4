"""Plans over images of uneven size, persistent launches and graph replay (needs an MI355X)."""
import numpy as np
import pytest
import torch

import oracle as O
from wvgen import get_config, make_weights, pack_weights, sinusoid_1f_planes
from gpu_common import PARAM_RTOL, XHAT_ATOL, check_cdf_rows, need_gpu, param_err, say

pytestmark = pytest.mark.gpu

SIZES = [(64, 96), (32, 48), (48, 80), (32, 48)]     # two images share a size; ragged subbands


def _images(sizes, seed=11):
    return [sinusoid_1f_planes(h, w, planes=3, seed=seed + k) for k, (h, w) in enumerate(sizes)]


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_plan_params_equal_per_group_calls_bitwise(prec):
    need_gpu()
    from paper_2405_12631_amd import codec, batch as B, WV_BF16, WV_FP32, WV_FP8
    say("plan vs per-group", prec)
    cfg = get_config("ycbcr512x768")
    model = codec.Model(cfg, pack_weights(cfg, make_weights(cfg)),
                        precision={"fp32": WV_FP32, "bf16": WV_BF16, "fp8": WV_FP8}[prec])
    imgs = _images(SIZES)
    bt = B.Batch(model, SIZES, nb_table=[1, 2, 4, 1])
    bt.load_images(imgs)
    # Reference: each group on its own through wv_context_params.
    refs = []
    for b, w in enumerate(bt.ws):
        ws = codec.Workspace(model, w.N, w.H, w.W)
        refs.append((ws, bt.q[b].clone()))
    K = cfg["mix_k"]
    for i in range(bt.nsub):
        for g in range(4):
            got = bt.context_params(i, g).clone()
            n, first = bt.rows(i, g)
            for b, (ws, q) in enumerate(refs):
                ref = codec.context_params(model, q, ws, i, g).reshape(-1)
                lo = first[b] * 3 * K
                assert torch.equal(got[lo:lo + ref.numel()], ref), (i, g, b)


def test_graph_replay_matches_eager_every_time():
    need_gpu()
    from paper_2405_12631_amd import codec, batch as B, WV_BF16
    say("graph replay")
    cfg = get_config("ycbcr512x768")
    model = codec.Model(cfg, pack_weights(cfg, make_weights(cfg)), precision=WV_BF16)
    bt = B.Batch(model, SIZES)
    bt.load_images(_images(SIZES, seed=21))
    known = [q.clone() for q in bt.q]
    syms = bt.known_symbols()
    eager = [x.clone() for x in bt.decode_elided(syms)]
    torch.cuda.synchronize()
    graph = bt.capture(syms)
    for rep in range(3):
        for q in bt.q:                       # eager work between replays
            q.fill_(7)
        for x in bt.xhat:
            x.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for b in range(len(bt.q)):
            assert torch.equal(bt.q[b], known[b]), (rep, b)
            assert torch.equal(bt.xhat[b], eager[b]), (rep, b)
    # Autotuning keeps the bits.
    tab, t = B.autotune(bt, syms, reps=1)
    say("autotune", tab, t)
    out = [x.clone() for x in bt.decode_elided(syms)]
    torch.cuda.synchronize()
    for b in range(len(out)):
        assert torch.equal(out[b], eager[b])


def test_batch_result_equals_single_image_decode():
    """Each image decodes to the same bits alone and inside the mixed batch."""
    need_gpu()
    from paper_2405_12631_amd import codec, batch as B, WV_BF16
    say("batch vs alone")
    cfg = get_config("ycbcr512x768")
    model = codec.Model(cfg, pack_weights(cfg, make_weights(cfg)), precision=WV_BF16)
    imgs = _images(SIZES, seed=31)
    bt = B.Batch(model, SIZES)
    bt.load_images(imgs)
    out = bt.decode_elided(bt.known_symbols())
    torch.cuda.synchronize()
    for k, (h, w) in enumerate(SIZES):
        ws = codec.Workspace(model, 3, h, w)
        q, _, _ = codec.analyze(model, torch.from_numpy(imgs[k]).cuda(), ws)
        syms = codec.prepare_elided(model, q, ws)
        q0 = torch.zeros_like(q)
        alone = codec.decode_elided(model, syms, ws, q0)
        gb, p0 = bt.where[k]
        assert torch.equal(alone, out[gb][p0:p0 + 3]), k


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_single_image_graph_replays_equal_eager(prec):
    # The bench times replays of one captured single-image decode; every replay, with eager
    # work and synchronisations in between, must equal the eager decode bit for bit.
    need_gpu()
    from paper_2405_12631_amd import codec, WV_BF16, WV_FP32
    say("single-image graph", prec)
    cfg = get_config("ycbcr512x768")
    model = codec.Model(cfg, pack_weights(cfg, make_weights(cfg)),
                        precision=WV_BF16 if prec == "bf16" else WV_FP32)
    x = sinusoid_1f_planes(64, 96, planes=3, seed=5)
    ws = codec.Workspace(model, 3, 64, 96)
    q_known, _, _ = codec.analyze(model, torch.from_numpy(x).cuda(), ws)
    syms = codec.prepare_elided(model, q_known, ws)
    q = torch.zeros_like(q_known)
    xhat = torch.empty((3, 64, 96), dtype=torch.float32, device="cuda")

    def step():
        codec.zero(q)
        codec.decode_elided(model, syms, ws, q, xhat)

    step()
    torch.cuda.synchronize()
    ref_q, ref_x = q.clone(), xhat.clone()
    assert torch.equal(ref_q, q_known)
    graph = codec.Graph(step)          # wv_graph_begin / wv_graph_end around the library calls
    for _ in range(3):
        q.fill_(7)
        xhat.fill_(-1.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(q, ref_q) and torch.equal(xhat, ref_x)


def test_wide_and_narrow_channel_blocking_bitwise():
    """The number of 16-channel output blocks per workgroup (and with it the item
    order over tiles and columns) never changes a result: a plan with four blocks
    per item everywhere (many segments, ragged subbands) and single-image calls on
    a 512x768 image (whose level-1 subbands take four blocks by the default rule)
    give the bits of a plan with two blocks everywhere (BF16 model)."""
    need_gpu()
    from paper_2405_12631_amd import codec, batch as B, WV_BF16
    say("wide vs narrow channel blocking")
    cfg = get_config("ycbcr512x768")
    model = codec.Model(cfg, pack_weights(cfg, make_weights(cfg)), precision=WV_BF16)
    sizes = [(512, 768), (64, 96), (48, 80), (64, 96)]
    imgs = _images(sizes, seed=41)
    narrow = B.Batch(model, sizes, nb_table=[2, 2, 2, 2])
    wide = B.Batch(model, sizes, nb_table=[4, 4, 4, 4])
    narrow.load_images(imgs)
    wide.load_images(imgs)
    for b in range(len(narrow.q)):
        assert torch.equal(narrow.q[b], wide.q[b])
    gb = narrow.where[0][0]
    ws = codec.Workspace(model, 3, 512, 768)
    q = narrow.q[gb].clone()
    K = cfg["mix_k"]
    for i in range(narrow.nsub):
        for g in range(4):
            a = narrow.context_params(i, g).clone()
            b = wide.context_params(i, g).clone()
            assert torch.equal(a, b), (i, g)
            n, first = narrow.rows(i, g)
            ref = codec.context_params(model, q, ws, i, g).reshape(-1)
            lo = first[gb] * 3 * K
            assert torch.equal(a[lo:lo + ref.numel()], ref), (i, g)


def test_plan_decode_matches_oracle_fp32():
    """A mixed-size FP32 plan (a 256 x 256 image, two 64 x 96 images, a 48 x 80 image and a
    1088 x 1920 image, three planes each) decoded through the persistent plan launches: every
    group's parameters (plane 0) against the FP64 oracle on the same symbols, at every
    (subband, step) (for 1088 x 1920 the level-4 and level-3 subbands, whose oracle finishes in
    seconds), one step's CDF rows against the oracle's tables of those parameters, and every
    group's reconstruction (plane 0; the wide 1088 x 1920 arrays take the row-streaming lifting
    kernel, the others the tiles)."""
    need_gpu()
    from paper_2405_12631_amd import codec, batch as B
    say("plan vs oracle fp32")
    cfg = get_config("ycbcr512x768")
    w = make_weights(cfg)
    model = codec.Model(cfg, pack_weights(cfg, w))
    sizes = [(256, 256), (64, 96), (48, 80), (1088, 1920), (64, 96)]
    bt = B.Batch(model, sizes)
    bt.load_images(_images(sizes, seed=51))
    syms = bt.known_symbols()
    K = cfg["mix_k"]
    qs = {b: O.unpack(bt.q[b][:1].cpu().numpy().astype(np.int64), cfg, ws.H, ws.W) for b, ws in enumerate(bt.ws)}
    checked = {b: (13 if ws.H * ws.W <= 256 * 256 else 7) for b, ws in enumerate(bt.ws)}
    got = {b: [] for b in qs}
    for q in bt.q:
        codec.zero(q)
    for i in range(bt.nsub):
        for g in range(4):
            prm = bt.context_params(i, g)
            n, first = bt.rows(i, g)
            for b, ws in enumerate(bt.ws):
                if i < checked[b]:
                    lay = ws.lay[i]
                    ng = codec.Model.group_count(lay["h"], lay["w"], g)
                    lo = first[b] * 3 * K
                    got[b].append(prm[lo:lo + ng * 3 * K].cpu().numpy().reshape(ng, 3 * K))
            cdf = bt.cdf_tables(prm)
            if (i, g) == (12, 2):
                check_cdf_rows(cdf[:n].cpu().numpy().view(np.uint16), prm[:n * 3 * K].cpu().numpy(), cfg)
            bt.scatter(syms[i][g], i, g)
    xh = bt.synthesize()
    torch.cuda.synchronize()
    for b, ws in enumerate(bt.ws):
        ls = O.long_context(qs[b], cfg, w, upto=checked[b])
        worst = 0.0
        for i in range(checked[b]):
            for g in range(4):
                ref = O.step_params(qs[b][i], ls[i], ws.lay[i]["type"], g, cfg, w)[0]
                worst = max(worst, param_err(got[b][4 * i + g], ref, K))
        say(f"group {ws.H}x{ws.W}: worst param rel err {worst:.2e} over {checked[b]} subbands")
        assert worst <= PARAM_RTOL, (ws.H, ws.W, worst)
        ref_x = O.synthesize(O.dequantize(qs[b], cfg), cfg, w)[0]
        err = float(np.max(np.abs(xh[b][0].cpu().numpy() - ref_x)))
        say(f"group {ws.H}x{ws.W}: xhat err {err:.2e}")
        assert err <= XHAT_ATOL, (ws.H, ws.W, err)


def test_fused_step_stacks_equal_layer_by_layer_bitwise():
    """The fused BF16 kernels (the ConvLSTM with weights in registers and input rows in an LDS
    ring; the step stacks: three ReLU layers and the head with activations in LDS) against the
    layer-by-layer launches, bit for bit: the parameters of every (subband, step) and the
    ConvLSTM's h and c after every subband, on a plan with tall subbands split into row pieces
    (1088 x 1920: level 1 is 544 rows in five pieces, 17 stack strips with a ragged last one),
    a 256 x 256 image, a small ragged one and a 16 x 32 one (level-4 subbands of 1 x 2: items of
    one row)."""
    import os
    need_gpu()
    from paper_2405_12631_amd import codec, batch as B, WV_BF16
    say("fused stacks vs layer by layer")
    cfg = get_config("ycbcr512x768")
    model = codec.Model(cfg, pack_weights(cfg, make_weights(cfg)), precision=WV_BF16)
    sizes = [(1088, 1920), (256, 256), (48, 80), (16, 32)]
    imgs = _images(sizes, seed=61)
    os.environ["WV_FUSED_STACKS"] = "0"
    try:
        layered = B.Batch(model, sizes)
    finally:
        del os.environ["WV_FUSED_STACKS"]
    fused = B.Batch(model, sizes)
    layered.load_images(imgs)
    fused.load_images(imgs)
    C = cfg["ctx_ch"]
    for i in range(fused.nsub):
        for g in range(4):
            a = fused.context_params(i, g)
            b = layered.context_params(i, g)
            assert torch.equal(a, b), (i, g)
            if g == 0:   # the state half of subband i: h (BF16) then, SS floats on, c (FP32)
                for wf, wl in zip(fused.ws, layered.ws):
                    lay = wf.lay[i]
                    n = wf.N * lay["h"] * lay["w"] * C
                    SS = wf.state.numel() // 4
                    h0, c0 = (i & 1) * 2 * SS, (i & 1) * 2 * SS + SS
                    assert torch.equal(wf.state[h0:h0 + n // 2], wl.state[h0:h0 + n // 2]), ("h", i)
                    assert torch.equal(wf.state[c0:c0 + n], wl.state[c0:c0 + n]), ("c", i)
