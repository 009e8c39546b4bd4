"""HIP path vs the FP64 oracle on identical seeded inputs (needs an MI355X)."""
import numpy as np
import pytest
import torch

import oracle as O
from wvgen import get_config, gradient_noise_image, sinusoid_1f_planes
from gpu_common import (PARAM_RTOL, REDUCED_BARS, XHAT_ATOL, check_cdf_rows, model_for, need_gpu, param_err,
                        q_to_device, reduced_errs, say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    need_gpu()
    from paper_2405_12631_amd import codec
    cfg = get_config("gray64")
    model, w = model_for(cfg)
    x = gradient_noise_image(64, 64, seed=1)[None]
    ys = O.analyze(x, cfg, w)
    qs, _ = O.quantize(ys, cfg)
    ws = codec.Workspace(model, 1, 64, 64)
    return dict(cfg=cfg, model=model, w=w, x=x, ys=ys, qs=qs, ws=ws, codec=codec)


def test_analyze_matches_oracle(small):
    say("analyze gray64")
    c = small["codec"]
    q, y, clip = c.analyze(small["model"], torch.from_numpy(small["x"]).cuda(), small["ws"], want_y=True)
    y_ref = O.pack(small["ys"])
    y_gpu = y.cpu().numpy()
    assert np.max(np.abs(y_gpu - y_ref)) < 2e-3
    check_q_near_ties(q.cpu().numpy(), y_gpu, y_ref, small["cfg"])
    assert int(clip.item()) == O.quantize(small["ys"], small["cfg"])[1]


def check_q_near_ties(q_gpu, y_gpu, y_ref, cfg):
    """q parity: the GPU's q is exactly clamp(rint(y_gpu * Delta)) of its own FP32 y, and
    differs from the oracle's q only by 1, only where the oracle's y * Delta lies within the
    measured FP32-vs-FP64 error of y (times Delta) of a rounding tie k + 1/2."""
    d = 1.0 / cfg["step"]
    q_gpu = np.asarray(q_gpu, np.int64)
    own = np.clip(np.rint(np.asarray(y_gpu, np.float32) * np.float32(d)), cfg["sym_min"], cfg["sym_max"])
    assert np.array_equal(q_gpu, own.astype(np.int64))
    q_ref = np.clip(np.rint(y_ref * d), cfg["sym_min"], cfg["sym_max"]).astype(np.int64)
    window = float(np.max(np.abs(np.asarray(y_gpu, np.float64) - y_ref))) * d
    bad = np.nonzero(q_gpu != q_ref)
    assert np.all(np.abs(q_gpu[bad] - q_ref[bad]) == 1)
    dist = np.abs(np.abs(y_ref[bad] * d - np.floor(y_ref[bad] * d)) - 0.5)
    assert np.all(dist <= window), (dist.max(initial=0), window)
    say(f"q: {len(bad[0])} of {q_gpu.size} differ from the oracle, all within {window:.2e} of a tie")


def test_synthesize_matches_oracle(small):
    say("synthesize gray64")
    c = small["codec"]
    xh, u8 = c.synthesize(small["model"], small["ws"], q=q_to_device(small["qs"]), want_u8=True)
    ref = O.synthesize(O.dequantize(small["qs"], small["cfg"]), small["cfg"], small["w"])
    assert np.max(np.abs(xh.cpu().numpy() - ref)) <= XHAT_ATOL
    assert np.array_equal(u8.cpu().numpy(), np.clip(np.rint(xh.cpu().numpy()), 0, 255).astype(np.uint8))


def test_context_params_match_oracle_every_step(small):
    say("context params gray64")
    c = small["codec"]
    cfg = small["cfg"]
    got = c.params_all(small["model"], q_to_device(small["qs"]), small["ws"])
    ref = O.context_params_all(small["qs"], cfg, small["w"])
    worst = 0.0
    for i in range(len(ref)):
        for g in range(4):
            e = param_err(got[i][g].cpu().numpy(), ref[i][g], cfg["mix_k"])
            worst = max(worst, e)
            assert e <= PARAM_RTOL, (i, g, e)
    say("worst param rel err", worst)


def test_cdf_tables_match_oracle_and_invariants(small):
    say("cdf gray64")
    c = small["codec"]
    model, cfg = small["model"], small["cfg"]
    got = c.params_all(model, q_to_device(small["qs"]), small["ws"])
    for i in (0, 3, 6):
        for g in range(4):
            cdf = c.cdf_tables(model, got[i][g])
            check_cdf_rows(cdf.cpu().numpy().view(np.uint16), got[i][g].cpu().numpy(), cfg)


def test_cdf_extreme_params():
    need_gpu()
    from paper_2405_12631_amd import codec
    cfg = get_config("gray64")
    model, _ = model_for(cfg)
    rng = np.random.default_rng(41)
    n = 5000
    logits = rng.normal(0, 4, (n, 3))
    w = np.exp(logits - logits.max(1, keepdims=True))
    w /= w.sum(1, keepdims=True)
    mu = rng.uniform(-90, 90, (n, 3))
    sg = np.exp(rng.uniform(np.log(0.11), np.log(400), (n, 3)))
    prm = torch.from_numpy(np.concatenate([w, mu, sg], 1).astype(np.float32)).cuda()
    for m in (1, 63, 64, 65, 1000, n):       # ragged last workgroup of rows
        say("cdf rows", m)
        cdf = codec.cdf_tables(model, prm[:m])
        check_cdf_rows(cdf.cpu().numpy().view(np.uint16), prm[:m].cpu().numpy(), cfg)
    empty = codec.cdf_tables(model, prm[:0])
    assert empty.shape[0] == 0


def test_cdf_row_split_forms_bitwise():
    """Launches of up to 256 Ki rows build each row with 4 lanes (slices of the entries and a
    prefix maximum), larger ones with one lane per row: identical tables."""
    need_gpu()
    from paper_2405_12631_amd import codec
    cfg = get_config("gray64")
    model, _ = model_for(cfg)
    rng = np.random.default_rng(47)
    n = 300_000                                  # one lane per row
    logits = rng.normal(0, 3, (n, 3))
    w = np.exp(logits - logits.max(1, keepdims=True))
    w /= w.sum(1, keepdims=True)
    mu = rng.uniform(-90, 90, (n, 3))
    sg = np.exp(rng.uniform(np.log(0.11), np.log(200), (n, 3)))
    prm = torch.from_numpy(np.concatenate([w, mu, sg], 1).astype(np.float32)).cuda()
    say("cdf rows", n)
    big = codec.cdf_tables(model, prm).cpu().numpy().view(np.uint16)
    check_cdf_rows(big[:1000], prm[:1000].cpu().numpy(), cfg)
    for m in (1, 65, 5000, 262_144):             # four lanes per row
        say("cdf rows (split)", m)
        part = codec.cdf_tables(model, prm[:m]).cpu().numpy().view(np.uint16)
        assert np.array_equal(part, big[:m]), m


@pytest.mark.parametrize("smin,smax", [(-3, 3), (-20, 21), (-127, 127)])
def test_cdf_alphabets_both_forms(smin, smax):
    """Other alphabet sizes: 7 symbols (the last of the 4 entry slices is empty), 42 (uneven
    slices), 255 (the largest table, 256 entries): one-lane and four-lane forms give the same
    tables, and they match the oracle."""
    need_gpu()
    from paper_2405_12631_amd import codec
    cfg = get_config("gray64", sym_min=smin, sym_max=smax)
    model, _ = model_for(cfg)
    rng = np.random.default_rng(53)
    n = 300_000
    logits = rng.normal(0, 3, (n, 3))
    w = np.exp(logits - logits.max(1, keepdims=True))
    w /= w.sum(1, keepdims=True)
    mu = rng.uniform(smin - 5, smax + 5, (n, 3))
    sg = np.exp(rng.uniform(np.log(0.11), np.log(2.0 * (smax - smin)), (n, 3)))
    prm = torch.from_numpy(np.concatenate([w, mu, sg], 1).astype(np.float32)).cuda()
    say("cdf alphabet", smin, smax)
    big = codec.cdf_tables(model, prm).cpu().numpy().view(np.uint16)
    assert big.shape == (n, smax - smin + 2)
    check_cdf_rows(big[:1000], prm[:1000].cpu().numpy(), cfg)
    for m in (1, 65, 5000):
        part = codec.cdf_tables(model, prm[:m]).cpu().numpy().view(np.uint16)
        assert np.array_equal(part, big[:m]), m


def test_cdf_trim_matches_oracle_definition():
    need_gpu()
    import ctypes
    from paper_2405_12631_amd import codec, _lib as L
    cfg = get_config("gray64")
    model, _ = model_for(cfg)
    rng = np.random.default_rng(43)
    n = 300_000                                  # > 1024 blocks of 256 rows: several scan chunks
    logits = rng.normal(0, 3, (n, 3))
    w = np.exp(logits - logits.max(1, keepdims=True))
    w /= w.sum(1, keepdims=True)
    mu = rng.uniform(-90, 90, (n, 3))
    sg = np.exp(rng.uniform(np.log(0.11), np.log(100), (n, 3)))
    prm = torch.from_numpy(np.concatenate([w, mu, sg], 1).astype(np.float32)).cuda()

    class WS:                                    # trim buffers sized for n rows
        pass
    ws = WS()
    tb = ctypes.c_size_t()
    L.call("wv_cdf_trim_scratch_bytes", n, ctypes.byref(tb))
    ws.lolen = torch.empty(2 * n, dtype=torch.uint8, device="cuda")
    ws.packed = torch.empty(n * 128, dtype=torch.int16, device="cuda")
    ws.trim_scratch = torch.empty(tb.value, dtype=torch.uint8, device="cuda")
    for m in (1, 255, 256, 257, 5000, n):
        say("cdf trim rows", m)
        cdf = codec.cdf_tables(model, prm[:m])
        full = cdf.cpu().numpy().view(np.uint16)
        tr = codec.cdf_trim_to_host(model, cdf, ws)
        k = min(m, 3000)                         # the oracle's definition, row by row, on a prefix
        lolen, packed = O.cdf_trim(full[:k].astype(np.int64) + np.r_[np.zeros(129, np.int64), 65536])
        assert np.array_equal(tr.lolen[:k], lolen)
        assert np.array_equal(tr.packed[:tr.off[k]], packed)
        assert np.array_equal(tr.full(), full)  # lossless at every size
    assert codec.cdf_trim_to_host(model, codec.cdf_tables(model, prm[:0]), ws).lolen.shape == (0, 2)


def test_encode_decode_roundtrip_bit_exact(small):
    say("roundtrip gray64")
    c = small["codec"]
    model = small["model"]
    data, q_enc = c.encode(model, small["x"])
    xh, u8, q_dec = c.decode(model, data)
    assert torch.equal(q_enc, q_dec)
    xs, _ = c.synthesize(model, c.Workspace(model, 1, 64, 64), q=q_enc)
    assert torch.equal(xs, xh)
    # The bitstream is close to the ideal code length of the tables.
    n_coef = 64 * 64
    assert len(data) * 8 / n_coef < 8.0
    # Corruption is reported, not crashed on.
    bad = bytearray(data)
    bad[-5] ^= 0xFF
    with pytest.raises(Exception):
        c.decode(model, bytes(bad))


def test_decode_elided_deterministic_and_matches_synthesis(small):
    say("elided decode determinism")
    c = small["codec"]
    model, ws = small["model"], small["ws"]
    qk = q_to_device(small["qs"])
    syms = c.prepare_elided(model, qk, ws)
    outs = []
    for _ in range(2):
        q = torch.zeros_like(qk)
        outs.append((c.decode_elided(model, syms, ws, q).clone(), q.clone(), ws.cdf.clone()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][2], outs[1][2])
    assert torch.equal(outs[0][1], qk)


@pytest.mark.parametrize("H,W,J", [(36, 52, 2), (48, 80, 4), (16, 16, 4)])
def test_ragged_and_odd_subbands(H, W, J):
    need_gpu()
    from paper_2405_12631_amd import codec
    say("ragged", H, W, J)
    cfg = get_config("gray64", levels=J)
    model, w = model_for(cfg)
    x = sinusoid_1f_planes(H, W, planes=2, seed=7)
    qs, _ = O.quantize(O.analyze(x, cfg, w), cfg)
    ws = codec.Workspace(model, 2, H, W)
    got = codec.params_all(model, q_to_device(qs), ws)
    ref = O.context_params_all(qs, cfg, w)
    for i in range(len(ref)):
        for g in range(4):
            assert param_err(got[i][g].cpu().numpy(), ref[i][g], 3) <= PARAM_RTOL, (i, g)
    xh, _ = codec.synthesize(model, ws, q=q_to_device(qs))
    assert np.max(np.abs(xh.cpu().numpy() - O.synthesize(O.dequantize(qs, cfg), cfg, w))) <= XHAT_ATOL


def test_large_model_small_image_parity():
    """The 64-channel, 4-layer context model and 32-channel lifting on a 64x96 3-plane image."""
    need_gpu()
    from paper_2405_12631_amd import codec
    say("ycbcr model 64x96")
    cfg = get_config("ycbcr512x768")
    model, w = model_for(cfg)
    x = sinusoid_1f_planes(64, 96, planes=3, seed=2)
    ys = O.analyze(x, cfg, w)
    qs, _ = O.quantize(ys, cfg)
    ws = codec.Workspace(model, 3, 64, 96)
    q, y, _ = codec.analyze(model, torch.from_numpy(x).cuda(), ws, want_y=True)
    assert np.max(np.abs(y.cpu().numpy() - O.pack(ys))) < 5e-3
    got = codec.params_all(model, q_to_device(qs), ws)
    ref = O.context_params_all(qs, cfg, w)
    worst = max(param_err(got[i][g].cpu().numpy(), ref[i][g], 3) for i in range(13) for g in range(4))
    say("worst param rel err", worst)
    assert worst <= PARAM_RTOL
    xh, _ = codec.synthesize(model, ws, q=q_to_device(qs))
    assert np.max(np.abs(xh.cpu().numpy() - O.synthesize(O.dequantize(qs, cfg), cfg, w))) <= XHAT_ATOL


def test_batch_invariance_bitwise():
    """A plane's parameters and reconstruction do not depend on the other planes of the batch."""
    need_gpu()
    from paper_2405_12631_amd import codec
    say("batch invariance")
    cfg = get_config("ycbcr512x768")
    model, w = model_for(cfg)
    x = sinusoid_1f_planes(64, 96, planes=3, seed=4)
    ws3 = codec.Workspace(model, 3, 64, 96)
    ws1 = codec.Workspace(model, 1, 64, 96)
    q3, _, _ = codec.analyze(model, torch.from_numpy(x).cuda(), ws3)
    q1, _, _ = codec.analyze(model, torch.from_numpy(x[1:2]).cuda(), ws1)
    assert torch.equal(q3[1:2], q1)
    p3 = codec.params_all(model, q3, ws3)
    p1 = codec.params_all(model, q1, ws1)
    for i in range(13):
        for g in range(4):
            assert torch.equal(p3[i][g][1:2], p1[i][g])
    x3, _ = codec.synthesize(model, ws3, q=q3)
    x1, _ = codec.synthesize(model, ws1, q=q1)
    assert torch.equal(x3[1:2], x1)


def test_integer_lifting_perfect_reconstruction_bit_exact():
    need_gpu()
    from paper_2405_12631_amd import codec
    say("integer lifting PR")
    cfg = get_config("ycbcr512x768", lift_int=1)
    model, w = model_for(cfg)
    x = sinusoid_1f_planes(64, 96, planes=3, seed=5)
    ws = codec.Workspace(model, 3, 64, 96)
    _, y, _ = codec.analyze(model, torch.from_numpy(x).cuda(), ws, want_y=True)
    yg = y.cpu().numpy()
    assert np.array_equal(yg, np.rint(yg))
    xh, u8 = codec.synthesize(model, ws, y=y, want_u8=True)
    assert np.array_equal(xh.cpu().numpy(), x.astype(np.float32))
    assert np.array_equal(u8.cpu().numpy(), x)
    y_ref = O.pack(O.analyze(x, cfg, w))
    assert np.mean(yg == y_ref) > 0.999


def test_float_lifting_reconstruction_from_y():
    need_gpu()
    from paper_2405_12631_amd import codec
    say("float lifting PR")
    cfg = get_config("ycbcr512x768")
    model, _ = model_for(cfg)
    x = sinusoid_1f_planes(64, 96, planes=3, seed=6)
    ws = codec.Workspace(model, 3, 64, 96)
    _, y, _ = codec.analyze(model, torch.from_numpy(x).cuda(), ws, want_y=True)
    xh, _ = codec.synthesize(model, ws, y=y)
    assert np.max(np.abs(xh.cpu().numpy() - x)) < 1e-3


def test_temporal_haar_matches_oracle():
    need_gpu()
    from paper_2405_12631_amd import codec
    say("temporal haar")
    rng = np.random.default_rng(9)
    f = rng.standard_normal((8, 5, 7)).astype(np.float32)
    t = torch.from_numpy(f).cuda()
    codec.temporal_haar(t)
    np.testing.assert_allclose(t.cpu().numpy(), O.temporal_haar_forward(f, 3), atol=1e-5)
    codec.temporal_haar(t, inverse=True)
    np.testing.assert_allclose(t.cpu().numpy(), f, atol=1e-5)


def test_device_entry_points_reject_bad_calls(small):
    from paper_2405_12631_amd import _lib as L
    c = small["codec"]
    ws = small["ws"]
    q = q_to_device(small["qs"])
    rc = L.lib().wv_context_params(small["model"].h, c._ptr(q), 1, 64, 64, 7, 0, c._ptr(ws.state),
                                   c._ptr(ws.scratch), c._ptr(ws.params), c._stream())
    assert rc == L.WV_EORDER
    rc = L.lib().wv_context_params(small["model"].h, c._ptr(q), 1, 62, 64, 0, 0, c._ptr(ws.state),
                                   c._ptr(ws.scratch), c._ptr(ws.params), c._stream())
    assert rc == L.WV_ESHAPE


def test_coding_order_is_enforced(small):
    """Sec. 3.2's dependent steps: a call that is not the successor of the last call on the
    same state buffer returns WV_EORDER and launches nothing; (0, 0) restarts at any time."""
    from paper_2405_12631_amd import _lib as L, batch as B
    say("coding order")
    c = small["codec"]
    model = small["model"]
    ws = c.Workspace(model, 1, 64, 64)
    q = q_to_device(small["qs"])

    def call(i, g):
        return L.lib().wv_context_params(model.h, c._ptr(q), 1, 64, 64, i, g, c._ptr(ws.state),
                                         c._ptr(ws.scratch), c._ptr(ws.params), c._stream())

    assert call(1, 2) == L.WV_EORDER                  # nothing decoded on this state yet
    assert call(0, 0) == L.WV_OK
    assert call(1, 2) == L.WV_EORDER                  # skips (0, 1) .. (1, 1)
    assert b"does not follow" in L.lib().wv_last_error()
    assert call(0, 2) == L.WV_EORDER                  # skips (0, 1)
    assert call(0, 1) == L.WV_OK                      # the failed calls left the cursor at (0, 0)
    assert call(0, 1) == L.WV_EORDER                  # a step may not run twice
    assert call(0, 0) == L.WV_OK                      # restart
    # The whole sequence in order, then only (0, 0) is accepted.
    for i in range(7):
        for g in range(4):
            if (i, g) != (0, 0):
                assert call(i, g) == L.WV_OK, (i, g)
    assert call(6, 3) == L.WV_EORDER and call(0, 1) == L.WV_EORDER
    assert call(0, 0) == L.WV_OK
    # Plans hold their own cursor.
    cfg = get_config("ycbcr512x768")
    bm, _ = model_for(cfg)
    bt = B.Batch(bm, [(32, 48), (64, 96)])
    with pytest.raises(L.WvError) as e:
        bt.context_params(0, 1)
    assert e.value.code == L.WV_EORDER
    bt.context_params(0, 0)
    with pytest.raises(L.WvError) as e:
        bt.context_params(1, 0)
    assert e.value.code == L.WV_EORDER
    bt.context_params(0, 1)
    torch.cuda.synchronize()


def test_laplace_model_params_cdf_and_roundtrip():
    """The paper's Laplacian probability model (K = 1) end to end."""
    need_gpu()
    from paper_2405_12631_amd import codec
    say("laplace K=1")
    cfg = get_config("gray64", mix_k=1, dist="laplace")
    model, w = model_for(cfg)
    x = gradient_noise_image(64, 64, seed=1)[None]
    qs, _ = O.quantize(O.analyze(x, cfg, w), cfg)
    ws = codec.Workspace(model, 1, 64, 64)
    got = codec.params_all(model, q_to_device(qs), ws)
    ref = O.context_params_all(qs, cfg, w)
    for i in range(len(ref)):
        for g in range(4):
            assert param_err(got[i][g].cpu().numpy(), ref[i][g], 1) <= PARAM_RTOL, (i, g)
            if i in (0, 6):
                cdf = codec.cdf_tables(model, got[i][g])
                check_cdf_rows(cdf.cpu().numpy().view(np.uint16), got[i][g].cpu().numpy(), cfg)
    data, q_enc = codec.encode(model, x)
    _, _, q_dec = codec.decode(model, data)
    assert torch.equal(q_enc, q_dec)


def test_subband_impulse_responses_match_oracle():
    """Sec. 3.4 impulse responses of the 13 subbands on a 16 x 16 grid."""
    need_gpu()
    from paper_2405_12631_amd import codec
    say("impulse responses")
    cfg = get_config("ycbcr512x768")
    model, w = model_for(cfg)
    x = sinusoid_1f_planes(64, 96, planes=1, seed=8)
    qs, _ = O.quantize(O.analyze(x, cfg, w), cfg)
    got = codec.impulse_responses(model, q_to_device(qs)[0], 64, 96).cpu().numpy()
    ref = O.subband_impulse_responses(qs, cfg, w, size=16)
    assert got.shape == (13, 16, 16)
    assert np.max(np.abs(got - ref)) <= XHAT_ATOL
    # A tie: two equal maxima in LL -> the first pooled cell in raster order wins.
    qt = [q.copy() for q in qs]
    qt[0][:] = 0
    qt[0][0, 3, 5] = 9
    qt[0][0, 1, 2] = -9
    got = codec.impulse_responses(model, q_to_device(qt)[0], 64, 96).cpu().numpy()
    ref = O.subband_impulse_responses(qt, cfg, w, size=16)
    assert np.max(np.abs(got - ref)) <= XHAT_ATOL


@pytest.mark.parametrize("name,H,W,N", [("gray64", 64, 64, 1), ("ycbcr512x768", 64, 96, 3)])
def test_block_architecture_params_match_oracle(name, H, W, N):
    """DepthConvBlock (step 0) and Residual Block (steps 1-3) stacks, Sec. 3.2."""
    need_gpu()
    from paper_2405_12631_amd import codec
    say("blocks", name)
    cfg = get_config(name, ctx_arch="blocks")
    model, w = model_for(cfg)
    x = gradient_noise_image(H, W, seed=1)[None] if N == 1 else sinusoid_1f_planes(H, W, planes=N, seed=2)
    qs, _ = O.quantize(O.analyze(x, cfg, w), cfg)
    ws = codec.Workspace(model, N, H, W)
    got = codec.params_all(model, q_to_device(qs), ws)
    ref = O.context_params_all(qs, cfg, w)
    worst = max(param_err(got[i][g].cpu().numpy(), ref[i][g], 3) for i in range(len(ref)) for g in range(4))
    say("blocks worst param rel err", worst)
    assert worst <= PARAM_RTOL
    data, q_enc = codec.encode(model, x)
    _, _, q_dec = codec.decode(model, data)
    assert torch.equal(q_enc, q_dec)


@pytest.mark.parametrize("name,H,W,N", [("gray64", 64, 64, 1), ("ycbcr512x768", 64, 96, 3)])
def test_autoregressive_ll_model(name, H, W, N):
    """The paper's default LL coding (Sec. 3.2): raster order, decoded on the GPU."""
    need_gpu()
    from paper_2405_12631_amd import codec, _lib as L
    say("ar ll", name)
    cfg = get_config(name, ll_ar=1)
    model, w = model_for(cfg)
    x = gradient_noise_image(H, W, seed=1)[None] if N == 1 else sinusoid_1f_planes(H, W, planes=N, seed=2)
    qs, _ = O.quantize(O.analyze(x, cfg, w), cfg)
    ws = codec.Workspace(model, N, H, W)
    got = codec.ar_params(model, q_to_device(qs), ws).cpu().numpy()
    ref = O.ar_params(qs[0], cfg, w)
    assert param_err(got, ref, 3) <= PARAM_RTOL
    check_cdf_rows(codec.cdf_tables(model, torch.from_numpy(got).cuda()).cpu().numpy().view(np.uint16),
                   got, cfg)
    data, q_enc = codec.encode(model, x)
    xh, _, q_dec = codec.decode(model, data)
    assert torch.equal(q_enc, q_dec)
    # A corrupted LL stream is reported through the kernel's status word.
    N_, H_, W_, streams = codec.unpack_stream(model, data)
    bad = [s.copy() if isinstance(s, list) else s for s in streams]
    ll = bytearray(bad[0][0][0])
    ll[len(ll) // 2] ^= 0xA5
    q = torch.zeros_like(q_enc)
    with pytest.raises(L.WvError):
        codec.ar_decode(model, q, codec.Workspace(model, N, H, W), [bytes(ll)] + [s[0][0] for s in bad[1:]])


@pytest.fixture(scope="module")
def full512():
    """512 x 768 x 3 through the FP32 encoder, and the oracle's parameters of plane 0 (all 13
    subbands x 4 steps) on the GPU encoder's own symbols."""
    need_gpu()
    from paper_2405_12631_amd import codec
    cfg = get_config("ycbcr512x768")
    model, w = model_for(cfg)
    x = sinusoid_1f_planes(512, 768, planes=3, seed=cfg["seed_image"])
    ws = codec.Workspace(model, 3, 512, 768)
    q, _, _ = codec.analyze(model, torch.from_numpy(x).cuda(), ws)
    qs = O.unpack(q.cpu().numpy().astype(np.int64)[:1], cfg, 512, 768)
    ref = O.context_params_all(qs, cfg, w)
    return dict(cfg=cfg, model=model, w=w, ws=ws, q=q, qs=qs, ref=ref, codec=codec)


def test_full_size_analysis_matches_oracle(full512):
    """512 x 768 x 3 analysis in the bench's three-plane launch: plane 0's subbands y and
    symbols q against the oracle's analysis of the same plane."""
    say("full size analysis 512x768")
    F = full512
    cfg, model, w, ws, codec = (F[k] for k in ("cfg", "model", "w", "ws", "codec"))
    x = sinusoid_1f_planes(512, 768, planes=3, seed=cfg["seed_image"])
    q, y, _ = codec.analyze(model, torch.from_numpy(x).cuda(), codec.Workspace(model, 3, 512, 768), want_y=True)
    assert torch.equal(q, F["q"])
    y_ref = O.pack(O.analyze(x[:1], cfg, w))[0]
    y_gpu = y[0].cpu().numpy()
    err = float(np.max(np.abs(y_gpu - y_ref)))
    say("full-size y err", err)
    assert err < 5e-3
    check_q_near_ties(q[0].cpu().numpy(), y_gpu, y_ref, cfg)


def test_full_size_plane_parity_in_bench_configuration(full512):
    """512 x 768, the benchmark's model and launch configuration (three planes per call):
    every parameter of plane 0 (all 13 subbands x 4 steps) and its reconstruction against
    the oracle; the oracle runs on the GPU encoder's own symbols."""
    say("full size 512x768")
    F = full512
    cfg, model, w, ws, q, qs, ref, codec = (F[k] for k in ("cfg", "model", "w", "ws", "q", "qs", "ref", "codec"))
    got = codec.params_all(model, q, ws)
    worst = max(param_err(got[i][g][:1].cpu().numpy(), ref[i][g], 3) for i in range(13) for g in range(4))
    say("full-size worst param rel err", worst)
    assert worst <= PARAM_RTOL
    cdf = codec.cdf_tables(model, got[12][3][:1].contiguous())
    check_cdf_rows(cdf.cpu().numpy().view(np.uint16), got[12][3][:1].cpu().numpy(), cfg)
    xh, _ = codec.synthesize(model, ws, q=q)
    ref_x = O.synthesize(O.dequantize(qs, cfg), cfg, w)
    assert np.max(np.abs(xh[:1].cpu().numpy() - ref_x)) <= XHAT_ATOL


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_full_size_reduced_precision_against_oracle(full512, prec):
    """The BF16 and FP8 context models at 512 x 768 x 3, where the level-1 subbands take the
    widest channel blocking and the ConvLSTM's column blocks run in XCD order: plane 0's
    parameters against the same oracle, within the reduced-precision bounds, and the CDF
    rows of the last subband valid."""
    from paper_2405_12631_amd import WV_BF16, WV_FP8
    from wvgen import make_weights, pack_weights
    F = full512
    cfg, q, ref, codec = F["cfg"], F["q"], F["ref"], F["codec"]
    say("full size 512x768", prec)
    model = codec.Model(cfg, pack_weights(cfg, make_weights(cfg)), precision={"bf16": WV_BF16, "fp8": WV_FP8}[prec])
    ws = codec.Workspace(model, 3, 512, 768)
    got = codec.params_all(model, q, ws)
    rels, wmax = [], 0.0
    for i in range(13):
        for g in range(4):
            r, wm = reduced_errs(got[i][g][:1].cpu().numpy(), ref[i][g], cfg["mix_k"])
            rels.append(r.ravel())
            wmax = max(wmax, wm)
    rel = np.concatenate(rels)
    say(f"{prec} 512x768: mean rel {rel.mean():.3e} max {rel.max():.3e} max |dw| {wmax:.3e}")
    assert rel.mean() < REDUCED_BARS[prec][0] and wmax < REDUCED_BARS[prec][1]
    cdf = codec.cdf_tables(model, got[12][3][:1].contiguous())
    check_cdf_rows(cdf.cpu().numpy().view(np.uint16), got[12][3][:1].cpu().numpy(), cfg)


def test_lifting_tile_forms_bitwise():
    """Analysis and synthesis of six 512 x 768 planes in one call take the 16 x 32-output lifting
    tile (at least 2048 such tiles per filter launch); three planes take the 8 x 16 one, whose
    results the full-size oracle test covers.  Both tile forms keep each output's arithmetic, so
    the symbols and the reconstruction of the shared planes are bitwise equal."""
    need_gpu()
    from paper_2405_12631_amd import codec
    say("lifting tile forms")
    cfg = get_config("ycbcr512x768")
    model, _ = model_for(cfg)
    x = np.concatenate([sinusoid_1f_planes(512, 768, planes=3, seed=s) for s in (7, 8)])
    ws6 = codec.Workspace(model, 6, 512, 768)
    ws3 = codec.Workspace(model, 3, 512, 768)
    q6, y6, _ = codec.analyze(model, torch.from_numpy(x).cuda(), ws6, want_y=True)
    q3, y3, _ = codec.analyze(model, torch.from_numpy(x[:3]).cuda(), ws3, want_y=True)
    assert torch.equal(q6[:3], q3) and torch.equal(y6[:3], y3)
    x6, _ = codec.synthesize(model, ws6, q=q6)
    x3, _ = codec.synthesize(model, ws3, q=q3)
    assert torch.equal(x6[:3], x3)


def test_lifting_tile_forms_bitwise_ragged():
    """Ragged 16 x 32 tiles: twelve 528 x 784 planes (level-1 arrays of 264 x 392, neither a
    multiple of the tile) take the big tile, three planes the 8 x 16 one; same bits."""
    need_gpu()
    from paper_2405_12631_amd import codec
    say("lifting tile forms, ragged")
    cfg = get_config("ycbcr512x768")
    model, _ = model_for(cfg)
    x = np.concatenate([sinusoid_1f_planes(528, 784, planes=3, seed=s) for s in (11, 12, 13, 14)])
    ws12 = codec.Workspace(model, 12, 528, 784)
    ws3 = codec.Workspace(model, 3, 528, 784)
    q12, y12, _ = codec.analyze(model, torch.from_numpy(x).cuda(), ws12, want_y=True)
    q3, y3, _ = codec.analyze(model, torch.from_numpy(x[:3]).cuda(), ws3, want_y=True)
    assert torch.equal(q12[:3], q3) and torch.equal(y12[:3], y3)
    x12, _ = codec.synthesize(model, ws12, q=q12)
    x3, _ = codec.synthesize(model, ws3, q=q3)
    assert torch.equal(x12[:3], x3)


@pytest.mark.parametrize("H,W,planes", [(512, 768, 3), (528, 784, 2), (1088, 1920, 1), (48, 80, 3)])
def test_lifting_row_form_bitwise(H, W, planes):
    """The row-streaming lifting kernel (taken for large arrays) forced on every filter
    launch of analysis and synthesis, against the tiled kernel forced likewise: the same
    coefficients, symbols and reconstruction, bit for bit.  Covers ragged 126-column strips
    (392, 784 and 960 columns), ragged row segments, and arrays smaller than one strip (the
    coarse levels, and 48 x 80)."""
    import os
    need_gpu()
    from paper_2405_12631_amd import codec
    say("lifting row form", H, W, planes)
    cfg = get_config("ycbcr512x768")
    model, _ = model_for(cfg)
    x = torch.from_numpy(sinusoid_1f_planes(H, W, planes=planes, seed=21)).cuda()
    ws = codec.Workspace(model, planes, H, W)
    res = {}
    for form in ("tile", "rows"):
        os.environ["WV_LIFT_FORM"] = form
        try:
            q, y, _ = codec.analyze(model, x, ws, want_y=True)
            xh, _ = codec.synthesize(model, ws, q=q)
            torch.cuda.synchronize()
            res[form] = (q.clone(), y.clone(), xh.clone())
        finally:
            del os.environ["WV_LIFT_FORM"]
    for name, a, b in zip(("q", "y", "xhat"), res["tile"], res["rows"]):
        assert torch.equal(a, b), name
