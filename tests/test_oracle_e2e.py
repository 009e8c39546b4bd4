"""Whole-image pins of the oracle: encode -> decode round trip on the 64x64 workload."""
import numpy as np

import oracle as O
from wvgen import gradient_noise_image


def test_oracle_encode_decode_roundtrip(cfg_small, weights_small):
    cfg, w = cfg_small, weights_small
    x = gradient_noise_image(64, 64, seed=1)[None]
    streams, qs, clips = O.encode(x, cfg, w)
    xr, qd = O.decode(streams, cfg, w, 64, 64, 1)
    for a, b in zip(qs, qd):
        assert np.array_equal(a, b)
    np.testing.assert_allclose(xr, O.synthesize(O.dequantize(qs, cfg), cfg, w), atol=0)
    nbytes = sum(len(s) for row in streams[0] for s in row)
    prm, tabs, _ = O.decode_path(qs, cfg, w)
    ideal = 0.0
    for i, q in enumerate(qs):
        for g in range(4):
            rr, cc = O.group_positions(q.shape[1], q.shape[2], g)
            ideal += O.ideal_bits(tabs[i][g], q[0][rr, cc] - cfg["sym_min"])
    assert 8 * nbytes <= ideal + 28 * 64 + 0.01 * ideal
    # Lossy but close: step 8 on a gradient image.
    assert np.sqrt(np.mean((xr - x) ** 2)) < 8.0


def test_decode_path_matches_encode_side_params(cfg_small, weights_small):
    # Encoder and decoder evaluate the same functions on the same symbols.
    x = gradient_noise_image(64, 64, seed=1)[None]
    qs, _ = O.quantize(O.analyze(x, cfg_small, weights_small), cfg_small)
    p1, t1, _ = O.decode_path(qs, cfg_small, weights_small)
    p2 = O.context_params_all([q.copy() for q in qs], cfg_small, weights_small)
    for a, b in zip(p1, p2):
        for u, v in zip(a, b):
            assert np.array_equal(u, v)
