"""The C-ABI library on the CPU: exported symbols, host-only entry points and
the host rANS coder (no GPU work is launched here)."""
import ctypes
import os
import re
import types

import numpy as np
import pytest

import oracle as O
from wvgen import CONFIGS, get_config, weights_nbytes

L = pytest.importorskip("paper_2405_12631_amd._lib")
from paper_2405_12631_amd import codec  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libwv.so not built")
    return L.lib()


def test_every_declared_symbol_is_exported_and_bound():
    lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "wv.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    declared = set(re.findall(r"\b(wv_[a-z0-9_]+)\s*\(", hdr))
    assert len(declared) >= 18
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(L.symbols())


@pytest.mark.parametrize("name,arch", [(n, a) for n in sorted(CONFIGS) for a in ("plain", "blocks")])
def test_weight_count_matches_manifest(name, arch):
    _lib()
    cfg = get_config(name, ctx_arch=arch)
    n = ctypes.c_longlong()
    L.call("wv_weights_count", ctypes.byref(codec.make_config(cfg)), ctypes.byref(n))
    assert n.value * 4 == weights_nbytes(cfg)


@pytest.mark.parametrize("H,W,J", [(64, 64, 2), (512, 768, 4), (48, 80, 4), (1088, 1920, 4), (16, 16, 4)])
def test_layout_matches_oracle(H, W, J):
    _lib()
    cfg = get_config("ycbcr512x768", levels=J)
    c = codec.make_config(cfg)
    n = 3 * J + 1
    arr = (L.wv_subband * n)()
    coefs = ctypes.c_longlong()
    L.call("wv_layout", ctypes.byref(c), H, W, arr, n, ctypes.byref(coefs))
    ref, total = O.subband_layout(cfg, H, W)
    assert coefs.value == total
    for a, r in zip(arr, ref):
        assert (a.h, a.w, a.level, a.type, a.offset) == (r["h"], r["w"], r["level"], r["type"], r["offset"])
        for g in range(4):
            rr, _ = O.group_positions(r["h"], r["w"], g)
            assert L.lib().wv_group_count(r["h"], r["w"], g) == len(rr)


def test_shape_and_argument_errors():
    _lib()
    c = codec.make_config(get_config("ycbcr512x768"))
    arr = (L.wv_subband * 13)()
    coefs = ctypes.c_longlong()
    assert L.lib().wv_layout(ctypes.byref(c), 520, 768, arr, 13, ctypes.byref(coefs)) == L.WV_ESHAPE
    assert L.lib().wv_layout(ctypes.byref(c), 0, 768, arr, 13, ctypes.byref(coefs)) == L.WV_ESHAPE
    assert L.lib().wv_layout(ctypes.byref(c), 512, 768, arr, 5, ctypes.byref(coefs)) == L.WV_ENOMEM
    bad = codec.make_config(get_config("ycbcr512x768", mix_k=7))
    assert L.lib().wv_layout(ctypes.byref(bad), 512, 768, arr, 13, ctypes.byref(coefs)) == L.WV_EUNSUPPORTED
    assert "mix_k" in L.lib().wv_last_error().decode()
    assert L.lib().wv_group_count(4, 4, 5) == -1
    nb = ctypes.c_size_t()
    assert L.lib().wv_pack_bytes(ctypes.byref(c), 9, ctypes.byref(nb)) == L.WV_EUNSUPPORTED
    # Reduced precision packs the context convs smaller than FP32 (BF16: 2 bytes, FP8: 1 byte
    # per weight plus per-channel scales) and needs the plain stacks.
    sizes = {}
    for prec in (L.WV_FP32, L.WV_BF16, L.WV_FP8):
        assert L.lib().wv_pack_bytes(ctypes.byref(c), prec, ctypes.byref(nb)) == L.WV_OK
        sizes[prec] = nb.value
    assert sizes[L.WV_FP8] < sizes[L.WV_BF16] < sizes[L.WV_FP32]
    blocks = codec.make_config(get_config("ycbcr512x768", ctx_arch="blocks"))
    assert L.lib().wv_pack_bytes(ctypes.byref(blocks), L.WV_FP8, ctypes.byref(nb)) == L.WV_EUNSUPPORTED
    # GPU entry points reject bad arguments on the host before any launch.
    assert L.lib().wv_cdf_tables(None, 5, 3, 0, -64, 64, 16, None, None) == L.WV_EINVAL
    assert L.lib().wv_cdf_tables(None, 0, 3, 0, -64, 64, 12, None, None) == L.WV_EUNSUPPORTED
    assert L.lib().wv_cdf_tables(None, 0, 3, 7, -64, 64, 16, None, None) == L.WV_EINVAL
    assert L.lib().wv_temporal_haar_forward(None, 6, 10, None) == L.WV_ESHAPE
    assert L.lib().wv_context_params(None, None, 1, 64, 64, 0, 0, None, None, None, None) == L.WV_EINVAL


def _tables(seed, n, cfg):
    rng = np.random.default_rng(seed)
    logits = rng.normal(0, 2, (n, 3))
    w = np.exp(logits) / np.exp(logits).sum(1, keepdims=True)
    mu = rng.uniform(-10, 10, (n, 3))
    sg = np.exp(rng.uniform(np.log(0.11), np.log(10), (n, 3)))
    cdf = O.cdf_tables(np.concatenate([w, mu, sg], 1), cfg)
    u = rng.integers(0, 65536, n)
    idx = np.array([np.searchsorted(cdf[k], u[k], side="right") - 1 for k in range(n)])
    return cdf, idx


def test_host_rans_roundtrip_matches_reference_coder(cfg_small):
    _lib()
    cdf, idx = _tables(31, 5000, cfg_small)
    u16 = O.cdf_to_u16(cdf)
    data = codec.rans_encode(u16, idx.astype(np.uint8), 129)
    assert data == O.rans_encode_ref(u16, idx)                 # same stream format
    back = codec.rans_decode(u16, data, len(idx), 129)
    assert np.array_equal(back, idx)
    assert 8 * len(data) <= O.ideal_bits(cdf, idx) * 1.002 + 64


def test_host_trimmed_tables_and_coder(cfg_small):
    _lib()
    cdf, idx = _tables(33, 3000, cfg_small)
    u16 = O.cdf_to_u16(cdf)
    lolen, packed = O.cdf_trim(cdf)
    tr = codec.Trimmed(lolen.astype(np.uint8), packed.astype(np.uint16), 129)
    assert np.array_equal(tr.full(), u16)                      # library untrim == oracle tables
    sym = idx.astype(np.uint8)
    full = codec.rans_encode(u16, sym, 129)
    for a, b in ((0, 3000), (0, 0), (1000, 2000), (2999, 3000)):
        data = codec.rans_encode_trim(tr, a, b, sym[a:b])
        assert data == codec.rans_encode(u16[a:b], sym[a:b], 129)
        assert np.array_equal(codec.rans_decode_trim(tr, a, b, data), sym[a:b])
    assert codec.rans_encode_trim(tr, 0, 3000, sym) == full
    # (lo, len) that do not describe a row are refused
    bad = lolen.astype(np.uint8).copy()
    bad[17, 0] = 0
    with pytest.raises(L.WvError) as e:
        codec.Trimmed(bad, packed.astype(np.uint16), 129).full()
    assert e.value.code == L.WV_ECORRUPT
    with pytest.raises(L.WvError):
        codec.rans_decode_trim(codec.Trimmed(bad, packed.astype(np.uint16), 129), 0, 3000, full)


def test_host_rans_edge_cases(cfg_small):
    _lib()
    cdf, idx = _tables(32, 300, cfg_small)
    u16 = O.cdf_to_u16(cdf)
    assert codec.rans_decode(u16[:0], codec.rans_encode(u16[:0], np.zeros(0, np.uint8), 129), 0, 129).size == 0
    ext = np.array([0, 128] * 150, np.uint8)
    assert np.array_equal(codec.rans_decode(u16, codec.rans_encode(u16, ext, 129), 300, 129), ext)
    data = codec.rans_encode(u16, idx.astype(np.uint8), 129)
    for bad in (data[:3], data[:-1], data + b"\x00", bytes([data[0] ^ 0x5A]) + data[1:]):
        with pytest.raises(L.WvError) as e:
            codec.rans_decode(u16, bad, 300, 129)
        assert e.value.code == L.WV_ECORRUPT
    buf = np.empty(8, np.uint8)
    ln = ctypes.c_size_t()
    sym = idx.astype(np.uint8)
    assert L.lib().wv_rans_encode(u16.ctypes.data, 129, sym.ctypes.data, 300, buf.ctypes.data, 8,
                                  ctypes.byref(ln)) == L.WV_ENOMEM
    sym[5] = 200
    big = np.empty(4096, np.uint8)
    assert L.lib().wv_rans_encode(u16.ctypes.data, 129, sym.ctypes.data, 300, big.ctypes.data, 4096,
                                  ctypes.byref(ln)) == L.WV_EINVAL


def test_bitstream_container_roundtrip_and_rejects_corruption():
    _lib()
    fake = types.SimpleNamespace(cfg=dict(levels=2, step=8.0), precision=0, blob_sha=bytes(range(32)),
                                 deltas=lambda: (0.125, 0.125))
    streams = [[[bytes([n, i, g]) * (g + 1) for g in range(4)] for i in range(7)] for n in range(2)]
    data = codec.pack_stream(fake, 2, 64, 64, streams)
    N, H, W, back = codec.unpack_stream(fake, data)
    assert (N, H, W) == (2, 64, 64) and back == streams
    for bad in (data[:10], data[:-1], b"XXXX" + data[4:], data + b"!"):
        with pytest.raises(L.WvError) as e:
            codec.unpack_stream(fake, bad)
        assert e.value.code == L.WV_ECORRUPT
    other = types.SimpleNamespace(cfg=dict(levels=2), precision=0, blob_sha=bytes(32))
    with pytest.raises(L.WvError):
        codec.unpack_stream(other, data)
