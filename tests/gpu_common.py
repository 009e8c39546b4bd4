"""Shared helpers of the GPU tests: model construction, oracle comparisons and tolerances."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from wvgen import make_weights, pack_weights

# Parameter parity bar (FP32 path vs FP64 oracle): max |a - b| / max(|b|, tau) <= 1e-4,
# tau = 1e-2 for the mixture weights and means, sigma >= sigma_min needs none.
PARAM_RTOL = 1e-4
TAU = 1e-2
# Reconstruction parity on the 0..255 scale after the inverse transform.
XHAT_ATOL = 1e-3
# Reduced-precision context convs: (mean relative parameter error, max |mixture weight error|).
# No parity bar is set for them; these bounds only catch a broken kernel (an FP32-accumulated
# BF16 conv stack stays far inside them; e4m3 has 3 mantissa bits, so its per-value rounding
# alone reaches 6 %).
REDUCED_BARS = {"bf16": (2e-2, 0.1), "fp8": (0.25, 0.5)}


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def model_for(cfg):
    from paper_2405_12631_amd import codec
    w = make_weights(cfg)
    return codec.Model(cfg, pack_weights(cfg, w)), w


def q_to_device(qs):
    return torch.from_numpy(O.pack(qs).astype(np.int16)).cuda()


def param_err(gpu, ref, K):
    """Elementwise relative error of [.., 3K] parameter arrays (see PARAM_RTOL)."""
    g = np.asarray(gpu, np.float64).reshape(-1, 3 * K)
    r = np.asarray(ref, np.float64).reshape(-1, 3 * K)
    if g.size == 0:
        return 0.0
    den = np.abs(r)
    den[:, :2 * K] = np.maximum(den[:, :2 * K], TAU)
    return float(np.max(np.abs(g - r) / den))


def check_cdf_rows(gpu_u16, prm_gpu, cfg, max_frac=0.01):
    """GPU tables vs the oracle's tables built from the GPU's own parameters."""
    ref = O.cdf_tables(np.asarray(prm_gpu, np.float64).reshape(-1, 3 * cfg["mix_k"]), cfg)
    got = np.asarray(gpu_u16, np.int64).reshape(ref.shape)
    got[:, -1] = np.where(got[:, -1] == 0, 65536, got[:, -1])
    d = np.abs(got - ref)
    assert d.max(initial=0) <= 1, d.max()
    assert np.mean(d != 0) <= max_frac, np.mean(d != 0)
    freq = np.diff(got, axis=1)
    assert np.all(got[:, 0] == 0) and np.all(freq >= 1) and np.all(got[:, -1] == 65536)
    return float(np.mean(d != 0))


def reduced_errs(gpu, ref, K):
    """Relative errors of [.., 3K] parameter arrays (denominators as in param_err) and the
    largest absolute error of a mixture weight."""
    g = np.asarray(gpu, np.float64).reshape(-1, 3 * K)
    r = np.asarray(ref, np.float64).reshape(-1, 3 * K)
    den = np.abs(r)
    den[:, :2 * K] = np.maximum(den[:, :2 * K], TAU)
    rel = np.abs(g - r) / den
    return rel, np.abs(g[:, :K] - r[:, :K]).max(initial=0)
