"""Pins of the oracle's CDF tables and reference rANS coder (CPU only)."""
import mpmath
import numpy as np
import pytest
import scipy.special

import oracle as O

mpmath.mp.dps = 50


def _random_params(rng, n, K=3, extreme=True):
    logits = rng.normal(0, 3, (n, K))
    w = np.exp(logits - logits.max(1, keepdims=True))
    w /= w.sum(1, keepdims=True)
    mu = rng.uniform(-20, 20, (n, K))
    sg = np.exp(rng.uniform(np.log(0.11), np.log(8.0), (n, K)))
    if extreme:
        mu[: n // 4] = rng.uniform(-90, 90, (n // 4, K))
        sg[n // 4: n // 2] = rng.choice([0.11, 0.2, 40.0, 300.0], (n // 2 - n // 4, K))
    return np.concatenate([w, mu, sg], 1)


def _exact_row(p, cfg):
    """High-precision floor(F_max * C_j) straight from the definition."""
    K = cfg["mix_k"]
    Ns = cfg["sym_max"] - cfg["sym_min"] + 1
    T = 1 << cfg["cdf_bits"]
    Fmax = T - Ns
    row = [0]
    wsum = mpmath.fsum(mpmath.mpf(float(p[k])) for k in range(K))
    for j in range(1, Ns):
        b = mpmath.mpf(cfg["sym_min"] + j) - mpmath.mpf("0.5")
        ws = [mpmath.mpf(float(p[k])) for k in range(K)]
        zs = [(b - mpmath.mpf(float(p[K + k]))) / mpmath.mpf(float(p[2 * K + k])) for k in range(K)]
        c = mpmath.fsum(ws[k] * mpmath.ncdf(zs[k]) for k in range(K)) / wsum
        if c <= mpmath.mpf("0.5"):
            row.append(j + int(mpmath.floor(Fmax * c)))
        else:
            # floor(F (1 - t)) = F - ceil(F t); t = 1 - c from the upper tails, which
            # keeps its digits where c itself rounds to 1 even at 50 digits.
            t = mpmath.fsum(ws[k] * mpmath.ncdf(-zs[k]) for k in range(K)) / wsum
            row.append(j + Fmax - int(mpmath.ceil(Fmax * t)))
    row.append(T)
    return np.array(row, np.int64)


def test_cdf_mixture_matches_high_precision(cfg_small):
    rng = np.random.default_rng(21)
    p = _random_params(rng, 24)
    got = O.cdf_tables(p, cfg_small)
    for n in range(p.shape[0]):
        np.testing.assert_array_equal(got[n], _exact_row(p[n], cfg_small), err_msg=str(p[n]))


def test_cdf_single_gaussian_matches_ndtr(cfg_small):
    cfg = dict(cfg_small, mix_k=1)
    rng = np.random.default_rng(22)
    mu = rng.uniform(-30, 30, 40)
    sg = np.exp(rng.uniform(np.log(0.2), np.log(20), 40))
    p = np.stack([np.ones(40), mu, sg], 1)
    got = O.cdf_tables(p, cfg)
    b = np.arange(1, 129) - 64.5
    c = scipy.special.ndtr((b[None] - mu[:, None]) / sg[:, None])
    # Away from the upper tail (where 1 - c loses digits in float64) the floor agrees.
    ok = c < 0.5
    want = np.arange(1, 129)[None] + np.floor(65407 * c)
    assert np.array_equal(got[:, 1:129][ok], want[ok])
    for n in range(4):
        np.testing.assert_array_equal(got[n], _exact_row(p[n], cfg))


def test_cdf_invariants_on_extreme_params(cfg_small):
    rng = np.random.default_rng(23)
    p = _random_params(rng, 4000)
    cdf = O.cdf_tables(p, cfg_small)
    assert cdf.shape == (4000, 130)
    assert np.all(cdf[:, 0] == 0) and np.all(cdf[:, 129] == 65536)
    freq = np.diff(cdf, axis=1)
    assert np.all(freq >= 1)
    assert np.all(freq.sum(1) == 65536)
    u16 = O.cdf_to_u16(cdf)
    assert u16.dtype == np.uint16 and np.all(u16[:, 129] == 0)


def test_cdf_concentrates_mass_near_mean(cfg_small):
    # One narrow component at mu = 3: symbol 3 gets almost all of the mass.
    p = np.array([[1.0, 0.0, 0.0, 3.0, 0.0, 0.0, 0.11, 1.0, 1.0]])
    cdf = O.cdf_tables(p, cfg_small)[0]
    freq = np.diff(cdf)
    assert np.argmax(freq) == 3 + 64
    assert freq[3 + 64] > 65536 - 200


def _sample(rng, cdf):
    u = rng.integers(0, 65536, cdf.shape[0])
    return np.array([np.searchsorted(cdf[n], u[n], side="right") - 1 for n in range(cdf.shape[0])])


def test_rans_reference_roundtrip_and_length(cfg_small):
    rng = np.random.default_rng(24)
    p = _random_params(rng, 3000, extreme=False)
    cdf = O.cdf_tables(p, cfg_small)
    idx = _sample(rng, cdf)
    data = O.rans_encode_ref(O.cdf_to_u16(cdf), idx)
    back = O.rans_decode_ref(O.cdf_to_u16(cdf), data, len(idx))
    assert np.array_equal(back, idx)
    ideal = O.ideal_bits(cdf, idx)
    assert 8 * len(data) <= ideal * 1.002 + 64
    assert 8 * len(data) >= ideal - 1


def test_rans_reference_edge_cases(cfg_small):
    rng = np.random.default_rng(25)
    p = _random_params(rng, 50)
    cdf = O.cdf_to_u16(O.cdf_tables(p, cfg_small))
    # Empty stream, extreme symbols, truncation.
    assert list(O.rans_decode_ref(cdf[:0], O.rans_encode_ref(cdf[:0], []), 0)) == []
    idx = np.array([0, 128] * 25)
    data = O.rans_encode_ref(cdf, idx)
    assert np.array_equal(O.rans_decode_ref(cdf, data, 50), idx)
    with pytest.raises(ValueError):
        O.rans_decode_ref(cdf, data[:3], 50)


def _exact_laplace_row(p, cfg):
    """High-precision floor(F_max * C_j) for a Laplace mixture, from its definition."""
    K = cfg["mix_k"]
    Ns = cfg["sym_max"] - cfg["sym_min"] + 1
    Fmax = (1 << cfg["cdf_bits"]) - Ns

    def lap(z):
        return mpmath.exp(z) / 2 if z < 0 else 1 - mpmath.exp(-z) / 2

    ws = [mpmath.mpf(float(p[k])) for k in range(K)]
    wsum = mpmath.fsum(ws)
    row = [0]
    for j in range(1, Ns):
        b = mpmath.mpf(cfg["sym_min"] + j) - mpmath.mpf("0.5")
        zs = [(b - mpmath.mpf(float(p[K + k]))) / mpmath.mpf(float(p[2 * K + k])) for k in range(K)]
        c = mpmath.fsum(ws[k] * lap(zs[k]) for k in range(K)) / wsum
        if c <= mpmath.mpf("0.5"):
            row.append(j + int(mpmath.floor(Fmax * c)))
        else:
            t = mpmath.fsum(ws[k] * lap(-zs[k]) for k in range(K)) / wsum
            row.append(j + Fmax - int(mpmath.ceil(Fmax * t)))
    row.append(1 << cfg["cdf_bits"])
    return np.array(row, np.int64)


def test_cdf_laplace_matches_high_precision_and_scipy(cfg_small):
    import scipy.stats
    cfg1 = dict(cfg_small, mix_k=1, dist="laplace")
    rng = np.random.default_rng(26)
    mu = rng.uniform(-40, 40, 30)
    b = np.exp(rng.uniform(np.log(0.11), np.log(30), 30))
    p = np.stack([np.ones(30), mu, b], 1)
    got = O.cdf_tables(p, cfg1)
    for n in range(p.shape[0]):
        np.testing.assert_array_equal(got[n], _exact_laplace_row(p[n], cfg1))
    edges = np.arange(1, 129) - 64.5
    c = scipy.stats.laplace.cdf(edges[None], loc=mu[:, None], scale=b[:, None])
    ok = c < 0.5
    want = np.arange(1, 129)[None] + np.floor(65407 * c)
    assert np.array_equal(got[:, 1:129][ok], want[ok])
    # Laplace mixtures, and the invariants on extreme parameters.
    cfg3 = dict(cfg_small, dist="laplace")
    p3 = _random_params(rng, 2000)
    cdf = O.cdf_tables(p3, cfg3)
    for n in range(6):
        np.testing.assert_array_equal(cdf[n], _exact_laplace_row(p3[n], cfg3))
    freq = np.diff(cdf, axis=1)
    assert np.all(freq >= 1) and np.all(cdf[:, -1] == 65536) and np.all(cdf[:, 0] == 0)
    # The two families differ (a dropped family switch would pass the checks above).
    assert not np.array_equal(cdf, O.cdf_tables(p3, cfg_small))


def test_cdf_trim_closed_form_single_gaussian(cfg_small):
    # One N(mu, 1) component: F_j > 0 exactly where F_max Phi(b_j - mu) >= 1, and
    # F_j < F_max - 1 exactly where F_max (1 - Phi(b_j - mu)) > 1, b_j = j - 64.5.
    import scipy.stats
    Fmax = 65536 - 129
    zq = scipy.stats.norm.ppf(1.0 / Fmax)                     # about -4.17
    for mu in (0.0, 10.25, -30.6):
        cdf = O.cdf_tables(np.array([[1.0, mu, 1.0]]), dict(cfg_small, mix_k=1))
        lolen, packed = O.cdf_trim(cdf)
        lo = int(np.ceil(64.5 + mu + zq))
        hi = int(np.ceil(64.5 + mu - zq)) - 1                  # last j with b_j - mu < -zq
        assert tuple(lolen[0]) == (lo, hi - lo + 1)
        assert np.array_equal(packed, cdf[0, lo:hi + 1] - np.arange(lo, hi + 1))


def test_cdf_trim_roundtrip_and_size(cfg_small):
    rng = np.random.default_rng(7)
    n = 400
    logits = rng.normal(0, 2, (n, 3))
    w = np.exp(logits) / np.exp(logits).sum(1, keepdims=True)
    mu = rng.uniform(-80, 80, (n, 3))                          # includes means beyond the alphabet
    sg = np.exp(rng.uniform(np.log(0.11), np.log(40), (n, 3)))
    cdf = O.cdf_tables(np.concatenate([w, mu, sg], 1), cfg_small)
    lolen, packed = O.cdf_trim(cdf)
    assert np.array_equal(O.cdf_untrim(lolen, packed, 129), cdf)
    assert lolen[:, 0].min() >= 1 and (lolen.sum(1) <= 129).all()
    assert packed.size == lolen[:, 1].sum() < cdf[:, 1:129].size
