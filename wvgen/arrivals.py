"""Seeded Poisson request arrivals for the serving workload."""
import numpy as np


def poisson_arrivals(rate_hz, duration_s, frac_video, sizes, seed=4):
    """Arrival times (s) and request kinds for a Poisson process.

    Returns a list of dicts {t, kind, size} where kind is "image" (size drawn
    uniformly from `sizes`) or "gop"; exponential inter-arrival times with mean
    1/rate_hz, truncated at duration_s.
    """
    rng = np.random.default_rng(seed)
    out, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        if rng.uniform() < frac_video:
            out.append(dict(t=t, kind="gop", size=None))
        else:
            out.append(dict(t=t, kind="image", size=tuple(sizes[rng.integers(0, len(sizes))])))
    return out
