"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds workload parameters and random-number generation only: image
and video generators, the random-init weight blob and its manifest, and
request arrival times.  It contains none of the coding method's arithmetic
(no lifting, no context model, no CDF), so that the FP64 oracle and the GPU
library can both consume it without sharing any code that computes a result.

Nothing from the paper's datasets (Kodak, UVG, Vimeo90K) is reproduced: the
1/f sinusoid textures stand in for natural images of the same shapes.
"""
from .configs import CONFIGS, get_config, subband_count
from .images import gradient_noise_image, sinusoid_1f_planes, video_gop_420, batch_sizes
from .weights import manifest, make_weights, pack_weights, weights_nbytes
from .arrivals import poisson_arrivals

__all__ = [
    "CONFIGS", "get_config", "subband_count",
    "gradient_noise_image", "sinusoid_1f_planes", "video_gop_420", "batch_sizes",
    "manifest", "make_weights", "pack_weights", "weights_nbytes",
    "poisson_arrivals",
]
