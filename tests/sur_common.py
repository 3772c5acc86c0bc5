"""Seeded surrogate parameters and data shared by the surrogate tests (CPU and
GPU).  Parameters are uniform draws scaled by 1/sqrt(fan-in) per tensor, so
both sides start from the same numbers."""

import numpy as np

from oracle import surrogate as osur
from synth import uniform_array


def init_params(cfg, seed):
    out = []
    for k, (name, shape) in enumerate(osur.layout(cfg)):
        n = int(np.prod(shape))
        if name.startswith("W"):
            fan_in = int(np.prod(shape[:-1]))
            bound = np.sqrt(3.0 / fan_in)
        else:
            bound = 0.05
        out.append(uniform_array(n, seed * 1000 + k, bound))
    return np.concatenate(out)


def random_maps(B, n_cells, seed, p=0.5):
    from synth import bernoulli_map
    return np.stack([bernoulli_map(n_cells, p, seed * 7919 + i) for i in range(B)])
