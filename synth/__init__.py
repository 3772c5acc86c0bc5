"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package holds only workload descriptions (geometry numbers, frequency
grids, seeds) and the seeded draws of pixel maps, via sites and candidate flip
lists.  It contains none of the method's arithmetic: no meshing, no basis
function classification, no Green's function, no solve, no S-parameters, no
figure of merit.  Both sides import it; neither side's code lives here.
"""

from .rng import SplitMix64, bernoulli_map, permutation, single_flips, pair_flips_3x3, uniform_array
from .configs import WorkloadSpec, PortSpec, get_spec, SPECS

__all__ = [
    "SplitMix64",
    "bernoulli_map",
    "permutation",
    "single_flips",
    "pair_flips_3x3",
    "uniform_array",
    "WorkloadSpec",
    "PortSpec",
    "get_spec",
    "SPECS",
]
