"""Counter-based random draws used to build synthetic workloads.

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) is used because its definition is short and
language independent: any implementation that follows the published
increment and mixing constants reproduces the same stream.

The paper starts each search from a random pixel map (Algorithm 1, restart
step) at 50 % metal density (Section III-C).  Maps are drawn here as
Bernoulli(p) per cell in canonical cell order.
"""

from __future__ import annotations

import numpy as np

_MASK = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15


class SplitMix64:
    """SplitMix64 stream.  ``next_u64`` returns the next 64-bit output."""

    def __init__(self, seed: int):
        self.state = seed & _MASK

    def next_u64(self) -> int:
        self.state = (self.state + _GOLDEN) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def next_unit(self) -> float:
        """Uniform double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)


def bernoulli_map(n_cells: int, p: float, seed: int) -> np.ndarray:
    """Pixel occupation vector: cell i is metal iff u_i < p (u_i from SplitMix64(seed))."""
    g = SplitMix64(seed)
    return np.array([1 if g.next_unit() < p else 0 for _ in range(n_cells)], dtype=np.uint8)


def permutation(n: int, seed: int) -> np.ndarray:
    """Fisher-Yates shuffle of 0..n-1 driven by SplitMix64(seed)."""
    g = SplitMix64(seed)
    a = list(range(n))
    for i in range(n - 1, 0, -1):
        j = int(g.next_unit() * (i + 1))
        a[i], a[j] = a[j], a[i]
    return np.array(a, dtype=np.int32)


def single_flips(cells) -> tuple[np.ndarray, np.ndarray]:
    """CSR flip list with one candidate per listed cell (the cell toggled)."""
    cells = np.asarray(cells, dtype=np.int32)
    offsets = np.arange(len(cells) + 1, dtype=np.int32)
    return offsets, cells.copy()


def pair_flips_3x3(n_layers: int, nx: int, ny: int) -> tuple[np.ndarray, np.ndarray]:
    """Pair-flip candidates restricted to a pixel's neighbourhood.

    Same-layer 4-adjacent pairs (horizontal then vertical, layer-major) followed
    by every pair of layers at the same (x, y).  Cells are canonical indices
    layer*ny*nx + y*nx + x; each pair is listed with the smaller index first.
    """
    pairs = []
    for l in range(n_layers):
        base = l * nx * ny
        for y in range(ny):
            for x in range(nx - 1):
                pairs.append((base + y * nx + x, base + y * nx + x + 1))
        for y in range(ny - 1):
            for x in range(nx):
                pairs.append((base + y * nx + x, base + (y + 1) * nx + x))
    for l0 in range(n_layers):
        for l1 in range(l0 + 1, n_layers):
            for y in range(ny):
                for x in range(nx):
                    c = y * nx + x
                    pairs.append((l0 * nx * ny + c, l1 * nx * ny + c))
    cells = np.array(pairs, dtype=np.int32).reshape(-1)
    offsets = np.arange(0, 2 * len(pairs) + 1, 2, dtype=np.int32)
    return offsets, cells


def uniform_array(n: int, seed: int, bound: float) -> np.ndarray:
    """n draws uniform in [-bound, bound) from SplitMix64(seed), as float64."""
    g = SplitMix64(seed)
    out = np.empty(n, np.float64)
    for i in range(n):
        out[i] = (2.0 * g.next_unit() - 1.0) * bound
    return out
