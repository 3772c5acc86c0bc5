"""Workload descriptions: geometry numbers, frequency grids and seeds.

Each workload is a stack of ``n_layers`` pixel grids (``nx`` by ``ny`` square
pixels of side ``a``), layer l lying in the plane z = -l*h, embedded in a
homogeneous medium of relative permittivity ``eps_r`` and loss tangent
``tan_d``.  Ports sit at the middle cell of a grid side on a given layer.
Optional vias join layers 0 and 1 at listed (x, y) sites.

The numbers follow the paper's workloads where it gives them (Table I stack
heights, the Rogers 4350B permittivity in Section IV, the 3-9 GHz FoM window
of Section III-B) and are otherwise chosen to be of the same shape.  None of
this is arithmetic of the method; it only says what to build.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .rng import bernoulli_map, pair_flips_3x3, permutation, single_flips

SIDES = ("right", "top", "left", "bottom")


@dataclass(frozen=True)
class PortSpec:
    side: str  # one of SIDES
    layer: int


@dataclass(frozen=True)
class WorkloadSpec:
    name: str
    n_layers: int
    nx: int
    ny: int
    a: float  # pixel side, metres
    h: float  # layer spacing, metres
    eps_r: float
    tan_d: float
    ports: tuple
    n_freq: int
    f_lo: float
    f_hi: float
    seed: int
    density: float = 0.5
    n_vias: int = 0
    z0: float = 50.0
    candidates: str = "single"  # "single" or "pair3x3"
    sub: int = 1  # squares per pixel side: 1, 2, 3 give 2, 8, 18 triangles per pixel

    @property
    def n_cells(self) -> int:
        return self.n_layers * self.nx * self.ny

    @property
    def freqs(self) -> np.ndarray:
        return np.linspace(self.f_lo, self.f_hi, self.n_freq)

    def via_sites(self) -> list:
        """(x, y) sites of the vias, the first n_vias cells of a seeded permutation."""
        if self.n_vias == 0:
            return []
        perm = permutation(self.nx * self.ny, self.seed * 1000 + 7)
        return [(int(c % self.nx), int(c // self.nx)) for c in perm[: self.n_vias]]

    def base_map(self) -> np.ndarray:
        return bernoulli_map(self.n_cells, self.density, self.seed)

    def flips(self):
        """(offsets, cells) CSR of the candidate flips for one search step."""
        if self.candidates == "single":
            return single_flips(np.arange(self.n_cells))
        if self.candidates == "pair3x3":
            return pair_flips_3x3(self.n_layers, self.nx, self.ny)
        raise ValueError(self.candidates)

    def uneven_batch(self, n_maps: int = 8, per_map: int = 100, p0: float = 0.55, dp: float = 0.04):
        """Maps of rising density, each with ``per_map`` single flips.

        Single flips change the active count by a handful of basis functions,
        so a spread of active sizes needs several base maps.  Returns a list of
        (map, offsets, cells).
        """
        out = []
        for i in range(n_maps):
            m = bernoulli_map(self.n_cells, p0 + dp * i, self.seed * 100 + i + 1)
            cells = permutation(self.n_cells, self.seed * 100 + 50 + i)[:per_map]
            off, cl = single_flips(np.sort(cells))
            out.append((m, off, cl))
        return out

    def uneven_maps(self, n_maps: int = 8, per_map: int = 100, p0: float = 0.55, dp: float = 0.04) -> np.ndarray:
        """The uneven batch as whole maps, one row per candidate (base map
        with its cell toggled), in batch order."""
        rows = []
        for m, off, cl in self.uneven_batch(n_maps, per_map, p0, dp):
            for c in range(len(off) - 1):
                r = m.copy()
                for cell in cl[off[c]:off[c + 1]]:
                    r[cell] ^= 1
                rows.append(r)
        return np.array(rows, dtype=np.uint8).reshape(len(rows), self.n_cells)


def _p(*pairs):
    return tuple(PortSpec(s, l) for s, l in pairs)


SPECS = {
    # One metal layer of 8x8 one-millimetre pixels in free space, two ports on
    # opposite sides, 11 frequencies over 1-6 GHz; one sweep of 64 single flips.
    "plain8": WorkloadSpec(
        name="plain8", n_layers=1, nx=8, ny=8, a=1.0e-3, h=0.0, eps_r=1.0, tan_d=0.0,
        ports=_p(("right", 0), ("left", 0)), n_freq=11, f_lo=1.0e9, f_hi=6.0e9, seed=1,
    ),
    # Two layers of 20x20 half-millimetre pixels in a lossy dielectric, three
    # ports (common right, low band top, high band left), 13 vias, 101
    # frequencies over 1-8 GHz; one sweep of all 800 single flips.
    "batched20": WorkloadSpec(
        name="batched20", n_layers=2, nx=20, ny=20, a=0.5e-3, h=0.5e-3, eps_r=3.5, tan_d=0.002,
        ports=_p(("right", 0), ("top", 0), ("left", 0)), n_freq=101, f_lo=1.0e9, f_hi=8.0e9,
        seed=2, n_vias=13,
    ),
    # Three layers of 24x24 pixels with the 0.4866 mm stack of Table I in
    # Rogers 4350B; ports on three different layers; 1728 single flips.
    "stress24": WorkloadSpec(
        name="stress24", n_layers=3, nx=24, ny=24, a=0.3e-3, h=0.4866e-3, eps_r=3.66, tan_d=0.004,
        ports=_p(("right", 1), ("left", 2), ("left", 0)), n_freq=101, f_lo=1.0e9, f_hi=8.0e9, seed=3,
    ),
    # Three layers of 32x32 pixels, 201 frequencies over 0.5-10 GHz, pair flips
    # in 3x3 neighbourhoods.
    "ceiling32": WorkloadSpec(
        name="ceiling32", n_layers=3, nx=32, ny=32, a=0.3e-3, h=0.4866e-3, eps_r=3.66, tan_d=0.004,
        ports=_p(("right", 1), ("left", 2), ("left", 0)), n_freq=201, f_lo=0.5e9, f_hi=10.0e9,
        seed=5, candidates="pair3x3",
    ),
    # The 8-triangle alternating mesh (every pixel a 2 x 2 grid of squares):
    # two layers of 12x12 pixels in the batched20 dielectric, 6 vias, 41
    # frequencies; and the paper-size stripline parent (two layers of 30x30
    # pixels, 8 triangles per pixel, about 21,500 functions) whose fill is
    # checked on sampled entries.
    "mesh8": WorkloadSpec(
        name="mesh8", n_layers=2, nx=12, ny=12, a=0.5e-3, h=0.5e-3, eps_r=3.5, tan_d=0.002,
        ports=_p(("right", 0), ("top", 0), ("left", 1)), n_freq=41, f_lo=1.0e9, f_hi=8.0e9,
        seed=6, n_vias=6, sub=2,
    ),
    "paper30": WorkloadSpec(
        name="paper30", n_layers=2, nx=30, ny=30, a=0.5e-3, h=0.5e-3, eps_r=3.66, tan_d=0.004,
        ports=_p(("right", 0), ("top", 0), ("left", 1)), n_freq=72, f_lo=1.0e9, f_hi=8.0e9,
        seed=7, n_vias=13, sub=2,
    ),
    # Small cases for CPU tests.
    "tiny4x2s2": WorkloadSpec(
        name="tiny4x2s2", n_layers=2, nx=4, ny=4, a=0.5e-3, h=0.5e-3, eps_r=3.5, tan_d=0.002,
        ports=_p(("right", 0), ("top", 0), ("left", 1)), n_freq=4, f_lo=5.0e9, f_hi=7.0e9,
        seed=12, n_vias=3, sub=2,
    ),
    "tiny3s3": WorkloadSpec(
        name="tiny3s3", n_layers=1, nx=3, ny=3, a=1.0e-3, h=0.0, eps_r=1.0, tan_d=0.0,
        ports=_p(("right", 0), ("left", 0)), n_freq=5, f_lo=3.5e9, f_hi=5.5e9, seed=11, sub=3,
    ),
    "tiny3": WorkloadSpec(
        name="tiny3", n_layers=1, nx=3, ny=3, a=1.0e-3, h=0.0, eps_r=1.0, tan_d=0.0,
        ports=_p(("right", 0), ("left", 0)), n_freq=5, f_lo=3.5e9, f_hi=5.5e9, seed=11,
    ),
    "tiny4x2": WorkloadSpec(
        name="tiny4x2", n_layers=2, nx=4, ny=4, a=0.5e-3, h=0.5e-3, eps_r=3.5, tan_d=0.002,
        ports=_p(("right", 0), ("top", 0), ("left", 1)), n_freq=4, f_lo=5.0e9, f_hi=7.0e9,
        seed=12, n_vias=3,
    ),
    "small6x3": WorkloadSpec(
        name="small6x3", n_layers=3, nx=6, ny=6, a=0.3e-3, h=0.4866e-3, eps_r=3.66, tan_d=0.004,
        ports=_p(("right", 1), ("left", 2), ("left", 0)), n_freq=5, f_lo=4.0e9, f_hi=8.0e9, seed=13,
    ),
}


def get_spec(name: str) -> WorkloadSpec:
    return SPECS[name]
