"""Brute-force pin of the sweep and accept rule (Algorithm 1) on a 3x3 grid."""

import itertools

import numpy as np
import pytest

from oracle import efie, geometry, search
from synth import get_spec, single_flips


@pytest.fixture(scope="module")
def table():
    spec = get_spec("tiny3")
    st = geometry.build_structure(spec)
    Zf = np.stack([efie.fill(st, f) for f in spec.freqs])
    maps = np.array(list(itertools.product((0, 1), repeat=spec.n_cells)), dtype=np.uint8)
    foms = np.array([search.evaluate_gather(st, Zf, m, spec.freqs)[1] for m in maps])
    return spec, st, Zf, maps, foms


def key(m):
    return int("".join(str(int(b)) for b in m), 2)


def test_every_map_is_finite(table):
    spec, st, Zf, maps, foms = table
    assert len(foms) == 512 and np.all(np.isfinite(foms)) and np.all(foms > 0)


@pytest.mark.parametrize("base_key", [0, 5, 170, 300, 511])
def test_sweep_argmin_is_exhaustive_neighbourhood_minimum(table, base_key):
    spec, st, Zf, maps, foms = table
    base = maps[base_key]
    off, cells = single_flips(np.arange(spec.n_cells))
    S, F = search.sweep(st, Zf, base, off, cells, spec.freqs)
    neigh = [key(search.apply_flips(base, [c])) for c in range(spec.n_cells)]
    assert np.array_equal(F, foms[neigh])
    i, ok = search.accept(foms[base_key], F)
    assert F[i] == foms[neigh].min()
    assert i == int(np.argmin(foms[neigh]))  # numpy's argmin also takes the first minimum
    assert ok == (foms[neigh].min() < foms[base_key])


def test_greedy_descent_ends_in_a_table_local_minimum(table):
    spec, st, Zf, maps, foms = table
    off, cells = single_flips(np.arange(spec.n_cells))
    m = maps[85].copy()
    cur = foms[85]
    for _ in range(600):
        _, F = search.sweep(st, Zf, m, off, cells, spec.freqs)
        i, ok = search.accept(cur, F)
        if not ok:
            break
        m = search.apply_flips(m, [i])
        cur = F[i]
    neigh = [key(search.apply_flips(m, [c])) for c in range(spec.n_cells)]
    assert foms[key(m)] == cur
    assert np.all(foms[neigh] >= cur)


def test_fresh_assembly_route_matches_gather(table):
    spec, st, Zf, maps, foms = table
    for k in (3, 77, 300, 511):
        S1, F1 = search.evaluate_gather(st, Zf, maps[k], spec.freqs)
        S2, F2 = search.evaluate_fresh(st, maps[k], spec.freqs)
        assert np.abs(S1 - S2).max() <= 1e-14
        assert abs(F1 - F2) <= 1e-13 * F1


def test_ties_go_to_lowest_index():
    assert search.argmin_lowest([3.0, 1.0, 1.0, 2.0]) == 1
    assert search.accept(1.0, [1.0, 2.0]) == (0, False)
