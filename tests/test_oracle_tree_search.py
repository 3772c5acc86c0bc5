"""Pins of the Algorithm 1 reference (CPU), on a table FoM so that every
property can be checked exactly."""

import itertools

import numpy as np

from oracle import search
from synth import bernoulli_map, permutation


def table_fom(n_cells, seed):
    """A fixed random FoM over all maps of a tiny grid (a lookup table)."""
    rng = np.random.default_rng(seed)
    vals = rng.random(1 << n_cells) + 0.1

    def f(m):
        return float(vals[int(sum(int(b) << i for i, b in enumerate(m)))])
    return f, vals


def restarts(n_cells, seed):
    k = 0
    while True:
        yield bernoulli_map(n_cells, 0.5, seed * 1000 + k)
        k += 1


def run(n_layers, n_pix, budget, seed=3, **kw):
    n_cells = n_layers * n_pix
    f, vals = table_fom(n_cells, seed)
    calls = []

    def ev(m):
        calls.append(np.array(m).copy())
        return f(m)
    out = search.tree_search(ev, bernoulli_map(n_cells, 0.5, seed), n_layers, n_pix, permutation(n_pix, seed),
                             restarts(n_cells, seed), budget, **kw)
    return out, calls, vals


def test_pixel_states_round_trip():
    m = np.array([1, 0, 0, 1, 1, 0], np.uint8)  # two layers of three pixels
    assert [search.pixel_state(m, 2, 3, j) for j in range(3)] == [3, 2, 0]
    for j, t in itertools.product(range(3), range(4)):
        assert search.pixel_state(search.with_state(m, 2, 3, j, t), 2, 3, j) == t


def test_evaluation_counts_follow_the_tree_shape():
    # two layers: 4 states, 3 children per pixel; depth 1 costs 3, depth 2 costs 3 + 9
    (best, P, evals, trace, nres), calls, _ = run(2, 4, 400, m_of_depth=(2, 2))
    assert evals == len(calls)
    steps = np.diff([1] + [e for e, _ in trace])
    assert set(steps.tolist()) <= {3, 12, 13, 4}  # depth 1, depth 2, and either plus a restart map


def test_accepted_fom_decreases_until_a_restart_and_best_is_the_minimum_seen():
    (best, P, evals, trace, nres), calls, vals = run(2, 4, 600, m_of_depth=(3, 2))
    seen = min(vals[int(sum(int(b) << i for i, b in enumerate(c)))] for c in calls)
    assert best == seen
    assert nres >= 1
    F = [f for _, f in trace]
    ups = sum(1 for a, b in zip(F, F[1:]) if b > a)
    assert ups <= nres  # the current FoM only rises at a restart


def test_finds_the_global_optimum_of_a_tiny_grid():
    """Brute force: one layer of 9 pixels (512 maps); with restarts and a
    budget of 3000 evaluations the search reaches the table's minimum."""
    (best, P, evals, trace, nres), calls, vals = run(1, 9, 3000, m_of_depth=(3, 2))
    assert best == vals.min()


def test_depth_two_leaves_change_exactly_two_pixels():
    n_layers, n_pix = 2, 4
    (best, P, evals, trace, nres), calls, _ = run(n_layers, n_pix, 60, m_of_depth=(1, 5))
    # after the first depth-1 failure the next tree has depth 2: 3 children then 9 leaves
    root = calls[0]
    first_tree = calls[1:4]
    for c in first_tree:
        assert np.count_nonzero(c.reshape(n_layers, n_pix) != root.reshape(n_layers, n_pix), axis=0).astype(bool).sum() == 1
