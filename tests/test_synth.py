"""The seeded generators shared by both sides."""

import numpy as np

from synth import SplitMix64, bernoulli_map, get_spec, pair_flips_3x3, permutation


def test_splitmix64_published_vector():
    # first outputs of SplitMix64 seeded with 1234567 (Steele, Lea, Flood 2014 reference code)
    g = SplitMix64(1234567)
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
            16408922859458223821]
    assert [g.next_u64() for _ in range(5)] == want


def test_bernoulli_density_and_determinism():
    a = bernoulli_map(20000, 0.5, 3)
    assert np.array_equal(a, bernoulli_map(20000, 0.5, 3))
    assert abs(a.mean() - 0.5) < 0.02
    assert abs(bernoulli_map(20000, 0.8, 4).mean() - 0.8) < 0.02


def test_permutation_is_a_permutation():
    p = permutation(800, 9)
    assert sorted(p.tolist()) == list(range(800))


def test_pair_candidate_count():
    off, cells = pair_flips_3x3(3, 32, 32)
    assert len(off) - 1 == 3 * (31 * 32 * 2) + 3 * 1024 == 9024
    assert np.all(cells[0::2] < cells[1::2])


def test_workload_sizes():
    s = get_spec("batched20")
    assert s.n_cells == 800 and len(s.freqs) == 101 and len(s.via_sites()) == 13
    assert len(set(s.via_sites())) == 13
    off, cells = s.flips()
    assert len(off) == 801
