"""Pins for the oracle figure of merit (Eqs. 8-9, Section III-B)."""

import json
import os

import numpy as np
import pytest

from oracle import fom
from synth import get_spec

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "fom_thresholds.json")))


def s_from_db(entries_db, P=3):
    S = np.full((P, P), 1e-3 + 0j)
    for (i, j), db in entries_db.items():
        S[i - 1, j - 1] = 10 ** (db / 20.0)
    return S


@pytest.mark.parametrize("term", list(GOLD["thresholds_db"]))
def test_each_reward_is_one_at_its_threshold(term):
    t = GOLD["thresholds_db"][term]
    S = s_from_db({tuple(t["entry"]): t["level_db"]})
    rw = fom.rewards(S)[term]
    assert abs(1.0 / rw - 1.0) <= 1e-12


def test_hand_value():
    # |S21| = 0.5: 1/rw_p1 = 10^-0.1 / 0.25 = 3.1773129389...
    S = np.full((3, 3), 0.1 + 0j)
    S[1, 0] = 0.5
    assert abs(1.0 / fom.rewards(S)["p1"] - 3.1773129388971) <= 1e-12
    # |S11| = 0.1 (-20 dB): 1/rw_m1 = 10^((-20 + 15)/10) = 10^-0.5
    assert abs(1.0 / fom.rewards(S)["m1"] - 10 ** -0.5) <= 1e-14
    # |S32| = 0.1: 1/rw_oi = 10^((-20 + 20)/15) = 1
    assert abs(1.0 / fom.rewards(S)["oi"] - 1.0) <= 1e-14


def test_barrier_directions():
    """Better S lowers each term: more transmission in band, less reflection,
    less leakage."""
    base = np.full((3, 3), 0.1 + 0j)
    hi = base.copy()
    hi[1, 0] = 0.9
    lo = base.copy()
    lo[1, 0] = 0.05
    r_hi, r_lo = fom.rewards(hi), fom.rewards(lo)
    assert 1 / r_hi["p1"] < 1 / r_lo["p1"]  # transmission rewarded in band 1
    assert 1 / r_hi["s1"] > 1 / r_lo["s1"]  # same entry punished as band-2 leakage


@pytest.mark.parametrize("name,counts", [
    ("plain8", (1, 0, 1, 5)),
    ("batched20", (11, 10, 7, 44)),
    ("stress24", (11, 10, 7, 44)),
    ("ceiling32", (17, 15, 10, 84)),
])
def test_band_counts(name, counts):
    f = get_spec(name).freqs
    got = tuple(int(m.sum()) for m in fom.band_sets(f))
    assert got == counts
    masks = np.stack(fom.band_sets(f))
    assert masks.sum(axis=0).max() <= 1  # bands are disjoint


def test_two_port_drops_missing_terms():
    f = get_spec("plain8").freqs
    S = np.tile(np.array([[0.3 + 0j, 0.6], [0.6, 0.3]]), (len(f), 1, 1))
    got = fom.fom(S, f)
    p1 = 10 ** -0.1 / 0.36 + 10 ** 1.5 * 0.09  # one band-1 point (5.5 GHz)
    s = 5 * 10 ** (10 / 9) * 0.6 ** (10 / 9)  # five f_s points
    assert abs(got - (p1 + s)) <= 1e-12 * got


def test_clamp_keeps_fom_finite():
    f = np.array([5.5e9])
    S = np.zeros((1, 3, 3), dtype=complex)
    assert np.isfinite(fom.fom(S, f))


def test_variant_tables_differ_from_eq8_by_exactly_their_terms():
    """Section III-D: 'rej' swaps rw_s1/rw_s2 for their -45 dB forms, 'iso'
    adds the isolation term over both passbands."""
    spec = get_spec("batched20")
    freqs = spec.freqs
    rng = np.random.default_rng(3)
    S = (rng.standard_normal((len(freqs), 3, 3)) + 1j * rng.standard_normal((len(freqs), 3, 3))) * 0.2
    p1, p2, fi, fs = fom.band_sets(freqs)
    base = fom.fom(S, freqs)
    rw = [fom.rewards(S[k]) for k in range(len(freqs))]
    iso_extra = sum(1.0 / rw[k]["oiiso"] for k in range(len(freqs)) if p1[k] or p2[k])
    assert abs(fom.fom(S, freqs, "iso") - (base + iso_extra)) <= 1e-12 * base
    rej = base - sum(1.0 / rw[k]["s2"] - 1.0 / rw[k]["s2rej"] for k in range(len(freqs)) if p1[k]) \
        - sum(1.0 / rw[k]["s1"] - 1.0 / rw[k]["s1rej"] for k in range(len(freqs)) if p2[k])
    assert abs(fom.fom(S, freqs, "rej") - rej) <= 1e-12 * base
