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


SLOPES = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "fom_slopes.json")))


@pytest.mark.parametrize("term", list(SLOPES["terms"]))
@pytest.mark.parametrize("level", ["0.5", "0.01"])
def test_each_reward_off_its_threshold(term, level):
    """Eq. 9 / Section III-D: 1/rw at two levels of its entry (|S| = 0.5 and
    0.01, on no threshold), against values written out from the exponents
    (tests/golden/fom_slopes.json).  A wrong denominator or offset in any
    exponent moves at least one of the two."""
    t = SLOPES["terms"][term]
    i, j = t["entry"]
    S = np.full((3, 3), 0.2 + 0j)
    S[i - 1, j - 1] = float(level)
    got = 1.0 / fom.rewards(S)[term]
    want = t["inv_rw"][level]
    assert abs(got - want) <= 1e-12 * want


def _const_s(level_of_entry, P=3):
    S = np.full((P, P), 0.2 + 0j)
    for (i, j), v in level_of_entry.items():
        S[i - 1, j - 1] = v
    return S


@pytest.mark.parametrize("variant", ["paper", "rej", "iso"])
def test_variant_tables_from_golden_terms(variant):
    """Eq. 8 and its Section III-D variants on an S that is the same at every
    frequency: the FoM is each band's point count times the sum of that
    band's golden 1/rw values.  The bands' terms (Eq. 8: p1 -> p1, m1, s2;
    p2 -> p2, m2, s1; f_i -> oi; f_s -> s3, s4; 'rej' swaps s1, s2 for their
    -45 dB forms; 'iso' adds the isolation term over p1 and p2) are typed in
    here from the equations, not taken from the oracle's table."""
    freqs = get_spec("batched20").freqs  # band counts (11, 10, 7, 44), pinned above
    counts = {"p1": 11, "p2": 10, "i": 7, "s": 44}
    lv = {(1, 1): 0.5, (2, 1): 0.01, (3, 1): 0.5, (3, 2): 0.01}
    g = {k: SLOPES["terms"][k]["inv_rw"]["0.5" if lv[tuple(v["entry"])] == 0.5 else "0.01"]
         for k, v in SLOPES["terms"].items()}
    table = {
        "paper": {"p1": ["p1", "m1", "s2"], "p2": ["p2", "m2", "s1"], "i": ["oi"], "s": ["s3", "s4"]},
        "rej": {"p1": ["p1", "m1", "s2rej"], "p2": ["p2", "m2", "s1rej"], "i": ["oi"], "s": ["s3", "s4"]},
        "iso": {"p1": ["p1", "m1", "s2", "oiiso"], "p2": ["p2", "m2", "s1", "oiiso"], "i": ["oi"],
                "s": ["s3", "s4"]},
    }[variant]
    want = sum(counts[b] * sum(g[t] for t in ts) for b, ts in table.items())
    S = np.tile(_const_s(lv), (len(freqs), 1, 1))
    got = fom.fom(S, freqs, variant)
    assert abs(got - want) <= 1e-12 * want
