"""Composite figure of merit (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Eq. 8 sums reciprocal rewards over four frequency sets and Eq. 9 defines each
reward as an exponential barrier in S_dB.  Lower is better (Algorithm 1 takes
the argmin).

Readings (the paper leaves these open):

* S_dB = 20 log10 |S|, so 10^(S_dB/10) = |S|^2 (power).
* Bands: f_p1 = [5.15, 5.925] GHz and f_p2 = [6.425, 7.125] GHz closed;
  f_i = (5.925, 6.425) GHz open; f_s = [3, 9] GHz minus the other three
  (Section III-B).  Frequencies outside 3-9 GHz add nothing.
* A term whose S entry does not exist (fewer than three ports) is dropped.
* |S| is clamped below at 1e-15 (|S|^2 >= 1e-30) so that 1/rw_p stays finite.

Parity: pinned by every term equalling exactly 1 at its threshold, by every
term's value at two levels off all thresholds (tests/golden/fom_slopes.json,
written out from the exponents, which fixes each slope), by the variant
tables summed from those values, and by band counts on the workload grids
(tests/test_oracle_fom.py).
"""

from __future__ import annotations

import numpy as np

P1 = (5.15e9, 5.925e9)
P2 = (6.425e9, 7.125e9)
FS = (3.0e9, 9.0e9)


def band_sets(freqs):
    """Boolean masks (p1, p2, i, s) over the frequency grid."""
    f = np.asarray(freqs, dtype=np.float64)
    p1 = (f >= P1[0]) & (f <= P1[1])
    p2 = (f >= P2[0]) & (f <= P2[1])
    fi = (f > P1[1]) & (f < P2[0])
    fs = (f >= FS[0]) & (f <= FS[1]) & ~p1 & ~p2 & ~fi
    return p1, p2, fi, fs


def s_db(S) -> np.ndarray:
    return 20.0 * np.log10(np.maximum(np.abs(S), 1e-15))


def rewards(S_f: np.ndarray) -> dict:
    """Eq. 9 for one frequency; S_f is P x P.  Ports are 1-based in the paper
    (S21 = S_f[1, 0]).  Missing entries give None."""
    P = S_f.shape[0]

    def db(i, j):
        return s_db(S_f[i - 1, j - 1]) if max(i, j) <= P else None

    def ten(x):
        return None if x is None else 10.0 ** x

    s11, s21, s31, s32 = db(1, 1), db(2, 1), db(3, 1), db(3, 2)
    return {
        "p1": ten(None if s21 is None else (s21 + 1.0) / 10.0),
        "p2": ten(None if s31 is None else (s31 + 1.0) / 10.0),
        "s1": ten(None if s21 is None else (-s21 - 35.0) / 15.0),
        "s2": ten(None if s31 is None else (-s31 - 35.0) / 15.0),
        "s3": ten(None if s21 is None else (-s21 - 20.0) / 18.0),
        "s4": ten(None if s31 is None else (-s31 - 20.0) / 18.0),
        "oi": ten(None if s32 is None else (-s32 - 20.0) / 15.0),
        "m1": ten((-15.0 - s11) / 10.0),
        "m2": ten((-15.0 - s11) / 10.0),
        # Section III-D variants: stricter rejection terms, and an isolation term
        "s1rej": ten(None if s21 is None else (-s21 - 45.0) / 10.0),
        "s2rej": ten(None if s31 is None else (-s31 - 45.0) / 10.0),
        "oiiso": ten(None if s32 is None else (-s32 - 35.0) / 15.0),
    }


BAND_TERMS = (("p1", ("p1", "m1", "s2")), ("p2", ("p2", "m2", "s1")), ("i", ("oi",)), ("s", ("s3", "s4")))

# Section III-D: "rej" replaces rw_s1 and rw_s2 by their stricter forms; "iso"
# adds the isolation term in both passbands.
VARIANT_TERMS = {
    "paper": BAND_TERMS,
    "rej": (("p1", ("p1", "m1", "s2rej")), ("p2", ("p2", "m2", "s1rej")), ("i", ("oi",)), ("s", ("s3", "s4"))),
    "iso": (("p1", ("p1", "m1", "s2", "oiiso")), ("p2", ("p2", "m2", "s1", "oiiso")), ("i", ("oi",)),
            ("s", ("s3", "s4"))),
}


def fom(S: np.ndarray, freqs, variant: str = "paper") -> float:
    """Eq. 8 for one candidate: S is (F, P, P); variant picks the term table."""
    masks = dict(zip(("p1", "p2", "i", "s"), band_sets(freqs)))
    total = 0.0
    for f_idx in range(len(freqs)):
        rw = rewards(S[f_idx])
        for band, terms in VARIANT_TERMS[variant]:
            if masks[band][f_idx]:
                for t in terms:
                    if rw[t] is not None:
                        total += 1.0 / rw[t]
    return total
