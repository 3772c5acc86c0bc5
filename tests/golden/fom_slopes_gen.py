"""Writes fom_slopes.json: the reciprocal reward 1/rw of every Eq. 9 term and
of the Section III-D variant terms at two magnitudes of its S entry.

Each value is 10^(-exponent) with the exponent typed in from the equation,
S_dB = 20 log10 |S|, evaluated in 40-digit decimal arithmetic.  Nothing here
imports the oracle or the library: the file pins the oracle from outside.
"""

import json
import os
from decimal import Decimal, getcontext

getcontext().prec = 40
TEN = Decimal(10)


def s_db(mag):
    return Decimal(20) * (Decimal(mag).ln() / TEN.ln())


def ten_to(x):
    return (x * TEN.ln()).exp()


# term: (S entry, exponent of rw as text, passage, exponent as a function of S_dB)
TERMS = {
    "p1": ((2, 1), "(S21_dB + 1) / 10", "Eq. 9", lambda s: (s + 1) / 10),
    "p2": ((3, 1), "(S31_dB + 1) / 10", "Eq. 9", lambda s: (s + 1) / 10),
    "s1": ((2, 1), "(-S21_dB - 35) / 15", "Eq. 9", lambda s: (-s - 35) / 15),
    "s2": ((3, 1), "(-S31_dB - 35) / 15", "Eq. 9", lambda s: (-s - 35) / 15),
    "s3": ((2, 1), "(-S21_dB - 20) / 18", "Eq. 9", lambda s: (-s - 20) / 18),
    "s4": ((3, 1), "(-S31_dB - 20) / 18", "Eq. 9", lambda s: (-s - 20) / 18),
    "oi": ((3, 2), "(-S32_dB - 20) / 15", "Eq. 9", lambda s: (-s - 20) / 15),
    "m1": ((1, 1), "(-15 - S11_dB) / 10", "Eq. 9", lambda s: (-15 - s) / 10),
    "m2": ((1, 1), "(-15 - S11_dB) / 10", "Eq. 9", lambda s: (-15 - s) / 10),
    "s1rej": ((2, 1), "(-S21_dB - 45) / 10", "Section III-D, rw_s1^rej", lambda s: (-s - 45) / 10),
    "s2rej": ((3, 1), "(-S31_dB - 45) / 10", "Section III-D, rw_s2^rej", lambda s: (-s - 45) / 10),
    "oiiso": ((3, 2), "(-S32_dB - 35) / 15", "Section III-D, rw_oi^iso", lambda s: (-s - 35) / 15),
}
LEVELS = ["0.5", "0.01"]  # -6.0206 dB and -40 dB: on no term's threshold


def main():
    out = {
        "source": "Eq. 9 and the Section III-D variant rewards of arXiv 2412.17617",
        "comment": ("Reciprocal reward 1/rw = 10^(-exponent) of every term at two magnitudes of its S entry "
                    "that lie on no term's threshold (|S| = 0.5 is -6.0206 dB, |S| = 0.01 is -40 dB), with "
                    "S_dB = 20 log10 |S|; two levels fix both the offset and the slope (the denominator) of "
                    "each exponent.  Written by fom_slopes_gen.py from the exponents typed in from the "
                    "equations."),
        "levels_abs": [float(x) for x in LEVELS],
        "terms": {},
    }
    for k, (e, expo, cite, f) in TERMS.items():
        out["terms"][k] = {"entry": list(e), "exponent_of_rw": expo, "passage": cite,
                           "inv_rw": {lv: float("%.15e" % ten_to(-f(s_db(lv)))) for lv in LEVELS}}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fom_slopes.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
