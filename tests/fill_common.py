"""Frequencies at which the near pairs of a structure straddle the switch
between the series and the exponential evaluation of the smooth remainder
(exp(-jkR) - 1)/(4 pi R) of the Green's function (switch at |kR| = 1e-3)."""

import numpy as np

from oracle import efie


def near_series_switch_freqs(st):
    """Returns ([f_mid / 3, f_mid], fraction of the near pairs' nonzero point
    distances below the switch at each): at f_mid half of them are below, at
    a third of it all are."""
    spec = st.spec
    td = efie.TriangleData(st.tri_xyz())
    t = np.arange(len(td.area))
    ip, iq = np.nonzero(efie.near_pairs(td, t, t))
    R = np.linalg.norm(td.qp[ip][:, :, None] - td.qp[iq][:, None], axis=-1)
    R = R[R > 0]
    k1 = abs(efie.wavenumber(1.0, spec.eps_r, spec.tan_d)[2])  # |k| at 1 Hz; k grows with f
    f_mid = 1e-3 / (np.median(R) * k1)
    freqs = np.array([f_mid / 3, f_mid])
    below = [float(np.mean(R * k1 * f < 1e-3)) for f in freqs]
    return freqs, below
