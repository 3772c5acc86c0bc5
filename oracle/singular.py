"""Closed-form potential integrals over a flat triangle (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

For a flat triangle T and an observation point r, with R = |r - r'|:

    I1(r)   = integral over T of 1/R dS'
    Irho(r) = integral over T of (rho' - rho)/R dS'

where rho is the projection of r onto the triangle's plane.  These are the
standard results of Wilton, Rao, Glisson et al. (IEEE Trans. Antennas Propag.
32(3), 1984) in the notation of Graglia (IEEE TAP 41(10), 1993).  They are used
to extract the 1/R part of the Green's function from near triangle pairs in
the EFIE fill (the paper delegates this to its MoM engine, Section II-D).

For each edge i of T (vertices taken counter-clockwise about the unit normal
n, edge running from vertex a to vertex b):

    t_i  = unit edge tangent,   u_i = t_i x n   (in-plane outward normal)
    l+_i = (r_b - rho).t_i,     l-_i = (r_a - rho).t_i
    P0_i = (r_a - rho).u_i,     d = n.(r - r_a)
    R0_i^2 = P0_i^2 + d^2,      R+-_i = sqrt(l+-_i^2 + R0_i^2)
    f_i  = ln[(R+_i + l+_i) / (R-_i + l-_i)]

    I1   = sum_i P0_i f_i - |d| sum_i [atan(P0_i l+_i / (R0_i^2 + |d| R+_i))
                                      - atan(P0_i l-_i / (R0_i^2 + |d| R-_i))]
    Irho = 1/2 sum_i u_i [R0_i^2 f_i + l+_i R+_i - l-_i R-_i]

f_i is evaluated as ln[(R-_i - l-_i)/(R+_i - l+_i)] when l+_i + l-_i < 0 (the
same value, without cancellation), and taken as 0 when R0_i vanishes (it is
then multiplied by zero).

Parity: pinned against Duffy-transformed Gauss-Legendre quadrature
(tests/test_oracle_singular.py).
"""

from __future__ import annotations

import numpy as np


def potential_integrals(tri: np.ndarray, r: np.ndarray):
    """tri: (..., 3, 3) vertex coordinates; r: (..., 3) observation points.

    Broadcasts over the leading axes.  Returns (I1 (...), Irho (..., 3)).
    """
    tri = np.asarray(tri, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    v = [tri[..., 0, :], tri[..., 1, :], tri[..., 2, :]]
    nrm = np.cross(v[1] - v[0], v[2] - v[0])
    n = nrm / np.linalg.norm(nrm, axis=-1, keepdims=True)
    d = np.sum(n * (r - v[0]), axis=-1)
    rho = r - d[..., None] * n
    ad = np.abs(d)
    I1 = np.zeros(np.broadcast_shapes(d.shape))
    Irho = np.zeros(I1.shape + (3,))
    for i in range(3):
        va, vb = v[i], v[(i + 1) % 3]
        edge = vb - va
        t = edge / np.linalg.norm(edge, axis=-1, keepdims=True)
        u = np.cross(t, n)
        lp = np.sum((vb - rho) * t, axis=-1)
        lm = np.sum((va - rho) * t, axis=-1)
        P0 = np.sum((va - rho) * u, axis=-1)
        R0sq = P0 * P0 + d * d
        Rp = np.sqrt(lp * lp + R0sq)
        Rm = np.sqrt(lm * lm + R0sq)
        scale = np.linalg.norm(edge, axis=-1)
        degenerate = R0sq <= (1e-14 * scale) ** 2
        with np.errstate(divide="ignore", invalid="ignore"):
            f_pos = np.log((Rp + lp) / (Rm + lm))
            f_neg = np.log((Rm - lm) / (Rp - lp))
        f = np.where(lp + lm >= 0.0, f_pos, f_neg)
        f = np.where(degenerate, 0.0, f)
        with np.errstate(divide="ignore", invalid="ignore"):
            b1 = np.arctan2(P0 * lp, R0sq + ad * Rp)
            b2 = np.arctan2(P0 * lm, R0sq + ad * Rm)
        beta = np.where(degenerate, 0.0, b1 - b2)
        I1 = I1 + P0 * f - ad * beta
        Irho = Irho + 0.5 * u * (R0sq * f + lp * Rp - lm * Rm)[..., None]
    return I1, Irho
