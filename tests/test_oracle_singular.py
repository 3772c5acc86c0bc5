"""Pin the closed-form potential integrals against Duffy quadrature.

The reference integrals split the triangle at the projection rho of the
observation point into three sub-triangles (rho, v_a, v_b) (signed, so rho may
lie outside) and map each from the unit square with the Duffy transform
x = rho + u (v_a - rho) + u v (v_b - v_a), whose Jacobian u * 2|area| cancels
the 1/R singularity at rho.  Each edge is cut into panels graded toward the point nearest rho, and each
panel's sub-triangle is integrated by Gauss-Legendre of order 32 per direction.
"""

import numpy as np
import pytest

from oracle.singular import potential_integrals


def _panels(rho, a, b):
    """Split edge [a, b] into segments graded geometrically toward the point of
    the segment closest to rho, so each sub-triangle (rho, p, q) sees a smooth
    angular integrand."""
    ab = b - a
    t = np.clip(np.dot(rho - a, ab) / np.dot(ab, ab), 0.0, 1.0)
    h = max(np.linalg.norm(rho - (a + t * ab)), 1e-300)
    L = np.linalg.norm(ab)
    cuts = {0.0, 1.0, t}
    for side, span in ((-1, t), (1, 1.0 - t)):
        s = span
        while s * L > h / 8 and s > 1e-16:
            s *= 0.5
            cuts.add(t + side * s)
    cuts = sorted(c for c in cuts if 0.0 <= c <= 1.0)
    return [(a + c0 * ab, a + c1 * ab) for c0, c1 in zip(cuts[:-1], cuts[1:]) if c1 > c0]


def duffy(tri, r, order=32):
    g, w = np.polynomial.legendre.leggauss(order)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    v0, v1, v2 = tri
    n = np.cross(v1 - v0, v2 - v0)
    n /= np.linalg.norm(n)
    d = np.dot(n, r - v0)
    rho = r - d * n
    I1 = 0.0
    Irho = np.zeros(3)
    U, V = np.meshgrid(g, g, indexing="ij")
    W = np.outer(w, w)
    for a0, b0 in ((v0, v1), (v1, v2), (v2, v0)):
        for a, b in _panels(rho, a0, b0):
            signed2A = np.dot(np.cross(a - rho, b - rho), n)  # twice the signed area
            x = rho + U[..., None] * (a - rho) + (U * V)[..., None] * (b - a)
            R = np.linalg.norm(r - x, axis=-1)
            jac = U * signed2A
            I1 += np.sum(W * jac / R)
            Irho += np.einsum("uv,uvd->d", W * jac / R, x - rho)
    return I1, Irho


TRI = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.3, 0.8, 0.0]])
TILT = np.array([[0.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 0.7]])  # a vertical triangle

POINTS = [
    (TRI, np.array([0.4, 0.3, 0.0])),  # inside, in plane
    (TRI, np.array([0.4, 0.3, 0.05])),  # just above
    (TRI, np.array([0.4, 0.3, -0.5])),  # well below
    (TRI, np.array([1.4, -0.3, 0.0])),  # outside, in plane
    (TRI, np.array([1.4, -0.3, 0.2])),  # outside, off plane
    (TRI, np.array([0.5, 0.001, 0.0])),  # near an edge
    (TRI, np.array([2.0, 0.0, 0.0])),  # on the line of an edge, beyond it
    (TILT, np.array([0.2, 0.3, 0.2])),  # vertical triangle, point beside it
    (TILT, np.array([0.0, 0.3, 0.2])),  # vertical triangle, point in its plane
]


@pytest.mark.parametrize("tri,r", POINTS)
def test_closed_form_matches_duffy(tri, r):
    I1, Irho = potential_integrals(tri, r)
    J1, Jrho = duffy(tri, r)
    assert abs(I1 - J1) <= 1e-10 * abs(J1)
    assert np.abs(Irho - Jrho).max() <= 1e-10 * max(1.0, np.abs(Jrho).max())


def test_far_point_tends_to_area_over_distance():
    r = np.array([0.4, 0.3, 1e4])
    I1, _ = potential_integrals(TRI, r)
    area = 0.5 * np.linalg.norm(np.cross(TRI[1] - TRI[0], TRI[2] - TRI[0]))
    c = TRI.mean(axis=0)
    assert abs(I1 - area / np.linalg.norm(r - c)) <= 1e-9 * I1


def test_broadcast_matches_single():
    pts = np.stack([p for _, p in POINTS[:6]])
    I1, Irho = potential_integrals(np.broadcast_to(TRI, (6, 3, 3)), pts)
    for i, p in enumerate(pts):
        a, b = potential_integrals(TRI, p)
        assert I1[i] == a and np.all(Irho[i] == b)
