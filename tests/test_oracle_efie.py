"""Pins for the oracle EFIE fill (Eqs. 1-2, RWG mixed-potential form).

The independent reference integrates the same Galerkin double integral with a
high-order rule: a collapsed-square Gauss-Legendre rule on the test triangle
and, for each test point, a Duffy-transformed Gauss-Legendre rule on the
source triangle applied to the full kernel exp(-jkR)/(4 pi R).  It shares
only the problem statement with the oracle.  The oracle's 4-point rule is a
low-order discretisation, so agreement is expected to the size of that rule's
error (a few parts in 1e3), while a dropped term, a wrong sign or a wrong
factor shows up at order one.
"""

import dataclasses

import numpy as np
import pytest

from oracle import efie, geometry, network, search
from synth import bernoulli_map, get_spec

MU0 = 4e-7 * np.pi
C0 = 299792458.0
EPS0 = 1.0 / (MU0 * C0 * C0)


def gl01(n):
    g, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (g + 1), 0.5 * w


def collapsed_rule(tri, n=10):
    """Points and weights (summing to the area) on a triangle."""
    g, w = gl01(n)
    U, V = np.meshgrid(g, g, indexing="ij")
    W = np.outer(w, w) * U
    v0, v1, v2 = tri
    pts = v0 + U[..., None] * (v1 - v0) + (U * V)[..., None] * (v2 - v1)
    A2 = np.linalg.norm(np.cross(v1 - v0, v2 - v0))
    return pts.reshape(-1, 3), (W * A2).reshape(-1)


def source_full(tri, r, k, n=16):
    """int over tri of G and of r' G, G = exp(-jkR)/(4 pi R), by Duffy panels
    from the projection of r."""
    g, w = gl01(n)
    U, V = np.meshgrid(g, g, indexing="ij")
    W = np.outer(w, w)
    v0, v1, v2 = tri
    nrm = np.cross(v1 - v0, v2 - v0)
    nrm /= np.linalg.norm(nrm)
    rho = r - np.dot(nrm, r - v0) * nrm
    s = 0j
    sv = np.zeros(3, dtype=complex)
    for a0, b0 in ((v0, v1), (v1, v2), (v2, v0)):
        ab = b0 - a0
        t = np.clip(np.dot(rho - a0, ab) / np.dot(ab, ab), 0, 1)
        h = max(np.linalg.norm(rho - (a0 + t * ab)), 1e-300)
        cuts = {0.0, 1.0, t}
        for side, span in ((-1, t), (1, 1 - t)):
            q = span
            while q * np.linalg.norm(ab) > h / 8 and q > 1e-16:
                q *= 0.5
                cuts.add(t + side * q)
        cuts = sorted(c for c in cuts if 0 <= c <= 1)
        for c0, c1 in zip(cuts[:-1], cuts[1:]):
            if c1 <= c0:
                continue
            a, b = a0 + c0 * ab, a0 + c1 * ab
            s2a = np.dot(np.cross(a - rho, b - rho), nrm)
            x = rho + U[..., None] * (a - rho) + (U * V)[..., None] * (b - a)
            R = np.linalg.norm(r - x, axis=-1)
            G = np.exp(-1j * k * R) / (4 * np.pi * R)
            jw = W * U * s2a * G
            s += jw.sum()
            sv += np.einsum("uv,uvd->d", jw, x)
    return s, sv


QUAD_BARY = np.array([[1 / 3, 1 / 3, 1 / 3], [0.6, 0.2, 0.2], [0.2, 0.6, 0.2], [0.2, 0.2, 0.6]])
QUAD_W = np.array([-27 / 48, 25 / 48, 25 / 48, 25 / 48])


def four_point_rule(tri):
    A = 0.5 * np.linalg.norm(np.cross(tri[1] - tri[0], tri[2] - tri[0]))
    return QUAD_BARY @ tri, QUAD_W * A


def z_reference(st, m, n, freq, test_rule=collapsed_rule, part="both"):
    spec = st.spec
    w = 2 * np.pi * freq
    eps = EPS0 * spec.eps_r * (1 - 1j * spec.tan_d)
    k = w * np.sqrt(MU0 * eps + 0j)
    length, tri, free = geometry.rwg_geometry(st)
    T = st.tri_xyz()
    total = 0j
    for a in range(2):
        ta = T[tri[m, a]]
        Aa = 0.5 * np.linalg.norm(np.cross(ta[1] - ta[0], ta[2] - ta[0]))
        pts, wts = test_rule(ta)
        for b in range(2):
            tb = T[tri[n, b]]
            Ab = 0.5 * np.linalg.norm(np.cross(tb[1] - tb[0], tb[2] - tb[0]))
            sa, sb = (1 - 2 * a), (1 - 2 * b)
            for r, wt in zip(pts, wts):
                s, sv = source_full(tb, r, k)
                fm = sa * length[m] / (2 * Aa) * (r - free[m, a])
                fn_int = sb * length[n] / (2 * Ab) * (sv - free[n, b] * s)
                div = (sa * length[m] / Aa) * (sb * length[n] / Ab)
                vec = 1j * w * MU0 * np.dot(fm, fn_int)
                sca = div * s / (1j * w * eps)
                total += wt * {"both": vec + sca, "vector": vec, "scalar": sca}[part]
    return total


def _picks(st):
    M = st.M
    picks = [(0, 0), (0, 1)]  # self, and two functions sharing a triangle
    inter = next(i for i, b in enumerate(st.bfs) if b.kind == geometry.KIND_INTER)
    picks += [(inter, inter), (0, inter), (0, M - 1), (M - 1, M - 1), (M - 2, M - 1)]
    if any(b.kind == geometry.KIND_VIA for b in st.bfs):
        v = next(i for i, b in enumerate(st.bfs) if b.kind == geometry.KIND_VIA)
        picks += [(v, v), (v, v + 1), (v, v + 2)]
    return picks


@pytest.mark.parametrize("name,freq", [("plain8", 4.0e9), ("tiny4x2", 6.0e9)])
def test_inner_integration_against_duffy(name, freq):
    """Same outer (test) rule as the oracle, exact inner integral: isolates the
    singularity extraction and the assembly coefficients.  The oracle's inner
    4-point rule on the smooth remainder leaves an error of a few parts in 1e4
    here, (ka)^2 / 20 at most; each potential term is checked on its own."""
    spec = get_spec(name)
    st = geometry.build_structure(spec)
    for part in ("vector", "scalar"):
        Z = efie.fill(st, freq, part=part)
        for m, n in _picks(st):
            ref = z_reference(st, m, n, freq, test_rule=four_point_rule, part=part)
            assert abs(Z[m, n] - ref) <= 2e-3 * abs(ref), (part, m, n, Z[m, n], ref)


@pytest.mark.parametrize("name,freq", [("plain8", 4.0e9)])
def test_entries_against_high_order_galerkin(name, freq):
    """High-order rule on both integrals.  The oracle's 4-point test rule
    misses the near-singular outer integral by several per cent on self and
    touching pairs; the radiative (real) part is smooth and must agree
    closely."""
    spec = get_spec(name)
    st = geometry.build_structure(spec)
    Z = efie.fill(st, freq)
    for m, n in _picks(st):
        ref = z_reference(st, m, n, freq)
        assert abs(Z[m, n] - ref) <= 0.15 * abs(ref), (m, n, Z[m, n], ref)
        assert abs(Z[m, n].real - ref.real) <= 1e-5 * abs(ref.real), (m, n, Z[m, n], ref)


def test_exact_symmetry_and_passive_hermitian_part():
    spec = get_spec("plain8")
    st = geometry.build_structure(spec)
    for f in (1e9, 6e9):
        Z = efie.fill(st, f)
        assert np.array_equal(Z, Z.T)
        H = 0.5 * (Z + Z.conj().T)
        e = np.linalg.eigvalsh(H)
        assert e.min() >= -1e-10 * e.max()  # radiated power is non-negative


def test_low_frequency_input_is_capacitive():
    """An open pad structure looks like a capacitor at low frequency: the
    input reactance is negative and grows like 1/f."""
    spec = get_spec("plain8")
    st = geometry.build_structure(spec)
    pm = np.ones(spec.n_cells, dtype=np.uint8)
    sel = st.active(pm)
    rows = network.port_positions(sel, st.port_bf)
    pl = search.port_lengths(st)
    zin = []
    for f in (1e8, 2e8):
        Z = network.reduce_matrix(efie.fill(st, f), sel)
        V = network.excitation(len(Z), rows, pl)
        X = np.linalg.solve(Z, V)
        zin.append(1.0 / (pl[0] * X[rows[0], 0]))  # unloaded, port 2 shorted
    assert zin[0].imag < 0 and zin[1].imag < 0
    assert abs(zin[0].imag / zin[1].imag - 2.0) < 0.05


def test_lossy_medium_dissipates():
    spec = get_spec("tiny4x2")
    st = geometry.build_structure(spec)
    Z = efie.fill(st, 6e9)
    lossless = efie.fill(st.__class__(dataclasses.replace(spec, tan_d=0.0), st.tri_keys, st.tri_owner,
                                      st.bfs, st.port_bf), 6e9)
    # adding loss raises the dissipated power for a uniform current pattern
    x = np.ones(st.M)
    assert np.real(x @ Z @ x) > np.real(x @ lossless @ x)


def test_near_pair_remainder_in_both_branches():
    """On near pairs the source integral takes the smooth remainder
    (exp(-jkR) - 1)/(4 pi R) from a short series where |kR| < 1e-3 and from
    the exponential above.  Both branches are pinned to the remainder's
    low-frequency expansion (-jk - k^2 R/2 + j k^3 R^2/6 - ...)/(4 pi),
    integrated over the source triangle (area A, centroid c):

    * first order: -jk A / (4 pi) (the weights sum to one), and nothing for
      the first moment (the points' weighted mean is the centroid);
    * second order: -k^2 A sum_j w_j R_j / (8 pi), and the same with
      (r_j - c) for the first moment;
    * third order: j k^3 A mean(R^2) / (24 pi), where the degree-3 rule
      integrates R^2 exactly: mean(R^2) = |r - c|^2 + (a^2 + b^2 + c^2) / 36
      (the polar moment of a triangle about its centroid).

    A dropped term, a wrong sign or a wrong coefficient up to the third order
    in either branch fails one of these."""
    spec = get_spec("plain8")
    st = geometry.build_structure(spec)
    T = st.tri_xyz()
    td = efie.TriangleData(T)
    tp = np.arange(0, len(T), 7)[:12]
    tq = np.arange(len(T))
    ip, iq = np.nonzero(efie.near_pairs(td, tp, tq))
    ri = td.qp[tp][ip]                                   # (K, 4, 3) test points
    rj = td.qp[tq][iq]                                   # (K, 4, 3) source points
    cq = td.centroid[tq][iq]                             # (K, 3)
    A = td.area[tq][iq][:, None]                         # (K, 1)
    R = np.linalg.norm(ri[:, :, None] - rj[:, None], axis=-1)  # (K, 4, 4)
    rel = rj - cq[:, None]
    v = T[tq][iq]
    e2 = sum(np.sum((v[:, (i + 1) % 3] - v[:, i]) ** 2, axis=-1) for i in range(3))
    mean_r2 = np.sum((ri - cq[:, None]) ** 2, axis=-1) + e2[:, None] / 36.0
    assert np.allclose(R ** 2 @ QUAD_W, mean_r2, rtol=1e-12)  # exactness of the rule on R^2

    o1 = -A / (4 * np.pi)
    o2 = -A * (R @ QUAD_W) / (8 * np.pi)
    o2v = -A[..., None] * np.einsum("kij,j,kjd->kid", R, QUAD_W, rel) / (8 * np.pi)
    o3 = A * mean_r2 / (24 * np.pi)
    o3v = A[..., None] * np.einsum("kij,j,kjd->kid", R ** 2, QUAD_W, rel) / (24 * np.pi)

    r_min, r_max = R[R > 0].min(), R.max()
    SS0, SV0 = efie.source_integrals(td, tp, tq, 0j)
    for k, branch in ((5e-4 / r_max, "series"), (1.5e-3 / r_min, "exponential")):
        kr = k * r_max
        nz = R > 0
        # every nonzero distance falls on the branch named
        assert (np.all(k * R[nz] < 1e-3) if branch == "series" else np.all(k * R[nz] > 1e-3)), branch
        assert kr < 0.1
        SS, SV = efie.source_integrals(td, tp, tq, k + 0j)
        D = (SS - SS0)[ip, iq]                           # (K, 4)
        DV = (SV - SV0)[ip, iq]                          # (K, 4, 3)
        # relative size of the first neglected order at this k
        tol = max(kr * kr, 1e-6)
        c1 = D.imag / k
        assert np.abs(c1 - o1).max() <= tol * np.abs(o1).max(), branch
        c3 = (D.imag / k - o1) / k ** 2
        assert np.abs(c3 - o3).max() <= 1e-2 * np.abs(o3).max(), branch
        c2 = D.real / k ** 2
        assert np.abs(c2 - o2).max() <= tol * np.abs(o2).max(), branch
        assert np.abs(DV.imag / k).max() <= tol * np.abs(o1).max() * r_max, branch
        c2v = DV.real / k ** 2
        assert np.abs(c2v - o2v).max() <= tol * np.abs(o2v).max(), branch
        c3v = DV.imag / k ** 3
        assert np.abs(c3v - o3v).max() <= 1e-2 * np.abs(o3v).max(), branch
