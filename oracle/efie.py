"""EFIE impedance matrix in RWG functions (oracle fill).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Discretises the EFIE of Eq. 1 into Z I = V (Eq. 2) with RWG functions
(Section II-B).  The paper's MoM engine uses a layered Sommerfeld Green's
function (Section II-D); this oracle uses the homogeneous-medium kernel
G(R) = exp(-jkR) / (4 pi R), time convention exp(+j w t), which is what the
synthetic workloads are built on (free space, or an unbounded lossy
dielectric).

Mixed-potential Galerkin form, for test function f_m and source f_n:

    Z_mn = j w mu  int int f_m(r).f_n(r') G dS' dS
         + 1/(j w eps) int int div f_m(r) div' f_n(r') G dS' dS

with eps = eps0 eps_r (1 - j tan_d), mu = mu0, k = w sqrt(mu eps) on the
principal branch (Im k < 0), and the RWG function on its + / - triangle

    f_n(r) = +- l_n / (2 A) (r - p),   div f_n = +- l_n / A

(p the triangle's free vertex).

Quadrature: the 4-point degree-3 triangle rule (centroid weight -27/48,
points (0.6, 0.2, 0.2) and permutations weight 25/48) on test and source
triangles.  For a pair of triangles whose centroids are closer than twice the
longer of their longest edges, the source integral splits G into
1/(4 pi R), integrated in closed form (``singular``), and the smooth remainder
(exp(-jkR) - 1)/(4 pi R), integrated by the 4-point rule.

Only Z_mn with m <= n is computed; the lower triangle is its mirror, so Z is
exactly symmetric.

Constants: c0 = 299792458 m/s, mu0 = 4 pi 1e-7 H/m, eps0 = 1 / (mu0 c0^2).

Parity: the singular integrals are pinned against Duffy quadrature; the
assembled matrix is pinned by exact symmetry, by a positive semi-definite
Hermitian part in free space (radiated power is non-negative), and through
the S-parameter invariants of ``network``.  Absolute accuracy against the
paper's solver: parity unpinned (its matrices are not published).
"""

from __future__ import annotations

import numpy as np

from .geometry import Structure, rwg_geometry
from .singular import potential_integrals

C0 = 299792458.0
MU0 = 4.0e-7 * np.pi
EPS0 = 1.0 / (MU0 * C0 * C0)

QUAD_BARY = np.array([[1.0 / 3, 1.0 / 3, 1.0 / 3], [0.6, 0.2, 0.2], [0.2, 0.6, 0.2], [0.2, 0.2, 0.6]])
QUAD_W = np.array([-27.0 / 48, 25.0 / 48, 25.0 / 48, 25.0 / 48])
NEAR_FACTOR = 2.0


def wavenumber(freq: float, eps_r: float, tan_d: float):
    w = 2.0 * np.pi * freq
    eps = EPS0 * eps_r * (1.0 - 1j * tan_d)
    k = w * np.sqrt(MU0 * eps + 0j)
    return w, eps, k


class TriangleData:
    def __init__(self, tri_xyz: np.ndarray):
        self.xyz = tri_xyz  # (T, 3, 3)
        e = [tri_xyz[:, 1] - tri_xyz[:, 0], tri_xyz[:, 2] - tri_xyz[:, 1], tri_xyz[:, 0] - tri_xyz[:, 2]]
        self.area = 0.5 * np.linalg.norm(np.cross(e[0], -e[2]), axis=-1)
        self.centroid = tri_xyz.mean(axis=1)
        self.maxedge = np.max(np.stack([np.linalg.norm(x, axis=-1) for x in e]), axis=0)
        self.qp = np.einsum("qv,tvd->tqd", QUAD_BARY, tri_xyz)  # (T, 4, 3)


def near_pairs(td: TriangleData, tp: np.ndarray, tq: np.ndarray) -> np.ndarray:
    """Boolean mask: centroids closer than NEAR_FACTOR times the longer max edge.

    A relative slack of 1e-9 keeps grid-exact ties on the near side."""
    d = np.linalg.norm(td.centroid[tp][:, None] - td.centroid[tq][None, :], axis=-1)
    lim = NEAR_FACTOR * np.maximum(td.maxedge[tp][:, None], td.maxedge[tq][None, :])
    return d < lim * (1.0 + 1e-9)


def source_integrals(td: TriangleData, tp: np.ndarray, tq: np.ndarray, k: complex):
    """For test triangles tp (P) and source triangles tq (Q) return, at each
    test quadrature point r_i of each test triangle,

        SS[p, q, i]    = int over T_q of G(r_i, r') dS'
        SV[p, q, i, :] = int over T_q of (r' - c_q) G(r_i, r') dS'

    with c_q the source centroid."""
    rp = td.qp[tp]  # (P, 4, 3)
    rq = td.qp[tq]  # (Q, 4, 3)
    diff = rp[:, None, :, None, :] - rq[None, :, None, :, :]  # (P, Q, 4, 4, 3)
    R = np.sqrt(np.einsum("pqijd,pqijd->pqij", diff, diff))
    near = near_pairs(td, tp, tq)  # (P, Q)
    with np.errstate(divide="ignore", invalid="ignore"):
        full = np.exp(-1j * k * R) / (4 * np.pi * R)  # far pairs: whole kernel
    ip, iq = np.nonzero(near)
    if len(ip):
        Rn = R[ip, iq]  # (K, 4, 4)
        kR = k * Rn
        x = -1j * kR
        small = np.abs(kR) < 1e-3
        em1 = np.where(small, x * (1 + x / 2 * (1 + x / 3 * (1 + x / 4))), np.exp(x) - 1.0)
        Rs = np.where(Rn > 0.0, Rn, 1.0)
        # near pairs: only the smooth part (exp(-jkR) - 1)/(4 pi R) by quadrature
        full[ip, iq] = np.where(Rn > 0.0, em1 / Rs, -1j * k) / (4 * np.pi)
    Aq = td.area[tq][None, :, None]
    fw = full * QUAD_W  # weight over source points j
    SS = Aq * fw.sum(axis=-1)
    rel = rq - td.centroid[tq][:, None, :]  # (Q, 4, 3)
    SV = Aq[..., None] * np.einsum("pqij,qjd->pqid", fw, rel, optimize=True)
    if len(ip):
        tri = td.xyz[tq[iq]][:, None]  # (K, 1, 3, 3)
        obs = rp[ip]  # (K, 4, 3)
        I1, Irho = potential_integrals(np.broadcast_to(tri, (len(ip), 4, 3, 3)), obs)
        # projection of r_i onto the source plane
        v = td.xyz[tq[iq]]
        n = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
        n /= np.linalg.norm(n, axis=-1, keepdims=True)
        dist = np.einsum("kid,kd->ki", obs - v[:, None, 0], n)
        rho = obs - dist[..., None] * n[:, None, :]
        cq = td.centroid[tq[iq]][:, None, :]
        SS[ip, iq] += I1 / (4 * np.pi)
        SV[ip, iq] += (Irho + (rho - cq) * I1[..., None]) / (4 * np.pi)
    return SS, SV


def fill(struct: Structure, freq: float, bf_subset=None, chunk: int = 128, part: str = "both") -> np.ndarray:
    """Impedance matrix (M x M, or N x N over ``bf_subset``) at one frequency.

    ``part`` keeps only the vector-potential (\"vector\") or scalar-potential
    (\"scalar\") term; used by tests to pin each term on its own."""
    spec = struct.spec
    w, eps, k = wavenumber(freq, spec.eps_r, spec.tan_d)
    length, tri, free = rwg_geometry(struct)
    bfs = np.arange(struct.M) if bf_subset is None else np.asarray(bf_subset)
    length, tri, free = length[bfs], tri[bfs], free[bfs]
    N = len(bfs)
    td = TriangleData(struct.tri_xyz())
    used = np.unique(tri)
    pos = -np.ones(len(td.area), dtype=np.int64)
    pos[used] = np.arange(len(used))
    # source integrals for every (test, source) pair of triangles in use
    SS = np.empty((len(used), len(used), 4), dtype=np.complex128)
    SV = np.empty((len(used), len(used), 4, 3), dtype=np.complex128)
    for p0 in range(0, len(used), chunk):
        SS[p0:p0 + chunk], SV[p0:p0 + chunk] = source_integrals(td, used[p0:p0 + chunk], used, k)
    sign = np.array([1.0, -1.0])
    jwmu4 = (1j * w * MU0 / 4.0) if part in ("both", "vector") else 0.0
    inv_jweps = (1.0 / (1j * w * eps)) if part in ("both", "scalar") else 0.0
    Z = np.zeros((N, N), dtype=np.complex128)
    for m0 in range(0, N, chunk):
        rows = np.arange(m0, min(N, m0 + chunk))
        block = np.zeros((len(rows), N), dtype=np.complex128)
        for a in range(2):  # test triangle: + then -
            tm = tri[rows, a]
            rt = td.qp[tm] - free[rows, a][:, None, :]  # (m, 4, 3): r_i - p_m
            for b in range(2):  # source triangle: + then -
                tn = tri[:, b]
                ss = SS[pos[tm][:, None], pos[tn][None, :]]  # (m, N, 4)
                sv = SV[pos[tm][:, None], pos[tn][None, :]]  # (m, N, 4, 3)
                off = free[:, b] - td.centroid[tn]  # (N, 3): p_n - c_n
                # (r_i - p_m) . int (r' - p_n) G  =  (r_i - p_m).SV - ((r_i - p_m).(p_n - c_n)) SS
                dot = np.einsum("mid,mnid->mni", rt, sv, optimize=True) - np.einsum(
                    "mid,nd->mni", rt, off, optimize=True) * ss
                term = (jwmu4 * dot + inv_jweps * ss) @ QUAD_W
                coef = sign[a] * sign[b] * length[rows][:, None] * length[None, :] / td.area[tn][None, :]
                block += coef * term
        Z[rows] = block
    iu = np.triu_indices(N, 1)
    Z[(iu[1], iu[0])] = Z[iu]
    return Z
