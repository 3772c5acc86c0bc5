"""Selection, dense solve and S-parameters (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* Eq. 3: the support set I = {i : (S_sub)_i = 1}, ascending.
* Eq. 4: the selection matrix (S_mat)_{m,n} = delta(m, i_n), M x N.
* Eq. 5: Z_sub = S_mat^T Z_parent S_mat.
* Eq. 2: Z I = V, solved by LU with partial pivoting (LAPACK zgesv through
  numpy.linalg.solve).
* Eqs. 6-7: S(i, j) = delta_ij - 2 Z0 I_i / V_j with I_i = l_i * i_i.

Reading of Eq. 6 used here (the paper names V_j "the voltage incident into
port j" and attributes the factor 2 to voltage division): every port is a
delta gap loaded by Z0 in series, so Z0 * l_p^2 is added to the port
function's diagonal entry, and the excitation of port j is a 1 V source EMF in
that gap, giving V = l_p at the port row.  With a_j = V_j / (2 sqrt Z0) and
b_i = (delta_ij V_j - 2 Z0 I_i) / (2 sqrt Z0), S_ij = b_i / a_j is exactly
Eq. 6.  Port current is positive into the structure.

A second route, used as a pin: solve the unloaded system with the same
excitations, read the short-circuit admittance Y_ij = l_i i_i^(j), and form
S = (I - Z0 Y)(I + Z0 Y)^-1.

Parity: pinned by the closed form on a pure port network, by reciprocity,
passivity, the agreement of the two routes, and by bitwise equality of the
gathered and freshly assembled sub-matrices (tests/test_oracle_network.py).
"""

from __future__ import annotations

import numpy as np


def support(selection: np.ndarray) -> np.ndarray:
    """Eq. 3: ascending indices of the selected basis functions."""
    return np.nonzero(np.asarray(selection).astype(bool))[0]


def selection_matrix(selection: np.ndarray) -> np.ndarray:
    """Eq. 4: M x N matrix with a single 1 per column at row i_n."""
    idx = support(selection)
    S = np.zeros((len(selection), len(idx)))
    S[idx, np.arange(len(idx))] = 1.0
    return S


def reduce_matrix(Z_parent: np.ndarray, selection: np.ndarray) -> np.ndarray:
    """Eq. 5 by index selection (rows and columns i_1 < ... < i_N)."""
    idx = support(selection)
    return Z_parent[np.ix_(idx, idx)]


def reduce_matrix_literal(Z_parent: np.ndarray, selection: np.ndarray) -> np.ndarray:
    """Eq. 5 as written, S_mat^T Z S_mat (slow; used to pin ``reduce_matrix``)."""
    S = selection_matrix(selection)
    return S.T @ Z_parent @ S


def port_positions(selection: np.ndarray, port_bf) -> np.ndarray:
    """Row of each port function inside the reduced system."""
    idx = support(selection)
    where = {int(m): n for n, m in enumerate(idx)}
    return np.array([where[int(p)] for p in port_bf])


def excitation(N: int, port_rows, port_len) -> np.ndarray:
    """V (N x P): 1 V source EMF in the gap of port j, V[row_j, j] = l_j."""
    V = np.zeros((N, len(port_rows)), dtype=np.complex128)
    for j, (r, l) in enumerate(zip(port_rows, port_len)):
        V[r, j] = l
    return V


def s_parameters(Z_sub: np.ndarray, port_rows, port_len, z0: float) -> np.ndarray:
    """Eqs. 6-7 with Z0-loaded ports.  Returns S (P x P, complex128)."""
    Zl = Z_sub.astype(np.complex128).copy()
    for r, l in zip(port_rows, port_len):
        Zl[r, r] += z0 * l * l
    V = excitation(len(Zl), port_rows, port_len)
    X = np.linalg.solve(Zl, V)
    P = len(port_rows)
    S = np.zeros((P, P), dtype=np.complex128)
    for i in range(P):
        I_i = port_len[i] * X[port_rows[i], :]  # Eq. 7, one entry per excitation j
        for j in range(P):
            S[i, j] = (1.0 if i == j else 0.0) - 2.0 * z0 * I_i[j] / 1.0  # Eq. 6, V_j = 1 V
    return S


def s_parameters_admittance(Z_sub: np.ndarray, port_rows, port_len, z0: float) -> np.ndarray:
    """Second route: unloaded solve, Y_ij = l_i i_i^(j), S = (I - Z0 Y)(I + Z0 Y)^-1."""
    V = excitation(len(Z_sub), port_rows, port_len)
    X = np.linalg.solve(Z_sub, V)
    P = len(port_rows)
    Y = np.array([[port_len[i] * X[port_rows[i], j] for j in range(P)] for i in range(P)])
    I = np.eye(P)
    return (I - z0 * Y) @ np.linalg.inv(I + z0 * Y)


def s_batch(Z_parent_f: np.ndarray, selection: np.ndarray, port_bf, port_len, z0: float) -> np.ndarray:
    """S over a stack of frequencies: Z_parent_f (F, M, M) -> (F, P, P)."""
    rows = port_positions(selection, port_bf)
    return np.stack([s_parameters(reduce_matrix(Z, selection), rows, port_len, z0) for Z in Z_parent_f])
