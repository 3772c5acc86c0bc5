"""Pins for the oracle's selection (Eqs. 3-5), solve (Eq. 2) and S (Eqs. 6-7)."""

import numpy as np
import pytest

from oracle import efie, geometry, network, search
from synth import bernoulli_map, get_spec


def rand_sym(n, seed):
    g = np.random.default_rng(seed)
    A = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
    return A + A.T


def test_pure_port_network_closed_form():
    """Every unknown a port with l = 1: Eq. 6 must give S = (Z - Z0)(Z + Z0)^-1."""
    z0 = 50.0
    for P, seed in ((1, 0), (2, 1), (3, 2), (5, 3)):
        Z = 40.0 * rand_sym(P, seed) + 80.0 * np.eye(P)
        S = network.s_parameters(Z, list(range(P)), np.ones(P), z0)
        ref = (Z - z0 * np.eye(P)) @ np.linalg.inv(Z + z0 * np.eye(P))
        assert np.abs(S - ref).max() <= 1e-13


@pytest.mark.parametrize("zin,want", [(50.0, 0.0), (1e14, 1.0), (1e-14, -1.0)])
def test_one_port_matched_open_short(zin, want):
    S = network.s_parameters(np.array([[zin + 0j]]), [0], [1.0], 50.0)
    assert abs(S[0, 0] - want) <= 1e-12


def test_port_length_scaling():
    """A port function of edge length l with Z_pp = l^2 z acts as impedance z."""
    l, z = 2.5e-3, 37.0 - 12.0j
    S = network.s_parameters(np.array([[l * l * z]]), [0], [l], 50.0)
    assert abs(S[0, 0] - (z - 50.0) / (z + 50.0)) <= 1e-13


def test_selection_literal_equals_index():
    g = np.random.default_rng(4)
    Z = rand_sym(40, 5)
    sel = g.random(40) < 0.4
    assert np.array_equal(network.reduce_matrix(Z, sel), network.reduce_matrix_literal(Z, sel))
    S = network.selection_matrix(sel)
    assert np.array_equal(S.sum(axis=0), np.ones(sel.sum()))
    idx = network.support(sel)
    assert np.all(np.diff(idx) > 0)


def _setup(name, f_idx=1, p=0.5, seed=None):
    spec = get_spec(name)
    st = geometry.build_structure(spec)
    pm = bernoulli_map(spec.n_cells, p, spec.seed if seed is None else seed)
    Z = efie.fill(st, spec.freqs[f_idx])
    sel = st.active(pm)
    rows = network.port_positions(sel, st.port_bf)
    pl = search.port_lengths(st)
    return spec, st, Z, sel, rows, pl


@pytest.mark.parametrize("name", ["plain8", "tiny4x2", "small6x3"])
def test_mom_s_invariants(name):
    spec, st, Z, sel, rows, pl = _setup(name)
    Zs = network.reduce_matrix(Z, sel)
    S = network.s_parameters(Zs, rows, pl, spec.z0)
    S2 = network.s_parameters_admittance(Zs, rows, pl, spec.z0)
    assert np.abs(S - S2).max() <= 1e-12  # two routes
    assert np.abs(S - S.T).max() <= 1e-12  # reciprocity (Z symmetric)
    sv = np.linalg.svd(S, compute_uv=False)
    assert sv.max() <= 1.0 + 1e-8  # passivity
    assert np.abs(S).max() <= 1.0 + 1e-8


@pytest.mark.parametrize("name", ["plain8", "tiny4x2"])
def test_gather_equals_fresh_assembly(name):
    """Eq. 5 from the parent is bitwise the matrix of the substructure itself."""
    spec, st, Z, sel, rows, pl = _setup(name)
    idx = network.support(sel)
    Zf = efie.fill(st, spec.freqs[1], bf_subset=idx)
    assert np.array_equal(Zf, network.reduce_matrix(Z, sel))


def test_lu_solve_backward_error():
    spec, st, Z, sel, rows, pl = _setup("plain8")
    Zs = network.reduce_matrix(Z, sel)
    V = network.excitation(len(Zs), rows, pl)
    X = np.linalg.solve(Zs, V)
    err = np.linalg.norm(Zs @ X - V) / (np.linalg.norm(Zs) * np.linalg.norm(X))
    assert err <= 1e-14
    Xi = np.linalg.inv(Zs) @ V
    assert np.abs(X - Xi).max() <= 1e-9 * np.abs(X).max()
