"""Pins for the oracle's mesh and basis-function classification (Section II-C)."""

import dataclasses

import numpy as np
import pytest

from oracle import geometry
from synth import bernoulli_map, get_spec


def per_layer(nx, ny):
    return nx * ny + (nx - 1) * ny + nx * (ny - 1)


def test_closed_form_counts():
    # one RWG function per interior edge of a two-triangle-per-pixel grid
    assert per_layer(8, 8) == 176
    assert 2 * per_layer(20, 20) == 2320
    assert 3 * per_layer(24, 24) == 5040
    assert 3 * per_layer(32, 32) == 9024


@pytest.mark.parametrize("name", ["plain8", "tiny3", "tiny4x2", "small6x3", "batched20", "stress24"])
def test_parent_size(name):
    spec = get_spec(name)
    st = geometry.build_structure(spec)
    assert st.M == geometry.expected_count(spec)
    # the parent size of the workloads
    want = {"plain8": 184, "batched20": 2371, "stress24": 5052}
    if name in want:
        assert st.M == want[name]


@pytest.mark.parametrize("name,seed", [("plain8", 5), ("tiny4x2", 7), ("tiny4x2", 8), ("small6x3", 9)])
def test_classification_equals_fresh_mesh(name, seed):
    """The functions the classification rule switches on are exactly the RWG
    functions of a mesh built from the metal alone."""
    spec = get_spec(name)
    st = geometry.build_structure(spec)
    for p in (0.3, 0.5, 0.8):
        pm = bernoulli_map(spec.n_cells, p, seed)
        act = st.active(pm)
        per_edge = {}
        for bf, on in zip(st.bfs, act):
            if on:
                e = tuple(sorted(bf.edge))
                per_edge[e] = per_edge.get(e, 0) + 1
        assert per_edge == geometry.fresh_submesh_edges(st, pm)


def test_all_on_is_parent_and_all_off_is_feeds():
    spec = get_spec("tiny4x2")
    st = geometry.build_structure(spec)
    assert st.active(np.ones(spec.n_cells)).all()
    off = st.active(np.zeros(spec.n_cells))
    kinds = np.array([b.kind for b in st.bfs])
    assert (off == (kinds == geometry.KIND_ALWAYS)).all()
    assert off.sum() == 3 * len(spec.ports)


def test_diagonal_contact_is_isolated():
    """Two pixels touching only at a corner share no basis function
    (Section VI-A, over-etch reading)."""
    spec = dataclasses.replace(get_spec("tiny3"), ports=())
    st = geometry.build_structure(spec)
    for a, b in [((0, 0), (1, 1)), ((1, 0), (0, 1)), ((1, 1), (2, 2)), ((2, 1), (1, 2))]:
        pm = np.zeros(spec.n_cells, dtype=np.uint8)
        ca, cb = st.cell_index(0, *a), st.cell_index(0, *b)
        pm[ca] = pm[cb] = 1
        act = st.active(pm)
        on = [bf for bf, x in zip(st.bfs, act) if x]
        assert all(bf.kind == geometry.KIND_INNER for bf in on)
        assert len(on) == 2


def test_canonical_order_ports_last():
    spec = get_spec("tiny4x2")
    st = geometry.build_structure(spec)
    P = len(spec.ports)
    assert st.port_bf == list(range(st.M - P, st.M))
    kinds = [b.kind for b in st.bfs]
    # inner, inter, pixel-port, via, always-present: non-decreasing blocks in that order
    order = {geometry.KIND_INNER: 0, geometry.KIND_INTER: 1, geometry.KIND_PIXPORT: 2, geometry.KIND_VIA: 3,
             geometry.KIND_ALWAYS: 4}
    ranks = [order[k] for k in kinds]
    assert ranks == sorted(ranks)


def test_rwg_edges_are_shared():
    spec = get_spec("tiny4x2")
    st = geometry.build_structure(spec)
    length, tri, free = geometry.rwg_geometry(st)
    assert np.all(length > 0)
    assert np.all(tri[:, 0] != tri[:, 1])
    # port edges have length a; vias add vertical triangles
    assert np.allclose(length[st.port_bf], spec.a)


# ---------------------------------------------------------------- 8- and 18-triangle meshes


def test_closed_form_counts_of_subdivided_pixels():
    # one pixel cut into s x s squares, each into two right triangles: s^2
    # diagonals and 2 s (s - 1) sides between squares are interior edges
    for s, inner in ((1, 1), (2, 8), (3, 21)):
        spec = dataclasses.replace(get_spec("tiny3"), nx=1, ny=1, ports=(), sub=s)
        assert geometry.build_structure(spec).M == inner
        assert len(geometry.build_structure(spec).tri_keys) == 2 * s * s
    # two pixels side by side share s edges
    spec = dataclasses.replace(get_spec("tiny3"), nx=2, ny=1, ports=(), sub=2)
    assert geometry.build_structure(spec).M == 2 * 8 + 2
    # the paper-size stripline parent: 2 layers of 30 x 30 pixels, 8 triangles
    # per pixel: 2 x (900 x 8 + 2 x 2 x 29 x 30) + 3 ports x 4 + 13 vias x 7
    assert geometry.expected_count(get_spec("paper30")) == 21463


@pytest.mark.parametrize("name", ["tiny4x2s2", "tiny3s3", "mesh8"])
def test_subdivided_parent_size(name):
    spec = get_spec(name)
    st = geometry.build_structure(spec)
    assert st.M == geometry.expected_count(spec)
    # the squares tile every pixel: triangle areas per pixel sum to a^2
    tx = st.tri_xyz()
    area = 0.5 * np.linalg.norm(np.cross(tx[:, 1] - tx[:, 0], tx[:, 2] - tx[:, 0]), axis=1)
    per_cell = np.zeros(spec.n_cells)
    for t, own in enumerate(st.tri_owner):
        if own[0] == "cell":
            per_cell[own[1]] += area[t]
    assert np.allclose(per_cell, spec.a ** 2, rtol=1e-12)
    length, tri, free = geometry.rwg_geometry(st)
    assert np.allclose(length[st.port_bf], spec.a / spec.sub)


@pytest.mark.parametrize("name,seed", [("tiny4x2s2", 7), ("tiny4x2s2", 8), ("tiny3s3", 9), ("mesh8", 10)])
def test_subdivided_classification_equals_fresh_mesh(name, seed):
    """With 8 or 18 triangles per pixel the classification rule still
    switches on exactly the RWG functions of a mesh built from the metal
    alone (vias and feeds included)."""
    spec = get_spec(name)
    st = geometry.build_structure(spec)
    for p in (0.3, 0.5, 0.8, 1.0):
        pm = bernoulli_map(spec.n_cells, p, seed)
        act = st.active(pm)
        per_edge = {}
        for bf, on in zip(st.bfs, act):
            if on:
                e = tuple(sorted(bf.edge))
                per_edge[e] = per_edge.get(e, 0) + 1
        assert per_edge == geometry.fresh_submesh_edges(st, pm)


def test_subdivided_diagonal_contact_is_isolated():
    spec = dataclasses.replace(get_spec("tiny3"), ports=(), sub=2)
    st = geometry.build_structure(spec)
    pm = np.zeros(spec.n_cells, dtype=np.uint8)
    pm[st.cell_index(0, 0, 0)] = pm[st.cell_index(0, 1, 1)] = 1
    on = [bf for bf, x in zip(st.bfs, st.active(pm)) if x]
    assert len(on) == 16 and all(bf.kind == geometry.KIND_INNER for bf in on)
