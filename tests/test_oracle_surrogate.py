"""Pins of the surrogate oracle: finite differences, closed forms, special
cases (CPU)."""

import numpy as np
import pytest

from oracle import surrogate as osur
from synth import uniform_array

from sur_common import init_params, random_maps

CFG = osur.SurrogateConfig(n_layers=2, ny=6, nx=5, channels=(3, 4, 5, 6), hidden=7, emb=4, n_out=4)


def test_layout_counts():
    c = (2, 3, 4, 5, 6)
    conv = sum(9 * c[i] * c[i + 1] + c[i + 1] for i in range(4))
    D = (6 // 4) * (5 // 4) * 6
    assert osur.n_params(CFG) == conv + D * 7 + 4 * 7 + 7 + 7 * 4 + 4
    p = np.arange(osur.n_params(CFG), dtype=float)
    assert np.array_equal(osur.pack(osur.unpack(p, CFG), CFG), p)


def test_identity_convolution_reproduces_input():
    X = uniform_array(2 * 4 * 5 * 3, 3, 1.0).reshape(2, 4, 5, 3)
    W = np.zeros((9, 3, 3))
    W[4] = np.eye(3)  # centre tap
    assert np.array_equal(osur.conv3x3(X, W, np.zeros(3)), X)
    # a pure shift: tap (dy, dx) = (0, 1) reads the row above
    W = np.zeros((9, 3, 3))
    W[1] = np.eye(3)
    Y = osur.conv3x3(X, W, np.zeros(3))
    assert np.array_equal(Y[:, 1:], X[:, :-1]) and np.all(Y[:, 0] == 0)


def test_convolution_against_direct_sum():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((1, 4, 3, 2))
    W = rng.standard_normal((9, 2, 3))
    b = rng.standard_normal(3)
    Y = osur.conv3x3(X, W, b)
    for y in range(4):
        for x in range(3):
            for o in range(3):
                s = b[o]
                for dy in range(3):
                    for dx in range(3):
                        yy, xx = y + dy - 1, x + dx - 1
                        if 0 <= yy < 4 and 0 <= xx < 3:
                            s += sum(X[0, yy, xx, i] * W[3 * dy + dx, i, o] for i in range(2))
                assert abs(Y[0, y, x, o] - s) < 1e-12


def test_pool_of_constant_and_odd_edges():
    X = np.full((1, 5, 7, 2), 3.5)
    P = osur.pool2(X)
    assert P.shape == (1, 2, 3, 2) and np.all(P == 3.5)
    X = np.zeros((1, 3, 3, 1))
    X[0, 2, :, 0] = 100.0  # dropped row
    assert np.all(osur.pool2(X) == 0)


def test_embedding_values():
    e = osur.embedding(np.array([0.0, 0.5, 1.0]), 4)
    assert np.allclose(e[0], [0, 1, 0, 1])
    assert np.allclose(e[1], [1, 0, 0, -1], atol=1e-15)
    assert np.allclose(e[2], [0, -1, 0, 1], atol=1e-15)


def test_zero_trunk_gives_map_independent_output():
    p = osur.unpack(init_params(CFG, 5), CFG)
    for i in range(1, 5):
        p[f"W{i}"][:] = 0
        p[f"b{i}"][:] = 0
    params = osur.pack(p, CFG)
    u = np.array([0.1, 0.7])
    maps = random_maps(3, 2 * 6 * 5, 1)
    out, _ = osur.forward(params, maps, u, CFG)
    e = osur.embedding(u, 4)
    want = np.maximum(e @ p["We"] + p["bh"], 0) @ p["Wo"] + p["bo"]
    for b in range(3):
        assert np.allclose(out[b], want, rtol=0, atol=1e-14)


def test_gradient_matches_central_differences():
    params = init_params(CFG, 7)
    maps = random_maps(3, 2 * 6 * 5, 2)
    u = np.array([0.0, 0.3, 0.9])
    target = uniform_array(3 * 3 * 4, 9, 1.0).reshape(3, 3, 4)
    L, g = osur.gradient(params, maps, u, target, CFG)
    idx = np.unique(np.concatenate([np.linspace(0, len(params) - 1, 40).astype(int),
                                    np.argsort(-np.abs(g))[:20]]))
    h = 1e-6
    for i in idx:
        pp, pm = params.copy(), params.copy()
        pp[i] += h
        pm[i] -= h
        fd = (osur.loss(osur.forward(pp, maps, u, CFG)[0], target) -
              osur.loss(osur.forward(pm, maps, u, CFG)[0], target)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-10, (i, fd, g[i])


def test_adamw_first_step_closed_form():
    rng = np.random.default_rng(1)
    p, g = rng.standard_normal(10), rng.standard_normal(10)
    lr, wd, eps = 1e-2, 0.1, 1e-8
    p1, m, v = osur.adamw_step(p, g, np.zeros(10), np.zeros(10), 1, lr, weight_decay=wd, eps=eps)
    # bias correction makes the first moments exactly g and g^2
    assert np.allclose(p1, p - lr * (g / (np.abs(g) + eps) + wd * p), rtol=0, atol=1e-15)
    p2, _, _ = osur.adamw_step(p, np.zeros(10), np.zeros(10), np.zeros(10), 1, lr, weight_decay=wd)
    assert np.allclose(p2, p * (1 - lr * wd), rtol=0, atol=1e-15)
