"""Candidate sweep and accept rule (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Algorithm 1 evaluates every child of a node, takes the argmin of F over the
children and accepts it only if it is strictly lower than the current F.  A
single-flip sweep is the depth-1, two-state case: each child toggles one
pixel.  Ties go to the lowest candidate index.

``sweep`` evaluates each candidate by the gather of Eq. 5 from a parent
matrix stack; ``evaluate_fresh`` assembles the candidate's own matrix from
scratch, which is the plain definition the gather must reproduce.

Parity: pinned by brute force over every map of a 3x3 grid
(tests/test_oracle_search.py).
"""

from __future__ import annotations

import numpy as np

from . import efie, fom as fom_mod, network
from .geometry import Structure, rwg_geometry


def apply_flips(base_map, cells) -> np.ndarray:
    m = np.asarray(base_map).astype(np.uint8).copy()
    for c in cells:
        m[c] ^= 1
    return m


def candidate_maps(base_map, offsets, cells):
    return [apply_flips(base_map, cells[offsets[c]:offsets[c + 1]]) for c in range(len(offsets) - 1)]


def port_lengths(struct: Structure) -> np.ndarray:
    length, _, _ = rwg_geometry(struct)
    return length[struct.port_bf]


def evaluate_gather(struct: Structure, Z_parent_f: np.ndarray, pixel_map, freqs):
    """S (F, P, P) and FoM of one map from the parent stack (Eq. 5 route)."""
    sel = struct.active(pixel_map)
    S = network.s_batch(Z_parent_f, sel, struct.port_bf, port_lengths(struct), struct.spec.z0)
    return S, fom_mod.fom(S, freqs)


def evaluate_fresh(struct: Structure, pixel_map, freqs):
    """S (F, P, P) and FoM of one map by assembling its own matrix."""
    sel = struct.active(pixel_map)
    idx = network.support(sel)
    rows = network.port_positions(sel, struct.port_bf)
    pl = port_lengths(struct)
    S = np.stack([
        network.s_parameters(efie.fill(struct, f, bf_subset=idx), rows, pl, struct.spec.z0) for f in freqs
    ])
    return S, fom_mod.fom(S, freqs)


def sweep(struct: Structure, Z_parent_f, base_map, offsets, cells, freqs):
    """Evaluate every candidate; returns (S (C, F, P, P), FoM (C,))."""
    out_S, out_F = [], []
    for m in candidate_maps(base_map, offsets, cells):
        S, F = evaluate_gather(struct, Z_parent_f, m, freqs)
        out_S.append(S)
        out_F.append(F)
    return np.stack(out_S), np.array(out_F)


def argmin_lowest(values) -> int:
    v = np.asarray(values)
    best = 0
    for i in range(1, len(v)):
        if v[i] < v[best]:
            best = i
    return best


def accept(current_fom: float, candidate_foms) -> tuple:
    """(index, accepted): argmin with ties to the lowest index, accepted only on
    strict improvement."""
    i = argmin_lowest(candidate_foms)
    return i, bool(candidate_foms[i] < current_fom)


# ---------------------------------------------------------------- Algorithm 1

def pixel_state(pixel_map, n_layers: int, n_pix: int, j: int) -> int:
    """Multi-state pixel (Section II-D, Fig. 4): the pixel at in-plane position j
    stacked over the layers, bit l set when layer l is metal there."""
    return sum(int(pixel_map[l * n_pix + j]) << l for l in range(n_layers))


def with_state(pixel_map, n_layers: int, n_pix: int, j: int, state: int) -> np.ndarray:
    m = np.array(pixel_map, dtype=np.uint8).copy()
    for l in range(n_layers):
        m[l * n_pix + j] = (state >> l) & 1
    return m


def tree_search(evaluate, start_map, n_layers: int, n_pix: int, pixel_order, restart_maps, max_evals: int,
                d_init: int = 1, d_max: int = 2, m_of_depth=(10, 3)):
    """Depth-increasing all-way tree navigation (Algorithm 1).

    evaluate(map) -> FoM of one map.  pixel_order: in-plane pixel indices taken
    in turn (cycled) for the tree levels; restart_maps: iterator of random maps
    for the restarts.  Readings: every node of one depth expands the same
    pixel; the restart happens when the non-improvement count saturates at the
    deepest depth; the budget counts every F evaluated.
    Returns (best FoM, best map, evaluations, trace of (evaluations, FoM of
    the current state) after each iteration, number of restarts)."""
    n_states = 1 << n_layers
    P = np.array(start_map, dtype=np.uint8)
    F = evaluate(P)
    evals = 1
    best_F, best_P = F, P.copy()
    D, count, restarts, cursor = d_init, 0, 0, 0
    trace = []
    while evals < max_evals:
        # the D pixels of this tree, distinct, in the given order
        path = []
        while len(path) < D:
            j = int(pixel_order[cursor % len(pixel_order)])
            cursor += 1
            if j not in path:
                path.append(j)
        level = [P]
        for j in path:
            children = []
            for parent in level:
                s = pixel_state(parent, n_layers, n_pix, j)
                for t in range(n_states):
                    if t != s:
                        children.append(with_state(parent, n_layers, n_pix, j, t))
            values = [evaluate(c) for c in children]
            evals += len(children)
            level, level_F = children, values
        k = argmin_lowest(level_F)
        if level_F[k] < F:
            P, F = level[k], level_F[k]
            count = 0
            if F < best_F:
                best_F, best_P = F, P.copy()
        else:
            count += 1
            if count >= m_of_depth[D - 1]:
                count = 0
                if D >= d_max:  # saturated at the deepest depth: restart
                    P = np.array(next(restart_maps), dtype=np.uint8)
                    F = evaluate(P)
                    evals += 1
                    if F < best_F:
                        best_F, best_P = F, P.copy()
                    D = d_init
                    restarts += 1
                else:
                    D += 1
        trace.append((evals, F))
    return best_F, best_P, evals, trace, restarts
