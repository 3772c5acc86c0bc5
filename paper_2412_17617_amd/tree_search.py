"""Depth-increasing all-way tree navigation (Algorithm 1) on the GPU evaluator.

The search state is a multi-state pixel map: the pixel at in-plane position j
stacked over the L layers takes one of 2^L states (bit l = metal on layer l,
Section II-D, Fig. 4).  One iteration builds the tree of depth D below the
current map: D distinct pixels (taken in turn from a caller-given order), and
for each level every other state of that level's pixel applied to every node
of the level above.  All nodes of all levels are candidate maps differing from
the root in at most D pixels, so the whole tree is one flip batch and one
persistent launch of the evaluator.  The best leaf of the deepest level is
accepted only if it improves strictly; M(D) failures raise D, and saturation
at the deepest depth restarts from a random map (caller-given).

Readings where the algorithm is silent: all nodes of one depth expand the same
pixel; the restart happens when the count saturates at the deepest depth; the
evaluation budget counts every candidate evaluated.  Optionally a surrogate
(``Surrogate``) ranks the deepest level and only its best k leaves are solved;
the exact evaluator still judges every accepted change and, when none of
those k leaves improves, solves the rest of the level before the iteration
counts as a failure.  Candidates with a failed solve (negative status) are
never selected.  Solving the trees
by the low-rank flip evaluation from the current map's inverse (``lowrank``)
is switched off: its one GPU run inside this driver made a memory fault
whose cause has not been shown, so the option raises.

Also here: steepest descent over a fixed move set (single and pair flips),
exhaustive or pruned by a ranker with the exact fallback (``descent``), and
the classical one-pixel-at-a-time direct binary search (``sequential_dbs``).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class SearchResult:
    best_fom: float
    best_map: np.ndarray
    evaluations: int
    trace: list = field(default_factory=list)  # (evaluations, current FoM) after each tree
    restarts: int = 0
    accepted: int = 0


class TreeSearch:
    def __init__(self, evaluator, n_layers: int, n_pix: int, d_init: int = 1, d_max: int = 2, m_of_depth=(10, 3),
                 lowrank: bool = False):
        if not (1 <= d_init <= d_max) or len(m_of_depth) < d_max:
            raise ValueError("need 1 <= d_init <= d_max and one M(D) per depth")
        if lowrank:
            raise NotImplementedError("low-rank evaluation inside the tree search is switched off: its only GPU run "
                                      "made a memory fault whose cause has not been shown")
        self.ev = evaluator
        self._eval = evaluator.evaluate_flips
        self.L, self.n_pix = n_layers, n_pix
        self.d_init, self.d_max, self.m = d_init, d_max, tuple(m_of_depth)

    def _tree(self, P, path):
        """Flip lists (CSR, relative to P) of every node below P, level by
        level, and the slice of the deepest level."""
        L, n = self.L, self.n_pix
        Pl = P.reshape(L, n)
        nodes = [np.zeros(0, np.int32)]  # cells toggled relative to P
        offs, cells, start = [0], [], 0
        for j in path:
            s = int(sum(int(Pl[l, j]) << l for l in range(L)))
            nxt = []
            for flips in nodes:
                for t in range(1 << L):
                    if t == s:
                        continue
                    diff = s ^ t
                    cj = np.array([l * n + j for l in range(L) if (diff >> l) & 1], np.int32)
                    nxt.append(np.concatenate([flips, cj]))
            start = len(offs) - 1
            for f in nxt:
                cells.append(f)
                offs.append(offs[-1] + len(f))
            nodes = nxt
        cells = np.concatenate(cells).astype(np.int32) if cells else np.zeros(0, np.int32)
        return np.asarray(offs, np.int32), cells, start, len(offs) - 1

    @staticmethod
    def _valid(Fc, st):
        """FoM of the evaluated candidates with every failed one (negative
        status: singular, non-finite, outside the size bound) at +inf, so
        that it can neither be the arg min nor be accepted."""
        Fc = np.array(Fc, np.float64)
        Fc[np.asarray(st) < 0] = np.inf
        return Fc

    def _solve_leaves(self, P, offs, cells, idx, res):
        """Exact FoM of the tree nodes idx (flip lists relative to P)."""
        if len(idx) == 0:
            return np.zeros(0)
        sub = np.zeros(len(idx) + 1, np.int32)
        sub[1:] = np.cumsum([offs[i + 1] - offs[i] for i in idx])
        sc = np.concatenate([cells[offs[i]:offs[i + 1]] for i in idx]).astype(np.int32)
        _, Fl, st, _ = self._eval(P, sub, sc, want_S=False)
        res.evaluations += len(idx)
        return self._valid(Fl, st)

    def _fom(self, m):
        _, F, _, _ = self._eval(m, np.array([0, 0], np.int32), np.zeros(0, np.int32), want_S=False)
        return float(F[0])

    def run(self, start_map, pixel_order, restart_maps, max_evals: int, prefilter=None) -> SearchResult:
        """prefilter: None, or (surrogate, k, rank) where rank(surrogate, P,
        offsets, cells) returns the surrogate's predicted FoM of each
        candidate; then only the best k of the deepest level are solved, and
        the rest of that level only when none of those k improves."""
        P = np.array(start_map, np.uint8)
        F = self._fom(P)
        res = SearchResult(F, P.copy(), 1)
        D, count, cursor = self.d_init, 0, 0
        order = np.asarray(pixel_order)
        while res.evaluations < max_evals:
            path = []
            while len(path) < D:
                j = int(order[cursor % len(order)])
                cursor += 1
                if j not in path:
                    path.append(j)
            offs, cells, lo, hi = self._tree(P, path)
            if prefilter is None:
                _, Fc, st, _ = self._eval(P, offs, cells, want_S=False)
                res.evaluations += len(offs) - 1
                leaves = np.arange(lo, hi)
                Fl = self._valid(Fc[lo:hi], st[lo:hi])
            else:
                # the surrogate scores the whole tree; only the deepest level
                # decides, so only its best k leaves are solved exactly
                sur, k, rank = prefilter
                pred = rank(sur, P, offs, cells)[lo:hi]
                order_l = np.argsort(pred, kind="stable") + lo
                pick = order_l[:k]
                Fl = self._solve_leaves(P, offs, cells, pick, res)
                leaves = pick
                if not (np.min(Fl) < F) and len(order_l) > len(pick):
                    # no verified leaf improves: the exact solve stays the
                    # fallback, so the rest of the level is solved before
                    # this iteration counts as a failure
                    rest = order_l[len(pick):]
                    Fl = np.concatenate([Fl, self._solve_leaves(P, offs, cells, rest, res)])
                    leaves = np.concatenate([pick, rest])
            k = int(np.argmin(Fl))  # lowest index among equal minima
            if np.isfinite(Fl[k]) and Fl[k] < F:
                leaf = leaves[k]
                P = P.copy()
                P[cells[offs[leaf]:offs[leaf + 1]]] ^= 1
                F = float(Fl[k])
                count = 0
                res.accepted += 1
                if F < res.best_fom:
                    res.best_fom, res.best_map = F, P.copy()
            else:
                count += 1
                if count >= self.m[D - 1]:
                    count = 0
                    if D >= self.d_max:
                        P = np.array(next(restart_maps), np.uint8)
                        F = self._fom(P)
                        res.evaluations += 1
                        res.restarts += 1
                        if F < res.best_fom:
                            res.best_fom, res.best_map = F, P.copy()
                        D = self.d_init
                    else:
                        D += 1
            res.trace.append((res.evaluations, F))
        return res


# ---------------------------------------------------------------- descent and DBS


@dataclass
class DescentResult:
    fom: float
    best_map: np.ndarray
    exact_solves: int
    trace: list = field(default_factory=list)  # per step: (seconds, exact solves, FoM, how the step ended)
    start_fom: float = np.inf


def _subset(offs, cells, idx):
    sub = np.zeros(len(idx) + 1, np.int32)
    sub[1:] = np.cumsum([offs[i + 1] - offs[i] for i in idx])
    sc = np.concatenate([cells[offs[i]:offs[i + 1]] for i in idx]).astype(np.int32) if len(idx) else \
        np.zeros(0, np.int32)
    return sub, sc


def descent(evaluator, start_map, offs, cells, max_steps, ranker=None, top_k=32, fallback=None, learn=None,
            clock=None):
    """Steepest descent over a fixed move set (flip lists relative to the
    current map, CSR offs / cells), accepting only strict improvements
    (Algorithm 1's accept rule at depth one, with pair moves when the set
    holds them).

    Exhaustive (ranker None): every move is solved exactly each step.
    Pruned: ranker(map, offs, cells) returns move indices best first; only
    its top_k are solved, and when none of them improves, the moves of
    `fallback` (CSR pair (offs, cells); default: the whole move set) are
    solved before the search stops, so the exact solve stays both the
    judge of every accepted move and the fallback.  learn(maps, S) receives
    every exact solve (candidate maps and their S) for fine-tuning.  Failed
    candidates (negative status) are never accepted.  Stops at a local
    minimum of the solved moves or after max_steps accepted moves."""
    import time

    clock = clock or time.perf_counter
    t0 = clock()
    m = np.array(start_map, np.uint8)
    _, F0, st0, _ = evaluator.evaluate_flips(m, np.array([0, 0], np.int32), np.zeros(0, np.int32), want_S=False)
    F = float(F0[0]) if st0[0] >= 0 else np.inf
    res = DescentResult(F, m.copy(), 1, start_fom=F)

    def solve(o, c):
        S, Fc, st, _ = evaluator.evaluate_flips(m, o, c, want_S=learn is not None)
        res.exact_solves += len(o) - 1
        if learn is not None:
            maps = np.repeat(m[None, :], len(o) - 1, axis=0)
            for r in range(len(o) - 1):
                maps[r, c[o[r]:o[r + 1]]] ^= 1
            learn(maps, S)
        return TreeSearch._valid(Fc, st)

    for _ in range(max_steps):
        how = "exhaustive"
        if ranker is None:
            Fc = solve(offs, cells)
            o_acc, c_acc = offs, cells
        else:
            pick = np.asarray(ranker(m, offs, cells))[:top_k]
            o_acc, c_acc = _subset(offs, cells, pick)
            Fc = solve(o_acc, c_acc)
            how = "verified"
            if not (np.min(Fc) < F):
                how = "fallback"
                if fallback is not None:
                    o_acc, c_acc = fallback
                    Fc = solve(o_acc, c_acc)
                else:  # the moves not verified yet
                    rest = np.setdiff1d(np.arange(len(offs) - 1), pick)
                    if len(rest):
                        both = np.concatenate([pick, rest])
                        o_r, c_r = _subset(offs, cells, rest)
                        Fc = np.concatenate([Fc, solve(o_r, c_r)])
                        o_acc, c_acc = _subset(offs, cells, both)
        k = int(np.argmin(Fc))
        if not (np.isfinite(Fc[k]) and Fc[k] < F):
            res.trace.append((clock() - t0, res.exact_solves, F, how + ", local minimum"))
            break
        m = m.copy()
        m[c_acc[o_acc[k]:o_acc[k + 1]]] ^= 1
        F = float(Fc[k])
        res.fom, res.best_map = F, m.copy()
        res.trace.append((clock() - t0, res.exact_solves, F, how))
    return res


def sequential_dbs(evaluator, start_map, order, sweeps=1):
    """Classical direct binary search (Section III-A): visit the pixels in
    `order`, toggle one, keep the toggle if the FoM improves strictly and
    undo it otherwise; one exact solve per visit.  Returns a DescentResult
    whose trace holds (visits, exact solves, FoM, "kept"/"undone")."""
    m = np.array(start_map, np.uint8)
    _, F0, st0, _ = evaluator.evaluate_flips(m, np.array([0, 0], np.int32), np.zeros(0, np.int32), want_S=False)
    F = float(F0[0]) if st0[0] >= 0 else np.inf
    res = DescentResult(F, m.copy(), 1, start_fom=F)
    visits = 0
    for _ in range(sweeps):
        for j in order:
            _, Fc, st, _ = evaluator.evaluate_flips(m, np.array([0, 1], np.int32), np.array([j], np.int32),
                                                    want_S=False)
            res.exact_solves += 1
            visits += 1
            Fj = TreeSearch._valid(Fc, st)[0]
            if Fj < F:
                m = m.copy()
                m[j] ^= 1
                F = float(Fj)
                res.fom, res.best_map = F, m.copy()
                res.trace.append((visits, res.exact_solves, F, "kept"))
            else:
                res.trace.append((visits, res.exact_solves, F, "undone"))
    return res
