"""Host-side logic of the Algorithm 1 driver that needs no GPU (CPU)."""

import numpy as np
import pytest

from paper_2412_17617_amd.tree_search import TreeSearch, descent, sequential_dbs


def test_tree_search_rejects_bad_depths():
    with pytest.raises(ValueError):
        TreeSearch(object(), 2, 16, d_init=3, d_max=2)
    with pytest.raises(ValueError):
        TreeSearch(object(), 2, 16, d_init=1, d_max=3, m_of_depth=(10, 3))


def test_low_rank_tree_search_stays_switched_off():
    # its only GPU run faulted with no cause shown: the option must refuse
    with pytest.raises(NotImplementedError):
        TreeSearch(object(), 2, 16, lowrank=True)


class _TableEvaluator:
    """Stands in for the GPU evaluator: the FoM of a map is a table lookup and
    the candidates listed in `bad` report a singular solve (status -2) with
    a FoM below every valid one, as a garbage S could produce."""

    def __init__(self, fom_of, bad=()):
        self.fom_of, self.bad, self.calls = fom_of, {bytes(b) for b in bad}, 0

    def evaluate_flips(self, base, offs, cells, want_S=True):
        self.calls += 1
        n = len(offs) - 1
        F = np.empty(n)
        st = np.zeros(n, np.int32)
        for c in range(n):
            m = np.array(base, np.uint8)
            m[cells[offs[c]:offs[c + 1]]] ^= 1
            F[c] = self.fom_of(m)
            if bytes(m) in self.bad:
                F[c], st[c] = -1e9, -2
        return None, F, st, int(np.argmin(F))


def _restarts(n):
    rng = np.random.default_rng(0)
    while True:
        yield (rng.random(n) < 0.5).astype(np.uint8)


def test_tree_search_never_accepts_a_failed_candidate():
    # one layer, 4 pixels: FoM = number of metal pixels, so every step down is
    # an improvement; the map with pixel 0 cleared is "singular"
    start = np.ones(4, np.uint8)
    bad = start.copy()
    bad[0] = 0
    ev = _TableEvaluator(lambda m: float(m.sum()) + 1.0, bad=[bad])
    res = TreeSearch(ev, 1, 4, d_init=1, d_max=1, m_of_depth=(2,)).run(start, [0, 1, 2, 3], _restarts(4), 3)
    # first tree expands pixel 0: its only child is the failed one -> rejected
    assert res.trace[0] == (2, 5.0)
    assert res.accepted == 0 or not np.array_equal(res.best_map, bad)
    assert res.best_fom >= 1.0


def test_prefilter_falls_back_to_exact_solves():
    """Two layers, two pixels (4-state pixels: three leaves per tree of depth
    one).  Only the leaf that puts metal on layer 1 of pixel 0 (cell 2)
    alone improves; the surrogate ranks every leaf with cell 2 last and only
    k = 1 leaf is verified.  The driver must solve the rest of the level
    before counting a failure, and then accept the improving leaf."""
    start = np.zeros(4, np.uint8)

    def fom_of(m):
        return 10.0 - 5.0 * m[2] + 1.0 * (m.sum() - m[2])

    ev = _TableEvaluator(fom_of)

    def rank(sur, P, offs, cells):  # worst prediction for every leaf with cell 2
        pred = np.zeros(len(offs) - 1)
        for c in range(len(offs) - 1):
            pred[c] = 100.0 if 2 in cells[offs[c]:offs[c + 1]] else 0.0
        return pred

    res = TreeSearch(ev, 2, 2, d_init=1, d_max=1, m_of_depth=(1,)).run(
        start, [0, 1], _restarts(4), 5, prefilter=(None, 1, rank))
    assert res.accepted >= 1 and res.best_fom == 5.0
    assert list(res.best_map) == [0, 0, 1, 0]
    # the verified leaf (state 1, FoM 11) failed, then the other two were solved
    assert res.trace[0] == (1 + 1 + 2, 5.0)


def _singles(n):
    return np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32)


def test_exhaustive_descent_takes_the_steepest_move_each_step():
    # FoM = 1 + sum of weights of the metal cells: the steepest move clears the
    # heaviest remaining cell; four steps reach the empty map, the fifth finds
    # no improving move
    w = np.array([1.0, 4.0, 2.0, 3.0])
    ev = _TableEvaluator(lambda m: 1.0 + float(w @ m))
    offs, cells = _singles(4)
    res = descent(ev, np.ones(4, np.uint8), offs, cells, max_steps=10)
    assert [round(t[2], 9) for t in res.trace[:4]] == [7.0, 4.0, 2.0, 1.0]
    assert res.trace[-1][3].endswith("local minimum") and res.fom == 1.0
    assert res.exact_solves == 1 + 5 * 4 and list(res.best_map) == [0, 0, 0, 0]


def test_pruned_descent_falls_back_and_never_accepts_a_failed_move():
    w = np.array([1.0, 4.0, 2.0, 3.0])
    start = np.ones(4, np.uint8)
    bad = start.copy()
    bad[1] = 0  # the steepest first move is a failed solve
    ev = _TableEvaluator(lambda m: 1.0 + float(w @ m), bad=[bad])
    offs, cells = _singles(4)
    # the ranker puts the moves that improve most last: the one verified move
    # (cell 0, the smallest weight) improves, so no fallback is needed
    res = descent(ev, start, offs, cells, max_steps=1, ranker=lambda m, o, c: [0, 2, 3, 1], top_k=1)
    assert res.trace[0][3] == "verified" and res.fom == 10.0 and res.exact_solves == 2
    # a ranker that only offers a non-improving move: the exact fallback over
    # the rest of the set runs and takes the best valid move (cell 3; cell 1 failed)
    start2 = np.array([0, 1, 1, 1], np.uint8)
    ev = _TableEvaluator(lambda m: 1.0 + float(w @ m), bad=[np.array([0, 0, 1, 1], np.uint8)])
    res = descent(ev, start2, offs, cells, max_steps=1, ranker=lambda m, o, c: [0], top_k=1)
    assert res.trace[0][3] == "fallback" and res.exact_solves == 1 + 1 + 3
    assert list(res.best_map) == [0, 1, 1, 0] and res.fom == 7.0


def test_sequential_dbs_keeps_only_improving_toggles():
    w = np.array([1.0, -4.0, 2.0, -3.0])  # clearing cells 1 and 3 makes it worse
    ev = _TableEvaluator(lambda m: 10.0 + float(w @ m))
    res = sequential_dbs(ev, np.ones(4, np.uint8), [0, 1, 2, 3])
    assert [t[3] for t in res.trace] == ["kept", "undone", "kept", "undone"]
    assert list(res.best_map) == [0, 1, 0, 1] and res.fom == 3.0 and res.exact_solves == 5


# ---------------------------------------------------------------- refinement rule

pxd = pytest.importorskip("paper_2412_17617_amd.pxd")


def test_refine_verdict_converges_on_fast_contraction():
    # changes 1e-2 then 1e-4: rho = 0.01, error left 1e-4 * 0.01 / 0.99 ~ 1e-6
    assert pxd.refine_verdict(2, 10, 1e-4, 1e-2, 1e-5) == 1
    assert pxd.refine_verdict(2, 10, 1e-4, 1e-2, 1e-7) == 0  # not yet below a tighter target


def test_refine_verdict_never_stops_after_one_step():
    # no contraction is known after one step (rho taken as 1)
    assert pxd.refine_verdict(1, 10, 1e-20, 0.0, 1.0) == 0


def test_refine_verdict_gives_up_on_divergence_from_step_three():
    assert pxd.refine_verdict(2, 10, 2.0, 1.0, 1e-9) == 0  # too early to give up
    assert pxd.refine_verdict(3, 10, 2.0, 1.0, 1e-9) == 2  # rho = 2
    assert pxd.refine_verdict(3, 10, 1.0, 1.0, 1e-9) == 2  # rho = 1
    assert pxd.refine_verdict(3, 10, float("nan"), 1.0, 1e-9) == 2


def test_refine_verdict_gives_up_when_the_budget_cannot_suffice():
    # rho = 0.8, left = 1e-3 * 0.8 / 0.2 = 4e-3; reaching 1e-9 needs
    # log(2.5e-7) / log(0.8) = 68.13 more steps
    m_prev, m = 1.25e-3, 1e-3
    assert pxd.refine_verdict(3, 10, m, m_prev, 1e-9) == 2
    assert pxd.refine_verdict(3, 71, m, m_prev, 1e-9) == 2  # 3 + 68.13 > 71
    assert pxd.refine_verdict(3, 72, m, m_prev, 1e-9) == 0  # 3 + 68.13 <= 72
    assert pxd.refine_verdict(3, 71, m, m_prev, 1e-9 / 0.8) == 0  # one step fewer needed


def test_refine_verdict_needs_rho_below_09():
    # rho = 0.95 with a tiny change: the bound m rho / (1 - rho) = 19 m decides
    assert pxd.refine_verdict(4, 100, 1e-12, 1e-12 / 0.95, 1e-6) == 0
    assert pxd.refine_verdict(4, 100, 1e-12, 1e-12 / 0.85, 1e-6) == 1


def test_refine_verdict_rejects_bad_arguments():
    with pytest.raises(pxd.PxdError):
        pxd.refine_verdict(0, 10, 1.0, 1.0, 1.0)


def test_bench_binding_roof():
    """The bench's roofline names the roof the dominant launch's floors
    select: at 56 flop per algorithmic byte (the 32x32x3 update, 572 GFLOP on
    10.2 GB per launch) the split-BF16 update (three BF16 products per real
    product at 2.5 PFLOP/s: 0.69 ms) is bound by the 1.27 ms its bytes need
    at 8 TB/s; the complex64 (FP32 MFMA, 3.64 ms) and FP64 (complex128
    bytes, 7.28 ms against 2.58 ms) updates by the MFMA rate."""
    import bench

    bound, comp, mem, issued = bench.binding_roof("bf16x3", 572.38, 10.19)
    assert bound == "hbm" and issued == 3.0
    assert comp == pytest.approx(3 * 572.38 / 2500.0 * 1e3) and mem == pytest.approx(10.19 / 8000.0 * 1e6)
    bound, comp, mem, _ = bench.binding_roof("mixed32", 572.38, 10.18)
    assert bound == "mfma" and comp == pytest.approx(572.38 / 157.3 * 1e3)
    bound, comp, mem, _ = bench.binding_roof("fp64", 572.38, 20.64)
    assert bound == "mfma" and comp > mem
    # the same launch with four times the bytes would be HBM-bound in complex64 too
    assert bench.binding_roof("mixed32", 572.38, 4 * 10.18)[0] == "hbm"
