"""Parity at the workloads' full sizes, on sampled outputs (GPU).

The GPU evaluates every candidate of the full batch in the bench's launch
configuration (persistent grid of 2 workgroups per CU, frequency-major
items), at one frequency in the FoM's first passband; the oracle fills its
own parent at that frequency and solves a seeded sample of the candidates
one by one (LAPACK).  Tolerances as in the small-size tests: FP64 1e-10,
the mixed forms 1e-4 (the metric's bar); per-frequency S only, so no FoM.
"""

import numpy as np
import pytest

from oracle import efie, geometry, network, search
from paper_2412_17617_amd import pxd
from synth import get_spec, permutation

pytestmark = pytest.mark.gpu


def sampled(name, precisions, n_sample, f_target=5.5e9):
    spec = get_spec(name)
    fi = int(np.argmin(np.abs(spec.freqs - f_target)))
    freqs = spec.freqs[fi:fi + 1]
    st = geometry.build_structure(spec)
    Z = efie.fill(st, freqs[0])[None]
    base = spec.base_map()
    off, cells = spec.flips()
    C = len(off) - 1
    pick = np.sort(permutation(C, 77)[:n_sample])
    maps = search.candidate_maps(base, off, cells)
    pl = search.port_lengths(st)
    S_o = {}
    for c in pick:
        sel = st.active(maps[c])
        S_o[c] = network.s_parameters(network.reduce_matrix(Z[0], sel), network.port_positions(sel, st.port_bf), pl,
                                      spec.z0)
    pb = pxd.Problem.from_spec(spec)
    out = {}
    for prec in precisions:
        ev = pxd.Evaluator(precision=prec, ir_max_iter=40)
        ev.load_parent(Z, freqs)
        ev.load_problem(pb, spec.z0)
        ev.set_fom_paper()
        S, F, status, am = ev.evaluate_flips(base, off, cells)
        stats = ev.stats()
        ev.close()
        dS = max(np.abs(S[c, 0] - S_o[c]).max() for c in pick)
        print(f"{name} precision {prec}: N {stats['min_active']}-{stats['max_active']}, {C} candidates, sampled "
              f"max |dS| {dS:.2e}, {stats['ir_iterations']} residuals, {stats['fallbacks']} fallbacks")
        out[prec] = (S, status, dS)
    return out


def test_batched20_full_batch():
    r = sampled("batched20", (pxd.PREC_FP64, pxd.PREC_MIXED32), 12)
    assert r[pxd.PREC_FP64][2] <= 1e-10
    assert r[pxd.PREC_MIXED32][2] <= 1e-4
    for prec, (S, status, dS) in r.items():
        assert np.all((status == 0) | (status == 1))


def test_stress24_full_batch_every_precision():
    precs = (pxd.PREC_FP64, pxd.PREC_MIXED32, pxd.PREC_MIXED_BF16, pxd.PREC_MIXED_F16)
    r = sampled("stress24", precs, 6)
    assert r[pxd.PREC_FP64][2] <= 1e-10
    for prec in precs[1:]:
        assert r[prec][2] <= 1e-4
    for prec, (S, status, dS) in r.items():
        assert np.all((status == 0) | (status == 1))


def test_active_size_above_the_tiled_limit_is_refused():
    """The all-metal 32x32x3 map has N = M = 9,036, above the mixed modes'
    5,696 (their solves keep the right-hand sides in LDS): the library
    refuses the batch instead of running it.  (The FP64 limit, 10,240, is
    checked on the paper-size parent in test_gpu_mesh.py.)"""
    spec = get_spec("ceiling32")
    pb = pxd.Problem.from_spec(spec)
    ev = pxd.Evaluator(precision=pxd.PREC_MIXED32)
    Z = np.zeros((1, pb.M, pb.M), np.complex128)
    ev.load_parent(Z, spec.freqs[:1])
    ev.load_problem(pb, spec.z0)
    ev.set_fom_paper()
    off = np.array([0, 0], np.int32)
    with pytest.raises(pxd.PxdError) as e:
        ev.evaluate_flips(np.ones(spec.n_cells, np.uint8), off, np.zeros(0, np.int32))
    assert e.value.code == pxd.ESHAPE
    ev.close()


def test_batched20_uneven_batch_at_size():
    """The 20 x 20 x 2 uneven batch (8 maps of density 0.55 ... 0.83, 100
    single flips each: 800 whole maps, active sizes ~915-1,740) in one call
    at one frequency of the first passband, in FP64 and complex64 + FP64
    refinement (the library picks the LU path per the autotuned table or
    its defaults); a seeded sample of 8 maps solved by the oracle."""
    spec = get_spec("batched20")
    fi = int(np.argmin(np.abs(spec.freqs - 5.5e9)))
    freqs = spec.freqs[fi:fi + 1]
    st = geometry.build_structure(spec)
    Z = efie.fill(st, freqs[0])[None]
    maps = spec.uneven_maps()
    pick = np.sort(permutation(len(maps), 79)[:8])
    pl = search.port_lengths(st)
    S_o = {}
    for c in pick:
        sel = st.active(maps[c])
        S_o[c] = network.s_parameters(network.reduce_matrix(Z[0], sel), network.port_positions(sel, st.port_bf), pl,
                                      spec.z0)
    pb = pxd.Problem.from_spec(spec)
    for prec, tol in ((pxd.PREC_FP64, 1e-10), (pxd.PREC_MIXED32, 1e-4)):
        ev = pxd.Evaluator(precision=prec, ir_max_iter=40)
        ev.load_parent(Z, freqs)
        ev.load_problem(pb, spec.z0)
        ev.set_fom_paper()
        S, F, status, am = ev.evaluate_maps(maps)
        stats = ev.stats()
        ev.close()
        dS = max(np.abs(S[c, 0] - S_o[c]).max() for c in pick)
        print(f"uneven batch precision {prec}: N {stats['min_active']}-{stats['max_active']}, {len(maps)} maps, "
              f"sampled max |dS| {dS:.2e}, {stats['fallbacks']} fallbacks", flush=True)
        assert stats["min_active"] < 1100 and 1600 < stats["max_active"] <= 2048
        assert np.all((status == 0) | (status == 1))
        assert dS <= tol
