"""GPU parity of the mixed-precision path (complex64 LU, FP64 residual and
iterative refinement) against the FP64 oracle, through the C ABI.

Bar: max |dS| <= 1e-4 (the accuracy the evaluation must reach) and the same
FoM ranking.  Refinement stops once a correction changes no S entry by more
than 1e-7; that correction is applied, so the returned S carries about 1e-7
times the complex64 contraction factor (well below 1e-9).  The FoM amplifies
the relative error of a small |S_ij| by at most ~2, so FoM agreement within
1e-6 relative, as on the FP64 path, is expected.
"""

import numpy as np
import pytest

from oracle import search
from paper_2412_17617_amd import pxd
from synth import PortSpec, bernoulli_map, get_spec, single_flips

from gpu_common import make_evaluator, oracle_parent, spec_variant

pytestmark = pytest.mark.gpu

S_BAR = 1e-4
FOM_RTOL = 1e-6


def run_mixed(spec, fidx=None, base=None, flips=None, **kw):
    st, Z, freqs = oracle_parent(spec, fidx)
    base = spec.base_map() if base is None else base
    off, cells = spec.flips() if flips is None else flips
    S_o, F_o = search.sweep(st, Z, base, off, cells, freqs)
    ev, _ = make_evaluator(spec, Z, freqs, precision=pxd.PREC_MIXED32, **kw)
    S, F, status, am = ev.evaluate_flips(base, off, cells)
    stats = ev.stats()
    ev.close()
    return S, F, status, am, S_o, F_o, stats


def check(S, F, status, am, S_o, F_o):
    assert np.all((status == pxd.STATUS_OK) | (status == pxd.STATUS_FALLBACK)), status
    dS = np.abs(S - S_o).max()
    assert dS <= S_BAR, dS
    assert np.all(np.abs(F - F_o) <= FOM_RTOL * F_o), np.max(np.abs(F - F_o) / F_o)
    assert np.array_equal(np.argsort(F, kind="stable"), np.argsort(F_o, kind="stable")) or \
        np.all(np.abs(np.sort(F) - np.sort(F_o)) <= FOM_RTOL * np.sort(F_o))
    assert F[am] == F.min()
    return dS


def test_mixed_plain8_sweep():
    S, F, status, am, S_o, F_o, stats = run_mixed(get_spec("plain8"))
    dS = check(S, F, status, am, S_o, F_o)
    assert dS <= 1e-8  # refinement reaches far below the bar
    assert stats["items"] == 64 * 11
    assert stats["ir_iterations"] >= stats["items"]  # at least one refinement step per item


def test_mixed_multilayer_and_vias():
    spec = get_spec("tiny4x2")
    check(*run_mixed(spec)[:6])
    check(*run_mixed(spec, base=bernoulli_map(spec.n_cells, 0.8, 99))[:6])
    check(*run_mixed(get_spec("small6x3"), fidx=(0, 4))[:6])


@pytest.mark.parametrize("nx,layers,p", [(11, 2, 0.6), (16, 2, 0.7), (26, 1, 0.9)])
def test_mixed_every_kernel_variant(nx, layers, p):
    ports = (PortSpec("right", 0), PortSpec("top", 0), PortSpec("left", layers - 1))
    spec = spec_variant("tiny4x2", nx=nx, ny=nx, n_layers=layers, density=p, n_vias=3 if layers > 1 else 0,
                        ports=ports, seed=40 + nx)
    cells = np.arange(0, spec.n_cells, max(1, spec.n_cells // 6))[:6]
    off, cl = single_flips(cells)
    check(*run_mixed(spec, fidx=(1,), flips=(off, cl))[:6])


def test_forced_fallback_returns_fp64_results():
    """One refinement step against an unreachable tolerance: every item is
    handed to the FP64 path, flagged FALLBACK, and matches the oracle to the
    FP64 tolerance."""
    S, F, status, am, S_o, F_o, stats = run_mixed(get_spec("tiny4x2"), ir_max_iter=1, ir_tol=1e-300)
    assert np.all(status == pxd.STATUS_FALLBACK)
    assert stats["fallbacks"] == stats["items"]
    assert np.abs(S - S_o).max() <= 1e-10
    assert np.all(np.abs(F - F_o) <= 1e-6 * F_o)
