"""GPU parity of the FP64 evaluation path against the oracle, through the C ABI.

Tolerances (FP64 path).  The GPU and LAPACK factor the same matrices with
different blockings, so results differ by rounding: backward error ~1e-16
amplified by kappa(Z_A) <= ~1e4 on these workloads.  S entries are bounded by
one, so |dS| <= 1e-10 leaves two decades of margin.  The FoM sums powers of
|S_ij| down to |S_ij|^-2 with |S21| as small as ~1e-5, so its relative error
is about 2 |dS| / |S|min <= 1e-5; 1e-6 relative is used, which measured
margins show holds.  Argmin must be identical unless the oracle's best two
candidates are within that tolerance (then either is accepted).
"""

import numpy as np
import pytest

from oracle import geometry, network, search
from paper_2412_17617_amd import pxd
from synth import PortSpec, bernoulli_map, get_spec, single_flips

from gpu_common import make_evaluator, oracle_active_sets, oracle_parent, spec_variant

pytestmark = pytest.mark.gpu

S_TOL = 1e-10
FOM_RTOL = 1e-6


def check_argmin(am, F_o):
    order = np.argsort(F_o, kind="stable")
    if am == order[0]:
        return
    assert abs(F_o[am] - F_o[order[0]]) <= FOM_RTOL * F_o[order[0]], (am, order[:3])


def test_expand_is_bit_exact():
    for name in ("plain8", "tiny4x2", "batched20"):
        spec = get_spec(name)
        st = geometry.build_structure(spec)
        Zdummy = np.zeros((1, st.M, st.M), np.complex128)
        ev, _ = make_evaluator(spec, Zdummy, spec.freqs[:1])
        base = spec.base_map()
        off, cells = spec.flips()
        N, idx = ev.expand(base, off, cells)
        want = oracle_active_sets(st, base, off, cells)
        assert list(N) == [len(w) for w in want]
        for a, b in zip(idx, want):
            assert np.array_equal(a, b)
        ev.close()


def test_expand_edge_cases():
    spec = get_spec("tiny4x2")
    st = geometry.build_structure(spec)
    ev, _ = make_evaluator(spec, np.zeros((1, st.M, st.M), np.complex128), spec.freqs[:1])
    n = spec.n_cells
    for base in (np.zeros(n, np.uint8), np.ones(n, np.uint8), spec.base_map()):
        # no flips, one flip, the same cell twice (toggles back), many flips
        off = np.array([0, 0, 1, 3, 3 + n], np.int32)
        cells = np.concatenate([[5], [7, 7], np.arange(n)]).astype(np.int32)
        N, idx = ev.expand(base, off, cells)
        want = oracle_active_sets(st, base, off, cells)
        assert [len(w) for w in want] == list(N)
        for a, b in zip(idx, want):
            assert np.array_equal(a, b)
    # zero candidates
    N, idx = ev.expand(spec.base_map(), np.zeros(1, np.int32), np.zeros(0, np.int32))
    assert len(N) == 0
    ev.close()


def test_gather_is_bitwise():
    for name in ("plain8", "tiny4x2"):
        spec = get_spec(name)
        st, Z, freqs = oracle_parent(spec, (0, 2))
        ev, _ = make_evaluator(spec, Z, freqs)
        for seed in (1, 2, 3):
            m = bernoulli_map(spec.n_cells, 0.5, seed)
            sel = st.active(m)
            idx = network.support(sel).astype(np.int32)
            for f in range(len(freqs)):
                assert np.array_equal(ev.gather(f, idx), network.reduce_matrix(Z[f], sel))
        ev.close()


def _sweep_parity(spec, fidx=None, flips=None, base=None):
    st, Z, freqs = oracle_parent(spec, fidx)
    base = spec.base_map() if base is None else base
    off, cells = spec.flips() if flips is None else flips
    S_o, F_o = search.sweep(st, Z, base, off, cells, freqs)
    ev, _ = make_evaluator(spec, Z, freqs)
    S, F, status, am = ev.evaluate_flips(base, off, cells)
    stats = ev.stats()
    ev.close()
    assert np.all(status == pxd.STATUS_OK)
    dS = np.abs(S - S_o).max()
    assert dS <= S_TOL, dS
    assert np.all(np.abs(F - F_o) <= FOM_RTOL * F_o), np.max(np.abs(F - F_o) / F_o)
    check_argmin(am, F_o)
    return stats, dS


def test_plain8_full_sweep():
    """The 8x8 free-space workload: all 64 single flips at all 11 frequencies."""
    stats, dS = _sweep_parity(get_spec("plain8"))
    assert stats["items"] == 64 * 11


def test_multilayer_with_vias():
    spec = get_spec("tiny4x2")
    _sweep_parity(spec)
    # denser base map, every single flip
    _sweep_parity(spec, base=bernoulli_map(spec.n_cells, 0.8, 99))


def test_three_layers_ports_on_three_layers():
    _sweep_parity(get_spec("small6x3"), fidx=(0, 4))


@pytest.mark.parametrize("nx,layers,p,expect_q", [(11, 2, 0.6, 2), (16, 2, 0.7, 4), (26, 1, 0.9, 8)])
def test_every_kernel_variant(nx, layers, p, expect_q):
    """Active sizes across the register-panel variants (rows per thread Q),
    ragged against the 32-wide panels and the 32 x 32 MFMA tiles."""
    ports = (PortSpec("right", 0), PortSpec("top", 0), PortSpec("left", layers - 1))
    spec = spec_variant("tiny4x2", nx=nx, ny=nx, n_layers=layers, density=p, n_vias=3 if layers > 1 else 0,
                        ports=ports, seed=40 + nx)
    base = spec.base_map()
    cells = np.arange(0, spec.n_cells, max(1, spec.n_cells // 6))[:6]
    off, cl = single_flips(cells)
    stats, _ = _sweep_parity(spec, fidx=(1,), flips=(off, cl), base=base)
    q = (stats["max_active"] + 255) // 256
    assert q == expect_q or (expect_q == 8 and q > 4), stats["max_active"]


def test_product_fill_end_to_end():
    """GPU path on the library's own parent fill vs the oracle on its own fill."""
    spec = get_spec("plain8")
    st, Zo, freqs = oracle_parent(spec)
    pb = pxd.Problem.from_spec(spec)
    Zp = pb.fill(freqs)
    base = spec.base_map()
    off, cells = spec.flips()
    S_o, F_o = search.sweep(st, Zo, base, off, cells, freqs)
    ev, _ = make_evaluator(spec, Zp, freqs)
    S, F, status, am = ev.evaluate_flips(base, off, cells)
    ev.close()
    assert np.abs(S - S_o).max() <= S_TOL
    assert np.all(np.abs(F - F_o) <= FOM_RTOL * F_o)
    check_argmin(am, F_o)


def test_status_codes_are_reported():
    """Host-forced faults: a zero row/column makes an exactly singular matrix,
    a NaN entry must surface as non-finite.  Other candidates are unaffected."""
    spec = get_spec("tiny3")
    st, Z, freqs = oracle_parent(spec)
    Zs = Z.copy()
    Zs[:, 0, :] = 0.0
    Zs[:, :, 0] = 0.0  # inner function of cell 0
    base = np.ones(spec.n_cells, np.uint8)
    off, cells = single_flips([0, 1])  # candidate 0 switches cell 0 off -> regular
    ev, _ = make_evaluator(spec, Zs, freqs)
    S, F, status, am = ev.evaluate_flips(base, off, cells)
    assert status[0] == pxd.STATUS_OK and status[1] == pxd.STATUS_SINGULAR
    # a failed candidate can never be selected (Algorithm 1 takes the arg min
    # of valid FoM values): its FoM is +inf and the argmin is the valid one
    assert np.isfinite(F[0]) and F[1] == np.inf and am == 0
    # listed first, the singular candidate still loses to the regular one
    off2, cells2 = single_flips([1, 0])
    S, F, status, am = ev.evaluate_flips(base, off2, cells2)
    assert status[0] == pxd.STATUS_SINGULAR and F[0] == np.inf and am == 1
    # no valid candidate at all: argmin -1
    off3, cells3 = single_flips([1, 2])
    S, F, status, am = ev.evaluate_flips(base, off3, cells3)
    assert np.all(status == pxd.STATUS_SINGULAR) and np.all(F == np.inf) and am == -1
    ev.close()
    Zn = Z.copy()
    Zn[2, 3, 4] = np.nan
    Zn[2, 4, 3] = np.nan
    ev, _ = make_evaluator(spec, Zn, freqs)
    S, F, status, am = ev.evaluate_flips(base, off, cells)
    assert np.all(status == pxd.STATUS_NONFINITE)
    assert np.all(F == np.inf) and am == -1
    ev.close()


def test_bad_arguments_return_codes():
    spec = get_spec("tiny3")
    st, Z, freqs = oracle_parent(spec)
    ev, _ = make_evaluator(spec, Z, freqs)
    with pytest.raises(pxd.PxdError) as e:
        ev.evaluate_flips(spec.base_map(), np.array([0, 1], np.int32), np.array([spec.n_cells], np.int32))
    assert e.value.code == pxd.EINVAL
    with pytest.raises(pxd.PxdError) as e:
        ev.gather(0, np.array([3, 2], np.int32))
    assert e.value.code == pxd.EINVAL
    with pytest.raises(pxd.PxdError) as e:
        ev.gather(len(freqs), np.array([1, 2], np.int32))
    assert e.value.code == pxd.EINVAL
    ev.close()
    fresh = pxd.Evaluator()
    with pytest.raises(pxd.PxdError) as e:
        fresh.evaluate_flips(spec.base_map(), np.array([0, 0], np.int32), np.zeros(0, np.int32))
    assert e.value.code == pxd.ENOTLOADED
    fresh.close()


@pytest.mark.parametrize("variant,name", [(pxd.FOM_REJ, "rej"), (pxd.FOM_ISO, "iso")])
def test_fom_variants(variant, name):
    """Section III-D term tables: the GPU FoM against the oracle's."""
    from oracle import fom as ofom

    spec = get_spec("tiny4x2")
    st, Z, freqs = oracle_parent(spec)
    base = spec.base_map()
    off, cells = spec.flips()
    S_o, _ = search.sweep(st, Z, base, off, cells, freqs)
    F_o = np.array([ofom.fom(S_o[c], freqs, name) for c in range(len(off) - 1)])
    ev, _ = make_evaluator(spec, Z, freqs)
    ev.set_fom_paper(variant)
    S, F, status, am = ev.evaluate_flips(base, off, cells)
    ev.close()
    assert np.abs(S - S_o).max() <= S_TOL
    assert np.all(np.abs(F - F_o) <= FOM_RTOL * F_o)
    check_argmin(am, F_o)
