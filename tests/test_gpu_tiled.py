"""GPU parity of the tiled LU (many workgroups per item, one launch per step
of each block column) against the oracle, through the C ABI.

Small and medium cases force the tiled path (lu_path = PXD_PATH_TILED) and
compare with the oracle's own fill and LAPACK solve, and with the persistent
one-workgroup-per-item path on the same inputs; the active sizes span one to
several 128-row output tiles with ragged tails, both block-column widths
(64, 128) and both the FP64 augmented system and the complex64 factor with
FP64 refinement.  Above 2,048 (where only the tiled path runs) the library's
own parent fill is compared with sampled oracle references written by
tests/golden/large_gen.py (oracle fill, Eq. 5 gather, LAPACK, Eqs. 6-7).
Tolerances as elsewhere: FP64 max |dS| <= 1e-10 (GPU and LAPACK differ only
in rounding order, ~kappa 1e-16 with kappa <= ~1e5), mixed forms 1e-4 (the
metric's bar), FoM 1e-6 relative.
"""

import os

import numpy as np
import pytest

from oracle import search
from paper_2412_17617_amd import pxd
from synth import PortSpec, get_spec, single_flips

from gpu_common import make_evaluator, oracle_parent, spec_variant

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
S_TOL = {pxd.PREC_FP64: 1e-10, pxd.PREC_MIXED32: 1e-4}
FOM_RTOL = 1e-6


def _check_fom(F, F_o, am):
    assert np.all(np.abs(F - F_o) <= FOM_RTOL * F_o), np.max(np.abs(F - F_o) / F_o)
    best = np.argsort(F_o, kind="stable")[0]
    assert am == best or abs(F_o[am] - F_o[best]) <= FOM_RTOL * F_o[best]


@pytest.mark.parametrize("name,prec,kb,shape", [
    ("tiny4x2", pxd.PREC_FP64, 64, 1), ("tiny4x2", pxd.PREC_MIXED32, 64, 2),
    ("small6x3", pxd.PREC_FP64, 128, 2), ("small6x3", pxd.PREC_MIXED32, 128, 1),
])
def test_tiled_matches_oracle_and_persistent_path(name, prec, kb, shape):
    spec = get_spec(name)
    st, Z, freqs = oracle_parent(spec)
    base = spec.base_map()
    off, cells = spec.flips()
    print(f"{name} precision {prec} block columns {kb} update tile {shape}", flush=True)
    S_o, F_o = search.sweep(st, Z, base, off, cells, freqs)
    ev, _ = make_evaluator(spec, Z, freqs, precision=prec, lu_path=pxd.PATH_TILED, tile_kb=kb, tile_shape=shape)
    S, F, status, am = ev.evaluate_flips(base, off, cells)
    stats = ev.stats()
    ev.close()
    ev, _ = make_evaluator(spec, Z, freqs, precision=prec, lu_path=pxd.PATH_PERSISTENT)
    S_p, F_p, _, _ = ev.evaluate_flips(base, off, cells)
    ev.close()
    print(f"  N {stats['min_active']}-{stats['max_active']}: max |dS| vs oracle {np.abs(S - S_o).max():.2e}, vs "
          f"persistent {np.abs(S - S_p).max():.2e}, fallbacks {stats['fallbacks']}", flush=True)
    assert np.all((status == pxd.STATUS_OK) | (status == pxd.STATUS_FALLBACK))
    assert np.abs(S - S_o).max() <= S_TOL[prec]
    assert np.abs(S - S_p).max() <= S_TOL[prec]
    _check_fom(F, F_o, am)
    if prec != pxd.PREC_FP64:
        assert stats["fallbacks"] == 0 and stats["ir_iterations"] >= stats["items"]


@pytest.mark.parametrize("shape", [1, 2, 3, 4])
@pytest.mark.parametrize("prec", [pxd.PREC_FP64, pxd.PREC_MIXED32])
@pytest.mark.parametrize("nx,layers,p", [(11, 2, 0.6), (16, 2, 0.7), (26, 1, 0.9)])
def test_tiled_sizes_span_several_tiles(prec, nx, layers, p, shape):
    """Active sizes ~150-700: one to six 128-row output tiles, several block
    columns, ragged last tiles; one frequency."""
    ports = (PortSpec("right", 0), PortSpec("top", 0), PortSpec("left", layers - 1))
    spec = spec_variant("tiny4x2", nx=nx, ny=nx, n_layers=layers, density=p, n_vias=3 if layers > 1 else 0,
                        ports=ports, seed=40 + nx)
    st, Z, freqs = oracle_parent(spec, (1,))
    base = spec.base_map()
    off, cells = single_flips(np.arange(0, spec.n_cells, max(1, spec.n_cells // 6))[:6])
    S_o, F_o = search.sweep(st, Z, base, off, cells, freqs)
    ev, _ = make_evaluator(spec, Z, freqs, precision=prec, lu_path=pxd.PATH_TILED, tile_shape=shape)
    print(f"nx {nx} layers {layers} precision {prec} update tile {shape}", flush=True)
    S, F, status, am = ev.evaluate_flips(base, off, cells)
    stats = ev.stats()
    ev.close()
    print(f"  N {stats['min_active']}-{stats['max_active']}: max |dS| {np.abs(S - S_o).max():.2e}", flush=True)
    assert np.all((status == pxd.STATUS_OK) | (status == pxd.STATUS_FALLBACK))
    assert np.abs(S - S_o).max() <= S_TOL[prec]
    _check_fom(F, F_o, am)


def test_tiled_reports_singular_items():
    """A zero row and column (host-forced) makes an exactly singular system:
    status SINGULAR, FoM +inf, never the argmin; the regular candidate is
    unaffected."""
    spec = get_spec("tiny3")
    st, Z, freqs = oracle_parent(spec)
    Zs = Z.copy()
    Zs[:, 0, :] = 0.0
    Zs[:, :, 0] = 0.0
    base = np.ones(spec.n_cells, np.uint8)
    off, cells = single_flips([0, 1])
    ev, _ = make_evaluator(spec, Zs, freqs, lu_path=pxd.PATH_TILED)
    S, F, status, am = ev.evaluate_flips(base, off, cells)
    ev.close()
    assert status[0] == pxd.STATUS_OK and status[1] == pxd.STATUS_SINGULAR
    assert np.isfinite(F[0]) and F[1] == np.inf and am == 0
    S_o, _ = search.sweep(st, Z, base, off[:2], cells[:1], freqs)
    assert np.abs(S[0] - S_o[0]).max() <= 1e-10


def _large(name, precisions, fill):
    g = np.load(os.path.join(GOLD, f"large_{name}.npz"))
    spec = get_spec("ceiling32") if name == "ceiling32" else spec_variant("stress24", density=float(g["density"]))
    fidx = list(g["fidx"])
    freqs = spec.freqs[fidx]
    pb = pxd.Problem.from_spec(spec)
    base = spec.base_map()
    off, cells = spec.flips()
    pick = g["pick"]
    sub_off = np.zeros(len(pick) + 1, np.int32)
    sub_off[1:] = np.cumsum([off[c + 1] - off[c] for c in pick])
    sub_cells = np.concatenate([cells[off[c]:off[c + 1]] for c in pick]).astype(np.int32)
    out = {}
    for prec in precisions:
        ev = pxd.Evaluator(precision=prec, ir_max_iter=40)
        ev.load_problem(pb, spec.z0)
        if fill == "device":
            ev.load_parent_problem(pb, freqs)
        else:
            ev.load_parent(pb.fill(freqs, n_threads=16), freqs)
        ev.set_fom_paper()
        print(f"{name} precision {prec}: {len(pick)} candidates x {len(fidx)} frequencies", flush=True)
        S, F, status, am = ev.evaluate_flips(base, sub_off, sub_cells)
        stats = ev.stats()
        ev.close()
        dS = float(np.abs(S - g["S"]).max())
        print(f"  N {stats['min_active']}-{stats['max_active']} (oracle {g['N'].min()}-{g['N'].max()}): max |dS| "
              f"{dS:.2e}, {stats['ir_iterations']} residuals, {stats['fallbacks']} fallbacks, "
              f"solve {stats['ms_solve']:.0f} ms", flush=True)
        assert stats["max_active"] == g["N"].max() and stats["min_active"] == g["N"].min()
        out[prec] = (S, status, dS)
    return out


def test_dense24_above_one_workgroup_limit():
    """24 x 24 x 3 stack at 0.65 density: active sizes ~2,530, above the
    persistent kernels' 2,048, so the tiled path takes them (auto)."""
    r = _large("dense24", (pxd.PREC_FP64, pxd.PREC_MIXED32), "host")
    for prec, (S, status, dS) in r.items():
        assert np.all((status == 0) | (status == 1))
        assert dS <= S_TOL[prec]


def test_ceiling32_sampled_against_oracle():
    """The 32 x 32 x 3 headline stack (M = 9,036): 16 seeded pair-flip
    candidates at 5 frequencies (the lowest grid point and one in each FoM
    band), parent filled on the GPU, active sizes ~3,035."""
    r = _large("ceiling32", (pxd.PREC_FP64, pxd.PREC_MIXED32), "device")
    for prec, (S, status, dS) in r.items():
        assert np.all((status == 0) | (status == 1))
        assert dS <= S_TOL[prec]


@pytest.mark.parametrize("name,nx,layers", [("tiny4x2", 4, 2), ("tiny4x2", 16, 2)])
def test_split_bf16_updates(name, nx, layers):
    """PXD_PREC_MIXED_BF16X3: trailing updates on split BF16 operands (three
    products, ~2^-16 relative), then FP64 refinement.  Every result meets the
    oracle to the mixed bar; on these small, well-conditioned systems the
    split factor settles on its own for most items (no FP64 hand-off)."""
    ports = (PortSpec("right", 0), PortSpec("top", 0), PortSpec("left", layers - 1))
    spec = spec_variant(name, nx=nx, ny=nx, n_layers=layers, density=0.7, n_vias=3, ports=ports, seed=60 + nx)
    st, Z, freqs = oracle_parent(spec, (1,))
    base = spec.base_map()
    off, cells = single_flips(np.arange(0, spec.n_cells, max(1, spec.n_cells // 6))[:6])
    S_o, F_o = search.sweep(st, Z, base, off, cells, freqs)
    ev, _ = make_evaluator(spec, Z, freqs, precision=pxd.PREC_MIXED_BF16X3, ir_max_iter=30)
    print(f"split BF16 nx {nx}", flush=True)
    S, F, status, am = ev.evaluate_flips(base, off, cells)
    stats = ev.stats()
    ev.close()
    print(f"  N {stats['max_active']}: {stats['ir_iterations']} refinement steps, {stats['fallbacks']} of "
          f"{stats['items']} items to FP64, max |dS| {np.abs(S - S_o).max():.2e}", flush=True)
    assert np.all((status == pxd.STATUS_OK) | (status == pxd.STATUS_FALLBACK))
    assert np.abs(S - S_o).max() <= 1e-4
    _check_fom(F, F_o, am)
    assert 2 * stats["fallbacks"] <= stats["items"], stats


def test_plain_half_modes_above_2048_are_refused():
    """The plain BF16 / FP16 block-update modes exist on the persistent LU
    only; a batch above its 2,048 limit is refused, not run in another
    arithmetic."""
    g = np.load(os.path.join(GOLD, "large_dense24.npz"))
    spec = spec_variant("stress24", density=float(g["density"]))
    pb = pxd.Problem.from_spec(spec)
    off, cells = single_flips([0])
    for prec in (pxd.PREC_MIXED_BF16, pxd.PREC_MIXED_F16):
        ev = pxd.Evaluator(precision=prec)
        ev.load_problem(pb, spec.z0)
        ev.load_parent(np.zeros((1, pb.M, pb.M), np.complex128), spec.freqs[:1])
        ev.set_fom_paper()
        with pytest.raises(pxd.PxdError) as e:
            ev.evaluate_flips(spec.base_map(), off, cells)
        assert e.value.code == pxd.ESHAPE
        ev.close()


@pytest.mark.parametrize("prec", [pxd.PREC_MIXED32, pxd.PREC_MIXED_BF16X3])
@pytest.mark.parametrize("maps", [False, True])
def test_lockstep_refinement_matches_per_item(prec, maps):
    """The lock-step refinement (the residuals of one frequency's items as
    one product over the union of the active sets) against the per-item form
    and the oracle.  Single flips of one map (union ~ one active set), or
    whole maps of densities 0.3-0.9 as flips of the empty map (union ~ the
    parent, candidates of very different sizes in one frequency group);
    five frequencies."""
    spec = get_spec("small6x3")
    st, Z, freqs = oracle_parent(spec)
    if maps:
        rng = np.random.default_rng(5)
        on = [np.nonzero(rng.random(spec.n_cells) < d)[0] for d in np.linspace(0.3, 0.9, 7)]
        base = np.zeros(spec.n_cells, np.uint8)
        off = np.zeros(len(on) + 1, np.int32)
        off[1:] = np.cumsum([len(c) for c in on])
        cells = np.concatenate(on).astype(np.int32)
    else:
        base = spec.base_map()
        off, cells = spec.flips()
        off, cells = off[:25], cells[:off[24]]
    print(f"small6x3 precision {prec} {'whole maps' if maps else 'single flips'}: {len(off) - 1} candidates",
          flush=True)
    S_o, F_o = search.sweep(st, Z, base, off, cells, freqs)
    out = {}
    for refine in (pxd.REFINE_PER_ITEM, pxd.REFINE_LOCKSTEP):
        ev, _ = make_evaluator(spec, Z, freqs, precision=prec, lu_path=pxd.PATH_TILED, refine=refine)
        S, F, status, am = ev.evaluate_flips(base, off, cells)
        stats = ev.stats()
        ev.close()
        out[refine] = (S, F, status, am, stats)
        print(f"  refine {refine}: N {stats['min_active']}-{stats['max_active']}, max |dS| vs oracle "
              f"{np.abs(S - S_o).max():.2e}, fallbacks {stats['fallbacks']}, steps {stats['ir_iterations']}",
              flush=True)
        assert np.all((status == pxd.STATUS_OK) | (status == pxd.STATUS_FALLBACK))
        assert np.abs(S - S_o).max() <= 1e-4
        _check_fom(F, F_o, am)
        if prec == pxd.PREC_MIXED32:
            assert stats["fallbacks"] == 0
    S1, S2 = out[pxd.REFINE_PER_ITEM][0], out[pxd.REFINE_LOCKSTEP][0]
    assert np.abs(S1 - S2).max() <= 1e-6
    # the same stop test on residuals that differ only in summation order
    assert abs(out[pxd.REFINE_PER_ITEM][4]["ir_iterations"] - out[pxd.REFINE_LOCKSTEP][4]["ir_iterations"]) <= \
        0.05 * out[pxd.REFINE_PER_ITEM][4]["ir_iterations"] + 2
