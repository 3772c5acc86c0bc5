"""GPU parent fill against the oracle's fill (GPU).

The GPU fill and the oracle implement the same discretisation (Section II-A:
mixed-potential EFIE, RWG functions, 4-point triangle rule, closed-form 1/R
extraction on near pairs) independently; they differ by the rounding of
their math libraries and summation orders, ~1e-15 relative per entry.  The
bar is 1e-12 of max |Z| (as for the host fill), and exact symmetry (the
upper triangle is mirrored).
"""

import numpy as np
import pytest
import torch

from oracle import efie, geometry, search
from paper_2412_17617_amd import pxd
from synth import get_spec

from fill_common import near_series_switch_freqs
from gpu_common import make_evaluator, oracle_parent

pytestmark = pytest.mark.gpu

Z_RTOL = 1e-12


def device_fill(pb, freqs):
    out = torch.empty((len(freqs), pb.M, pb.M), dtype=torch.complex128, device="cuda:0")
    pb.fill_device(freqs, out)
    return out.cpu().numpy()


@pytest.mark.parametrize("name", ["plain8", "tiny4x2", "small6x3"])
def test_device_fill_matches_oracle(name):
    spec = get_spec(name)
    pb = pxd.Problem.from_spec(spec)
    st = geometry.build_structure(spec)
    freqs = spec.freqs[[0, -1]]
    Z = device_fill(pb, freqs)
    Zo = np.stack([efie.fill(st, f) for f in freqs])
    err = np.abs(Z - Zo).max() / np.abs(Zo).max()
    print(f"{name}: M {pb.M}, max |dZ| / max |Z| = {err:.2e}")
    assert np.array_equal(Z, np.transpose(Z, (0, 2, 1)))
    assert err <= Z_RTOL


@pytest.mark.parametrize("name", ["plain8", "tiny4x2"])
def test_device_fill_across_the_near_series_switch(name):
    """Near pairs evaluate the smooth remainder (exp(-jkR) - 1)/(4 pi R) by a
    short series where |kR| < 1e-3 and by the exponential above; the band-edge
    cases use the exponential only.  Here half of the near pairs' point
    distances fall below the switch (f_mid), then all of them (f_mid / 3).
    At f_mid a wrong second- or third-order coefficient of the series moves
    the oracle's Z by 3e-8 or 6e-12 of max |Z| (tiny4x2; plain8 4e-8 and
    1e-11), past the bar; the fourth order stays at rounding level."""
    spec = get_spec(name)
    pb = pxd.Problem.from_spec(spec)
    st = geometry.build_structure(spec)
    freqs, below = near_series_switch_freqs(st)
    assert below[0] == 1.0 and 0.3 < below[1] < 0.7, below
    Z = device_fill(pb, freqs)
    Zo = np.stack([efie.fill(st, f) for f in freqs])
    err = np.abs(Z - Zo).max(axis=(1, 2)) / np.abs(Zo).max(axis=(1, 2))
    print(f"{name}: f {freqs[0]:.3e} {freqs[1]:.3e} Hz, near distances below the switch {below}, "
          f"max |dZ| / max |Z| = {err[0]:.2e} {err[1]:.2e}")
    assert np.array_equal(Z, np.transpose(Z, (0, 2, 1)))
    assert err.max() <= Z_RTOL


def test_device_fill_full_size():
    """20 x 20 x 2 stack (M = 2,371) at one frequency in the first passband."""
    spec = get_spec("batched20")
    pb = pxd.Problem.from_spec(spec)
    st = geometry.build_structure(spec)
    fi = int(np.argmin(np.abs(spec.freqs - 5.5e9)))
    freqs = spec.freqs[fi:fi + 1]
    Z = device_fill(pb, freqs)
    Zo = efie.fill(st, freqs[0])[None]
    err = np.abs(Z - Zo).max() / np.abs(Zo).max()
    print(f"batched20: M {pb.M}, max |dZ| / max |Z| = {err:.2e}")
    assert np.array_equal(Z, np.transpose(Z, (0, 2, 1)))
    assert err <= Z_RTOL


def test_load_parent_problem_end_to_end():
    """An evaluator whose parent is filled on the GPU gives the oracle's S."""
    spec = get_spec("small6x3")
    st, Zo, freqs = oracle_parent(spec)
    base = spec.base_map()
    off, cells = spec.flips()
    S_o, F_o = search.sweep(st, Zo, base, off, cells, freqs)
    pb = pxd.Problem.from_spec(spec)
    for prec in (pxd.PREC_FP64, pxd.PREC_MIXED32):
        ev = pxd.Evaluator(precision=prec)
        ev.load_problem(pb, spec.z0)
        ev.load_parent_problem(pb, freqs)
        ev.set_fom_paper()
        S, F, status, am = ev.evaluate_flips(base, off, cells)
        ev.close()
        tol = 1e-10 if prec == pxd.PREC_FP64 else 1e-4
        print(f"precision {prec}: max |dS| {np.abs(S - S_o).max():.2e}")
        assert np.all((status == 0) | (status == 1))
        assert np.abs(S - S_o).max() <= tol
