"""The no-allocation entry point (pxd_evaluate_flips_device_noalloc) against
the allocating one it varies (pxd_evaluate_flips_device), through the C ABI
(GPU).  Both run the same kernels on the same inputs; only where the
workspace lives and how many persistent workgroups run differ, and neither
changes any item's arithmetic, so S, FoM, status and argmin must agree to the
FP64 path's bar (max |dS| <= 1e-10; in fact bit for bit).  Two calls in a row,
the second with a smaller batch, check that what the first leaves in the
shared scratch array does not leak into the second.  The oracle pins the
first call too.
"""

import numpy as np
import pytest

from oracle import search
from paper_2412_17617_amd import pxd
from synth import get_spec, single_flips

from gpu_common import make_evaluator, oracle_parent

pytestmark = pytest.mark.gpu

S_TOL = 1e-10
FOM_RTOL = 1e-6


def _dev(a, torch):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _run(ev, entry, base, off, cells, F, P, torch):
    C = len(off) - 1
    S = torch.full((C, F, P, P, 2), 7.0, dtype=torch.float64, device="cuda:0")
    fom = torch.full((C,), 7.0, dtype=torch.float64, device="cuda:0")
    st = torch.full((C,), 7, dtype=torch.int32, device="cuda:0")
    am = torch.full((1,), 7, dtype=torch.int32, device="cuda:0")
    stream = torch.cuda.current_stream()
    getattr(ev, entry)(stream, _dev(base, torch), _dev(off, torch), _dev(cells, torch), S, fom, st, am)
    torch.cuda.synchronize()
    return (torch.view_as_complex(S).cpu().numpy(), fom.cpu().numpy(), st.cpu().numpy(), int(am.cpu().numpy()[0]))


@pytest.mark.parametrize("prec", [pxd.PREC_FP64, pxd.PREC_MIXED32])
def test_no_alloc_matches_allocating_entry(prec):
    torch = pytest.importorskip("torch")
    spec = get_spec("tiny4x2")
    st, Z, freqs = oracle_parent(spec)
    P = len(spec.ports)
    base = spec.base_map()
    off1, cells1 = spec.flips()                 # all 32 single flips
    off2, cells2 = single_flips([3, 8, 21])     # then a smaller batch
    ev, _ = make_evaluator(spec, Z, freqs, precision=prec)
    print(f"precision {prec}: call 1 ({len(off1) - 1} candidates), call 2 ({len(off2) - 1})", flush=True)
    a1 = _run(ev, "evaluate_flips_device_noalloc", base, off1, cells1, len(freqs), P, torch)
    a2 = _run(ev, "evaluate_flips_device_noalloc", base, off2, cells2, len(freqs), P, torch)
    r1 = _run(ev, "evaluate_flips_device", base, off1, cells1, len(freqs), P, torch)
    r2 = _run(ev, "evaluate_flips_device", base, off2, cells2, len(freqs), P, torch)
    ev.close()
    for a, r in ((a1, r1), (a2, r2)):
        assert np.abs(a[0] - r[0]).max() <= S_TOL
        assert np.all(np.abs(a[1] - r[1]) <= FOM_RTOL * np.abs(r[1]))
        assert np.array_equal(a[2], r[2]) and a[3] == r[3]
        assert np.all(a[2] >= 0)
    S_o, F_o = search.sweep(st, Z, base, off1, cells1, freqs)
    bar = S_TOL if prec == pxd.PREC_FP64 else 1e-4
    assert np.abs(a1[0] - S_o).max() <= bar
    assert np.all(np.abs(a1[1] - F_o) <= FOM_RTOL * F_o)


def test_no_alloc_refuses_a_batch_beyond_its_scratch():
    """100,000 candidates of the 8x8 workload need 100,000 x (184 + 2) x 4
    bytes of active lists alone, above the 64 MiB array: refused before any
    kernel runs, and the next call still works."""
    torch = pytest.importorskip("torch")
    spec = get_spec("plain8")
    st, Z, freqs = oracle_parent(spec, fidx=(5,))
    P = len(spec.ports)
    ev, _ = make_evaluator(spec, Z, freqs)
    base = spec.base_map()
    C = 100_000
    off = np.arange(C + 1, dtype=np.int32)
    cells = (np.arange(C) % spec.n_cells).astype(np.int32)
    S = torch.empty((C, 1, P, P, 2), dtype=torch.float64, device="cuda:0")
    fom = torch.empty(C, dtype=torch.float64, device="cuda:0")
    with pytest.raises(pxd.PxdError) as e:
        ev.evaluate_flips_device_noalloc(torch.cuda.current_stream(), _dev(base, torch), _dev(off, torch),
                                         _dev(cells, torch), S, fom)
    assert e.value.code == pxd.ESHAPE
    del S, fom
    off2, cells2 = single_flips([0, 5])
    a = _run(ev, "evaluate_flips_device_noalloc", base, off2, cells2, 1, P, torch)
    r = _run(ev, "evaluate_flips_device", base, off2, cells2, 1, P, torch)
    ev.close()
    assert np.abs(a[0] - r[0]).max() <= S_TOL and a[3] == r[3]
