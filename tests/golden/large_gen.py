"""Writes the sampled oracle references of the large workloads.

Only the oracle (``oracle/``) and the seeded inputs (``synth/``) are used:
its own mesh, classification and EFIE fill at each listed frequency, Eq. 5's
gather, LAPACK's solve and Eqs. 6-7.  The GPU tests compare the library's S
on the same candidates and frequencies against these numbers, since one
oracle fill of these parents takes minutes.

  large_ceiling32.npz : the 32 x 32 x 3 stack (201 frequencies over
                        0.5-10 GHz, 3 x 3 pair-flip candidates): 16 seeded
                        candidates at 5 frequencies, one in each FoM band
                        and the lowest grid frequency (active size ~3,035).
  large_dense24.npz   : the 24 x 24 x 3 stack with a 0.65-density map
                        (active size ~2,530, above one workgroup's 2,048):
                        6 seeded single flips at 2 frequencies.
  large_paper30.npz   : the paper-size 8-triangle parent (2 layers of 30 x
                        30 pixels, M = 21,463): 2 seeded single flips at
                        5.5 GHz (active size ~9,460; the oracle fills the
                        union of their active sets only).
  large_mesh8.npz     : the 8-triangle mesh (2 layers of 12 x 12 pixels, each
                        a 2 x 2 grid of squares; M = 3,414, active size
                        ~1,400): 8 seeded single flips at 4 frequencies.

Usage: python tests/golden/large_gen.py [ceiling32] [dense24] [mesh8] [paper30]
"""

import dataclasses
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import efie, geometry, network, search  # noqa: E402
from synth import get_spec, permutation  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def cases():
    c32 = get_spec("ceiling32")
    d24 = dataclasses.replace(get_spec("stress24"), density=0.65)
    return {
        # name: (spec, number of candidates, candidate seed, frequency indices)
        "ceiling32": (c32, 16, 505, [0, 63, 105, 120, 133]),
        "dense24": (d24, 6, 506, [0, 64]),
        "mesh8": (get_spec("mesh8"), 8, 507, [0, 24, 29, 40]),
        "paper30": (get_spec("paper30"), 2, 508, [47]),
    }


def run(name):
    spec, n_pick, seed, fidx = cases()[name]
    st = geometry.build_structure(spec)
    base = spec.base_map()
    off, cells = spec.flips()
    C = len(off) - 1
    pick = np.sort(permutation(C, seed)[:n_pick]).astype(np.int32)
    maps = search.candidate_maps(base, off, cells)
    pl = search.port_lengths(st)
    P = len(st.port_bf)
    S = np.zeros((n_pick, len(fidx), P, P), np.complex128)
    N = np.zeros(n_pick, np.int32)
    # large parents: the oracle fills only the union of the sampled candidates' active sets
    union = np.zeros(st.M, bool)
    for c in pick:
        union |= st.active(maps[c])
    idx = network.support(union) if st.M > 12000 else np.arange(st.M)
    pos = -np.ones(st.M, np.int64)
    pos[idx] = np.arange(len(idx))
    for k, fi in enumerate(fidx):
        t = time.time()
        Z = efie.fill(st, spec.freqs[fi], bf_subset=idx if len(idx) < st.M else None)
        print(f"{name}: fill {k + 1}/{len(fidx)} ({spec.freqs[fi] / 1e9:.4f} GHz, M = {st.M}, "
              f"{len(idx)} functions filled) {time.time() - t:.0f} s", flush=True)
        for i, c in enumerate(pick):
            sel = st.active(maps[c])
            N[i] = int(sel.sum())
            rows = pos[network.support(sel)]
            S[i, k] = network.s_parameters(Z[np.ix_(rows, rows)], network.port_positions(sel, st.port_bf), pl,
                                           spec.z0)
        del Z
    np.savez(os.path.join(HERE, f"large_{name}.npz"), pick=pick, fidx=np.asarray(fidx, np.int32), S=S, N=N,
             density=np.float64(spec.density))
    print(f"{name}: N {N.min()}-{N.max()}, written", flush=True)


if __name__ == "__main__":
    for name in (sys.argv[1:] or ["dense24", "ceiling32"]):
        run(name)
