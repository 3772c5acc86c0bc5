"""Helpers shared by the GPU tests: oracle reference data and evaluator setup.

Oracle data is always computed by ``oracle/`` from the seeded inputs of
``synth/``; the GPU side may be handed the oracle's parent matrices as input
(never the other way round).
"""

import dataclasses
import functools

import numpy as np

from oracle import efie, geometry, network, search
from paper_2412_17617_amd import pxd
from synth import get_spec


def spec_variant(name, **kw):
    return dataclasses.replace(get_spec(name), **kw)


@functools.lru_cache(maxsize=None)
def _oracle_parent_cached(key):
    spec, fidx = key
    st = geometry.build_structure(spec)
    freqs = spec.freqs[list(fidx)]
    return st, np.stack([efie.fill(st, f) for f in freqs]), freqs


def oracle_parent(spec, fidx=None):
    fidx = tuple(range(spec.n_freq)) if fidx is None else tuple(fidx)
    return _oracle_parent_cached((spec, fidx))


def oracle_sweep(st, Z, base, off, cells, freqs):
    return search.sweep(st, Z, base, off, cells, freqs)


def make_evaluator(spec, Z, freqs, precision=pxd.PREC_FP64, **kw):
    pb = pxd.Problem.from_spec(spec)
    ev = pxd.Evaluator(precision=precision, **kw)
    ev.load_parent(Z, freqs)
    ev.load_problem(pb, spec.z0)
    ev.set_fom_paper()
    return ev, pb


def oracle_active_sets(st, base, off, cells):
    out = []
    for m in search.candidate_maps(base, off, cells):
        out.append(network.support(st.active(m)).astype(np.int32))
    return out


def fom_close(a, b, rtol):
    return np.all(np.abs(a - b) <= rtol * np.abs(b))
