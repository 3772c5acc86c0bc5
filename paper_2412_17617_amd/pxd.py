"""Python binding of ``libpxd.so`` (ctypes).  Argument marshalling only.

Every computation runs in the library: the structure builder and parent fill
on the host (C++), everything else in the gfx950 kernels.  There is no Python
or CPU fallback; if the library is missing the import fails.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PXD_LIB_PATH") or os.path.join(_HERE, "libpxd.so")

OK, EINVAL, ENOMEM, ENOTLOADED, EDEVICE, ESHAPE = 0, -1, -2, -3, -4, -5
PREC_FP64, PREC_MIXED32, PREC_MIXED_BF16, PREC_MIXED_F16, PREC_MIXED_BF16X3 = 0, 1, 2, 3, 4
KIND_ALWAYS, KIND_INNER, KIND_INTER, KIND_PIXPORT, KIND_VIA = 0, 1, 2, 3, 4
STATUS_OK, STATUS_FALLBACK, STATUS_NONFINITE, STATUS_SINGULAR, STATUS_SIZE = 0, 1, -1, -2, -3
SCHED_AUTO, SCHED_FREQ_MAJOR, SCHED_SIZE_MAJOR = 0, 1, 2
PATH_AUTO, PATH_PERSISTENT, PATH_TILED = 0, 1, 2
REFINE_AUTO, REFINE_PER_ITEM, REFINE_LOCKSTEP = 0, 1, 2
FOM_PAPER, FOM_REJ, FOM_ISO = 0, 1, 2
SIDES = {"right": 0, "top": 1, "left": 2, "bottom": 3}


class PxdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pxd error {code}: {msg}")
        self.code = code


class Geometry(C.Structure):
    _fields_ = [
        ("n_layers", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
        ("a", C.c_double), ("h", C.c_double), ("eps_r", C.c_double), ("tan_d", C.c_double),
        ("n_ports", C.c_int32), ("port_side", C.POINTER(C.c_int32)), ("port_layer", C.POINTER(C.c_int32)),
        ("n_vias", C.c_int32), ("via_x", C.POINTER(C.c_int32)), ("via_y", C.POINTER(C.c_int32)),
        ("sub", C.c_int32),
    ]


class Options(C.Structure):
    _fields_ = [
        ("device", C.c_int32), ("precision", C.c_int32), ("ir_max_iter", C.c_int32), ("ir_tol", C.c_double),
        ("wg_per_cu", C.c_int32), ("half_subpanel", C.c_int32), ("schedule", C.c_int32),
        ("lu_path", C.c_int32), ("tile_kb", C.c_int32), ("tile_shape", C.c_int32), ("ws_gib", C.c_double),
        ("refine", C.c_int32),
    ]


class FomTerm(C.Structure):
    _fields_ = [("band", C.c_int32), ("i", C.c_int32), ("j", C.c_int32), ("log10_factor", C.c_double),
                ("power", C.c_double)]


class Stats(C.Structure):
    _fields_ = [
        ("items", C.c_int64), ("fallbacks", C.c_int64), ("ir_iterations", C.c_int64),
        ("max_active", C.c_int32), ("min_active", C.c_int32),
        ("ms_expand", C.c_double), ("ms_solve", C.c_double), ("ms_fallback", C.c_double), ("ms_fom", C.c_double),
        ("ms_base_inverse", C.c_double), ("base_reused", C.c_int32), ("update_launches", C.c_int32),
        ("ms_update", C.c_double), ("update_gflop", C.c_double), ("update_gbyte", C.c_double),
    ]


class TuneEntry(C.Structure):
    _fields_ = [("rows_per_thread", C.c_int32), ("wg_per_cu", C.c_int32), ("half_subpanel", C.c_int32),
                ("schedule", C.c_int32), ("lu_path", C.c_int32), ("tile_kb", C.c_int32), ("tile_shape", C.c_int32),
                ("reserved", C.c_int32), ("ms", C.c_double)]


_VP = C.c_void_p
_SIGS = {
    "pxd_problem_create": (C.c_int, [C.POINTER(Geometry), C.POINTER(_VP)]),
    "pxd_problem_destroy": (None, [_VP]),
    "pxd_problem_sizes": (C.c_int, [_VP, _VP, _VP, _VP]),
    "pxd_problem_classification": (C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "pxd_problem_fill": (C.c_int, [_VP, C.c_int32, _VP, _VP, C.c_int32]),
    "pxd_problem_fill_device": (C.c_int, [_VP, C.c_int32, _VP, C.c_int32, _VP, _VP]),
    "pxd_load_parent_problem": (C.c_int, [_VP, _VP, C.c_int32, _VP]),
    "pxd_create": (C.c_int, [C.POINTER(Options), C.POINTER(_VP)]),
    "pxd_destroy": (None, [_VP]),
    "pxd_last_error": (C.c_char_p, [_VP]),
    "pxd_load_parent": (C.c_int, [_VP, C.c_int32, C.c_int32, _VP, _VP]),
    "pxd_load_map": (C.c_int, [_VP, C.c_int32, C.c_int32, _VP, _VP, _VP, C.c_int32, _VP, _VP, C.c_double]),
    "pxd_set_fom": (C.c_int, [_VP, C.c_int32, _VP, _VP]),
    "pxd_set_fom_paper": (C.c_int, [_VP]),
    "pxd_set_fom_variant": (C.c_int, [_VP, C.c_int32]),
    "pxd_evaluate_flips": (C.c_int, [_VP, _VP, C.c_int32, _VP, _VP, _VP, _VP, _VP, _VP]),
    "pxd_evaluate_flips_lowrank": (C.c_int, [_VP, _VP, C.c_int32, _VP, _VP, _VP, _VP, _VP, _VP]),
    "pxd_evaluate_flips_device": (C.c_int, [_VP, _VP, _VP, C.c_int32, _VP, _VP, C.c_int32, _VP, _VP, _VP, _VP]),
    "pxd_evaluate_flips_device_noalloc": (C.c_int, [_VP, _VP, _VP, C.c_int32, _VP, _VP, C.c_int32, _VP, _VP, _VP,
                                                    _VP]),
    "pxd_expand": (C.c_int, [_VP, _VP, C.c_int32, _VP, _VP, _VP, _VP]),
    "pxd_gather": (C.c_int, [_VP, C.c_int32, C.c_int32, _VP, _VP]),
    "pxd_get_stats": (C.c_int, [_VP, C.POINTER(Stats)]),
    "pxd_set_profiling": (C.c_int, [_VP, C.c_int32]),
    "pxd_refine_verdict": (C.c_int, [C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_double]),
    "pxd_evaluate_maps": (C.c_int, [_VP, C.c_int32, _VP, _VP, _VP, _VP, _VP]),
    "pxd_evaluate_maps_device": (C.c_int, [_VP, _VP, C.c_int32, _VP, _VP, _VP, _VP, _VP]),
    "pxd_autotune": (C.c_int, [_VP, _VP, C.c_int32, _VP, _VP, C.c_int32, _VP, C.c_int32, _VP]),
    "pxd_tune_save": (C.c_int, [_VP, C.c_char_p]),
    "pxd_tune_load": (C.c_int, [_VP, C.c_char_p]),
    "pxd_graph_create": (C.c_int, [_VP, _VP, C.c_int64, C.c_int32, _VP, _VP, C.c_int32, _VP, _VP, _VP, _VP,
                                   C.POINTER(_VP)]),
    "pxd_graph_launch": (C.c_int, [_VP, _VP]),
    "pxd_graph_destroy": (None, [_VP]),
}

_lib_handle = None


def lib():
    """Load libpxd.so (built by ``python -m paper_2412_17617_amd.build``)."""
    global _lib_handle
    if _lib_handle is None:
        # One HIP runtime per process: PyTorch ships its own libamdhip64.so.7
        # under the same soname as the system one the library links.  Loading
        # torch first makes the library bind to torch's copy, so device
        # pointers and streams from torch are valid here; loaded the other
        # way round, torch would run on a runtime it was not built for.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2412_17617_amd.build")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib_handle = h
    return _lib_handle


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_VP)


def _check(rc, ctx=None):
    if rc != OK:
        msg = lib().pxd_last_error(ctx)
        raise PxdError(rc, msg.decode() if msg else "")


def refine_verdict(iters, ir_max, m, m_prev, target):
    """The mixed-precision refinement's stop / give-up rule for one step
    (pxd_refine_verdict): 1 converged, 2 hand to FP64, 0 continue."""
    rc = lib().pxd_refine_verdict(iters, ir_max, m, m_prev, target)
    if rc < 0:
        _check(rc)
    return rc


class Problem:
    """Mesh + RWG classification + host EFIE fill of one workload geometry."""

    def __init__(self, n_layers, nx, ny, a, h, eps_r, tan_d, ports, vias=(), sub=1):
        L = lib()
        self._keep = [
            np.array([SIDES[s] if isinstance(s, str) else int(s) for s, _ in ports] or [0], dtype=np.int32),
            np.array([l for _, l in ports] or [0], dtype=np.int32),
            np.array([x for x, _ in vias] or [0], dtype=np.int32),
            np.array([y for _, y in vias] or [0], dtype=np.int32),
        ]
        g = Geometry(n_layers, nx, ny, a, h, eps_r, tan_d, len(ports),
                     self._keep[0].ctypes.data_as(C.POINTER(C.c_int32)),
                     self._keep[1].ctypes.data_as(C.POINTER(C.c_int32)), len(vias),
                     self._keep[2].ctypes.data_as(C.POINTER(C.c_int32)),
                     self._keep[3].ctypes.data_as(C.POINTER(C.c_int32)), int(sub))
        h_ = _VP()
        _check(L.pxd_problem_create(C.byref(g), C.byref(h_)))
        self._h = h_
        M, nc, npo = C.c_int32(), C.c_int32(), C.c_int32()
        _check(L.pxd_problem_sizes(self._h, C.byref(M), C.byref(nc), C.byref(npo)))
        self.M, self.n_cells, self.n_ports = M.value, nc.value, npo.value

    @classmethod
    def from_spec(cls, spec):
        """Build from any object with the workload attributes (n_layers, nx, ny,
        a, h, eps_r, tan_d, ports with .side/.layer, via_sites(), optionally
        sub)."""
        return cls(spec.n_layers, spec.nx, spec.ny, spec.a, spec.h, spec.eps_r, spec.tan_d,
                   [(p.side, p.layer) for p in spec.ports], list(spec.via_sites()), getattr(spec, "sub", 1))

    def classification(self):
        kind = np.zeros(self.M, np.uint8)
        ca = np.zeros(self.M, np.int32)
        cb = np.zeros(self.M, np.int32)
        pbf = np.zeros(self.n_ports, np.int32)
        plen = np.zeros(self.n_ports, np.float64)
        _check(lib().pxd_problem_classification(self._h, _ptr(kind), _ptr(ca), _ptr(cb), _ptr(pbf), _ptr(plen)))
        return kind, ca, cb, pbf, plen

    def fill(self, freqs, n_threads=0, out=None):
        freqs = np.ascontiguousarray(freqs, dtype=np.float64)
        Z = out if out is not None else np.empty((len(freqs), self.M, self.M), np.complex128)
        assert Z.shape == (len(freqs), self.M, self.M) and Z.dtype == np.complex128 and Z.flags.c_contiguous
        _check(lib().pxd_problem_fill(self._h, len(freqs), _ptr(freqs), _ptr(Z), n_threads))
        return Z

    def fill_device(self, freqs, out, stream=None, device=0):
        """Fill on the GPU into `out`: a device buffer of F x M x M complex128
        (a torch CUDA tensor, complex128 or float64 with a trailing 2, or any
        object with data_ptr()).  Returns when the fill is finished."""
        freqs = np.ascontiguousarray(freqs, dtype=np.float64)
        sp = getattr(stream, "cuda_stream", stream)
        _check(lib().pxd_problem_fill_device(self._h, device, _VP(sp) if sp else None, len(freqs), _ptr(freqs),
                                             _VP(out.data_ptr())))
        return out

    def __del__(self):
        if getattr(self, "_h", None) and _lib_handle is not None:
            _lib_handle.pxd_problem_destroy(self._h)
            self._h = None


class Evaluator:
    """GPU evaluator context (one per device and host thread)."""

    def __init__(self, device=0, precision=PREC_FP64, ir_max_iter=10, ir_tol=1e-7, wg_per_cu=0, half_subpanel=0,
                 schedule=SCHED_AUTO, lu_path=0, tile_kb=0, tile_shape=0, ws_gib=0.0, refine=0):
        o = Options(device, precision, ir_max_iter, ir_tol, wg_per_cu, half_subpanel, schedule, lu_path, tile_kb,
                    tile_shape, ws_gib, refine)
        h_ = _VP()
        _check(lib().pxd_create(C.byref(o), C.byref(h_)))
        self._h = h_
        self.M = self.F = self.P = self.n_cells = 0

    def _c(self, rc):
        _check(rc, self._h)

    def load_parent(self, Z, freqs):
        Z = np.ascontiguousarray(Z, dtype=np.complex128)
        freqs = np.ascontiguousarray(freqs, dtype=np.float64)
        F, M, M2 = Z.shape
        assert M == M2 and F == len(freqs)
        self._c(lib().pxd_load_parent(self._h, M, F, _ptr(freqs), _ptr(Z)))
        self.M, self.F = M, F

    def load_parent_problem(self, problem, freqs):
        """Parent filled on this context's GPU from the structure (no host matrix)."""
        freqs = np.ascontiguousarray(freqs, dtype=np.float64)
        self._c(lib().pxd_load_parent_problem(self._h, problem._h, len(freqs), _ptr(freqs)))
        self.M, self.F = problem.M, len(freqs)

    def load_map(self, n_cells, kind, cell_a, cell_b, port_bf, port_len, z0=50.0):
        kind = np.ascontiguousarray(kind, np.uint8)
        ca = np.ascontiguousarray(cell_a, np.int32)
        cb = np.ascontiguousarray(cell_b, np.int32)
        pbf = np.ascontiguousarray(port_bf, np.int32)
        pl = np.ascontiguousarray(port_len, np.float64)
        self._c(lib().pxd_load_map(self._h, n_cells, len(ca), _ptr(kind), _ptr(ca), _ptr(cb), len(pbf), _ptr(pbf),
                                   _ptr(pl), z0))
        self.n_cells, self.P, self.M = n_cells, len(pbf), len(ca)

    def load_problem(self, problem: Problem, z0=50.0):
        kind, ca, cb, pbf, pl = problem.classification()
        self.load_map(problem.n_cells, kind, ca, cb, pbf, pl, z0)

    def set_fom_paper(self, variant=0):
        """variant: FOM_PAPER (Eqs. 8-9), FOM_REJ or FOM_ISO (Section III-D)."""
        self._c(lib().pxd_set_fom_variant(self._h, variant))

    def set_fom(self, terms, band_of_freq):
        arr = (FomTerm * max(1, len(terms)))(*[FomTerm(*t) for t in terms])
        band = np.ascontiguousarray(band_of_freq, np.int8)
        self._c(lib().pxd_set_fom(self._h, len(terms), C.cast(arr, _VP), _ptr(band)))

    def evaluate_flips(self, base_map, offsets, cells, want_S=True):
        base = np.ascontiguousarray(base_map, np.uint8)
        off = np.ascontiguousarray(offsets, np.int32)
        cl = np.ascontiguousarray(cells, np.int32)
        n = len(off) - 1
        S = np.empty((n, self.F, self.P, self.P), np.complex128) if want_S else None
        fom = np.empty(n, np.float64)
        st = np.empty(n, np.int32)
        am = np.zeros(1, np.int32)
        self._c(lib().pxd_evaluate_flips(self._h, _ptr(base), n, _ptr(off), _ptr(cl if len(cl) else
                                         np.zeros(1, np.int32)), _ptr(S), _ptr(fom), _ptr(st), _ptr(am)))
        return S, fom, st, int(am[0])

    def evaluate_flips_lowrank(self, base_map, offsets, cells, want_S=True):
        """As evaluate_flips, solved from the cached inverse of the base map."""
        base = np.ascontiguousarray(base_map, np.uint8)
        off = np.ascontiguousarray(offsets, np.int32)
        cl = np.ascontiguousarray(cells, np.int32)
        n = len(off) - 1
        S = np.empty((n, self.F, self.P, self.P), np.complex128) if want_S else None
        fom = np.empty(n, np.float64)
        st = np.empty(n, np.int32)
        am = np.zeros(1, np.int32)
        self._c(lib().pxd_evaluate_flips_lowrank(self._h, _ptr(base), n, _ptr(off), _ptr(cl if len(cl) else
                                                 np.zeros(1, np.int32)), _ptr(S), _ptr(fom), _ptr(st), _ptr(am)))
        return S, fom, st, int(am[0])

    def evaluate_flips_device(self, stream, base_map, offsets, cells, S_out, fom_out, status_out=None,
                              argmin_out=None):
        """All arrays are torch CUDA tensors (or objects with data_ptr());
        stream is a torch.cuda.Stream or a raw hipStream_t integer."""
        sp = getattr(stream, "cuda_stream", stream)

        def dp(t):
            return None if t is None else _VP(t.data_ptr())

        n = offsets.numel() - 1
        self._c(lib().pxd_evaluate_flips_device(self._h, _VP(sp), dp(base_map), n, dp(offsets), dp(cells),
                                                cells.numel(), dp(S_out), dp(fom_out), dp(status_out),
                                                dp(argmin_out)))

    def evaluate_flips_device_noalloc(self, stream, base_map, offsets, cells, S_out, fom_out, status_out=None,
                                      argmin_out=None):
        """As evaluate_flips_device, with every internal buffer taken from the
        library's static scratch array (no device allocation)."""
        sp = getattr(stream, "cuda_stream", stream)

        def dp(t):
            return None if t is None else _VP(t.data_ptr())

        n = offsets.numel() - 1
        self._c(lib().pxd_evaluate_flips_device_noalloc(self._h, _VP(sp), dp(base_map), n, dp(offsets), dp(cells),
                                                        cells.numel(), dp(S_out), dp(fom_out), dp(status_out),
                                                        dp(argmin_out)))

    def evaluate_maps(self, maps, want_S=True):
        """Candidates given as whole maps (n_maps x n_cells uint8)."""
        maps = np.ascontiguousarray(maps, np.uint8)
        n = maps.shape[0]
        assert maps.ndim == 2 and maps.shape[1] == self.n_cells
        S = np.empty((n, self.F, self.P, self.P), np.complex128) if want_S else None
        fom = np.empty(n, np.float64)
        st = np.empty(n, np.int32)
        am = np.zeros(1, np.int32)
        self._c(lib().pxd_evaluate_maps(self._h, n, _ptr(maps), _ptr(S), _ptr(fom), _ptr(st), _ptr(am)))
        return S, fom, st, int(am[0])

    def evaluate_maps_device(self, stream, maps, S_out, fom_out, status_out=None, argmin_out=None):
        sp = getattr(stream, "cuda_stream", stream)

        def dp(t):
            return None if t is None else _VP(t.data_ptr())

        self._c(lib().pxd_evaluate_maps_device(self._h, _VP(sp), maps.shape[0], dp(maps), dp(S_out), dp(fom_out),
                                               dp(status_out), dp(argmin_out)))

    def autotune(self, base_map, offsets, cells, n_reps=1):
        """Time every launch configuration on this batch; the fastest becomes
        the context's choice for its precision and size class.  Returns the
        tried configurations, fastest first."""
        base = np.ascontiguousarray(base_map, np.uint8)
        off = np.ascontiguousarray(offsets, np.int32)
        cl = np.ascontiguousarray(cells, np.int32)
        rep = (TuneEntry * 64)()
        n = C.c_int32()
        self._c(lib().pxd_autotune(self._h, _ptr(base), len(off) - 1, _ptr(off),
                                   _ptr(cl if len(cl) else np.zeros(1, np.int32)), n_reps, C.cast(rep, _VP), 64,
                                   C.byref(n)))
        return [{k: getattr(rep[i], k) for k, _ in TuneEntry._fields_} for i in range(n.value)]

    def tune_save(self, path):
        self._c(lib().pxd_tune_save(self._h, os.fsencode(path)))

    def tune_load(self, path):
        self._c(lib().pxd_tune_load(self._h, os.fsencode(path)))

    def graph(self, base_map, offsets, cells, n_max_active, S_out, fom_out, status_out=None, argmin_out=None,
              maps=False):
        """Capture the device-side evaluation of this batch (torch CUDA
        tensors) into a HIP graph; returns a Graph to launch repeatedly."""
        return Graph(self, base_map, offsets, cells, n_max_active, S_out, fom_out, status_out, argmin_out, maps)

    def expand(self, base_map, offsets, cells):
        base = np.ascontiguousarray(base_map, np.uint8)
        off = np.ascontiguousarray(offsets, np.int32)
        cl = np.ascontiguousarray(cells, np.int32)
        n = len(off) - 1
        N = np.empty(n, np.int32)
        idx = np.empty((n, self.M), np.int32)
        self._c(lib().pxd_expand(self._h, _ptr(base), n, _ptr(off), _ptr(cl if len(cl) else np.zeros(1, np.int32)),
                                 _ptr(N), _ptr(idx)))
        return N, [idx[c, :N[c]].copy() for c in range(n)]

    def gather(self, f, idx):
        idx = np.ascontiguousarray(idx, np.int32)
        out = np.empty((len(idx), len(idx)), np.complex128)
        self._c(lib().pxd_gather(self._h, f, len(idx), _ptr(idx), _ptr(out)))
        return out

    def set_profiling(self, on=True):
        """Time every trailing-update launch of the tiled path (stats()['ms_update'])
        and count its algorithmic work (stats()['update_gflop'])."""
        self._c(lib().pxd_set_profiling(self._h, 1 if on else 0))

    def stats(self):
        s = Stats()
        self._c(lib().pxd_get_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def close(self):
        if getattr(self, "_h", None) and _lib_handle is not None:
            _lib_handle.pxd_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


class Graph:
    """A captured evaluation (pxd_graph_*).  Holds references to the tensors it
    reads and writes so they outlive it."""

    def __init__(self, ev, base_map, offsets, cells, n_max_active, S_out, fom_out, status_out, argmin_out, maps):
        def dp(t):
            return None if t is None else _VP(t.data_ptr())

        self._ev = ev
        self._keep = (base_map, offsets, cells, S_out, fom_out, status_out, argmin_out)
        if maps:
            n, stride = base_map.shape[0], base_map.shape[1]
            off_p, cells_p = None, None
        else:
            n, stride = offsets.numel() - 1, 0
            off_p, cells_p = dp(offsets), dp(cells)
        h_ = _VP()
        ev._c(lib().pxd_graph_create(ev._h, dp(base_map), stride, n, off_p, cells_p, n_max_active, dp(S_out),
                                     dp(fom_out), dp(status_out), dp(argmin_out), C.byref(h_)))
        self._h = h_

    def launch(self, stream=None):
        sp = 0 if stream is None else getattr(stream, "cuda_stream", stream)
        _check(lib().pxd_graph_launch(self._h, _VP(sp)))

    def close(self):
        if getattr(self, "_h", None) and _lib_handle is not None:
            _lib_handle.pxd_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


SUR_FP32, SUR_BF16 = 0, 1
SUR_INFER_AUTO, SUR_INFER_GENERIC, SUR_INFER_FUSED = 0, 1, 2


class SurConfig(C.Structure):
    _fields_ = [
        ("device", C.c_int32), ("n_layers", C.c_int32), ("ny", C.c_int32), ("nx", C.c_int32),
        ("channels", C.c_int32 * 4), ("hidden", C.c_int32), ("emb", C.c_int32), ("n_entries", C.c_int32),
        ("entry_i", C.c_int32 * 4), ("entry_j", C.c_int32 * 4), ("precision", C.c_int32), ("max_batch", C.c_int32),
        ("inference", C.c_int32),
    ]


class AdamW(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("weight_decay", C.c_double)]


_SIGS.update({
    "pxd_sur_create": (C.c_int, [C.POINTER(SurConfig), C.c_int32, _VP, C.c_double, C.c_double, C.POINTER(_VP)]),
    "pxd_sur_destroy": (None, [_VP]),
    "pxd_sur_last_error": (C.c_char_p, [_VP]),
    "pxd_sur_num_params": (C.c_int, [_VP, C.POINTER(C.c_int64)]),
    "pxd_sur_init_params": (C.c_int, [_VP, C.c_uint64]),
    "pxd_sur_set_params": (C.c_int, [_VP, _VP, C.c_int64]),
    "pxd_sur_get_params": (C.c_int, [_VP, _VP, C.c_int64]),
    "pxd_sur_forward": (C.c_int, [_VP, _VP, C.c_int32, _VP, _VP]),
    "pxd_sur_gradient": (C.c_int, [_VP, _VP, C.c_int32, _VP, _VP, _VP, _VP]),
    "pxd_sur_train_step": (C.c_int, [_VP, _VP, C.c_int32, _VP, _VP, C.POINTER(AdamW), _VP]),
    "pxd_sur_rank": (C.c_int, [_VP, _VP, _VP, _VP, C.c_int32, _VP, _VP, C.c_int32, _VP, _VP]),
    "pxd_sur_encode": (C.c_int, [_VP, _VP, C.c_int32, _VP, C.c_int32, _VP]),
    "pxd_sur_inference_path": (C.c_int, [_VP, _VP]),
})


class Surrogate:
    """CNN surrogate (pxd_sur_*).  Device arrays are torch CUDA tensors (or any
    object with data_ptr()); stream is a torch.cuda.Stream, a raw handle or
    None (HIP's default stream)."""

    def __init__(self, n_layers, ny, nx, freqs, f_lo, f_hi, entries=((0, 0), (1, 0), (2, 0)),
                 channels=(32, 32, 64, 64), hidden=256, emb=16, precision=SUR_BF16, max_batch=64, device=0,
                 inference=SUR_INFER_AUTO):
        c = SurConfig()
        c.device, c.n_layers, c.ny, c.nx = device, n_layers, ny, nx
        for i in range(4):
            c.channels[i] = channels[i]
        c.hidden, c.emb, c.n_entries = hidden, emb, len(entries)
        for k, (i, j) in enumerate(entries):
            c.entry_i[k], c.entry_j[k] = i, j
        c.precision, c.max_batch, c.inference = precision, max_batch, inference
        freqs = np.ascontiguousarray(freqs, np.float64)
        h_ = _VP()
        _check(lib().pxd_sur_create(C.byref(c), len(freqs), _ptr(freqs), f_lo, f_hi, C.byref(h_)))
        self._h = h_
        self.F, self.n_out, self.max_batch = len(freqs), 3 * len(entries), max_batch
        n = C.c_int64()
        self._c(lib().pxd_sur_num_params(self._h, C.byref(n)))
        self.n_params = n.value
        path = C.c_int32()
        self._c(lib().pxd_sur_inference_path(self._h, C.byref(path)))
        self.inference = path.value

    def _c(self, rc):
        if rc != OK:
            msg = lib().pxd_sur_last_error(self._h)
            raise PxdError(rc, msg.decode() if msg else "")

    @staticmethod
    def _s(stream):
        return _VP(0 if stream is None else getattr(stream, "cuda_stream", stream))

    @staticmethod
    def _d(t):
        return None if t is None else _VP(t.data_ptr())

    def init_params(self, seed):
        self._c(lib().pxd_sur_init_params(self._h, seed))

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        self._c(lib().pxd_sur_set_params(self._h, _ptr(p), len(p)))

    def get_params(self):
        p = np.empty(self.n_params, np.float32)
        self._c(lib().pxd_sur_get_params(self._h, _ptr(p), len(p)))
        return p

    def forward(self, maps, out, stream=None):
        self._c(lib().pxd_sur_forward(self._h, self._s(stream), maps.shape[0], self._d(maps), self._d(out)))

    def gradient(self, maps, target, grad=None, loss=None, stream=None):
        self._c(lib().pxd_sur_gradient(self._h, self._s(stream), maps.shape[0], self._d(maps), self._d(target),
                                       self._d(grad), self._d(loss)))

    def train_step(self, maps, target, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0, loss=None,
                   stream=None):
        hp = AdamW(lr, beta1, beta2, eps, weight_decay)
        self._c(lib().pxd_sur_train_step(self._h, self._s(stream), maps.shape[0], self._d(maps), self._d(target),
                                         C.byref(hp), self._d(loss)))

    def rank(self, evaluator, base_map, offsets, cells, k, fom_pred, top, stream=None):
        self._c(lib().pxd_sur_rank(self._h, evaluator._h, self._s(stream), self._d(base_map), offsets.numel() - 1,
                                   self._d(offsets), self._d(cells), k, self._d(fom_pred), self._d(top)))

    def encode_device(self, S, target, stream=None):
        """Training targets on the device from exact S (torch CUDA tensors:
        S n x F x P x P x 2 float64, target n x F x 3 n_entries float32)."""
        n, P = S.shape[0], S.shape[2]
        self._c(lib().pxd_sur_encode(self._h, self._s(stream), n, self._d(S), P, self._d(target)))

    @staticmethod
    def encode(S, entries=((0, 0), (1, 0), (2, 0))):
        """Training targets from S (..., P, P): per entry ln|S|, cos arg S, sin arg S."""
        out = []
        for i, j in entries:
            v = S[..., i, j]
            a = np.maximum(np.abs(v), 1e-30)
            out += [np.log(a), v.real / a, v.imag / a]
        return np.stack(out, axis=-1).astype(np.float32)

    def close(self):
        if getattr(self, "_h", None) and _lib_handle is not None:
            _lib_handle.pxd_sur_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()
