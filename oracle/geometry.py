"""Pixel mesh, feeds, vias and RWG basis-function classification (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Follows Section II-C and Fig. 2(a) of the paper: every RWG function
(Section II-B, one per interior triangle edge) is classified as

* always present  -- feed-line functions that exist for every pixel map,
* inner pixel     -- the edge inside one pixel; active iff that pixel is on,
* inter pixel     -- the edge between two side-adjacent pixels; active iff
                     both are on,
* pixel port      -- the edge joining a feed to its adjacent pixel; active iff
                     that pixel is on,

plus a via class (a vertical strip joining layers 0 and 1, active iff the two
pixels it joins are on).  Each pixel carries two triangles whose diagonals
alternate in a checkerboard, the mesh the paper selects in Section V.
Pixels that touch only at a corner share no edge, so they are not connected
(the over-etch reading of Section VI-A).

Vertices are identified by exact integer keys (2x, 2y, layer) in units of
half a pixel, so topology can be checked without floating-point tolerances.

Parity: pinned by closed-form counts, by the equality of the classification
rule's active set with the interior edges of a freshly meshed substructure,
and by the diagonal-contact rule (tests/test_oracle_geometry.py).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

KIND_ALWAYS, KIND_INNER, KIND_INTER, KIND_PIXPORT, KIND_VIA = 0, 1, 2, 3, 4


@dataclass
class BasisFunction:
    kind: int
    cells: tuple  # canonical cell indices that must all be on
    edge: tuple  # (key0, key1), the shared edge
    tplus: int  # triangle on the + side (current leaves it across the edge)
    tminus: int
    port: int = -1  # port number if this is a port (delta-gap) edge


@dataclass
class Structure:
    spec: object
    tri_keys: list  # list of 3-tuples of vertex keys
    tri_owner: list  # ("cell", c) / ("feed", port, "inner"|"outer") / ("via", site)
    bfs: list  # list of BasisFunction in canonical order
    port_bf: list  # index of port k's delta-gap function

    def xyz(self, key):
        s = self.spec
        return np.array([key[0] * s.a / 2.0, key[1] * s.a / 2.0, -key[2] * s.h])

    def tri_xyz(self) -> np.ndarray:
        return np.array([[self.xyz(k) for k in t] for t in self.tri_keys])

    @property
    def M(self) -> int:
        return len(self.bfs)

    def cell_index(self, layer, x, y) -> int:
        s = self.spec
        return layer * s.ny * s.nx + y * s.nx + x

    def active(self, pixel_map) -> np.ndarray:
        """Boolean selection vector S_sub of Fig. 2(c): a function is present iff
        every cell it depends on is on."""
        pm = np.asarray(pixel_map).astype(bool)
        return np.array([all(pm[c] for c in bf.cells) for bf in self.bfs], dtype=bool)


def _pixel_tris(x, y, l):
    LL, LR, UR, UL = (2 * x, 2 * y, l), (2 * x + 2, 2 * y, l), (2 * x + 2, 2 * y + 2, l), (2 * x, 2 * y + 2, l)
    if (x + y) % 2 == 0:  # diagonal from lower-left to upper-right
        return (LL, LR, UR), (LL, UR, UL), (LL, UR)
    return (LL, LR, UL), (LR, UR, UL), (LR, UL)  # diagonal from lower-right to upper-left


def _pixel_side_tri(x, y, side):
    """Which of the pixel's two triangles (0 = lower, 1 = upper) holds a side."""
    even = (x + y) % 2 == 0
    if side == "bottom":
        return 0
    if side == "top":
        return 1
    if side == "left":
        return 1 if even else 0
    if side == "right":
        return 0 if even else 1
    raise ValueError(side)


def _rect_tris(x0, x1, y0, y1, l):
    """Rectangle (half-pixel key units) split by its lower-left/upper-right
    diagonal; the lower triangle holds the bottom and right sides."""
    LL, LR, UR, UL = (x0, y0, l), (x1, y0, l), (x1, y1, l), (x0, y1, l)
    return (LL, LR, UR), (LL, UR, UL), (LL, UR)


def build_structure(spec) -> Structure:
    nx, ny, L = spec.nx, spec.ny, spec.n_layers
    tri_keys, tri_owner = [], []
    cell_tris = {}
    for l in range(L):
        for y in range(ny):
            for x in range(nx):
                lo, up, _ = _pixel_tris(x, y, l)
                c = l * ny * nx + y * nx + x
                cell_tris[c] = (len(tri_keys), len(tri_keys) + 1)
                tri_keys += [lo, up]
                tri_owner += [("cell", c), ("cell", c)]

    def cidx(l, x, y):
        return l * ny * nx + y * nx + x

    def side_tri(l, x, y, side):
        return cell_tris[cidx(l, x, y)][_pixel_side_tri(x, y, side)]

    inner, inter_h, inter_v = [], [], []
    for l in range(L):
        for y in range(ny):
            for x in range(nx):
                c = cidx(l, x, y)
                _, _, diag = _pixel_tris(x, y, l)
                inner.append(BasisFunction(KIND_INNER, (c,), diag, cell_tris[c][0], cell_tris[c][1]))
    for l in range(L):
        for y in range(ny):
            for x in range(nx - 1):
                e = ((2 * x + 2, 2 * y, l), (2 * x + 2, 2 * y + 2, l))
                inter_h.append(BasisFunction(KIND_INTER, (cidx(l, x, y), cidx(l, x + 1, y)), e,
                                             side_tri(l, x, y, "right"), side_tri(l, x + 1, y, "left")))
    for l in range(L):
        for y in range(ny - 1):
            for x in range(nx):
                e = ((2 * x, 2 * y + 2, l), (2 * x + 2, 2 * y + 2, l))
                inter_v.append(BasisFunction(KIND_INTER, (cidx(l, x, y), cidx(l, x, y + 1)), e,
                                             side_tri(l, x, y, "top"), side_tri(l, x, y + 1, "bottom")))

    # Feeds: a one-pixel pad beyond the middle cell of a grid side, cut into an
    # inner and an outer half strip.  The delta-gap port sits on the line
    # between the two half strips; + side is the outer (source) side.
    pixport, feed_diag, port_edge = [], [], []
    for k, ps in enumerate(spec.ports):
        l = ps.layer
        if ps.side in ("right", "left"):
            j = ny // 2
            cx = nx - 1 if ps.side == "right" else 0
            cell = (cx, j)
            if ps.side == "right":
                inner_r = (2 * nx, 2 * nx + 1, 2 * j, 2 * j + 2)
                outer_r = (2 * nx + 1, 2 * nx + 2, 2 * j, 2 * j + 2)
            else:
                inner_r = (-1, 0, 2 * j, 2 * j + 2)
                outer_r = (-2, -1, 2 * j, 2 * j + 2)
        else:
            j = nx // 2
            cy = ny - 1 if ps.side == "top" else 0
            cell = (j, cy)
            if ps.side == "top":
                inner_r = (2 * j, 2 * j + 2, 2 * ny, 2 * ny + 1)
                outer_r = (2 * j, 2 * j + 2, 2 * ny + 1, 2 * ny + 2)
            else:
                inner_r = (2 * j, 2 * j + 2, -1, 0)
                outer_r = (2 * j, 2 * j + 2, -2, -1)
        ilo, iup, idiag = _rect_tris(*inner_r, l)
        olo, oup, odiag = _rect_tris(*outer_r, l)
        t0 = len(tri_keys)
        tri_keys += [ilo, iup, olo, oup]
        tri_owner += [("feed", k, "inner"), ("feed", k, "inner"), ("feed", k, "outer"), ("feed", k, "outer")]
        T_ilo, T_iup, T_olo, T_oup = t0, t0 + 1, t0 + 2, t0 + 3
        x0i, x1i, y0i, y1i = inner_r
        if ps.side == "right":
            pe = ((x1i, y0i, l), (x1i, y1i, l))
            port_pair = (T_oup, T_ilo)  # outer strip's left side / inner strip's right side
            ppe = ((x0i, y0i, l), (x0i, y1i, l))
            pp_pair = (T_iup, side_tri(l, cell[0], cell[1], "right"))
        elif ps.side == "left":
            pe = ((x0i, y0i, l), (x0i, y1i, l))
            port_pair = (T_olo, T_iup)
            ppe = ((x1i, y0i, l), (x1i, y1i, l))
            pp_pair = (T_ilo, side_tri(l, cell[0], cell[1], "left"))
        elif ps.side == "top":
            pe = ((x0i, y1i, l), (x1i, y1i, l))
            port_pair = (T_olo, T_iup)
            ppe = ((x0i, y0i, l), (x1i, y0i, l))
            pp_pair = (T_ilo, side_tri(l, cell[0], cell[1], "top"))
        else:  # bottom
            pe = ((x0i, y0i, l), (x1i, y0i, l))
            port_pair = (T_oup, T_ilo)
            ppe = ((x0i, y1i, l), (x1i, y1i, l))
            pp_pair = (T_iup, side_tri(l, cell[0], cell[1], "bottom"))
        c = cidx(l, cell[0], cell[1])
        pixport.append(BasisFunction(KIND_PIXPORT, (c,), ppe, pp_pair[0], pp_pair[1]))
        feed_diag.append(BasisFunction(KIND_ALWAYS, (), idiag, T_ilo, T_iup))
        feed_diag.append(BasisFunction(KIND_ALWAYS, (), odiag, T_olo, T_oup))
        port_edge.append(BasisFunction(KIND_ALWAYS, (), pe, port_pair[0], port_pair[1], port=k))

    # Vias: a vertical strip under the lower side line of cell (x, y), from
    # layer 0 down to layer 1, split by its top-left/bottom-right diagonal.
    vias = []
    for s_i, (x, y) in enumerate(spec.via_sites()):
        TL, TR, BR, BL = (2 * x, 2 * y, 0), (2 * x + 2, 2 * y, 0), (2 * x + 2, 2 * y, 1), (2 * x, 2 * y, 1)
        t0 = len(tri_keys)
        tri_keys += [(TL, TR, BR), (TL, BR, BL)]
        tri_owner += [("via", s_i), ("via", s_i)]
        tU, tLo = t0, t0 + 1
        cells = (cidx(0, x, y), cidx(1, x, y))
        vias.append(BasisFunction(KIND_VIA, cells, (TL, TR), side_tri(0, x, y, "bottom"), tU))
        vias.append(BasisFunction(KIND_VIA, cells, (TL, BR), tU, tLo))
        vias.append(BasisFunction(KIND_VIA, cells, (BL, BR), tLo, side_tri(1, x, y, "bottom")))

    bfs = inner + inter_h + inter_v + pixport + vias + feed_diag + port_edge
    port_bf = [i for i, b in enumerate(bfs) if b.port >= 0]
    return Structure(spec, tri_keys, tri_owner, bfs, port_bf)


def expected_count(spec) -> int:
    """Closed-form parent size: per layer nx*ny inner + (nx-1)*ny + nx*(ny-1)
    inter functions; four functions per port; three per via."""
    per_layer = spec.nx * spec.ny + (spec.nx - 1) * spec.ny + spec.nx * (spec.ny - 1)
    return spec.n_layers * per_layer + 4 * len(spec.ports) + 3 * spec.n_vias


def fresh_submesh_edges(struct: Structure, pixel_map) -> dict:
    """Mesh only what is metal under ``pixel_map`` (on pixels, feeds, vias whose
    two pixels are on) and return {edge: number of RWG functions it carries}
    (k-1 for an edge shared by k triangles)."""
    pm = np.asarray(pixel_map).astype(bool)
    keep = []
    for t, own in enumerate(struct.tri_owner):
        if own[0] == "cell":
            ok = pm[own[1]]
        elif own[0] == "feed":
            ok = True
        else:
            x, y = struct.spec.via_sites()[own[1]]
            ok = pm[struct.cell_index(0, x, y)] and pm[struct.cell_index(1, x, y)]
        if ok:
            keep.append(t)
    count = {}
    for t in keep:
        a, b, c = struct.tri_keys[t]
        for e in ((a, b), (b, c), (c, a)):
            key = tuple(sorted(e))
            count[key] = count.get(key, 0) + 1
    return {e: n - 1 for e, n in count.items() if n >= 2}


def rwg_geometry(struct: Structure):
    """Per-function arrays for the fill: edge length, + and - triangles and the
    free vertex (the triangle vertex off the edge) of each."""
    M = struct.M
    length = np.zeros(M)
    tri = np.zeros((M, 2), dtype=np.int64)
    free = np.zeros((M, 2, 3))
    for i, bf in enumerate(struct.bfs):
        e0, e1 = bf.edge
        length[i] = np.linalg.norm(struct.xyz(e1) - struct.xyz(e0))
        for s, t in enumerate((bf.tplus, bf.tminus)):
            tk = struct.tri_keys[t]
            assert e0 in tk and e1 in tk, "edge not on its triangle"
            fv = [k for k in tk if k != e0 and k != e1]
            assert len(fv) == 1
            tri[i, s] = t
            free[i, s] = struct.xyz(fv[0])
    return length, tri, free
