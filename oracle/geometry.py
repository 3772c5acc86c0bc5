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
alternate in a checkerboard, the mesh the paper selects in Section V; with
``spec.sub`` = s > 1 every pixel is an s x s grid of such squares (8 or 18
triangles per pixel, the denser meshes of the mesh study), the checkerboard
taken over the squares.  Pixels that touch only at a corner share no edge,
so they are not connected (the over-etch reading of Section VI-A).

Vertices are identified by exact integer keys in units of half a square
side (2 s x, 2 s y, layer at pixel corners), so topology can be checked
without floating-point tolerances.

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
        u = s.a / (2.0 * _sub(s))  # key unit: half a square side
        return np.array([key[0] * u, key[1] * u, -key[2] * s.h])

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


def _sub(spec) -> int:
    """Sub-squares per pixel side: 1 (2 triangles per pixel), 2 (8), 3 (18)."""
    return int(getattr(spec, "sub", 1) or 1)


def _square_tris(X0, Y0, l, parity):
    """One square of side 2 key units at (X0, Y0) split into two right
    triangles: parity 0 along the lower-left/upper-right diagonal, 1 along
    the lower-right/upper-left one.  Returns (lower, upper, diagonal edge);
    the lower triangle holds the bottom side, the upper the top side."""
    LL, LR, UR, UL = (X0, Y0, l), (X0 + 2, Y0, l), (X0 + 2, Y0 + 2, l), (X0, Y0 + 2, l)
    if parity == 0:
        return (LL, LR, UR), (LL, UR, UL), (LL, UR)
    return (LL, LR, UL), (LR, UR, UL), (LR, UL)


def _square_side(parity, side):
    """Which triangle of a square (0 = lower, 1 = upper) holds a side."""
    if side == "bottom":
        return 0
    if side == "top":
        return 1
    if side == "left":
        return 1 if parity == 0 else 0
    if side == "right":
        return 0 if parity == 0 else 1
    raise ValueError(side)


def _rect_tris(x0, x1, y0, y1, l):
    """Rectangle (key units) split by its lower-left/upper-right diagonal;
    the lower triangle holds the bottom and right sides."""
    LL, LR, UR, UL = (x0, y0, l), (x1, y0, l), (x1, y1, l), (x0, y1, l)
    return (LL, LR, UR), (LL, UR, UL), (LL, UR)


def _centroid(tri):
    return tuple(sum(v[i] for v in tri) / 3.0 for i in range(3))


def _lower_first(tri_keys, t1, t2):
    """(+, -) triangles of an in-plane edge: the lower centroid y first, the
    smaller centroid x on a tie."""
    c1, c2 = _centroid(tri_keys[t1]), _centroid(tri_keys[t2])
    return (t1, t2) if (c1[1], c1[0]) < (c2[1], c2[0]) else (t2, t1)


def build_structure(spec) -> Structure:
    """Mesh of the parent structure: every pixel an s x s grid of squares
    (s = spec.sub, default 1), each square split into two right triangles
    whose diagonals alternate in a checkerboard over the squares (the
    alternating mesh of Section V; s = 1, 2, 3 give 2, 8, 18 triangles per
    pixel).  Vertex keys are integers in units of half a square side."""
    nx, ny, L = spec.nx, spec.ny, spec.n_layers
    s = _sub(spec)
    W = 2 * s  # pixel side in key units
    tri_keys, tri_owner = [], []
    sq = {}  # (cell, u, v) -> (lower, upper, parity)

    def cidx(l, x, y):
        return l * ny * nx + y * nx + x

    for l in range(L):
        for y in range(ny):
            for x in range(nx):
                c = cidx(l, x, y)
                for v in range(s):
                    for u in range(s):
                        par = (s * x + u + s * y + v) % 2
                        lo, up, _ = _square_tris(W * x + 2 * u, W * y + 2 * v, l, par)
                        sq[(c, u, v)] = (len(tri_keys), len(tri_keys) + 1, par)
                        tri_keys += [lo, up]
                        tri_owner += [("cell", c), ("cell", c)]

    def side_tri(c, u, v, side):
        lo, up, par = sq[(c, u, v)]
        return (lo, up)[_square_side(par, side)]

    inner, inter_h, inter_v = [], [], []
    for l in range(L):
        for y in range(ny):
            for x in range(nx):
                c = cidx(l, x, y)
                fs = []
                for v in range(s):
                    for u in range(s):
                        lo, up, par = sq[(c, u, v)]
                        fs.append(((lo, up), _square_tris(W * x + 2 * u, W * y + 2 * v, l, par)[2]))
                        X0, Y0 = W * x + 2 * u, W * y + 2 * v
                        if u + 1 < s:  # side between squares (u, v) and (u + 1, v)
                            fs.append((_lower_first(tri_keys, side_tri(c, u, v, "right"),
                                                    side_tri(c, u + 1, v, "left")),
                                       ((X0 + 2, Y0, l), (X0 + 2, Y0 + 2, l))))
                        if v + 1 < s:  # side between squares (u, v) and (u, v + 1)
                            fs.append(((side_tri(c, u, v, "top"), side_tri(c, u, v + 1, "bottom")),
                                       ((X0, Y0 + 2, l), (X0 + 2, Y0 + 2, l))))
                # order inside the pixel: by the edge's midpoint, y first
                fs.sort(key=lambda f: (f[1][0][1] + f[1][1][1], f[1][0][0] + f[1][1][0]))
                for (tp, tm), e in fs:
                    inner.append(BasisFunction(KIND_INNER, (c,), e, tp, tm))
    for l in range(L):
        for y in range(ny):
            for x in range(nx - 1):
                a, b = cidx(l, x, y), cidx(l, x + 1, y)
                for v in range(s):
                    e = ((W * (x + 1), W * y + 2 * v, l), (W * (x + 1), W * y + 2 * v + 2, l))
                    inter_h.append(BasisFunction(KIND_INTER, (a, b), e, side_tri(a, s - 1, v, "right"),
                                                 side_tri(b, 0, v, "left")))
    for l in range(L):
        for y in range(ny - 1):
            for x in range(nx):
                a, b = cidx(l, x, y), cidx(l, x, y + 1)
                for u in range(s):
                    e = ((W * x + 2 * u, W * (y + 1), l), (W * x + 2 * u + 2, W * (y + 1), l))
                    inter_v.append(BasisFunction(KIND_INTER, (a, b), e, side_tri(a, u, s - 1, "top"),
                                                 side_tri(b, u, 0, "bottom")))

    # Feeds: a pad one square wide beyond square m = s // 2 of the middle
    # cell's grid side (the whole pixel side when s = 1), cut into an inner
    # and an outer half strip.  The delta-gap port sits on the line between
    # the two half strips; + side is the outer (source) side.
    m = s // 2
    pixport, feed_diag, port_edge = [], [], []
    for k, ps in enumerate(spec.ports):
        l = ps.layer
        if ps.side in ("right", "left"):
            j = ny // 2
            cx = nx - 1 if ps.side == "right" else 0
            cell = (cx, j)
            ya, yb = W * j + 2 * m, W * j + 2 * m + 2
            if ps.side == "right":
                inner_r = (W * nx, W * nx + 1, ya, yb)
                outer_r = (W * nx + 1, W * nx + 2, ya, yb)
            else:
                inner_r = (-1, 0, ya, yb)
                outer_r = (-2, -1, ya, yb)
        else:
            j = nx // 2
            cy = ny - 1 if ps.side == "top" else 0
            cell = (j, cy)
            xa, xb = W * j + 2 * m, W * j + 2 * m + 2
            if ps.side == "top":
                inner_r = (xa, xb, W * ny, W * ny + 1)
                outer_r = (xa, xb, W * ny + 1, W * ny + 2)
            else:
                inner_r = (xa, xb, -1, 0)
                outer_r = (xa, xb, -2, -1)
        ilo, iup, idiag = _rect_tris(*inner_r, l)
        olo, oup, odiag = _rect_tris(*outer_r, l)
        t0 = len(tri_keys)
        tri_keys += [ilo, iup, olo, oup]
        tri_owner += [("feed", k, "inner"), ("feed", k, "inner"), ("feed", k, "outer"), ("feed", k, "outer")]
        T_ilo, T_iup, T_olo, T_oup = t0, t0 + 1, t0 + 2, t0 + 3
        x0i, x1i, y0i, y1i = inner_r
        c = cidx(l, cell[0], cell[1])
        if ps.side == "right":
            pe = ((x1i, y0i, l), (x1i, y1i, l))
            port_pair = (T_oup, T_ilo)  # outer strip's left side / inner strip's right side
            ppe = ((x0i, y0i, l), (x0i, y1i, l))
            pp_pair = (T_iup, side_tri(c, s - 1, m, "right"))
        elif ps.side == "left":
            pe = ((x0i, y0i, l), (x0i, y1i, l))
            port_pair = (T_olo, T_iup)
            ppe = ((x1i, y0i, l), (x1i, y1i, l))
            pp_pair = (T_ilo, side_tri(c, 0, m, "left"))
        elif ps.side == "top":
            pe = ((x0i, y1i, l), (x1i, y1i, l))
            port_pair = (T_olo, T_iup)
            ppe = ((x0i, y0i, l), (x1i, y0i, l))
            pp_pair = (T_ilo, side_tri(c, m, s - 1, "top"))
        else:  # bottom
            pe = ((x0i, y0i, l), (x1i, y0i, l))
            port_pair = (T_oup, T_ilo)
            ppe = ((x0i, y1i, l), (x1i, y1i, l))
            pp_pair = (T_iup, side_tri(c, m, 0, "bottom"))
        pixport.append(BasisFunction(KIND_PIXPORT, (c,), ppe, pp_pair[0], pp_pair[1]))
        feed_diag.append(BasisFunction(KIND_ALWAYS, (), idiag, T_ilo, T_iup))
        feed_diag.append(BasisFunction(KIND_ALWAYS, (), odiag, T_olo, T_oup))
        port_edge.append(BasisFunction(KIND_ALWAYS, (), pe, port_pair[0], port_pair[1], port=k))

    # Vias: a vertical strip under the lower side line of cell (x, y), from
    # layer 0 down to layer 1, one sub-strip per square, each split by its
    # top-left/bottom-right diagonal.  Per via: the top junctions, then the
    # diagonals and the sides between sub-strips (by position), then the
    # bottom junctions.
    vias = []
    for s_i, (x, y) in enumerate(spec.via_sites()):
        c0, c1 = cidx(0, x, y), cidx(1, x, y)
        top, mid, bot = [], [], []
        prev_up = None
        for u in range(s):
            X0, Y = W * x + 2 * u, W * y
            TL, TR, BR, BL = (X0, Y, 0), (X0 + 2, Y, 0), (X0 + 2, Y, 1), (X0, Y, 1)
            t0 = len(tri_keys)
            tri_keys += [(TL, TR, BR), (TL, BR, BL)]
            tri_owner += [("via", s_i), ("via", s_i)]
            tU, tLo = t0, t0 + 1
            top.append(BasisFunction(KIND_VIA, (c0, c1), (TL, TR), side_tri(c0, u, 0, "bottom"), tU))
            if prev_up is not None:  # the side shared with the previous sub-strip
                mid.append(BasisFunction(KIND_VIA, (c0, c1), (TL, BL), prev_up, tLo))
            mid.append(BasisFunction(KIND_VIA, (c0, c1), (TL, BR), tU, tLo))
            bot.append(BasisFunction(KIND_VIA, (c0, c1), (BL, BR), tLo, side_tri(c1, u, 0, "bottom")))
            prev_up = tU
        vias += top + mid + bot

    bfs = inner + inter_h + inter_v + pixport + vias + feed_diag + port_edge
    port_bf = [i for i, b in enumerate(bfs) if b.port >= 0]
    return Structure(spec, tri_keys, tri_owner, bfs, port_bf)


def expected_count(spec) -> int:
    """Closed-form parent size with s squares per pixel side: per layer
    (3 s^2 - 2 s) inner functions per pixel (s^2 diagonals and 2 s (s - 1)
    sides between squares) and s per side between two pixels; four
    functions per port; 4 s - 1 per via (s top and s bottom junctions, s
    diagonals, s - 1 sides between sub-strips)."""
    s = _sub(spec)
    per_layer = spec.nx * spec.ny * (3 * s * s - 2 * s) + s * ((spec.nx - 1) * spec.ny + spec.nx * (spec.ny - 1))
    return spec.n_layers * per_layer + 4 * len(spec.ports) + (4 * s - 1) * spec.n_vias


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
