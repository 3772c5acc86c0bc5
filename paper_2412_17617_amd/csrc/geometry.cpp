// Structure builder: pixel mesh, feeds, vias, RWG functions (Section II-B)
// and their classification into always-present, inner-pixel, inter-pixel,
// pixel-port and via functions (Section II-C, Fig. 2(a)).
//
// The mesh is generated triangle by triangle; RWG functions are then found as
// the interior edges of the whole (all-metal) parent mesh and classified from
// the owners of the triangles that share each edge.  Two pixels touching only
// at a corner share no edge, hence no function (Section VI-A).
#include <algorithm>
#include <cmath>
#include <map>
#include <string>
#include <vector>

#include "problem.hpp"

namespace pxd {
namespace {

struct EdgeKey {
  VKey a, b;
  bool operator<(const EdgeKey& o) const {
    if (!(a == o.a)) return a < o.a;
    return b < o.b;
  }
};

EdgeKey make_edge(const VKey& p, const VKey& q) { return (p < q) ? EdgeKey{p, q} : EdgeKey{q, p}; }

void add_rect(std::vector<Tri>& tris, int x0, int x1, int y0, int y1, int l, int okind, int owner) {
  // lower triangle holds the bottom and right sides, upper the top and left
  VKey LL{x0, y0, l}, LR{x1, y0, l}, UR{x1, y1, l}, UL{x0, y1, l};
  tris.push_back(Tri{{LL, LR, UR}, okind, owner, 0});
  tris.push_back(Tri{{LL, UR, UL}, okind, owner, 1});
}

double centroid_coord(const Tri& t, int axis) {
  double s = 0;
  for (auto& v : t.v) s += (axis == 0 ? v.x2 : axis == 1 ? v.y2 : -v.l);
  return s;  // only compared, scale irrelevant
}

}  // namespace

int build_problem(const pxd_geometry* g, Problem* P, std::string* err) {
  if (!g || g->n_layers < 1 || g->nx < 1 || g->ny < 1 || !(g->a > 0) || g->n_ports < 0 || g->n_vias < 0 ||
      (g->n_ports > 0 && (!g->port_side || !g->port_layer)) || (g->n_vias > 0 && (!g->via_x || !g->via_y)) ||
      (g->n_layers > 1 && !(g->h > 0))) {
    *err = "invalid geometry";
    return PXD_EINVAL;
  }
  if (g->sub < 0 || g->sub > 8) {
    *err = "invalid geometry: sub must be 0..8";
    return PXD_EINVAL;
  }
  const int nx = g->nx, ny = g->ny, L = g->n_layers;
  const int S = g->sub > 1 ? g->sub : 1;  // squares per pixel side
  const int W = 2 * S;                      // pixel side in key units (half a square side)
  P->g = *g;
  P->sub = S;
  P->port_side.assign(g->port_side, g->port_side + g->n_ports);
  P->port_layer.assign(g->port_layer, g->port_layer + g->n_ports);
  P->via_x.assign(g->via_x, g->via_x + g->n_vias);
  P->via_y.assign(g->via_y, g->via_y + g->n_vias);
  P->g.port_side = P->port_side.data();
  P->g.port_layer = P->port_layer.data();
  P->g.via_x = P->via_x.data();
  P->g.via_y = P->via_y.data();
  P->n_cells = L * nx * ny;
  for (int k = 0; k < g->n_ports; ++k)
    if (P->port_side[k] < 0 || P->port_side[k] > 3 || P->port_layer[k] < 0 || P->port_layer[k] >= L) {
      *err = "invalid port";
      return PXD_EINVAL;
    }
  for (int v = 0; v < g->n_vias; ++v)
    if (L < 2 || P->via_x[v] < 0 || P->via_x[v] >= nx || P->via_y[v] < 0 || P->via_y[v] >= ny) {
      *err = "invalid via";
      return PXD_EINVAL;
    }

  auto& tris = P->tris;
  tris.clear();
  // every pixel an S x S grid of squares, each cut into two right triangles
  // along the diagonal that alternates in a checkerboard over the squares
  for (int l = 0; l < L; ++l)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int c = (l * ny + y) * nx + x;
        for (int v = 0; v < S; ++v)
          for (int u = 0; u < S; ++u) {
            const int X0 = W * x + 2 * u, Y0 = W * y + 2 * v;
            VKey LL{X0, Y0, l}, LR{X0 + 2, Y0, l}, UR{X0 + 2, Y0 + 2, l}, UL{X0, Y0 + 2, l};
            if (((S * x + u + S * y + v) & 1) == 0) {
              tris.push_back(Tri{{LL, LR, UR}, OWN_CELL, c, 0});
              tris.push_back(Tri{{LL, UR, UL}, OWN_CELL, c, 1});
            } else {
              tris.push_back(Tri{{LL, LR, UL}, OWN_CELL, c, 0});
              tris.push_back(Tri{{LR, UR, UL}, OWN_CELL, c, 1});
            }
          }
      }
  // feeds: a pad one square wide beyond square S / 2 of the middle cell's
  // side, cut in an inner and an outer half strip
  std::vector<int> port_cell(g->n_ports);
  const int m = S / 2;
  for (int k = 0; k < g->n_ports; ++k) {
    int side = P->port_side[k], l = P->port_layer[k];
    int jy = ny / 2, jx = nx / 2;
    int ix[2][2], iy[2][2];  // [inner/outer][lo/hi]
    int cx, cy;
    switch (side) {
      case 0:  // right
        cx = nx - 1, cy = jy;
        ix[0][0] = W * nx, ix[0][1] = W * nx + 1, ix[1][0] = W * nx + 1, ix[1][1] = W * nx + 2;
        iy[0][0] = iy[1][0] = W * jy + 2 * m, iy[0][1] = iy[1][1] = W * jy + 2 * m + 2;
        break;
      case 2:  // left
        cx = 0, cy = jy;
        ix[0][0] = -1, ix[0][1] = 0, ix[1][0] = -2, ix[1][1] = -1;
        iy[0][0] = iy[1][0] = W * jy + 2 * m, iy[0][1] = iy[1][1] = W * jy + 2 * m + 2;
        break;
      case 1:  // top
        cx = jx, cy = ny - 1;
        ix[0][0] = ix[1][0] = W * jx + 2 * m, ix[0][1] = ix[1][1] = W * jx + 2 * m + 2;
        iy[0][0] = W * ny, iy[0][1] = W * ny + 1, iy[1][0] = W * ny + 1, iy[1][1] = W * ny + 2;
        break;
      default:  // bottom
        cx = jx, cy = 0;
        ix[0][0] = ix[1][0] = W * jx + 2 * m, ix[0][1] = ix[1][1] = W * jx + 2 * m + 2;
        iy[0][0] = -1, iy[0][1] = 0, iy[1][0] = -2, iy[1][1] = -1;
        break;
    }
    port_cell[k] = (l * ny + cy) * nx + cx;
    add_rect(tris, ix[0][0], ix[0][1], iy[0][0], iy[0][1], l, OWN_FEED_INNER, k);
    add_rect(tris, ix[1][0], ix[1][1], iy[1][0], iy[1][1], l, OWN_FEED_OUTER, k);
  }
  // vias: vertical strip under the lower side of cell (x, y), layers 0 -> 1,
  // one sub-strip per square of that side
  for (int v = 0; v < g->n_vias; ++v) {
    int x = P->via_x[v], y = P->via_y[v];
    for (int u = 0; u < S; ++u) {
      const int X0 = W * x + 2 * u, Y = W * y;
      VKey TL{X0, Y, 0}, TR{X0 + 2, Y, 0}, BR{X0 + 2, Y, 1}, BL{X0, Y, 1};
      tris.push_back(Tri{{TL, TR, BR}, OWN_VIA, v, 1});
      tris.push_back(Tri{{TL, BR, BL}, OWN_VIA, v, 0});
    }
  }

  // interior edges of the parent mesh
  std::map<EdgeKey, std::vector<int>> edges;
  for (int t = 0; t < (int)tris.size(); ++t)
    for (int e = 0; e < 3; ++e) edges[make_edge(tris[t].v[e], tris[t].v[(e + 1) % 3])].push_back(t);

  auto cell_xyz = [&](int c, int& l, int& x, int& y) {
    x = c % nx;
    y = (c / nx) % ny;
    l = c / (nx * ny);
  };
  auto via_cell = [&](int v, int layer) { return (layer * ny + P->via_y[v]) * nx + P->via_x[v]; };

  auto& R = P->rwg;
  R.clear();
  auto emit_pair = [&](const EdgeKey& ek, int t1, int t2) -> bool {
    const Tri& A = tris[t1];
    const Tri& B = tris[t2];
    Rwg f{};
    f.e0 = ek.a;
    f.e1 = ek.b;
    f.cell_a = f.cell_b = -1;
    f.port = -1;
    auto lower_y_first = [&](int p, int q) {  // lower centroid y, then smaller x
      const double yp = centroid_coord(tris[p], 1), yq = centroid_coord(tris[q], 1);
      const bool p_first = yp < yq || (yp == yq && centroid_coord(tris[p], 0) < centroid_coord(tris[q], 0));
      if (p_first) f.tp = p, f.tm = q;
      else f.tp = q, f.tm = p;
    };
    auto higher_z_first = [&](int p, int q) {
      if (centroid_coord(tris[p], 2) > centroid_coord(tris[q], 2)) f.tp = p, f.tm = q;
      else f.tp = q, f.tm = p;
    };
    int ka = A.owner_kind, kb = B.owner_kind;
    if (ka == OWN_CELL && kb == OWN_CELL) {
      if (A.owner == B.owner) {
        int l, x, y;
        cell_xyz(A.owner, l, x, y);
        f.kind = PXD_KIND_INNER;
        f.cell_a = A.owner;
        lower_y_first(t1, t2);
        // inside the pixel: by the edge's midpoint, y first
        const int my = ek.a.y2 + ek.b.y2 - 2 * W * y, mx = ek.a.x2 + ek.b.x2 - 2 * W * x;
        f.cls = 0, f.k0 = l, f.k1 = y, f.k2 = x, f.k3 = my * (2 * W + 1) + mx;
      } else {
        int la, xa, ya, lb, xb, yb;
        cell_xyz(A.owner, la, xa, ya);
        cell_xyz(B.owner, lb, xb, yb);
        if (la != lb || std::abs(xa - xb) + std::abs(ya - yb) != 1) return false;
        bool first_a = (xa < xb) || (ya < yb);  // + side: smaller x (horizontal pair) or smaller y
        int c0 = first_a ? A.owner : B.owner, c1 = first_a ? B.owner : A.owner;
        f.kind = PXD_KIND_INTER;
        f.cell_a = c0;
        f.cell_b = c1;
        f.tp = first_a ? t1 : t2;
        f.tm = first_a ? t2 : t1;
        int l, x, y;
        cell_xyz(c0, l, x, y);
        if (ya == yb) f.cls = 1; else f.cls = 2;
        // the side's squares in order along it
        f.k0 = l, f.k1 = y, f.k2 = x, f.k3 = (ya == yb) ? ek.a.y2 + ek.b.y2 : ek.a.x2 + ek.b.x2;
      }
    } else if ((ka == OWN_FEED_INNER || ka == OWN_FEED_OUTER) && (kb == OWN_FEED_INNER || kb == OWN_FEED_OUTER)) {
      if (A.owner != B.owner) return false;
      f.kind = PXD_KIND_ALWAYS;
      if (ka == kb) {  // diagonal of one half strip
        lower_y_first(t1, t2);
        f.cls = 5, f.k0 = A.owner, f.k1 = (ka == OWN_FEED_INNER ? 0 : 1), f.k2 = f.k3 = 0;
      } else {  // the delta-gap port edge; + side is the outer strip
        f.tp = (ka == OWN_FEED_OUTER) ? t1 : t2;
        f.tm = (ka == OWN_FEED_OUTER) ? t2 : t1;
        f.port = A.owner;
        f.cls = 6, f.k0 = A.owner, f.k1 = f.k2 = f.k3 = 0;
      }
    } else if ((ka == OWN_FEED_INNER && kb == OWN_CELL) || (kb == OWN_FEED_INNER && ka == OWN_CELL)) {
      const Tri& F = (ka == OWN_FEED_INNER) ? A : B;
      const Tri& C = (ka == OWN_FEED_INNER) ? B : A;
      if (port_cell[F.owner] != C.owner) return false;
      f.kind = PXD_KIND_PIXPORT;
      f.cell_a = C.owner;
      f.tp = (ka == OWN_FEED_INNER) ? t1 : t2;  // + side on the feed
      f.tm = (ka == OWN_FEED_INNER) ? t2 : t1;
      f.cls = 3, f.k0 = F.owner, f.k1 = f.k2 = f.k3 = 0;
    } else if (ka == OWN_VIA || kb == OWN_VIA) {
      int v = (ka == OWN_VIA) ? A.owner : B.owner;
      if (ka == OWN_VIA && kb == OWN_VIA && A.owner != B.owner) return false;
      if (ka != kb) {
        const Tri& C = (ka == OWN_VIA) ? B : A;
        if (C.owner_kind != OWN_CELL || C.owner != via_cell(v, ek.a.l)) return false;
      }
      f.kind = PXD_KIND_VIA;
      f.cell_a = via_cell(v, 0);
      f.cell_b = via_cell(v, 1);
      higher_z_first(t1, t2);
      int sub;
      if (ka == OWN_VIA && kb == OWN_VIA) sub = 1;
      else sub = (ek.a.l == 0) ? 0 : 2;  // junction on layer 0 (top) or layer 1 (bottom)
      f.cls = 4, f.k0 = v, f.k1 = sub, f.k2 = ek.a.x2 + ek.b.x2, f.k3 = 0;  // by position along the strip
    } else {
      return false;
    }
    R.push_back(f);
    return true;
  };

  for (auto& kv : edges) {
    const auto& ts = kv.second;
    if (ts.size() < 2) continue;
    bool ok = true;
    if (ts.size() == 2) {
      ok = emit_pair(kv.first, ts[0], ts[1]);
    } else if (ts.size() == 3) {
      // a via junction edge that is also the side between two pixels: the via
      // triangle pairs with the triangle of its own cell, the two pixel
      // triangles form the ordinary inter-pixel function
      int tv = -1;
      std::vector<int> cells;
      for (int t : ts) {
        if (tris[t].owner_kind == OWN_VIA) tv = t;
        else cells.push_back(t);
      }
      if (tv < 0 || cells.size() != 2) ok = false;
      else {
        int v = tris[tv].owner, layer = kv.first.a.l;
        int own = via_cell(v, layer);
        int tc = (tris[cells[0]].owner == own) ? cells[0] : (tris[cells[1]].owner == own ? cells[1] : -1);
        if (tc < 0) ok = false;
        else ok = emit_pair(kv.first, cells[0], cells[1]) && emit_pair(kv.first, tv, tc);
      }
    } else {
      ok = false;
    }
    if (!ok) {
      *err = "unexpected edge topology while classifying basis functions";
      return PXD_EINVAL;
    }
  }
  std::sort(R.begin(), R.end(), [](const Rwg& p, const Rwg& q) {
    if (p.cls != q.cls) return p.cls < q.cls;
    if (p.k0 != q.k0) return p.k0 < q.k0;
    if (p.k1 != q.k1) return p.k1 < q.k1;
    if (p.k2 != q.k2) return p.k2 < q.k2;
    return p.k3 < q.k3;
  });
  P->port_bf.assign(g->n_ports, -1);
  for (int i = 0; i < (int)R.size(); ++i)
    if (R[i].port >= 0) P->port_bf[R[i].port] = i;
  for (int k = 0; k < g->n_ports; ++k)
    if (P->port_bf[k] != (int)R.size() - g->n_ports + k) {
      *err = "port functions are not last in port order";
      return PXD_EINVAL;
    }
  return PXD_OK;
}

}  // namespace pxd
