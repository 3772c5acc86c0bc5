// Host-side structure: mesh, RWG functions and their classification.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "pxd.h"

namespace pxd {

// Vertex in integer units of half a square side (a / (2 sub)): pixel corners
// at (2 sub x, 2 sub y, layer).
struct VKey {
  int x2, y2, l;
  bool operator<(const VKey& o) const {
    if (x2 != o.x2) return x2 < o.x2;
    if (y2 != o.y2) return y2 < o.y2;
    return l < o.l;
  }
  bool operator==(const VKey& o) const { return x2 == o.x2 && y2 == o.y2 && l == o.l; }
};

enum OwnerKind { OWN_CELL = 0, OWN_FEED_INNER = 1, OWN_FEED_OUTER = 2, OWN_VIA = 3 };

struct Tri {
  std::array<VKey, 3> v;
  int owner_kind;  // OwnerKind
  int owner;       // cell index, port index or via index
  int half;        // pixel/strip triangle: 0 = lower (holds the bottom side), 1 = upper
};

struct Rwg {
  int kind;           // PXD_KIND_*
  int cell_a, cell_b; // -1 if unused
  int tp, tm;         // + and - triangles
  VKey e0, e1;        // shared edge
  int port;           // port number for a delta-gap edge, else -1
  // canonical sort key
  int cls, k0, k1, k2, k3;
};

struct Problem {
  pxd_geometry g{};
  std::vector<int> port_side, port_layer, via_x, via_y;
  std::vector<Tri> tris;
  std::vector<Rwg> rwg;
  std::vector<int> port_bf;
  int n_cells = 0;
  int sub = 1;  // squares per pixel side

  std::array<double, 3> xyz(const VKey& k) const {
    const double u = g.a / (2.0 * sub);
    return {k.x2 * u, k.y2 * u, -k.l * g.h};
  }
};

int build_problem(const pxd_geometry* g, Problem* out, std::string* err);
int fill_problem(const Problem& p, int F, const double* freqs, double* Z, int n_threads, std::string* err);
// The same fill on the current device: Zdev is a device pointer (F x M x M
// complex128), work enqueued on `stream` (a hipStream_t) and finished on return.
int fill_problem_device(const Problem& p, int F, const double* freqs, double* Zdev, void* stream, std::string* err);

}  // namespace pxd

struct pxd_problem {
  pxd::Problem p;
};
