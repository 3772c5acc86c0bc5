// Parent impedance matrix fill (Phase 2 of the paper's flow, Section II-A):
// the EFIE (Eq. 1) in RWG functions (Eq. 2), mixed-potential Galerkin form,
// homogeneous-medium kernel G = exp(-jkR)/(4 pi R), time convention exp(jwt).
//
//   Z_mn = jw mu <f_m, G f_n> + 1/(jw eps) <div f_m, G div f_n>
//
// Both integrals use the 4-point degree-3 triangle rule.  For triangle pairs
// whose centroids are closer than twice the longer of their longest edges the
// inner integral splits G into 1/(4 pi R), integrated in closed form over the
// source triangle (Wilton et al. 1984; Graglia 1993), plus the smooth
// remainder (exp(-jkR) - 1)/(4 pi R) on the 4-point rule.  Z_mn is computed
// for m <= n and mirrored.
//
// Work is split in two phases per frequency: (1) for every test triangle, the
// source integrals over every source triangle at its four test points;
// (2) assembly of the rows of Z from those integrals.  Both phases are spread
// over host threads with an atomic work counter.
#include <atomic>
#include <cmath>
#include <complex>
#include <string>
#include <thread>
#include <vector>

#include "problem.hpp"

namespace pxd {
namespace {

using cd = std::complex<double>;
using V3 = std::array<double, 3>;

constexpr double kC0 = 299792458.0;
constexpr double kPi = 3.14159265358979323846;
constexpr double kMu0 = 4.0e-7 * kPi;

// 4-point rule: barycentric weights of each point and its weight
constexpr double kBary[4][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {0.6, 0.2, 0.2}, {0.2, 0.6, 0.2}, {0.2, 0.2, 0.6}};
constexpr double kW[4] = {-27.0 / 48, 25.0 / 48, 25.0 / 48, 25.0 / 48};

inline V3 sub(const V3& a, const V3& b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
inline double dot(const V3& a, const V3& b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline V3 cross(const V3& a, const V3& b) {
  return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
inline double norm(const V3& a) { return std::sqrt(dot(a, a)); }

struct TriGeo {
  V3 v[3];
  V3 c;       // centroid
  V3 q[4];    // quadrature points
  V3 n;       // unit normal
  double area, maxedge;
  // per edge: unit tangent t and in-plane outward normal u = t x n
  V3 t[3], u[3];
};

TriGeo make_tri(const Problem& P, const Tri& T) {
  TriGeo g{};
  for (int i = 0; i < 3; ++i) g.v[i] = P.xyz(T.v[i]);
  for (int d = 0; d < 3; ++d) g.c[d] = (g.v[0][d] + g.v[1][d] + g.v[2][d]) / 3.0;
  for (int p = 0; p < 4; ++p)
    for (int d = 0; d < 3; ++d)
      g.q[p][d] = kBary[p][0] * g.v[0][d] + kBary[p][1] * g.v[1][d] + kBary[p][2] * g.v[2][d];
  V3 nn = cross(sub(g.v[1], g.v[0]), sub(g.v[2], g.v[0]));
  double nl = norm(nn);
  g.area = 0.5 * nl;
  g.n = {nn[0] / nl, nn[1] / nl, nn[2] / nl};
  g.maxedge = 0;
  for (int i = 0; i < 3; ++i) {
    V3 e = sub(g.v[(i + 1) % 3], g.v[i]);
    double L = norm(e);
    g.maxedge = std::max(g.maxedge, L);
    g.t[i] = {e[0] / L, e[1] / L, e[2] / L};
    g.u[i] = cross(g.t[i], g.n);
  }
  return g;
}

// Closed-form integrals over triangle T of 1/R and of (rho' - rho)/R at r.
void static_integrals(const TriGeo& T, const V3& r, double* I1, V3* Irho) {
  double d = dot(T.n, sub(r, T.v[0]));
  V3 rho = {r[0] - d * T.n[0], r[1] - d * T.n[1], r[2] - d * T.n[2]};
  double ad = std::fabs(d);
  double s1 = 0;
  V3 sv = {0, 0, 0};
  for (int i = 0; i < 3; ++i) {
    const V3& a = T.v[i];
    const V3& b = T.v[(i + 1) % 3];
    V3 ar = sub(a, rho), br = sub(b, rho);
    double lp = dot(br, T.t[i]);
    double lm = dot(ar, T.t[i]);
    double P0 = dot(ar, T.u[i]);
    double R0sq = P0 * P0 + d * d;
    double Rp = std::sqrt(lp * lp + R0sq);
    double Rm = std::sqrt(lm * lm + R0sq);
    double elen = norm(sub(b, a));
    double f = 0, beta = 0;
    if (R0sq > (1e-14 * elen) * (1e-14 * elen)) {
      // ln[(R+ + l+)/(R- + l-)], written without cancellation when l < 0
      f = (lp + lm >= 0) ? std::log((Rp + lp) / (Rm + lm)) : std::log((Rm - lm) / (Rp - lp));
      beta = std::atan2(P0 * lp, R0sq + ad * Rp) - std::atan2(P0 * lm, R0sq + ad * Rm);
    }
    s1 += P0 * f - ad * beta;
    double w = 0.5 * (R0sq * f + lp * Rp - lm * Rm);
    for (int k = 0; k < 3; ++k) sv[k] += w * T.u[i][k];
  }
  *I1 = s1;
  *Irho = sv;
}

struct SrcInt {
  cd s[4];     // int G over the source triangle at each test point
  cd v[4][3];  // int (r' - c_src) G
};

}  // namespace

int fill_problem(const Problem& P, int F, const double* freqs, double* Zout, int n_threads, std::string* err) {
  const int M = (int)P.rwg.size();
  const int T = (int)P.tris.size();
  if (F < 1 || !freqs || !Zout) {
    *err = "invalid fill arguments";
    return PXD_EINVAL;
  }
  if (n_threads <= 0) n_threads = std::max(1u, std::thread::hardware_concurrency());
  std::vector<TriGeo> tg(T);
  for (int t = 0; t < T; ++t) tg[t] = make_tri(P, P.tris[t]);
  // per function: edge length, triangles, free vertices
  std::vector<double> len(M);
  std::vector<int> tri2(2 * M);
  std::vector<V3> freev(2 * M);
  for (int m = 0; m < M; ++m) {
    const Rwg& f = P.rwg[m];
    len[m] = norm(sub(P.xyz(f.e1), P.xyz(f.e0)));
    int ts[2] = {f.tp, f.tm};
    for (int s = 0; s < 2; ++s) {
      tri2[2 * m + s] = ts[s];
      const Tri& tr = P.tris[ts[s]];
      for (int i = 0; i < 3; ++i)
        if (!(tr.v[i] == f.e0) && !(tr.v[i] == f.e1)) freev[2 * m + s] = P.xyz(tr.v[i]);
    }
  }
  const double eps0 = 1.0 / (kMu0 * kC0 * kC0);
  std::vector<SrcInt> SI((size_t)T * T);

  auto run = [&](int n_items, auto&& body) {
    std::atomic<int> next{0};
    std::vector<std::thread> pool;
    for (int w = 0; w < n_threads; ++w)
      pool.emplace_back([&] {
        for (int it = next.fetch_add(1); it < n_items; it = next.fetch_add(1)) body(it);
      });
    for (auto& th : pool) th.join();
  };

  for (int fi = 0; fi < F; ++fi) {
    const double w = 2.0 * kPi * freqs[fi];
    const cd eps = eps0 * P.g.eps_r * cd(1.0, -P.g.tan_d);
    const cd k = w * std::sqrt(cd(kMu0, 0.0) * eps);  // principal root: Im k <= 0
    const cd jwmu4 = cd(0.0, w * kMu0 / 4.0);
    const cd inv_jweps = 1.0 / (cd(0.0, w) * eps);
    const cd mjk4pi = cd(0.0, -1.0) * k / (4.0 * kPi);

    // phase 1: source integrals for every (test p, source q)
    run(T, [&](int p) {
      const TriGeo& A = tg[p];
      for (int q = 0; q < T; ++q) {
        const TriGeo& B = tg[q];
        SrcInt& out = SI[(size_t)p * T + q];
        double dc = norm(sub(A.c, B.c));
        bool near = dc < 2.0 * std::max(A.maxedge, B.maxedge) * (1.0 + 1e-9);
        for (int i = 0; i < 4; ++i) {
          cd s = 0;
          cd sv[3] = {0, 0, 0};
          for (int j = 0; j < 4; ++j) {
            V3 dr = sub(A.q[i], B.q[j]);
            double R = norm(dr);
            cd g;
            if (!near) {
              g = std::exp(cd(0.0, -1.0) * k * R) / (4.0 * kPi * R);
            } else if (R == 0.0) {
              g = mjk4pi;  // limit of (exp(-jkR) - 1)/(4 pi R)
            } else {
              cd x = cd(0.0, -1.0) * k * R;
              cd em1 = (std::abs(k * R) < 1e-3) ? x * (1.0 + x / 2.0 * (1.0 + x / 3.0 * (1.0 + x / 4.0)))
                                                : std::exp(x) - 1.0;
              g = em1 / (4.0 * kPi * R);
            }
            cd wg = kW[j] * g;
            s += wg;
            for (int d = 0; d < 3; ++d) sv[d] += wg * (B.q[j][d] - B.c[d]);
          }
          s *= B.area;
          for (int d = 0; d < 3; ++d) sv[d] *= B.area;
          if (near) {
            double I1;
            V3 Ir;
            static_integrals(B, A.q[i], &I1, &Ir);
            double dd = dot(B.n, sub(A.q[i], B.v[0]));
            V3 rho = {A.q[i][0] - dd * B.n[0], A.q[i][1] - dd * B.n[1], A.q[i][2] - dd * B.n[2]};
            s += I1 / (4.0 * kPi);
            for (int d = 0; d < 3; ++d) sv[d] += (Ir[d] + (rho[d] - B.c[d]) * I1) / (4.0 * kPi);
          }
          out.s[i] = s;
          for (int d = 0; d < 3; ++d) out.v[i][d] = sv[d];
        }
      }
    });

    // phase 2: Z_mn for n >= m, mirrored
    cd* Z = reinterpret_cast<cd*>(Zout) + (size_t)fi * M * M;
    run(M, [&](int m) {
      for (int n = m; n < M; ++n) {
        cd acc = 0;
        for (int a = 0; a < 2; ++a) {
          int tp = tri2[2 * m + a];
          const TriGeo& A = tg[tp];
          const V3& pm = freev[2 * m + a];
          for (int b = 0; b < 2; ++b) {
            int tq = tri2[2 * n + b];
            const TriGeo& B = tg[tq];
            const SrcInt& si = SI[(size_t)tp * T + tq];
            V3 off = sub(freev[2 * n + b], B.c);  // p_n - c_n
            cd term = 0;
            for (int i = 0; i < 4; ++i) {
              V3 rt = sub(A.q[i], pm);
              cd vec = 0;
              for (int d = 0; d < 3; ++d) vec += rt[d] * (si.v[i][d] - off[d] * si.s[i]);
              term += kW[i] * (jwmu4 * vec + inv_jweps * si.s[i]);
            }
            double sign = (a == b) ? 1.0 : -1.0;
            acc += sign * len[m] * len[n] / B.area * term;
          }
        }
        Z[(size_t)m * M + n] = acc;
        Z[(size_t)n * M + m] = acc;
      }
    });
  }
  return PXD_OK;
}

}  // namespace pxd
