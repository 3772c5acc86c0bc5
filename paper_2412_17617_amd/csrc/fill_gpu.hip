// Parent impedance matrix fill on the GPU: the discretisation of fill.cpp
// (mixed-potential EFIE of Eq. 1 in the RWG functions of Eq. 2, kernel
// exp(-jkR)/(4 pi R), 4-point degree-3 triangle rule, closed-form 1/R
// extraction on near triangle pairs, upper triangle computed and mirrored),
// in FP64 with one thread per item:
//   k_fill_source:   per (test triangle p, source triangle q, test point i)
//                    the source integrals of G and (r' - c_q) G;
//   k_fill_assemble: per (m, n >= m) the four triangle-pair terms of Z_mn,
//                    written to Z[m][n] and Z[n][m].
// The source table (T x T x 4 entries of 64 bytes, T triangles) is built
// once per frequency and read by the assembly from L2 / HBM.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "problem.hpp"
#include "pxd.h"

namespace pxd {
namespace {

constexpr double kC0g = 299792458.0;
constexpr double kPig = 3.14159265358979323846;
constexpr double kMu0g = 4.0e-7 * kPig;

// Triangle data for the kernels (FP64).
struct TriDev {
  double v[3][3];
  double c[3];
  double q[4][3];  // quadrature points
  double n[3];     // unit normal
  double t[3][3];  // unit edge tangents
  double u[3][3];  // in-plane outward edge normals t x n
  double area, maxedge;
};

// Quadrature weights of the 4-point rule (points at barycentric (1/3,1/3,1/3),
// (3/5,1/5,1/5) and its permutations).
__constant__ double cW[4] = {-27.0 / 48, 25.0 / 48, 25.0 / 48, 25.0 / 48};

struct FillConst {
  double kr, ki;             // wavenumber k = kr + j ki (ki <= 0)
  double2 jwmu4, inv_jweps;  // j w mu / 4 and 1 / (j w eps)
};

__device__ __forceinline__ double2 cm(double2 a, double2 b) { return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

// Closed-form integrals over triangle T of 1/R and of (rho' - rho)/R at r
// (Wilton et al. 1984; Graglia 1993).
__device__ void static_integrals_dev(const TriDev& T, const double* r, double* I1, double* Irho) {
  const double d = T.n[0] * (r[0] - T.v[0][0]) + T.n[1] * (r[1] - T.v[0][1]) + T.n[2] * (r[2] - T.v[0][2]);
  const double rho[3] = {r[0] - d * T.n[0], r[1] - d * T.n[1], r[2] - d * T.n[2]};
  const double ad = fabs(d);
  double s1 = 0, sv[3] = {0, 0, 0};
  for (int i = 0; i < 3; ++i) {
    const double* a = T.v[i];
    const double* b = T.v[(i + 1) % 3];
    const double ar[3] = {a[0] - rho[0], a[1] - rho[1], a[2] - rho[2]};
    const double br[3] = {b[0] - rho[0], b[1] - rho[1], b[2] - rho[2]};
    const double lp = br[0] * T.t[i][0] + br[1] * T.t[i][1] + br[2] * T.t[i][2];
    const double lm = ar[0] * T.t[i][0] + ar[1] * T.t[i][1] + ar[2] * T.t[i][2];
    const double P0 = ar[0] * T.u[i][0] + ar[1] * T.u[i][1] + ar[2] * T.u[i][2];
    const double R0sq = P0 * P0 + d * d;
    const double Rp = sqrt(lp * lp + R0sq), Rm = sqrt(lm * lm + R0sq);
    const double ex = b[0] - a[0], ey = b[1] - a[1], ez = b[2] - a[2];
    const double elen = sqrt(ex * ex + ey * ey + ez * ez);
    double f = 0, beta = 0;
    if (R0sq > (1e-14 * elen) * (1e-14 * elen)) {
      f = (lp + lm >= 0) ? log((Rp + lp) / (Rm + lm)) : log((Rm - lm) / (Rp - lp));
      beta = atan2(P0 * lp, R0sq + ad * Rp) - atan2(P0 * lm, R0sq + ad * Rm);
    }
    s1 += P0 * f - ad * beta;
    const double w = 0.5 * (R0sq * f + lp * Rp - lm * Rm);
    for (int k = 0; k < 3; ++k) sv[k] += w * T.u[i][k];
  }
  *I1 = s1;
  for (int k = 0; k < 3; ++k) Irho[k] = sv[k];
}

// SI[(p T + q) 4 + i] = {int_q G, int_q (r' - c_q) G} at test point i of p.
__global__ __launch_bounds__(256) void k_fill_source(const TriDev* __restrict__ tg, int T, FillConst fc,
                                                     double2* __restrict__ SI) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long long)T * T * 4) return;
  const int i = (int)(gid & 3);
  const long long pq = gid >> 2;
  const int p = (int)(pq / T), q = (int)(pq - (long long)p * T);
  const TriDev& A = tg[p];
  const TriDev& B = tg[q];
  const double r[3] = {A.q[i][0], A.q[i][1], A.q[i][2]};
  const double dcx = A.c[0] - B.c[0], dcy = A.c[1] - B.c[1], dcz = A.c[2] - B.c[2];
  const double dc = sqrt(dcx * dcx + dcy * dcy + dcz * dcz);
  const bool near = dc < 2.0 * fmax(A.maxedge, B.maxedge) * (1.0 + 1e-9);
  double2 s{0, 0}, sv[3] = {{0, 0}, {0, 0}, {0, 0}};
  for (int j = 0; j < 4; ++j) {
    const double dx = r[0] - B.q[j][0], dy = r[1] - B.q[j][1], dz = r[2] - B.q[j][2];
    const double R = sqrt(dx * dx + dy * dy + dz * dz);
    double2 g;
    if (!near) {
      // exp(-j k R) = exp(ki R) (cos(kr R) - j sin(kr R))
      double sn, cs;
      sincos(fc.kr * R, &sn, &cs);
      const double mag = exp(fc.ki * R) / (4.0 * kPig * R);
      g = double2{mag * cs, -mag * sn};
    } else if (R == 0.0) {
      g = double2{fc.ki / (4.0 * kPig), -fc.kr / (4.0 * kPig)};  // limit of (exp(-jkR) - 1)/(4 pi R)
    } else {
      const double2 x{fc.ki * R, -fc.kr * R};  // -j k R
      double2 em1;
      if (sqrt(fc.kr * fc.kr + fc.ki * fc.ki) * R < 1e-3) {  // exp(x) - 1 by its series
        double2 t = cm(x, double2{0.25, 0.0});
        t = cm(x, double2{(1.0 + t.x) / 3.0, t.y / 3.0});
        t = cm(x, double2{(1.0 + t.x) / 2.0, t.y / 2.0});
        em1 = cm(x, double2{1.0 + t.x, t.y});
      } else {
        double sn, cs;
        sincos(-x.y, &sn, &cs);
        const double e = exp(x.x);
        em1 = double2{e * cs - 1.0, -e * sn};
      }
      g = double2{em1.x / (4.0 * kPig * R), em1.y / (4.0 * kPig * R)};
    }
    const double2 wg{cW[j] * g.x, cW[j] * g.y};
    s.x += wg.x, s.y += wg.y;
    for (int d = 0; d < 3; ++d) {
      const double o = B.q[j][d] - B.c[d];
      sv[d].x += wg.x * o, sv[d].y += wg.y * o;
    }
  }
  s.x *= B.area, s.y *= B.area;
  for (int d = 0; d < 3; ++d) sv[d].x *= B.area, sv[d].y *= B.area;
  if (near) {
    double I1, Ir[3];
    static_integrals_dev(B, r, &I1, Ir);
    const double dd = B.n[0] * (r[0] - B.v[0][0]) + B.n[1] * (r[1] - B.v[0][1]) + B.n[2] * (r[2] - B.v[0][2]);
    s.x += I1 / (4.0 * kPig);
    for (int d = 0; d < 3; ++d) {
      const double rho = r[d] - dd * B.n[d];
      sv[d].x += (Ir[d] + (rho - B.c[d]) * I1) / (4.0 * kPig);
    }
  }
  double2* o = SI + gid * 4;
  o[0] = s;
  o[1] = sv[0];
  o[2] = sv[1];
  o[3] = sv[2];
}

// Z_mn for n >= m over 16 x 16 tiles of the upper triangle, mirrored.
__global__ __launch_bounds__(256) void k_fill_assemble(const TriDev* __restrict__ tg, int T, int M,
                                                       const double* __restrict__ len, const int* __restrict__ tri2,
                                                       const double* __restrict__ freev, FillConst fc,
                                                       const double2* __restrict__ SI, double2* __restrict__ Z) {
  const int bm = blockIdx.y, bn = blockIdx.x;
  if (bn < bm) return;
  const int m = bm * 16 + (threadIdx.x >> 4), n = bn * 16 + (threadIdx.x & 15);
  if (m >= M || n >= M || n < m) return;
  double2 acc{0, 0};
  for (int a = 0; a < 2; ++a) {
    const int tp = tri2[2 * m + a];
    const TriDev& A = tg[tp];
    const double* pm = freev + (size_t)(2 * m + a) * 3;
    for (int b = 0; b < 2; ++b) {
      const int tq = tri2[2 * n + b];
      const TriDev& B = tg[tq];
      const double* pn = freev + (size_t)(2 * n + b) * 3;
      const double off[3] = {pn[0] - B.c[0], pn[1] - B.c[1], pn[2] - B.c[2]};
      const double2* si = SI + ((size_t)tp * T + tq) * 16;
      double2 term{0, 0};
      for (int i = 0; i < 4; ++i) {
        const double2 s = si[4 * i];
        double2 vec{0, 0};
        for (int d = 0; d < 3; ++d) {
          const double rt = A.q[i][d] - pm[d];
          const double2 v = si[4 * i + 1 + d];
          vec.x += rt * (v.x - off[d] * s.x);
          vec.y += rt * (v.y - off[d] * s.y);
        }
        const double2 t1 = cm(fc.jwmu4, vec), t2 = cm(fc.inv_jweps, s);
        term.x += cW[i] * (t1.x + t2.x);
        term.y += cW[i] * (t1.y + t2.y);
      }
      const double sc = ((a == b) ? 1.0 : -1.0) * len[m] * len[n] / B.area;
      acc.x += sc * term.x;
      acc.y += sc * term.y;
    }
  }
  Z[(size_t)m * M + n] = acc;
  Z[(size_t)n * M + m] = acc;
}

struct DevMem {
  void* p = nullptr;
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

int fill_problem_device(const Problem& P, int F, const double* freqs, double* Zdev, void* stream, std::string* err) {
  const int M = (int)P.rwg.size();
  const int T = (int)P.tris.size();
  if (F < 1 || !freqs || !Zdev || M < 1) {
    *err = "invalid fill arguments";
    return PXD_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto hip_err = [&](hipError_t e, const char* where) {
    *err = std::string(where) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? PXD_ENOMEM : PXD_EDEVICE;
  };
  using V3 = std::array<double, 3>;
  std::vector<TriDev> tg(T);
  static const double bary[4][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {0.6, 0.2, 0.2}, {0.2, 0.6, 0.2}, {0.2, 0.2, 0.6}};
  for (int t = 0; t < T; ++t) {
    TriDev& g = tg[t];
    V3 v[3];
    for (int i = 0; i < 3; ++i) v[i] = P.xyz(P.tris[t].v[i]);
    for (int i = 0; i < 3; ++i)
      for (int d = 0; d < 3; ++d) g.v[i][d] = v[i][d];
    for (int d = 0; d < 3; ++d) g.c[d] = (v[0][d] + v[1][d] + v[2][d]) / 3.0;
    for (int p = 0; p < 4; ++p)
      for (int d = 0; d < 3; ++d) g.q[p][d] = bary[p][0] * v[0][d] + bary[p][1] * v[1][d] + bary[p][2] * v[2][d];
    const V3 e1{v[1][0] - v[0][0], v[1][1] - v[0][1], v[1][2] - v[0][2]};
    const V3 e2{v[2][0] - v[0][0], v[2][1] - v[0][1], v[2][2] - v[0][2]};
    const V3 nn{e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double nl = std::sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
    g.area = 0.5 * nl;
    for (int d = 0; d < 3; ++d) g.n[d] = nn[d] / nl;
    g.maxedge = 0;
    for (int i = 0; i < 3; ++i) {
      const V3& a = v[i];
      const V3& b = v[(i + 1) % 3];
      const V3 e{b[0] - a[0], b[1] - a[1], b[2] - a[2]};
      const double L = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
      g.maxedge = std::max(g.maxedge, L);
      for (int d = 0; d < 3; ++d) g.t[i][d] = e[d] / L;
      g.u[i][0] = g.t[i][1] * g.n[2] - g.t[i][2] * g.n[1];
      g.u[i][1] = g.t[i][2] * g.n[0] - g.t[i][0] * g.n[2];
      g.u[i][2] = g.t[i][0] * g.n[1] - g.t[i][1] * g.n[0];
    }
  }
  std::vector<double> len(M), freev((size_t)6 * M);
  std::vector<int> tri2(2 * M);
  for (int m = 0; m < M; ++m) {
    const Rwg& f = P.rwg[m];
    const V3 a = P.xyz(f.e0), b = P.xyz(f.e1);
    len[m] = std::sqrt((a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1]) + (a[2] - b[2]) * (a[2] - b[2]));
    const int ts[2] = {f.tp, f.tm};
    for (int sd = 0; sd < 2; ++sd) {
      tri2[2 * m + sd] = ts[sd];
      const Tri& tr = P.tris[ts[sd]];
      for (int i = 0; i < 3; ++i)
        if (!(tr.v[i] == f.e0) && !(tr.v[i] == f.e1)) {
          const V3 x = P.xyz(tr.v[i]);
          for (int d = 0; d < 3; ++d) freev[(size_t)(2 * m + sd) * 3 + d] = x[d];
        }
    }
  }
  DevMem d_tg, d_len, d_tri2, d_freev, d_SI;
  hipError_t e;
  const size_t si_bytes = (size_t)T * T * 4 * 4 * sizeof(double2);
  if ((e = hipMalloc(&d_tg.p, sizeof(TriDev) * T)) != hipSuccess) return hip_err(e, "hipMalloc");
  if ((e = hipMalloc(&d_len.p, sizeof(double) * M)) != hipSuccess) return hip_err(e, "hipMalloc");
  if ((e = hipMalloc(&d_tri2.p, sizeof(int) * 2 * M)) != hipSuccess) return hip_err(e, "hipMalloc");
  if ((e = hipMalloc(&d_freev.p, sizeof(double) * 6 * M)) != hipSuccess) return hip_err(e, "hipMalloc");
  if ((e = hipMalloc(&d_SI.p, si_bytes)) != hipSuccess) return hip_err(e, "hipMalloc (source table)");
  if ((e = hipMemcpyAsync(d_tg.p, tg.data(), sizeof(TriDev) * T, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(d_len.p, len.data(), sizeof(double) * M, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(d_tri2.p, tri2.data(), sizeof(int) * 2 * M, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(d_freev.p, freev.data(), sizeof(double) * 6 * M, hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_err(e, "hipMemcpyAsync");
  const double eps0 = 1.0 / (kMu0g * kC0g * kC0g);
  const long long n1 = (long long)T * T * 4;
  const int nt = (M + 15) / 16;
  for (int fi = 0; fi < F; ++fi) {
    using cd = std::complex<double>;
    const double w = 2.0 * kPig * freqs[fi];
    const cd eps = eps0 * P.g.eps_r * cd(1.0, -P.g.tan_d);
    const cd k = w * std::sqrt(cd(kMu0g, 0.0) * eps);  // principal root: Im k <= 0
    const cd jwmu4 = cd(0.0, w * kMu0g / 4.0);
    const cd inv_jweps = 1.0 / (cd(0.0, w) * eps);
    FillConst fc{k.real(), k.imag(), double2{jwmu4.real(), jwmu4.imag()},
                 double2{inv_jweps.real(), inv_jweps.imag()}};
    hipLaunchKernelGGL(k_fill_source, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s,
                       static_cast<const TriDev*>(d_tg.p), T, fc, static_cast<double2*>(d_SI.p));
    if ((e = hipGetLastError()) != hipSuccess) return hip_err(e, "k_fill_source");
    hipLaunchKernelGGL(k_fill_assemble, dim3(nt, nt), dim3(256), 0, s, static_cast<const TriDev*>(d_tg.p), T, M,
                       static_cast<const double*>(d_len.p), static_cast<const int*>(d_tri2.p),
                       static_cast<const double*>(d_freev.p), fc, static_cast<const double2*>(d_SI.p),
                       reinterpret_cast<double2*>(Zdev) + (size_t)fi * M * M);
    if ((e = hipGetLastError()) != hipSuccess) return hip_err(e, "k_fill_assemble");
  }
  // the temporaries are freed on return: wait for the kernels that read them
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_err(e, "hipStreamSynchronize");
  return PXD_OK;
}

}  // namespace pxd
