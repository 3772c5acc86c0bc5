// Exact evaluation of flip candidates from the base map's inverse (a variant
// the paper does not use): the same S as a dense solve of each candidate's
// Z_A, up to rounding.
//
// With G = Z_B^-1 on the base active set A_B (port loads included; Z_B and G
// are complex symmetric), a candidate that keeps K = A_B \ R and adds E has
//   H   = (Z_B[K,K])^-1 = G_KK - G_KR M^-1 G_RK,          M = G_RR,
//   Z_c = [[Z_KK, B], [B^T, D]],   B = Z[K,E], D = Z[E,E],
//   S_m = D - B^T H B,
//   (Z_c^-1)_pp = H_pp + (H B)_p S_m^-1 (H B)_p^T           (block inverse).
// With B~ = B padded by zero rows at R and T = G B~ (|A_B| x |E|):
//   H B = T_K - G_KR M^-1 T_R,   B^T H B = B~^T T - T_R^T M^-1 T_R.
// Only T needs O(N^2 |E|) work; everything else is k x k algebra.  The port
// currents then give S_ij = delta_ij - 2 Z0 l_i l_j X_ij (Eqs. 6-7 with
// V_j = l_j e_pj).
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernels.hpp"

namespace pxd {

constexpr int KR_MAX = 16;  // removed functions handled per candidate
constexpr int KE_MAX = 8;   // added functions handled per candidate
constexpr int KE_CH = 4;    // added columns per pass over G
constexpr int ICH = 256;    // rows of B~ staged per chunk

struct LrShared {
  unsigned bits[64];  // base positions still active (N <= 2048)
  int R[KR_MAX], E[KE_MAX];
  int nr, ne, item;
  double2 Mr[KR_MAX * KR_MAX];
  double2 GpR[4 * KR_MAX];
  double2 Gpp[16];
  double2 TR[KR_MAX * KE_MAX];
  double2 Tp[4 * KE_MAX];
  double2 BtT[KE_MAX * KE_MAX];
  double2 D[KE_MAX * KE_MAX];
  double2 Y[KR_MAX * (4 + KE_MAX)];
  double2 b[ICH * KE_CH];
  double2 red[kWaves * KE_CH];
  // thread 0's k x k algebra
  double2 Hpp[16], HBp[4 * KE_MAX], Sm[KE_MAX * KE_MAX], X[16], Wv[KE_MAX * 4];
};

// Solve A X = Bm in place by Gaussian elimination with partial pivoting
// (one thread; A is n x n with leading dimension lda, Bm n x m with ldb).
// Returns false on an exactly zero pivot.
__device__ bool small_solve(double2* A, int lda, int n, double2* Bm, int ldb, int m) {
  bool ok = true;
  for (int c = 0; c < n; ++c) {
    int p = c;
    double best = fabs(A[c * lda + c].x) + fabs(A[c * lda + c].y);
    for (int r = c + 1; r < n; ++r) {
      const double v = fabs(A[r * lda + c].x) + fabs(A[r * lda + c].y);
      if (v > best) best = v, p = r;
    }
    if (!(best > 0.0)) {
      ok = false;
      continue;
    }
    if (p != c) {
      for (int j = 0; j < n; ++j) {
        const double2 t = A[c * lda + j];
        A[c * lda + j] = A[p * lda + j];
        A[p * lda + j] = t;
      }
      for (int j = 0; j < m; ++j) {
        const double2 t = Bm[c * ldb + j];
        Bm[c * ldb + j] = Bm[p * ldb + j];
        Bm[p * ldb + j] = t;
      }
    }
    const double2 inv = crecip(A[c * lda + c]);
    for (int r = c + 1; r < n; ++r) {
      const double2 l = cmul(A[r * lda + c], inv);
      for (int j = c + 1; j < n; ++j) A[r * lda + j] = cfms(A[r * lda + j], l, A[c * lda + j]);
      for (int j = 0; j < m; ++j) Bm[r * ldb + j] = cfms(Bm[r * ldb + j], l, Bm[c * ldb + j]);
    }
  }
  for (int j = 0; j < m; ++j)
    for (int r = n - 1; r >= 0; --r) {
      double2 acc = Bm[r * ldb + j];
      for (int t = r + 1; t < n; ++t) acc = cfms(acc, A[r * lda + t], Bm[t * ldb + j]);
      Bm[r * ldb + j] = cmul(acc, crecip(A[r * lda + r]));
    }
  return ok;
}

template <int QR>
__global__ __launch_bounds__(kThreads, 2) void k_lowrank(LrParams p) {
  __shared__ LrShared sh;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int NB = p.NB, P = p.P;
  const int n_items = p.C * p.F;
  for (;;) {
    if (tid == 0) sh.item = atomicAdd(p.counter, 1);
    __syncthreads();
    const int it = sh.item;
    __syncthreads();
    if (it >= n_items) break;
    const int f = it / p.C;
    const int c = p.order[it - f * p.C];
    const double2* Zf = p.Z128 + (size_t)f * p.M * p.M;
    const double2* G = p.G + (size_t)f * NB * NB;
    // 1. removed base positions R and added functions E
    for (int w = tid; w < 64; w += kThreads) sh.bits[w] = 0u;
    if (tid == 0) sh.nr = 0, sh.ne = 0;
    __syncthreads();
    const int Nc = p.Nc[c];
    const int* list = p.Ilist + (size_t)c * p.M;
    for (int s = tid; s < Nc; s += kThreads) {
      const int m = list[s];
      const int q = p.pos_of[m];
      if (q >= 0) {
        atomicOr(&sh.bits[q >> 5], 1u << (q & 31));
      } else {
        const int e = atomicAdd(&sh.ne, 1);
        if (e < KE_MAX) sh.E[e] = m;
      }
    }
    __syncthreads();
    for (int q = tid; q < NB; q += kThreads)
      if (!((sh.bits[q >> 5] >> (q & 31)) & 1u)) {
        const int r = atomicAdd(&sh.nr, 1);
        if (r < KR_MAX) sh.R[r] = q;
      }
    __syncthreads();
    const int nr = sh.nr, ne = sh.ne;
    if (nr > KR_MAX || ne > KE_MAX) {  // outside the low-rank limits: the dense FP64 path takes it
      if (tid == 0) {
        const int slot = atomicAdd(p.fb_count, 1);
        p.fb_list[slot] = c * p.F + f;
      }
      continue;
    }
    if (tid == 0) {  // ascending order, so results do not depend on the atomics' order
      for (int a = 1; a < nr; ++a)
        for (int b = a; b > 0 && sh.R[b - 1] > sh.R[b]; --b) {
          const int t = sh.R[b];
          sh.R[b] = sh.R[b - 1];
          sh.R[b - 1] = t;
        }
      for (int a = 1; a < ne; ++a)
        for (int b = a; b > 0 && sh.E[b - 1] > sh.E[b]; --b) {
          const int t = sh.E[b];
          sh.E[b] = sh.E[b - 1];
          sh.E[b - 1] = t;
        }
    }
    __syncthreads();
    // 2. the small blocks of G
    for (int e = tid; e < nr * nr; e += kThreads) sh.Mr[e] = G[(size_t)sh.R[e / nr] * NB + sh.R[e % nr]];
    for (int e = tid; e < P * nr; e += kThreads) sh.GpR[e] = G[(size_t)(NB - P + e / nr) * NB + sh.R[e % nr]];
    for (int e = tid; e < P * P; e += kThreads) sh.Gpp[e] = G[(size_t)(NB - P + e / P) * NB + NB - P + e % P];
    for (int e = tid; e < ne * ne; e += kThreads) sh.D[e] = Zf[(size_t)sh.E[e / ne] * p.M + sh.E[e % ne]];
    __syncthreads();
    // 3. T = G B~ in passes of KE_CH added columns; keep T_R, T_p and B~^T T
    for (int e0 = 0; e0 < ne; e0 += KE_CH) {
      const int nch = min(KE_CH, ne - e0);
      double2 t[QR][KE_CH];
#pragma unroll
      for (int q = 0; q < QR; ++q)
#pragma unroll
        for (int ee = 0; ee < KE_CH; ++ee) t[q][ee] = double2{0.0, 0.0};
      for (int i0 = 0; i0 < NB; i0 += ICH) {
        __syncthreads();
        for (int e = tid; e < ICH * KE_CH; e += kThreads) {
          const int ii = e / KE_CH, ee = e - ii * KE_CH, i = i0 + ii;
          const bool kept = i < NB && ((sh.bits[i >> 5] >> (i & 31)) & 1u);
          sh.b[e] = (kept && ee < nch) ? Zf[(size_t)sh.E[e0 + ee] * p.M + p.IB[i]] : double2{0.0, 0.0};
        }
        __syncthreads();
        const int iend = min(ICH, NB - i0);
        for (int ii = 0; ii < iend; ++ii) {
          const double2* grow = G + (size_t)(i0 + ii) * NB;  // G symmetric: row i holds column i
#pragma unroll
          for (int q = 0; q < QR; ++q) {
            const int r = tid + kThreads * q;
            if (r < NB) {
              const double2 g = grow[r];
#pragma unroll
              for (int ee = 0; ee < KE_CH; ++ee) {
                const double2 bv = sh.b[ii * KE_CH + ee];
                t[q][ee].x += g.x * bv.x - g.y * bv.y;
                t[q][ee].y += g.x * bv.y + g.y * bv.x;
              }
            }
          }
        }
      }
      // rows of T at R and at the ports
#pragma unroll
      for (int q = 0; q < QR; ++q) {
        const int r = tid + kThreads * q;
        if (r < NB) {
          if (!((sh.bits[r >> 5] >> (r & 31)) & 1u))
            for (int a = 0; a < nr; ++a)
              if (sh.R[a] == r) {
#pragma unroll
                for (int ee = 0; ee < KE_CH; ++ee)
                  if (ee < nch) sh.TR[a * KE_MAX + e0 + ee] = t[q][ee];
              }
          if (r >= NB - P) {
#pragma unroll
            for (int ee = 0; ee < KE_CH; ++ee)
              if (ee < nch) sh.Tp[(r - (NB - P)) * KE_MAX + e0 + ee] = t[q][ee];
          }
        }
      }
      // B~^T T for these columns: one block reduction per added function e1
      for (int e1 = 0; e1 < ne; ++e1) {
        double2 part[KE_CH];
#pragma unroll
        for (int ee = 0; ee < KE_CH; ++ee) part[ee] = double2{0.0, 0.0};
#pragma unroll
        for (int q = 0; q < QR; ++q) {
          const int r = tid + kThreads * q;
          if (r < NB && ((sh.bits[r >> 5] >> (r & 31)) & 1u)) {
            const double2 bv = Zf[(size_t)sh.E[e1] * p.M + p.IB[r]];
#pragma unroll
            for (int ee = 0; ee < KE_CH; ++ee) {
              part[ee].x += bv.x * t[q][ee].x - bv.y * t[q][ee].y;
              part[ee].y += bv.x * t[q][ee].y + bv.y * t[q][ee].x;
            }
          }
        }
#pragma unroll
        for (int ee = 0; ee < KE_CH; ++ee) {
#pragma unroll
          for (int off = 32; off >= 1; off >>= 1) {
            part[ee].x += __shfl_xor(part[ee].x, off, 64);
            part[ee].y += __shfl_xor(part[ee].y, off, 64);
          }
          if (lane == 0) sh.red[wid * KE_CH + ee] = part[ee];
        }
        __syncthreads();
        if (tid < nch) {
          double2 sum = double2{0.0, 0.0};
          for (int w = 0; w < kWaves; ++w) {
            sum.x += sh.red[w * KE_CH + tid].x;
            sum.y += sh.red[w * KE_CH + tid].y;
          }
          sh.BtT[e1 * KE_MAX + e0 + tid] = sum;
        }
        __syncthreads();
      }
    }
    __syncthreads();
    // 4. the k x k algebra and S (one thread)
    if (tid == 0) {
      bool ok = true;
      double2 *Hpp = sh.Hpp, *HBp = sh.HBp, *Sm = sh.Sm, *X = sh.X, *Wv = sh.Wv;
      for (int e = 0; e < P * P; ++e) Hpp[e] = sh.Gpp[e];
      for (int i = 0; i < P; ++i)
        for (int e = 0; e < ne; ++e) HBp[i * KE_MAX + e] = sh.Tp[i * KE_MAX + e];
      for (int a = 0; a < ne; ++a)
        for (int b = 0; b < ne; ++b) Sm[a * KE_MAX + b] = csub(sh.D[a * ne + b], sh.BtT[a * KE_MAX + b]);
      if (nr > 0) {
        // Y = M^-1 [G_Rp | T_R]   (G_Rp = G_pR^T)
        const int m = P + ne, ldy = 4 + KE_MAX;
        for (int a = 0; a < nr; ++a) {
          for (int i = 0; i < P; ++i) sh.Y[a * ldy + i] = sh.GpR[i * nr + a];
          for (int e = 0; e < ne; ++e) sh.Y[a * ldy + P + e] = sh.TR[a * KE_MAX + e];
        }
        ok = small_solve(sh.Mr, nr, nr, sh.Y, ldy, m) && ok;
        for (int i = 0; i < P; ++i) {
          for (int j = 0; j < P; ++j)
            for (int a = 0; a < nr; ++a) Hpp[i * P + j] = cfms(Hpp[i * P + j], sh.GpR[i * nr + a], sh.Y[a * ldy + j]);
          for (int e = 0; e < ne; ++e)
            for (int a = 0; a < nr; ++a)
              HBp[i * KE_MAX + e] = cfms(HBp[i * KE_MAX + e], sh.GpR[i * nr + a], sh.Y[a * ldy + P + e]);
        }
        for (int a = 0; a < ne; ++a)  // + T_R^T M^-1 T_R
          for (int b = 0; b < ne; ++b)
            for (int r = 0; r < nr; ++r)
              Sm[a * KE_MAX + b] = cadd(Sm[a * KE_MAX + b], cmul(sh.TR[r * KE_MAX + a], sh.Y[r * ldy + P + b]));
      }
      for (int e = 0; e < P * P; ++e) X[e] = Hpp[e];
      if (ne > 0) {
        // Wv = S_m^-1 (H B)_p^T
        for (int e = 0; e < ne; ++e)
          for (int j = 0; j < P; ++j) Wv[e * 4 + j] = HBp[j * KE_MAX + e];
        ok = small_solve(Sm, KE_MAX, ne, Wv, 4, P) && ok;
        for (int i = 0; i < P; ++i)
          for (int j = 0; j < P; ++j)
            for (int e = 0; e < ne; ++e) X[i * P + j] = cadd(X[i * P + j], cmul(HBp[i * KE_MAX + e], Wv[e * 4 + j]));
      }
      double2* Sout = p.S + ((size_t)c * p.F + f) * P * P;
      bool finite = true;
      for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j) {
          const double g = 2.0 * p.z0 * p.port_len[i] * p.port_len[j];
          const double2 sv = double2{(i == j ? 1.0 : 0.0) - g * X[i * P + j].x, -g * X[i * P + j].y};
          finite = finite && isfinite(sv.x) && isfinite(sv.y);
          Sout[i * P + j] = sv;
        }
      int st = PXD_STATUS_OK;
      if (!finite) st = PXD_STATUS_NONFINITE;
      else if (!ok || p.base_status[f] != PXD_STATUS_OK) st = PXD_STATUS_SINGULAR;
      p.status[(size_t)c * p.F + f] = st;
    }
    __syncthreads();
  }
}

// base position of every parent function (-1 if inactive in the base map)
__global__ void k_positions(int M, int* pos_of) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < M) pos_of[m] = -1;
}

__global__ void k_positions_set(const int* IB, int NB, int* pos_of) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < NB) pos_of[IB[i]] = i;
}

hipError_t launch_positions(hipStream_t s, const int* IB, int NB, int M, int* pos_of) {
  hipLaunchKernelGGL(k_positions, dim3((M + 255) / 256), dim3(256), 0, s, M, pos_of);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || NB <= 0) return e;
  hipLaunchKernelGGL(k_positions_set, dim3((NB + 255) / 256), dim3(256), 0, s, IB, NB, pos_of);
  return hipGetLastError();
}

hipError_t launch_lowrank(hipStream_t s, const LrParams& p, int grid) {
  const int Q = rows_per_thread(p.NB);
  if (Q <= 1) hipLaunchKernelGGL((k_lowrank<1>), dim3(grid), dim3(kThreads), 0, s, p);
  else if (Q <= 2) hipLaunchKernelGGL((k_lowrank<2>), dim3(grid), dim3(kThreads), 0, s, p);
  else if (Q <= 4) hipLaunchKernelGGL((k_lowrank<4>), dim3(grid), dim3(kThreads), 0, s, p);
  else if (Q <= 8) hipLaunchKernelGGL((k_lowrank<8>), dim3(grid), dim3(kThreads), 0, s, p);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace pxd
