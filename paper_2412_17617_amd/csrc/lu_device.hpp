// Device routines of the dense LU solve shared by the evaluator kernels:
// gather of Z_A (Eq. 5), the two-level right-looking LU with partial
// pivoting (Eq. 2) and its pieces, the port-block solve and S (Eqs. 6-7),
// and the complex64 solve / FP64 residual / port-correction steps of the
// mixed-precision refinement.  Included by the kernel sources only.
#pragma once

#include "device.hpp"
#include "kernels.hpp"

namespace pxd {

constexpr int NB = 32;     // inner panel width
constexpr int KBMAX = 128; // widest outer block column
constexpr int CS = 32;     // column slab of the wide trailing update staged in LDS
constexpr int KB_PLAIN = 64;  // block column of the complex128 LU
constexpr int KB_MIXED = 64;  // block column of the complex64 LU

template <typename R>
struct LuShared {
  using T = typename Cx<R>::T;
  T prow[NB];
  T crow[NB];
  T buf[2 * NB * NB];  // L11 (first half) and the sub-panel U block (second half), or a wide-update slab
  R red_v[kWaves];
  int red_i[kWaves];
  int piv[NB];
  int bpiv[KBMAX];  // pivots of the current block column (absolute rows)
  int bad;
};

// Z_A = Z_f[I, I] into the slot, plus the Z0 loads of the port functions and,
// for the augmented system, the excitation columns V (1 V source EMF in each
// port gap: V[row of port j, j] = l_j).
template <typename T, typename TP>
__device__ __forceinline__ void gather_item(T* __restrict__ W, int ld, const TP* __restrict__ Zf, int M, const int* sI, int N,
                            int P, const double* __restrict__ plen, double z0, bool augment) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int r = wid; r < N; r += kWaves) {
    const TP* zrow = Zf + (size_t)sI[r] * M;
    T* wrow = W + (size_t)r * ld;
    int s = lane;
    for (; s + 192 < N; s += 256) {
      const TP v0 = zrow[sI[s]], v1 = zrow[sI[s + 64]], v2 = zrow[sI[s + 128]], v3 = zrow[sI[s + 192]];
      wrow[s] = T{(decltype(T::x))v0.x, (decltype(T::x))v0.y};
      wrow[s + 64] = T{(decltype(T::x))v1.x, (decltype(T::x))v1.y};
      wrow[s + 128] = T{(decltype(T::x))v2.x, (decltype(T::x))v2.y};
      wrow[s + 192] = T{(decltype(T::x))v3.x, (decltype(T::x))v3.y};
    }
    for (; s < N; s += 64) {
      const TP v = zrow[sI[s]];
      wrow[s] = T{(decltype(T::x))v.x, (decltype(T::x))v.y};
    }
    if (augment && lane < P) wrow[N + lane] = T{(r == N - P + lane) ? (decltype(T::x))plen[lane] : 0, 0};
  }
  __syncthreads();
  if (tid < P) {
    const int r = N - P + tid;
    W[(size_t)r * ld + r].x += (decltype(T::x))(z0 * plen[tid] * plen[tid]);
  }
  __syncthreads();
}

// ------------------------------------------------------------------ LU pieces

// Unblocked LU with partial pivoting of the sub-panel rows [c0, N), columns
// [c0, c0 + sbw), held in registers: thread t owns rows c0 + t + 256 q.
template <typename R, int Q, int SB>
__device__ __forceinline__ void factor_subpanel(typename Cx<R>::T* __restrict__ W, int ld, int N, int c0, int sbw,
                                LuShared<R>& sm, int pbase) {
  using T = typename Cx<R>::T;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  T reg[Q][SB];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int r = c0 + tid + kThreads * q;
#pragma unroll
    for (int j = 0; j < SB; ++j) reg[q][j] = (r < N && j < sbw) ? W[(size_t)r * ld + c0 + j] : T{0, 0};
  }
#pragma unroll
  for (int j = 0; j < SB; ++j) {
    if (j < sbw) {
      const int c = c0 + j;
      R best = R(-1);
      int bi = 0x7fffffff;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int r = c0 + tid + kThreads * q;
        if (r >= c && r < N) {
          const R v = fabs(reg[q][j].x) + fabs(reg[q][j].y);
          if (v > best) {
            best = v;
            bi = r;
          }
        }
      }
      wave_argmax(best, bi);
      if (lane == 0) {
        sm.red_v[wid] = best;
        sm.red_i[wid] = bi;
      }
      __syncthreads();
      best = sm.red_v[0];
      bi = sm.red_i[0];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) {
        const R ov = sm.red_v[w];
        const int oi = sm.red_i[w];
        if (ov > best || (ov == best && oi < bi)) {
          best = ov;
          bi = oi;
        }
      }
      if (bi >= N) bi = c;  // no finite candidate: keep the diagonal, flagged below
      const int p = bi;
      const int oc = c - c0, op = p - c0;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int rr = tid + kThreads * q;
        if (rr == op) {
#pragma unroll
          for (int jj = 0; jj < SB; ++jj) sm.prow[jj] = reg[q][jj];
        }
        if (rr == oc) {
#pragma unroll
          for (int jj = 0; jj < SB; ++jj) sm.crow[jj] = reg[q][jj];
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int rr = tid + kThreads * q;
        if (rr == oc) {
#pragma unroll
          for (int jj = 0; jj < SB; ++jj) reg[q][jj] = sm.prow[jj];
        } else if (rr == op) {
#pragma unroll
          for (int jj = 0; jj < SB; ++jj) reg[q][jj] = sm.crow[jj];
        }
      }
      const T pv = sm.prow[j];
      if (tid == 0) {
        sm.piv[pbase + j] = p;
        if (!(fabs(pv.x) + fabs(pv.y) > R(0))) sm.bad = 1;  // zero or non-finite pivot
      }
      const T inv = crecip(pv);
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int r = c0 + tid + kThreads * q;
        if (r > c && r < N) {
          const T l = cmul(reg[q][j], inv);
          reg[q][j] = l;
#pragma unroll
          for (int jj = j + 1; jj < SB; ++jj) reg[q][jj] = cfms(reg[q][jj], l, sm.prow[jj]);
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int r = c0 + tid + kThreads * q;
    if (r < N) {
#pragma unroll
      for (int j = 0; j < SB; ++j)
        if (j < sbw) W[(size_t)r * ld + c0 + j] = reg[q][j];
    }
  }
}

// Factor panel columns [k, k + kb) over rows [k, N); pivots of the panel end
// in sm.piv[0 .. kb) (absolute rows), applied to every panel column.
template <typename R, int Q, int SB>
__device__ __forceinline__ void factor_panel(typename Cx<R>::T* __restrict__ W, int ld, int N, int k, int kb, LuShared<R>& sm) {
  using T = typename Cx<R>::T;
  const int tid = threadIdx.x;
  for (int s = 0; s < kb; s += SB) {
    const int c0 = k + s, sbw = min(SB, kb - s);
    factor_subpanel<R, Q, SB>(W, ld, N, c0, sbw, sm, s);
    __syncthreads();
    // this sub-block's interchanges on the other columns of the panel
    for (int t = tid; t < kb; t += kThreads) {
      const int col = k + t;
      if (col >= c0 && col < c0 + sbw) continue;
      for (int j = 0; j < sbw; ++j) {
        const int r = c0 + j, p = sm.piv[s + j];
        if (p != r) {
          const T a = W[(size_t)r * ld + col];
          W[(size_t)r * ld + col] = W[(size_t)p * ld + col];
          W[(size_t)p * ld + col] = a;
        }
      }
    }
    __syncthreads();
    const int w2 = kb - s - sbw;
    if (w2 > 0) {
      // U block of the columns right of the sub-block: unit-lower solve
      for (int t = tid; t < w2; t += kThreads) {
        const int col = c0 + sbw + t;
        T u[SB];
#pragma unroll
        for (int i = 0; i < SB; ++i) u[i] = (i < sbw) ? W[(size_t)(c0 + i) * ld + col] : T{0, 0};
#pragma unroll
        for (int i = 1; i < SB; ++i) {
          if (i < sbw) {
            T acc = u[i];
#pragma unroll
            for (int j = 0; j < i; ++j) acc = cfms(acc, W[(size_t)(c0 + i) * ld + c0 + j], u[j]);
            u[i] = acc;
          }
        }
#pragma unroll
        for (int i = 0; i < SB; ++i)
          if (i < sbw) {
            W[(size_t)(c0 + i) * ld + col] = u[i];
            sm.buf[NB * NB + i * NB + t] = u[i];
          }
      }
      __syncthreads();
      {
        // rows below: the 32 lanes of a half-wave span a row's w2 columns
        // (one contiguous segment per load and store; the row's L entries are
        // broadcast loads), RU rows per half-wave and step, all their loads
        // issued before any product
        constexpr int RW = SB * (int)sizeof(R) / 4;  // register words of one row's L entries
        constexpr int RU = RW >= 32 ? 1 : RW >= 16 ? 2 : RW >= 8 ? 4 : 8;
        const int lane = tid & 63, wid = tid >> 6, t = lane & 31, half = lane >> 5;
        const int step = 2 * kWaves;
        T u[SB];
#pragma unroll
        for (int j = 0; j < SB; ++j) u[j] = (t < w2 && j < sbw) ? sm.buf[NB * NB + j * NB + t] : T{0, 0};
        for (int rb = c0 + sbw + 2 * wid + half; rb < N; rb += step * RU) {
          T lv[RU][SB], v[RU];
#pragma unroll
          for (int q = 0; q < RU; ++q) {
            const int r = rb + q * step;
            const bool ok = t < w2 && r < N;
#pragma unroll
            for (int j = 0; j < SB; ++j) lv[q][j] = (ok && j < sbw) ? W[(size_t)r * ld + c0 + j] : T{0, 0};
            v[q] = ok ? W[(size_t)r * ld + c0 + sbw + t] : T{0, 0};
          }
#pragma unroll
          for (int q = 0; q < RU; ++q) {
            const int r = rb + q * step;
            if (t < w2 && r < N) {
              T acc{0, 0};
#pragma unroll
              for (int j = 0; j < SB; ++j) acc = cfms(acc, lv[q][j], u[j]);
              W[(size_t)r * ld + c0 + sbw + t] = T{v[q].x + acc.x, v[q].y + acc.y};
            }
          }
        }
      }
      __syncthreads();
    }
  }
}

// Interchanges of panel rows [k, k + kb) (pivots in piv, absolute rows; no
// interchanges when piv is null) on columns [c0, c1), then U = L11^-1 A for
// those rows and columns (L11 unit lower, from the panel), one thread per
// column, in blocks of 8 rows held in registers.
template <typename R>
__device__ __forceinline__ void swap_trsm(typename Cx<R>::T* __restrict__ W, int ld, int k, int kb, int c0, int c1,
                                          LuShared<R>& sm, const int* piv) {
  using T = typename Cx<R>::T;
  constexpr int B = 8;
  const int tid = threadIdx.x;
  for (int e = tid; e < kb * kb; e += kThreads) {
    const int i = e / kb, j = e - i * kb;
    sm.buf[i * NB + j] = (j < i) ? W[(size_t)(k + i) * ld + k + j] : T{0, 0};
  }
  __syncthreads();
  for (int col = c0 + tid; col < c1; col += kThreads) {
    if (piv)
      for (int i = 0; i < kb; ++i) {
        const int r = k + i, p = piv[i];
        if (p != r) {
          const T a = W[(size_t)r * ld + col];
          W[(size_t)r * ld + col] = W[(size_t)p * ld + col];
          W[(size_t)p * ld + col] = a;
        }
      }
    for (int b0 = 0; b0 < kb; b0 += B) {
      T u[B];
#pragma unroll
      for (int i = 0; i < B; ++i) u[i] = (b0 + i < kb) ? W[(size_t)(k + b0 + i) * ld + col] : T{0, 0};
      for (int j = 0; j < b0; ++j) {  // contributions of the solved rows above the block
        const T uj = W[(size_t)(k + j) * ld + col];
#pragma unroll
        for (int i = 0; i < B; ++i) u[i] = cfms(u[i], sm.buf[(b0 + i) * NB + j], uj);
      }
#pragma unroll
      for (int i = 1; i < B; ++i)
#pragma unroll
        for (int j = 0; j < i; ++j) u[i] = cfms(u[i], sm.buf[(b0 + i) * NB + b0 + j], u[j]);
#pragma unroll
      for (int i = 0; i < B; ++i)
        if (b0 + i < kb) W[(size_t)(k + b0 + i) * ld + col] = u[i];
    }
  }
  __syncthreads();
}

// U = L11^-1 A on rows [k, k + kb) and columns [c0, c1), L11 the unit-lower
// panel block: its inverse is formed in LDS (row by row, all entries of a row
// at once) and applied as an MFMA product, each wave taking 16-column tiles
// (the tile's A rows are in registers before any of them is overwritten).
template <typename R>
__device__ __forceinline__ void trsm_inverse(typename Cx<R>::T* __restrict__ W, int ld, int k, int kb, int c0, int c1,
                                             LuShared<R>& sm) {
  using T = typename Cx<R>::T;
  using MF = Mfma<R>;
  using acc_t = typename MF::acc_t;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  T* L = sm.buf;             // L11, strictly lower part (zero elsewhere)
  T* Li = sm.buf + NB * NB;  // its inverse, zero outside [0, kb)^2
  for (int e = tid; e < NB * NB; e += kThreads) {
    const int i = e / NB, j = e - i * NB;
    L[e] = (i < kb && j < i) ? W[(size_t)(k + i) * ld + k + j] : T{0, 0};
    Li[e] = (i == j && i < kb) ? T{1, 0} : T{0, 0};
  }
  __syncthreads();
  for (int i = 1; i < kb; ++i) {  // Li[i][j] = -sum_{j <= t < i} L[i][t] Li[t][j]
    if (tid < i) {
      const int j = tid;
      T acc{0, 0};
      for (int t = j; t < i; ++t) acc = cfms(acc, L[i * NB + t], Li[t * NB + j]);
      Li[i * NB + j] = acc;
    }
    __syncthreads();
  }
  // A operand: Li rows 16 a + l16, k-columns 4 kq + lk
  R ar[2][NB / 4], ai[2][NB / 4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int kq = 0; kq < NB / 4; ++kq) {
      const T v = Li[(16 * a + l16) * NB + 4 * kq + lk];
      ar[a][kq] = v.x;
      ai[a][kq] = v.y;
    }
  const int ntile = (c1 - c0 + 15) >> 4;
  for (int tn = wid; tn < ntile; tn += kWaves) {
    const int col = c0 + 16 * tn + l16;
    T bq[NB / 4];
#pragma unroll
    for (int kq = 0; kq < NB / 4; ++kq) {
      const int kk = 4 * kq + lk;
      bq[kq] = (kk < kb && col < c1) ? W[(size_t)(k + kk) * ld + col] : T{0, 0};
    }
    acc_t cr[2], ci[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      cr[a] = acc_t{0, 0, 0, 0};
      ci[a] = acc_t{0, 0, 0, 0};
    }
#pragma unroll
    for (int kq = 0; kq < NB / 4; ++kq)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        cr[a] = MF::run(ar[a][kq], bq[kq].x, cr[a]);
        cr[a] = MF::run(ai[a][kq], -bq[kq].y, cr[a]);
        ci[a] = MF::run(ar[a][kq], bq[kq].y, ci[a]);
        ci[a] = MF::run(ai[a][kq], bq[kq].x, ci[a]);
      }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 16 * a + MF::row(lane, i);
        if (r < kb && col < c1) W[(size_t)(k + r) * ld + col] = T{cr[a][i], ci[a][i]};
      }
  }
  __syncthreads();
}

// Interchanges of rows [k, k + kb) with piv[0 .. kb) on columns [c0, c1), in order.
template <typename T>
__device__ __forceinline__ void apply_swaps(T* __restrict__ W, int ld, int k, int kb, const int* piv, int c0, int c1) {
  for (int col = c0 + (int)threadIdx.x; col < c1; col += kThreads)
    for (int i = 0; i < kb; ++i) {
      const int r = k + i, p = piv[i];
      if (p != r) {
        const T a = W[(size_t)r * ld + col];
        W[(size_t)r * ld + col] = W[(size_t)p * ld + col];
        W[(size_t)p * ld + col] = a;
      }
    }
  __syncthreads();
}

// A22 -= L21 U12 on rows [k + kb, r1), columns [c0, c1), with L21 the panel
// columns [k, k + kb) and U12 the panel rows.
// Wave w owns block rows w, w + 4, ... of 32 rows and keeps their (negated)
// L21 fragments in registers while sweeping the block columns; the four waves
// sweep the columns in the same order, so a U12 block is fetched from memory
// once and served to the other waves from cache.  Each 32 x 32 output tile
// issues its U12 fragment loads before its 128 MFMAs (the products are
// summed from zero and added to C once at the end), so the two waves sharing
// a SIMD overlap one tile's memory latency with the other's arithmetic.
template <typename R>
__device__ __forceinline__ void trailing_update(typename Cx<R>::T* __restrict__ W, int ld, int k, int kb, int N,
                                                int c0, int ncols) {
  using T = typename Cx<R>::T;
  using MF = Mfma<R>;
  using acc_t = typename MF::acc_t;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  const int r0 = k + kb;
  const int mr = N - r0, nc = ncols - c0;
  if (mr <= 0 || nc <= 0) return;
  const int tmn = (mr + 31) >> 5, tnn = (nc + 31) >> 5;
  for (int tm = wid; tm < tmn; tm += kWaves) {
    // -L21 fragments of this block row: A operand lane l holds row l % 16, k l / 16
    R anr[2][NB / 4], ani[2][NB / 4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int kq = 0; kq < NB / 4; ++kq) {
        const int r = r0 + 32 * tm + 16 * a + l16;
        const int kk = 4 * kq + lk;
        const T v = (r < N && kk < kb) ? W[(size_t)r * ld + k + kk] : T{0, 0};
        anr[a][kq] = -v.x;
        ani[a][kq] = -v.y;
      }
    for (int tn = 0; tn < tnn; ++tn) {
      acc_t cr[2][2], ci[2][2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            cr[a][b][i] = R(0);  // the products are summed apart from C (one rounding into C)
            ci[a][b][i] = R(0);
          }
      auto load_b = [&](int kq, int b) -> T {
        const int kk = 4 * kq + lk;
        const int col = c0 + 32 * tn + 16 * b + l16;
        return (kk < kb && col < ncols) ? W[(size_t)(k + kk) * ld + col] : T{0, 0};
      };
      // C -= A B:  Cr += (-Ar) Br + (-Ai)(-Bi),  Ci += (-Ar) Bi + (-Ai) Br
      auto mma = [&](int kq, const T (&bq)[2]) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            cr[a][b] = MF::run(anr[a][kq], bq[b].x, cr[a][b]);
            cr[a][b] = MF::run(ani[a][kq], -bq[b].y, cr[a][b]);
            ci[a][b] = MF::run(anr[a][kq], bq[b].y, ci[a][b]);
            ci[a][b] = MF::run(ani[a][kq], bq[b].x, ci[a][b]);
          }
      };
      if constexpr (sizeof(R) == 4) {
        // complex64: every U12 fragment of the tile in flight at once
        T bfr[NB / 4][2];
#pragma unroll
        for (int kq = 0; kq < NB / 4; ++kq)
#pragma unroll
          for (int b = 0; b < 2; ++b) bfr[kq][b] = load_b(kq, b);
#pragma unroll
        for (int kq = 0; kq < NB / 4; ++kq) mma(kq, bfr[kq]);
      } else {
        // complex128: stream the fragments one k-step ahead (register budget)
        T cur[2] = {load_b(0, 0), load_b(0, 1)};
#pragma unroll
        for (int kq = 0; kq < NB / 4; ++kq) {
          T nxt[2];
          if (kq + 1 < NB / 4) {
            nxt[0] = load_b(kq + 1, 0);
            nxt[1] = load_b(kq + 1, 1);
          }
          mma(kq, cur);
          if (kq + 1 < NB / 4) {
            cur[0] = nxt[0];
            cur[1] = nxt[1];
          }
        }
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int r = r0 + 32 * tm + 16 * a + MF::row(lane, i);
            const int col = c0 + 32 * tn + 16 * b + l16;
            if (r < N && col < ncols) {
              const T v = W[(size_t)r * ld + col];
              W[(size_t)r * ld + col] = T{v.x + cr[a][b][i], v.y + ci[a][b][i]};
            }
          }
    }
  }
}

// A[r0:r1, c0:c1] -= A[r0:r1, k:k+kb] A[k:k+kb, c0:c1] for a block column of
// width kb <= KB.  The U12 rows are staged in LDS (Us, KB x CS complex) one
// column slab at a time; each wave owns RT consecutive 16-row tiles of a
// 64 RT-row group and keeps their (negated) L21 fragments in registers for
// the whole group, so the trailing block is read and written once per block
// column and U12 once per row group.
template <typename R, int KB, int RT>
__device__ __forceinline__ void wide_update(typename Cx<R>::T* __restrict__ W, int ld, int k, int kb, int r0, int r1,
                                            int c0, int c1, typename Cx<R>::T* Us) {
  using T = typename Cx<R>::T;
  using MF = Mfma<R>;
  using acc_t = typename MF::acc_t;
  constexpr int KQ = KB / 4;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  if (r1 <= r0 || c1 <= c0 || kb <= 0) return;
  constexpr int GROUP = kWaves * 16 * RT;
  for (int g0 = r0; g0 < r1; g0 += GROUP) {
    const int rb = g0 + wid * 16 * RT;
    R anr[RT][KQ], ani[RT][KQ];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int kq = 0; kq < KQ; ++kq) {
        const int r = rb + 16 * t + l16, kk = 4 * kq + lk;
        const T v = (r < r1 && kk < kb) ? W[(size_t)r * ld + k + kk] : T{0, 0};
        anr[t][kq] = -v.x;
        ani[t][kq] = -v.y;
      }
    for (int s0 = c0; s0 < c1; s0 += CS) {
      __syncthreads();  // the previous slab is consumed
      for (int e = tid; e < KB * CS; e += kThreads) {
        const int i = e / CS, j = e - i * CS;
        Us[e] = (i < kb && s0 + j < c1) ? W[(size_t)(k + i) * ld + s0 + j] : T{0, 0};
      }
      __syncthreads();
      if (rb < r1) {
        acc_t cr[RT][2], ci[RT][2];
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              cr[t][b][i] = 0;  // the products are summed apart from C (one rounding into C)
              ci[t][b][i] = 0;
            }
#pragma unroll
        for (int kq = 0; kq < KQ; ++kq) {
          if (4 * kq < kb) {
            T bq[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) bq[b] = Us[(4 * kq + lk) * CS + 16 * b + l16];
#pragma unroll
            for (int t = 0; t < RT; ++t)
#pragma unroll
              for (int b = 0; b < 2; ++b) {
                cr[t][b] = MF::run(anr[t][kq], bq[b].x, cr[t][b]);
                cr[t][b] = MF::run(ani[t][kq], -bq[b].y, cr[t][b]);
                ci[t][b] = MF::run(anr[t][kq], bq[b].y, ci[t][b]);
                ci[t][b] = MF::run(ani[t][kq], bq[b].x, ci[t][b]);
              }
          }
        }
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int r = rb + 16 * t + MF::row(lane, i), col = s0 + 16 * b + l16;
              if (r < r1 && col < c1) {
                const T v = W[(size_t)r * ld + col];
                W[(size_t)r * ld + col] = T{v.x + cr[t][b][i], v.y + ci[t][b][i]};
              }
            }
      }
    }
  }
  __syncthreads();
}

// Half-precision operands for the 16x16x16 MFMA: lane l holds A[l % 16][4 (l / 16) + j]
// and B[4 (l / 16) + j][l % 16] for j < 4; the accumulator layout is the FP32 one.
template <int H>
struct Half;
template <>
struct Half<PXD_HALF_BF16> {
  typedef short v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ short one(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (short)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (short)(u >> 16);
  }
  static __device__ __forceinline__ fx4 run(v4 a, v4 b, fx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
};
template <>
struct Half<PXD_HALF_F16> {
  typedef _Float16 v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ _Float16 one(float f) { return (_Float16)f; }
  static __device__ __forceinline__ fx4 run(v4 a, v4 b, fx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
  }
};

// wide_update for the complex64 factor with L21 and U12 rounded to BF16 or
// FP16 (the products accumulate in FP32 on top of the FP32 trailing block).
template <int KB, int RT, int H>
__device__ __forceinline__ void wide_update_half(float2* __restrict__ W, int ld, int k, int kb, int r0, int r1, int c0,
                                                 int c1, float2* Us) {
  using HM = Half<H>;
  using v4 = typename HM::v4;
  using MF = Mfma<float>;
  constexpr int KC = KB / 16;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  if (r1 <= r0 || c1 <= c0 || kb <= 0) return;
  constexpr int GROUP = kWaves * 16 * RT;
  for (int g0 = r0; g0 < r1; g0 += GROUP) {
    const int rb = g0 + wid * 16 * RT;
    v4 anr[RT][KC], ani[RT][KC];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int c = 0; c < KC; ++c)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = rb + 16 * t + l16, kk = 16 * c + 4 * lk + j;
          const float2 v = (r < r1 && kk < kb) ? W[(size_t)r * ld + k + kk] : float2{0, 0};
          anr[t][c][j] = HM::one(-v.x);
          ani[t][c][j] = HM::one(-v.y);
        }
    for (int s0 = c0; s0 < c1; s0 += CS) {
      __syncthreads();
      for (int e = tid; e < KB * CS; e += kThreads) {
        const int i = e / CS, j = e - i * CS;
        Us[e] = (i < kb && s0 + j < c1) ? W[(size_t)(k + i) * ld + s0 + j] : float2{0, 0};
      }
      __syncthreads();
      if (rb < r1) {
        fx4 cr[RT][2], ci[RT][2];
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              cr[t][b][i] = 0;  // the products are summed apart from C (one rounding into C)
              ci[t][b][i] = 0;
            }
#pragma unroll
        for (int c = 0; c < KC; ++c) {
          if (16 * c < kb) {
            v4 br[2], bi[2], bin[2];
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
              for (int j = 0; j < 4; ++j) {
                const float2 u = Us[(16 * c + 4 * lk + j) * CS + 16 * b + l16];
                br[b][j] = HM::one(u.x);
                bi[b][j] = HM::one(u.y);
                bin[b][j] = HM::one(-u.y);
              }
#pragma unroll
            for (int t = 0; t < RT; ++t)
#pragma unroll
              for (int b = 0; b < 2; ++b) {
                cr[t][b] = HM::run(anr[t][c], br[b], cr[t][b]);
                cr[t][b] = HM::run(ani[t][c], bin[b], cr[t][b]);
                ci[t][b] = HM::run(anr[t][c], bi[b], ci[t][b]);
                ci[t][b] = HM::run(ani[t][c], br[b], ci[t][b]);
              }
          }
        }
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int r = rb + 16 * t + MF::row(lane, i), col = s0 + 16 * b + l16;
              if (r < r1 && col < c1) {
                const float2 v = W[(size_t)r * ld + col];
                W[(size_t)r * ld + col] = float2{v.x + cr[t][b][i], v.y + ci[t][b][i]};
              }
            }
      }
    }
  }
  __syncthreads();
}

// Two-level right-looking LU with partial pivoting of columns [0, Ne) of the
// N x ncols row-major matrix.  Block columns of KB are factored with 32-wide
// panels (interchanges applied across the whole block column, so its L is
// stored in the block's final row order); then the block's interchanges, the
// solve for its U rows and one rank-KB update reach the columns to its right.
// Columns left of a block are not permuted by later blocks: solves replay
// the interchanges block by block.  When piv_out is given the pivots are
// stored there (absolute rows).
template <typename R, int Q, int SB, int KB, int RT>
__device__ __forceinline__ void lu_factor(typename Cx<R>::T* __restrict__ W, int ld, int N, int Ne, int ncols, LuShared<R>& sm,
                          int* __restrict__ piv_out, int half = PXD_HALF_NONE) {
  using T = typename Cx<R>::T;
  static_assert(KB % NB == 0 && KB <= KBMAX, "block column width");
  static_assert(sizeof(sm.buf) >= sizeof(T) * KB * CS, "LDS slab must fit the panel buffer");
  T* Us = sm.buf;  // idle during the wide update
  for (int K = 0; K < Ne; K += KB) {
    const int kbb = min(KB, Ne - K), Kend = K + kbb;
    for (int k = K; k < Kend; k += NB) {
      const int kb = min(NB, Kend - k);
      factor_panel<R, Q, SB>(W, ld, N, k, kb, sm);
      for (int i = threadIdx.x; i < kb; i += kThreads) {
        sm.bpiv[k - K + i] = sm.piv[i];
        if (piv_out) piv_out[k + i] = sm.piv[i];
      }
      apply_swaps<T>(W, ld, k, kb, sm.piv, K, k);        // block columns left of the panel
      swap_trsm<R>(W, ld, k, kb, k + kb, Kend, sm, sm.piv);  // and right of it, inside the block
      trailing_update<R>(W, ld, k, kb, N, k + kb, Kend);
      __syncthreads();
    }
    if (Kend < ncols) {
      apply_swaps<T>(W, ld, K, kbb, sm.bpiv, Kend, ncols);
      for (int k = K; k < Kend; k += NB) {  // U rows of the block: L11^-1 A12, 32 rows at a time
        const int kb = min(NB, Kend - k);
        trsm_inverse<R>(W, ld, k, kb, Kend, ncols, sm);
        trailing_update<R>(W, ld, k, kb, Kend, Kend, ncols);
        __syncthreads();
      }
      if constexpr (sizeof(R) == 4) {
        if (half == PXD_HALF_BF16)
          wide_update_half<KB, RT, PXD_HALF_BF16>(W, ld, K, kbb, Kend, N, Kend, ncols, Us);
        else if (half == PXD_HALF_F16)
          wide_update_half<KB, RT, PXD_HALF_F16>(W, ld, K, kbb, Kend, N, Kend, ncols, Us);
        else
          wide_update<R, KB, RT>(W, ld, K, kbb, Kend, N, Kend, ncols, Us);
      } else {
        wide_update<R, KB, RT>(W, ld, K, kbb, Kend, N, Kend, ncols, Us);
      }
    }
  }
}

// P x P system of the port unknowns left after eliminating the first N - P
// columns of [Z_A | V]; thread 0 solves it with partial pivoting and writes
// S = I - 2 Z0 diag(l) X (Eqs. 6-7).
__device__ __forceinline__ int port_solve_and_s(const double2* __restrict__ W, int ld, int N, int P,
                                const double* __restrict__ plen, double z0, double2* __restrict__ S) {
  __shared__ double2 A[4][8];
  const int tid = threadIdx.x;
  if (tid < P * 2 * P) {
    const int i = tid / (2 * P), j = tid - i * 2 * P;
    A[i][j] = W[(size_t)(N - P + i) * ld + (N - P + j)];
  }
  __syncthreads();
  int st = PXD_STATUS_OK;
  if (tid == 0) {
    for (int c = 0; c < P; ++c) {
      int p = c;
      double best = fabs(A[c][c].x) + fabs(A[c][c].y);
      for (int r = c + 1; r < P; ++r) {
        const double v = fabs(A[r][c].x) + fabs(A[r][c].y);
        if (v > best) best = v, p = r;
      }
      if (!(best > 0.0)) st = PXD_STATUS_SINGULAR;
      if (p != c)
        for (int j = 0; j < 2 * P; ++j) {
          const double2 t = A[c][j];
          A[c][j] = A[p][j];
          A[p][j] = t;
        }
      const double2 inv = crecip(A[c][c]);
      for (int r = c + 1; r < P; ++r) {
        const double2 l = cmul(A[r][c], inv);
        for (int j = c; j < 2 * P; ++j) A[r][j] = cfms(A[r][j], l, A[c][j]);
      }
    }
    for (int j = 0; j < P; ++j)
      for (int i = P - 1; i >= 0; --i) {
        double2 acc = A[i][P + j];
        for (int t = i + 1; t < P; ++t) acc = cfms(acc, A[i][t], A[t][P + j]);
        A[i][P + j] = cmul(acc, crecip(A[i][i]));
      }
    bool finite = true;
    for (int i = 0; i < P; ++i)
      for (int j = 0; j < P; ++j) {
        const double2 x = A[i][P + j];
        double2 s = double2{(i == j ? 1.0 : 0.0) - 2.0 * z0 * plen[i] * x.x, -2.0 * z0 * plen[i] * x.y};
        finite = finite && isfinite(s.x) && isfinite(s.y);
        S[i * P + j] = s;
      }
    if (!finite) st = PXD_STATUS_NONFINITE;
  }
  __syncthreads();
  return st;
}

// ------------------------------------------------------------------ mixed precision

// b[r] -= sum over j < kb of W[r][k + j] y[j] for the rows r_lo <= r < r_hi,
// all waves of the workgroup: eight lanes per row, each lane four
// consecutive entries (contiguous 16-byte loads across the row), eight row
// groups per wave in flight (a lone workgroup is bound by load latency), the
// eight partial sums reduced over the row's lanes and added to b once.
// y (kb x P) and b may be in LDS.
__device__ __forceinline__ void rows_update_block(const float2* __restrict__ W, int ld, int k, int kb, int r_lo,
                                                  int r_hi, const float2* y, float2* b, int P) {
  constexpr int RG = 8;  // row groups per wave per step
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int sub = lane >> 3, l8 = lane & 7, j0 = 4 * l8;
  const bool vec = ((ld & 1) == 0) && j0 + 3 < kb;  // 16-byte aligned and inside the block
  float2 yv[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int jr = 0; jr < 4; ++jr) yv[u][jr] = (jr < P && j0 + u < kb) ? y[(j0 + u) * P + jr] : float2{0, 0};
  for (int r0 = r_lo + 8 * RG * wid; r0 < r_hi; r0 += 8 * RG * kWaves) {
    float2 w[RG][4];
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      const int r = r0 + 8 * g + sub;
      const float2* row = W + (size_t)r * ld + k + j0;
      if (r < r_hi && vec) {
        const float4 a = reinterpret_cast<const float4*>(row)[0], c = reinterpret_cast<const float4*>(row)[1];
        w[g][0] = float2{a.x, a.y}, w[g][1] = float2{a.z, a.w}, w[g][2] = float2{c.x, c.y}, w[g][3] = float2{c.z, c.w};
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) w[g][u] = (r < r_hi && j0 + u < kb) ? row[u] : float2{0, 0};
      }
    }
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      const int r = r0 + 8 * g + sub;
      float2 acc[4] = {};  // the products are summed apart from b (one rounding into it)
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int jr = 0; jr < 4; ++jr)
          if (jr < P) acc[jr] = cfms(acc[jr], w[g][u], yv[u][jr]);
#pragma unroll
      for (int jr = 0; jr < 4; ++jr) {
        if (jr >= P) continue;
#pragma unroll
        for (int off = 4; off >= 1; off >>= 1) {
          acc[jr].x += __shfl_xor(acc[jr].x, off, 64);
          acc[jr].y += __shfl_xor(acc[jr].y, off, 64);
        }
        if (l8 == 0 && r < r_hi) b[(size_t)r * P + jr] = float2{b[(size_t)r * P + jr].x + acc[jr].x,
                                                                 b[(size_t)r * P + jr].y + acc[jr].y};
      }
    }
  }
}

constexpr int kTlKbMaxSolve = 128;  // widest block column whose interchanges lu_solve_c64 replays

__device__ __forceinline__ void lu_solve_c64(const float2* __restrict__ W, int ld, int N, const int* __restrict__ piv,
                                             float2* b, int P, int kblock = KB_MIXED) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  __shared__ int s_piv[kTlKbMaxSolve];  // the block column's pivots, read in parallel before the serial swaps
  // forward: b <- L^-1 P b; a block column's interchanges all precede its
  // eliminations (its L is stored in the block's final row order)
  for (int k = 0; k < N; k += NB) {
    const int kb = min(NB, N - k);
    if (k % kblock == 0) {
      const int nk = min(kblock, N - k);
      for (int i = tid; i < nk; i += kThreads) s_piv[i] = piv[k + i];
      __syncthreads();
      if (tid < P)
        for (int i = 0; i < nk; ++i) {
          const int r = k + i, q = s_piv[i];
          if (q != r) {
            const float2 t = b[r * P + tid];
            b[r * P + tid] = b[q * P + tid];
            b[q * P + tid] = t;
          }
        }
    }
    __syncthreads();
    if (wid == 0) {
      float2 l[NB];
      const bool mine = lane < kb;
#pragma unroll
      for (int j = 0; j < NB; ++j) l[j] = (mine && j < lane) ? W[(size_t)(k + lane) * ld + k + j] : float2{0, 0};
      for (int jr = 0; jr < P; ++jr) {
        float2 v = mine ? b[(k + lane) * P + jr] : float2{0, 0};
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          const float2 bj = float2{__shfl(v.x, j, 64), __shfl(v.y, j, 64)};
          if (j < lane) v = cfms(v, l[j], bj);
        }
        if (mine) b[(k + lane) * P + jr] = v;
      }
    }
    __syncthreads();
    rows_update_block(W, ld, k, kb, k + kb, N, b + (size_t)k * P, b, P);
    __syncthreads();
  }
  // backward: b <- U^-1 b
  const int nblk = (N + NB - 1) / NB;
  for (int bi = nblk - 1; bi >= 0; --bi) {
    const int k = bi * NB, kb = min(NB, N - k);
    if (wid == 0) {
      float2 u[NB];
      const bool mine = lane < kb;
#pragma unroll
      for (int j = 0; j < NB; ++j) u[j] = (mine && j >= lane && j < kb) ? W[(size_t)(k + lane) * ld + k + j] : float2{0, 0};
      float2 diag = float2{1, 0};
#pragma unroll
      for (int j = 0; j < NB; ++j)
        if (j == lane) diag = u[j];
      const float2 rdiag = crecip(diag);
      for (int jr = 0; jr < P; ++jr) {
        float2 v = mine ? b[(k + lane) * P + jr] : float2{0, 0};
#pragma unroll
        for (int j = NB - 1; j >= 0; --j) {
          if (j < kb) {
            // row j is final once the columns right of it are eliminated
            float2 xj = cmul(v, rdiag);
            xj = float2{__shfl(xj.x, j, 64), __shfl(xj.y, j, 64)};
            if (lane == j) v = xj;
            else if (lane < j) v = cfms(v, u[j], xj);
          }
        }
        if (mine) b[(k + lane) * P + jr] = v;
      }
    }
    __syncthreads();
    rows_update_block(W, ld, k, kb, 0, k, b + (size_t)k * P, b, P);
    __syncthreads();
  }
}

// r = V - Z_A x in FP64, Z_A gathered on the fly from the complex128 parent
// (with the Z0 loads of the port functions); the result, rounded to
// complex64, replaces b.  Sixteen lanes per row (four rows per wave), each
// lane keeping eight independent gathers in flight.
__device__ __forceinline__ void residual_fp64(const double2* __restrict__ Zf, int M, const int* sI, int N, int P,
                                              const double* __restrict__ plen, double z0,
                                              const double2* __restrict__ x, float2* b) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int sub = lane >> 4, l16 = lane & 15;
  for (int i0 = 4 * wid; i0 < N; i0 += 4 * kWaves) {
    const int i = i0 + sub;
    double2 acc[4] = {};
    if (i < N) {
      const double2* zrow = Zf + (size_t)sI[i] * M;
      int j = l16;
      for (; j + 112 < N; j += 128) {  // eight gathers in flight per lane
        double2 z[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) z[u] = zrow[sI[j + 16 * u]];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int jr = 0; jr < 4; ++jr)
            if (jr < P) {
              const double2 xv = x[(size_t)(j + 16 * u) * P + jr];
              acc[jr].x += z[u].x * xv.x - z[u].y * xv.y;
              acc[jr].y += z[u].x * xv.y + z[u].y * xv.x;
            }
      }
      for (; j < N; j += 16) {
        const double2 zv = zrow[sI[j]];
#pragma unroll
        for (int jr = 0; jr < 4; ++jr)
          if (jr < P) {
            const double2 xv = x[(size_t)j * P + jr];
            acc[jr].x += zv.x * xv.x - zv.y * xv.y;
            acc[jr].y += zv.x * xv.y + zv.y * xv.x;
          }
      }
    }
#pragma unroll
    for (int jr = 0; jr < 4; ++jr) {
#pragma unroll
      for (int off = 8; off >= 1; off >>= 1) {
        acc[jr].x += __shfl_xor(acc[jr].x, off, 16);
        acc[jr].y += __shfl_xor(acc[jr].y, off, 16);
      }
    }
    if (i < N && l16 < P) {
      const int jr = l16;
      double2 a = acc[0];
#pragma unroll
      for (int t = 1; t < 4; ++t)
        if (t == jr) a = acc[t];
      const int pi = i - (N - P);  // port index of this row, if it is a port row
      double2 r = double2{-a.x, -a.y};
      if (pi >= 0) {
        const double2 xv = x[(size_t)i * P + jr];
        const double load = z0 * plen[pi] * plen[pi];
        r.x -= load * xv.x;
        r.y -= load * xv.y;
        if (pi == jr) r.x += plen[pi];  // V: 1 V source EMF in the gap of port jr
      }
      b[i * P + jr] = float2{(float)r.x, (float)r.y};
    }
  }
  __syncthreads();
}

// Port-current corrections from a residual without a solve.  Z_A is
// symmetric, so row p_i of Z_A^-1 is x_i^T / l_i (x_i the solution for port
// i's excitation l_i e_{p_i}); the correction of x[p_i][j] is therefore
// x_i^T r_j / l_i, exact up to a term second order in the solution error
// (dual-weighted residual).  x is the current solution (FP64), r = b the
// residual rounded to complex64.  delta[i P + j] receives the corrections.
__device__ __forceinline__ void port_corrections(const double2* __restrict__ x, const float2* b, int N, int P,
                                                 const double* __restrict__ plen, double2* delta, double2* part) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  double2 acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = double2{0.0, 0.0};
  for (int n = tid; n < N; n += kThreads) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (i < P) {
        const double2 xi = x[(size_t)n * P + i];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (j < P) {
            const float2 rj = b[n * P + j];
            acc[i * 4 + j].x += xi.x * rj.x - xi.y * rj.y;
            acc[i * 4 + j].y += xi.x * rj.y + xi.y * rj.x;
          }
      }
  }
#pragma unroll
  for (int q = 0; q < 16; ++q)
    if ((q >> 2) < P && (q & 3) < P) {
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        acc[q].x += __shfl_xor(acc[q].x, off, 64);
        acc[q].y += __shfl_xor(acc[q].y, off, 64);
      }
    }
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < 16; ++q) part[wid * 16 + q] = acc[q];
  __syncthreads();
  if (tid < P * P) {
    const int i = tid / P, j = tid - i * P;
    double2 sum = double2{0.0, 0.0};
    for (int w = 0; w < kWaves; ++w) {
      sum.x += part[w * 16 + i * 4 + j].x;
      sum.y += part[w * 16 + i * 4 + j].y;
    }
    delta[tid] = double2{sum.x / plen[i], sum.y / plen[i]};
  }
  __syncthreads();
}

// Absolute floor of the refinement target on S, above what FP64 residuals of
// these systems resolve (~kappa x 1e-16 with kappa up to ~1e5).
constexpr double kIrAbsFloor = 1e-11;


// Mixed-precision item after its complex64 factorisation (W, pivots of a
// factorisation in block columns of kblock): x0 = (LU)^-1 V in complex64,
// then refinement with FP64 residuals.  After each step the error left in
// every S_ij = delta_ij - 2 Z0 l_i x_ij is bounded by rho / (1 - rho) times
// the largest change the step made to any S entry, rho being the observed
// contraction (refine_verdict).  Each step first forms the FP64 residual and
// the port corrections it implies (no solve); when the stop test passes on
// those, they are applied and the step ends there, otherwise the full
// correction is solved.  A converged item writes S (Eqs. 6-7) and its status;
// one that does not is appended to fb_list (as `item`) for the FP64 path.
// b: N x P complex64 in LDS; sI: the item's active list in LDS; x: N x P
// complex128 in the slot.  All threads of the workgroup call it.
__device__ __forceinline__ void refine_item(const float2* __restrict__ W, int ld, int N, const int* __restrict__ piv,
                                         int kblock, float2* b, const int* sI, double2* __restrict__ x,
                                         const double2* __restrict__ Zf128, int M, int P,
                                         const double* __restrict__ plen, double z0, int ir_max, double ir_tol,
                                         int bad, int item, double2* __restrict__ Sout, int* __restrict__ status_out,
                                         int* ir_iters, int* fb_count, int* fb_list) {
  __shared__ int s_conv;
  __shared__ double s_ds[16], s_sabs[16], s_mprev;
  __shared__ double2 s_delta[16], s_part[kWaves * 16];
  const int tid = threadIdx.x;
  // x0 = (LU)^-1 V
  for (int e = tid; e < N * P; e += kThreads) {
    const int i = e / P, jr = e - i * P;
    b[e] = float2{(i == N - P + jr) ? (float)plen[jr] : 0.0f, 0.0f};
  }
  __syncthreads();
  lu_solve_c64(W, ld, N, piv, b, P, kblock);
  for (int e = tid; e < N * P; e += kThreads) x[e] = double2{(double)b[e].x, (double)b[e].y};
  __syncthreads();
  int iters = 0;
  bool conv = false;
  if (tid == 0) s_mprev = 0.0;
  while (iters < ir_max) {
    residual_fp64(Zf128, M, sI, N, P, plen, z0, x, b);
    ++iters;
    // what this step would change at the ports, without solving
    port_corrections(x, b, N, P, plen, s_delta, s_part);
    if (tid == 0) {
      double m = 0.0;
      for (int q = 0; q < P * P; ++q) {
        const int i = q / P, j = q - i * P;
        const double g = 2.0 * z0 * plen[i];
        const double ds = g * sqrt(s_delta[q].x * s_delta[q].x + s_delta[q].y * s_delta[q].y);
        m = (ds > m || ds != ds) ? ds : m;
        const double2 xv = x[(size_t)(N - P + i) * P + j];
        const double sr = (i == j ? 1.0 : 0.0) - g * (xv.x + s_delta[q].x), si = -g * (xv.y + s_delta[q].y);
        s_sabs[q] = sqrt(sr * sr + si * si);
      }
      // the contraction acts on the whole error, so what is left in any
      // entry is bounded by rho times the largest change, not its own change
      double target = 1e300;
      for (int q = 0; q < P * P; ++q) target = fmin(target, ir_tol * s_sabs[q] + kIrAbsFloor);
      const int verdict = refine_verdict(iters, ir_max, m, s_mprev, target);
      s_conv = verdict;
    }
    __syncthreads();
    conv = s_conv == 1;
    if (s_conv == 2) break;
    if (conv) {  // converged: the port corrections finish the step
      if (tid < P * P) {
        double2* xv = x + (size_t)(N - P + tid / P) * P + tid % P;
        xv->x += s_delta[tid].x;
        xv->y += s_delta[tid].y;
      }
      __syncthreads();
      break;
    }
    lu_solve_c64(W, ld, N, piv, b, P, kblock);
    for (int e = tid; e < N * P; e += kThreads) {
      const double2 d = double2{(double)b[e].x, (double)b[e].y};
      double2 xv = x[e];
      xv.x += d.x;
      xv.y += d.y;
      x[e] = xv;
      if (e >= (N - P) * P) {  // port rows: the change of S_ij (Eq. 6) this step made
        const int pi = e / P - (N - P), jr = e - (e / P) * P;
        s_ds[pi * P + jr] = 2.0 * z0 * plen[pi] * sqrt(d.x * d.x + d.y * d.y);
      }
    }
    __syncthreads();
    if (tid == 0) {
      double m = 0.0;
      for (int q = 0; q < P * P; ++q) m = (s_ds[q] > m || s_ds[q] != s_ds[q]) ? s_ds[q] : m;
      s_mprev = m;
    }
    __syncthreads();
  }
  if (tid == 0) {
    atomicAdd(ir_iters, iters);
    int st = PXD_STATUS_OK;
    if (!conv) {
      st = PXD_STATUS_FALLBACK;
      const int slotn = atomicAdd(fb_count, 1);
      fb_list[slotn] = item;
    } else {
      bool finite = true;
      for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j) {
          const double2 xv = x[(size_t)(N - P + i) * P + j];
          const double2 sv = double2{(i == j ? 1.0 : 0.0) - 2.0 * z0 * plen[i] * xv.x,
                                     -2.0 * z0 * plen[i] * xv.y};
          finite = finite && isfinite(sv.x) && isfinite(sv.y);
          Sout[i * P + j] = sv;
        }
      if (!finite) st = PXD_STATUS_NONFINITE;
      else if (bad) st = PXD_STATUS_SINGULAR;
    }
    *status_out = st;
  }
  __syncthreads();
}

}  // namespace pxd
