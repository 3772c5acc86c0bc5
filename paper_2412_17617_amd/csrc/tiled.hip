// Tiled LU for large active sizes: the items of a chunk are factored in lock
// step, one launch per step of each block column, with many workgroups per
// item (Eq. 2's dense solve when one item's matrix is far larger than what
// one compute unit can hold or stream efficiently).
//
// Per item the layout is that of the persistent evaluator: the matrix
// row-major in its slot, ports ordered last, right-looking LU with partial
// pivoting in block columns of kb (64 or 128), factored in 32-wide panels.
// Per block column [K, K + kb):
//   k_tl_panel   one workgroup per item: factor the block column over rows
//                [K, N) (register sub-panels, interchanges applied across the
//                block column), store the pivots, the inverse of its
//                unit-lower diagonal block L11 and, for the columns to its
//                right, which rows the block's interchanges touch and where
//                each one's new content comes from;
//   k_tl_trsm    per (item, 64- or 32-column tile): apply those interchanges
//                to the tile and form U12 = L11^-1 A12 on MFMA;
//   k_tl_update  per (item, output tile): A22 -= L21 U12, a complex GEMM of
//                four real MFMA products on LDS-staged planar tiles.
// Columns left of a block column are not permuted by later blocks (solves
// replay the interchanges block by block), as in the persistent kernels.
// Then per item: the port block and S (FP64 augmented system) or the
// complex64 solve with FP64 refinement (mixed modes).
#include <algorithm>

#include "device.hpp"
#include "kernels.hpp"
#include "lu_device.hpp"

namespace pxd {

namespace {

struct TlItem {
  int c, f, N, Ne, ncols;
};

__device__ __forceinline__ TlItem tl_item(const TlParams& p, int b) {
  const int it = p.items[b];
  TlItem r;
  r.c = it / p.F;
  r.f = it - r.c * p.F;
  r.N = p.Nc[r.c];
  r.Ne = p.mixed ? r.N : r.N - p.P;
  r.ncols = p.mixed ? r.N : r.N + p.P;
  return r;
}

__device__ __forceinline__ int* tl_aux(const TlParams& p, int b) {
  return reinterpret_cast<int*>(p.ws + (size_t)b * p.slot_bytes + p.lay.aux_off);
}
// aux: [0] zero-pivot flag, [1] touched-row count, tr[2 kTlKbMax], src[2 kTlKbMax],
// then the lock-step refinement's state: still refining, steps taken, and (as
// a double) the largest change of the last step
constexpr int kAuxTr = 4;
constexpr int kAuxSrc = 4 + 2 * kTlKbMax;
constexpr int kAuxIr = 4 + 4 * kTlKbMax;

// ------------------------------------------------------------------ gather

// Z_A = Z_f[I, I] (Eq. 5) with the Z0 loads of the port functions added on
// the diagonal; FP64 path: the excitation columns V (1 V in each port gap)
// appended.  16 rows per workgroup, 4 per wave.
template <typename T, typename TP>
__global__ __launch_bounds__(256) void k_tl_gather(TlParams p, const TP* __restrict__ Zpar) {
  using R = decltype(T::x);
  const int b = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const TlItem t = tl_item(p, b);
  const int r0 = blockIdx.x * 16;
  if (blockIdx.x == 0 && tid == 0) {
    int* aux = tl_aux(p, b);
    aux[0] = 0;
    aux[1] = 0;
  }
  if (r0 >= t.N) return;
  T* W = reinterpret_cast<T*>(p.ws + (size_t)b * p.slot_bytes);
  const int* I = p.Ilist + (size_t)t.c * p.M;
  const TP* Zf = Zpar + (size_t)t.f * p.M * p.M;
  const int P = p.P;
  for (int rr = wid; rr < 16; rr += kWaves) {
    const int r = r0 + rr;
    if (r >= t.N) break;
    const TP* zrow = Zf + (size_t)I[r] * p.M;
    T* wrow = W + (size_t)r * p.lay.ld;
    const int pi = r - (t.N - P);  // port index of this row, if it is a port row
    const double load = (pi >= 0) ? p.z0 * p.port_len[pi] * p.port_len[pi] : 0.0;
    for (int s = lane; s < t.N; s += 64) {
      const TP v = zrow[I[s]];
      const double re = (double)v.x + ((s == r) ? load : 0.0);
      wrow[s] = T{(R)re, (R)v.y};
    }
    if (!p.mixed && lane < P) wrow[t.N + lane] = T{(pi == lane) ? (R)p.port_len[lane] : (R)0, (R)0};
  }
}

// ------------------------------------------------------------------ panel

template <typename R, int Q, int SB>
__global__ __launch_bounds__(256) void k_tl_panel(TlParams p, int K) {
  using T = typename Cx<R>::T;
  __shared__ LuShared<R> sm;
  __shared__ T sY[NB * NB];
  const int b = blockIdx.x, tid = threadIdx.x;
  const TlItem t = tl_item(p, b);
  if (K >= t.Ne) return;
  const int kbb = min(p.kb, t.Ne - K), Kend = K + kbb;
  const int ld = p.lay.ld;
  char* slot = p.ws + (size_t)b * p.slot_bytes;
  T* W = reinterpret_cast<T*>(slot);
  int* piv = reinterpret_cast<int*>(slot + p.lay.piv_off);
  int* aux = reinterpret_cast<int*>(slot + p.lay.aux_off);
  T* Li = reinterpret_cast<T*>(slot + p.lay.li_off);
  if (tid == 0) sm.bad = aux[0];
  __syncthreads();
  for (int k = K; k < Kend; k += NB) {
    const int kb = min(NB, Kend - k);
    factor_panel<R, Q, SB>(W, ld, t.N, k, kb, sm);
    for (int i = tid; i < kb; i += kThreads) {
      sm.bpiv[k - K + i] = sm.piv[i];
      piv[k + i] = sm.piv[i];
    }
    apply_swaps<T>(W, ld, k, kb, sm.piv, K, k);          // block columns left of the panel
    swap_trsm<R>(W, ld, k, kb, k + kb, Kend, sm, sm.piv);  // and right of it, inside the block
    trailing_update<R>(W, ld, k, kb, t.N, k + kb, Kend);
    __syncthreads();
  }
  // rows the block's interchanges touch and the source of each one's final
  // content: the interchanges applied in order to an identity map
  if (tid == 0) {
    aux[0] = sm.bad;
    int* tr = aux + kAuxTr;
    int* src = aux + kAuxSrc;
    int n = kbb;
    for (int i = 0; i < kbb; ++i) tr[i] = src[i] = K + i;
    for (int i = 0; i < kbb; ++i) {
      const int q = sm.bpiv[i];
      if (q == K + i) continue;
      int jq = q - K;
      if (q >= Kend) {
        jq = -1;
        for (int j = kbb; j < n; ++j)
          if (tr[j] == q) {
            jq = j;
            break;
          }
        if (jq < 0) {
          tr[n] = src[n] = q;
          jq = n++;
        }
      }
      const int s0 = src[i];
      src[i] = src[jq];
      src[jq] = s0;
    }
    aux[1] = n;
  }
  // Li = L11^-1 (unit lower, kbb x kbb) by 32 x 32 blocks: the diagonal
  // blocks' inverses by substitution, then block row bi, column bj < bi:
  //   Li[bi][bj] = -Li[bi][bi] sum_{bj <= tb < bi} L[bi][tb] Li[tb][bj]
  const int nbk = (kbb + NB - 1) / NB;
  T* Lb = sm.buf;            // diagonal block of L (strictly lower part)
  T* Db = sm.buf + NB * NB;  // its inverse
  for (int bi = 0; bi < nbk; ++bi) {
    const int r0 = K + bi * NB, kbi = min(NB, kbb - bi * NB);
    for (int e = tid; e < NB * NB; e += kThreads) {
      const int i = e / NB, j = e - i * NB;
      Lb[e] = (i < kbi && j < i) ? W[(size_t)(r0 + i) * ld + r0 + j] : T{0, 0};
      Db[e] = (i == j && i < kbi) ? T{1, 0} : T{0, 0};
    }
    __syncthreads();
    for (int i = 1; i < kbi; ++i) {  // Db[i][j] = -sum_{j <= u < i} Lb[i][u] Db[u][j]
      if (tid < i) {
        const int j = tid;
        T acc{0, 0};
        for (int u = j; u < i; ++u) acc = cfms(acc, Lb[i * NB + u], Db[u * NB + j]);
        Db[i * NB + j] = acc;
      }
      __syncthreads();
    }
    for (int e = tid; e < NB * NB; e += kThreads) {
      const int i = e / NB, j = e - i * NB;
      Li[(size_t)(bi * NB + i) * kTlKbMax + bi * NB + j] = Db[e];
      for (int bj = bi + 1; bj < nbk; ++bj) Li[(size_t)(bi * NB + i) * kTlKbMax + bj * NB + j] = T{0, 0};
    }
    __syncthreads();
    for (int bj = 0; bj < bi; ++bj) {
      // Y = sum over the block columns tb in [bj, bi) of L[bi][tb] Li[tb][bj]
      for (int e = tid; e < NB * NB; e += kThreads) {
        const int i = e / NB, j = e - i * NB;
        T acc{0, 0};
        if (i < kbi)
          for (int u = bj * NB; u < bi * NB; ++u)
            acc = cfms(acc, W[(size_t)(r0 + i) * ld + K + u], Li[(size_t)u * kTlKbMax + bj * NB + j]);
        sY[e] = acc;  // holds -Y
      }
      __syncthreads();
      for (int e = tid; e < NB * NB; e += kThreads) {
        const int i = e / NB, j = e - i * NB;
        T acc{0, 0};
        for (int u = 0; u <= i; ++u) acc = cfms(acc, Db[i * NB + u], sY[u * NB + j]);
        Li[(size_t)(bi * NB + i) * kTlKbMax + bj * NB + j] = T{-acc.x, -acc.y};  // = Db (-Y)
      }
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------------ interchanges + U12

// One workgroup per (item, CT-column tile of [Kend, ncols)).  The block's
// interchanges reach the tile as a gather from the source rows (all old
// values are read before any is written), then U12 = L11^-1 (P A12) on MFMA:
// the right-hand block in LDS, L11^-1 fragments from the slot (cache).
template <typename R, int CT>
__global__ __launch_bounds__(256) void k_tl_trsm(TlParams p, int K) {
  using T = typename Cx<R>::T;
  using MF = Mfma<R>;
  using acc_t = typename MF::acc_t;
  constexpr int SBS = CT + 16;  // LDS row stride (conflict-free B fragments)
  constexpr int NSUB = CT / 16;
  constexpr int MAXD = kTlKbMax * CT / kThreads;  // displaced (row, column) pairs per thread
  __shared__ R Br[kTlKbMax * SBS], Bi[kTlKbMax * SBS];
  const int b = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  const TlItem t = tl_item(p, b);
  if (K >= t.Ne) return;
  const int kbb = min(p.kb, t.Ne - K), Kend = K + kbb;
  const int c0 = Kend + blockIdx.x * CT;
  if (c0 >= t.ncols) return;
  const int c1 = min(c0 + CT, t.ncols);
  const int ld = p.lay.ld;
  char* slot = p.ws + (size_t)b * p.slot_bytes;
  T* W = reinterpret_cast<T*>(slot);
  const int* aux = reinterpret_cast<const int*>(slot + p.lay.aux_off);
  const int* tr = aux + kAuxTr;
  const int* src = aux + kAuxSrc;
  const T* Li = reinterpret_cast<const T*>(slot + p.lay.li_off);
  const int ntouch = aux[1];
  const int kpad = (kbb + 3) & ~3;
  for (int e = tid; e < kpad * CT; e += kThreads) {
    const int kr = e / CT, cc = e - kr * CT;
    const T v = (kr < kbb && c0 + cc < c1) ? W[(size_t)src[kr] * ld + c0 + cc] : T{0, 0};
    Br[kr * SBS + cc] = v.x;
    Bi[kr * SBS + cc] = v.y;
  }
  T dv[MAXD];
#pragma unroll
  for (int i = 0; i < MAXD; ++i) {
    const int e = tid + kThreads * i;
    const int j = kbb + e / CT, cc = e % CT;
    dv[i] = (j < ntouch && c0 + cc < c1) ? W[(size_t)src[j] * ld + c0 + cc] : T{0, 0};
  }
  __syncthreads();  // every old value has been read
#pragma unroll
  for (int i = 0; i < MAXD; ++i) {
    const int e = tid + kThreads * i;
    const int j = kbb + e / CT, cc = e % CT;
    if (j < ntouch && c0 + cc < c1) W[(size_t)tr[j] * ld + c0 + cc] = dv[i];
  }
  const int nrs = (kbb + 15) >> 4;
  for (int rs = wid; rs < nrs; rs += kWaves) {
    acc_t cr[NSUB], ci[NSUB];
#pragma unroll
    for (int sn = 0; sn < NSUB; ++sn) {
      cr[sn] = acc_t{0, 0, 0, 0};
      ci[sn] = acc_t{0, 0, 0, 0};
    }
    const int row = 16 * rs + l16;
    for (int kq0 = 0; kq0 < kpad / 4; kq0 += 8) {
      // eight k-steps of L11^-1 fragments in flight together
      T a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int kk = 4 * (kq0 + u) + lk;
        a[u] = (row < kbb && kk < kbb) ? Li[(size_t)row * kTlKbMax + kk] : T{0, 0};
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int kk = 4 * (kq0 + u) + lk;
        if (kq0 + u >= kpad / 4) break;
#pragma unroll
        for (int sn = 0; sn < NSUB; ++sn) {
          const R br = Br[kk * SBS + 16 * sn + l16], bi = Bi[kk * SBS + 16 * sn + l16];
          cr[sn] = MF::run(a[u].x, br, cr[sn]);
          ci[sn] = MF::run(a[u].x, bi, ci[sn]);
          cr[sn] = MF::run(-a[u].y, bi, cr[sn]);
          ci[sn] = MF::run(a[u].y, br, ci[sn]);
        }
      }
    }
#pragma unroll
    for (int sn = 0; sn < NSUB; ++sn)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 16 * rs + MF::row(lane, i), col = c0 + 16 * sn + l16;
        if (r < kbb && col < c1) W[(size_t)(K + r) * ld + col] = T{cr[sn][i], ci[sn][i]};
      }
  }
}

// ------------------------------------------------------------------ trailing update

// A22 -= L21 U12 for one TM x TN output tile of one item, rows [Kend, N),
// columns [Kend, ncols).  WGM x WGN waves, each owning a (TM/WGM) x (TN/WGN)
// block of 16 x 16 MFMA tiles (real and imaginary accumulators).  L21 and U12 are staged in LDS as planar real/imaginary
// tiles, KC columns of L21 (rows as stored, row stride KC + pad) and KC rows
// of U12 (row stride TN + 16) at a time; the strides make the fragment reads
// of a wave hit distinct banks.  The next stage's tiles are fetched into
// registers while the current stage's MFMAs run, and the four real products
// of the complex update are issued product by product over all of the
// wave's tiles, so no MFMA waits on the one before it.  The block id is
// remapped so that the tiles of one item run on one XCD (workgroups are
// dealt to the XCDs in turn).
template <typename R, int TM, int TN, int KC, int OCC, int WGM = 2, int WGN = 2>
__global__ __launch_bounds__(64 * WGM * WGN, OCC) void k_tl_update(TlParams p, int K, int tiles_m, int tiles_n, int cb,
                                                                   int ce) {
  using T = typename Cx<R>::T;
  using MF = Mfma<R>;
  using acc_t = typename MF::acc_t;
  constexpr int NT = 64 * WGM * WGN;
  constexpr int WM = TM / WGM, WN = TN / WGN, SM = WM / 16, SN = WN / 16;
  constexpr int SA = (sizeof(R) == 4) ? KC + 4 : KC + 2;  // A row stride: 4 x odd (f32), 2 x odd (f64)
  constexpr int SBS = TN + 16;
  constexpr int NA = TM * KC / NT, NBV = KC * TN / NT;  // stage elements per thread
  static_assert(TM * KC % NT == 0 && KC * TN % NT == 0 && WM % 16 == 0 && WN % 16 == 0, "stage split");
  __shared__ R Ar[TM * SA], Ai[TM * SA], Br[KC * SBS], Bi[KC * SBS];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  // XCD-grouped block order
  const int total = gridDim.x * gridDim.y;
  const int lid = blockIdx.x + blockIdx.y * gridDim.x;
  const int gid = (lid & 7) * (total >> 3) + (lid >> 3);
  const int b = gid / gridDim.x, tile = gid - b * gridDim.x;
  if (b >= p.B || tile >= tiles_m * tiles_n) return;
  const TlItem t = tl_item(p, b);
  if (K >= t.Ne) return;
  const int kbb = min(p.kb, t.Ne - K), Kend = K + kbb;
  const int tm = tile % tiles_m, tn = tile / tiles_m;
  const int cend = min(t.ncols, Kend + ce);  // this launch's columns: [Kend + cb, Kend + ce)
  const int r0 = Kend + tm * TM, c0 = Kend + cb + tn * TN;
  if (r0 >= t.N || c0 >= cend) return;
  const int ld = p.lay.ld;
  T* W = reinterpret_cast<T*>(p.ws + (size_t)b * p.slot_bytes);
  T ra[NA], rb[NBV];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = tid + NT * i, row = e / KC, kk = e - row * KC;
      const int r = r0 + row, k = k0 + kk;
      ra[i] = (r < t.N && k < Kend) ? W[(size_t)r * ld + k] : T{0, 0};
    }
#pragma unroll
    for (int i = 0; i < NBV; ++i) {
      const int e = tid + NT * i, kr = e / TN, col = e - kr * TN;
      const int k = k0 + kr, cc = c0 + col;
      rb[i] = (k < Kend && cc < cend) ? W[(size_t)k * ld + cc] : T{0, 0};
    }
  };
  fetch(K);
  const int wm = wid % WGM, wn = wid / WGM;
  const int rw = r0 + wm * WM, cw = c0 + wn * WN;
  // complex64: C is read with the first stage's operands, so its latency is
  // not paid after the products (complex128 has no registers to spare for it)
  constexpr bool kEarlyC = sizeof(R) == 4;
  T cv[SM][SN][4];
  if constexpr (kEarlyC) {
#pragma unroll
    for (int a = 0; a < SM; ++a)
#pragma unroll
      for (int s = 0; s < SN; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = rw + 16 * a + MF::row(lane, i), col = cw + 16 * s + l16;
          cv[a][s][i] = (r < t.N && col < cend) ? W[(size_t)r * ld + col] : T{0, 0};
        }
  }
  acc_t cr[SM][SN], ci[SM][SN];
#pragma unroll
  for (int a = 0; a < SM; ++a)
#pragma unroll
    for (int s = 0; s < SN; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        cr[a][s][i] = 0;  // the products are summed apart from C (one rounding into C)
        ci[a][s][i] = 0;
      }
  for (int k0 = K; k0 < Kend; k0 += KC) {
    __syncthreads();  // the previous stage is consumed
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = tid + NT * i, row = e / KC, kk = e - row * KC;
      Ar[row * SA + kk] = ra[i].x;
      Ai[row * SA + kk] = ra[i].y;
    }
#pragma unroll
    for (int i = 0; i < NBV; ++i) {
      const int e = tid + NT * i, kr = e / TN, col = e - kr * TN;
      Br[kr * SBS + col] = rb[i].x;
      Bi[kr * SBS + col] = rb[i].y;
    }
    __syncthreads();
    if (k0 + KC < Kend) fetch(k0 + KC);  // in flight during this stage's products
#pragma unroll
    for (int kq = 0; kq < KC / 4; ++kq) {
      R nar[SM], ai[SM], nai[SM], br[SN], bi[SN];
#pragma unroll
      for (int a = 0; a < SM; ++a) {
        const int row = wm * WM + 16 * a + l16;
        nar[a] = -Ar[row * SA + 4 * kq + lk];
        ai[a] = Ai[row * SA + 4 * kq + lk];
        nai[a] = -ai[a];
      }
#pragma unroll
      for (int s = 0; s < SN; ++s) {
        const int col = wn * WN + 16 * s + l16;
        br[s] = Br[(4 * kq + lk) * SBS + col];
        bi[s] = Bi[(4 * kq + lk) * SBS + col];
      }
      // C -= A B:  Cr += (-Ar) Br + Ai Bi,  Ci += (-Ar) Bi + (-Ai) Br,
      // one real product at a time over every tile of the wave
#pragma unroll
      for (int a = 0; a < SM; ++a)
#pragma unroll
        for (int s = 0; s < SN; ++s) cr[a][s] = MF::run(nar[a], br[s], cr[a][s]);
#pragma unroll
      for (int a = 0; a < SM; ++a)
#pragma unroll
        for (int s = 0; s < SN; ++s) ci[a][s] = MF::run(nar[a], bi[s], ci[a][s]);
#pragma unroll
      for (int a = 0; a < SM; ++a)
#pragma unroll
        for (int s = 0; s < SN; ++s) cr[a][s] = MF::run(ai[a], bi[s], cr[a][s]);
#pragma unroll
      for (int a = 0; a < SM; ++a)
#pragma unroll
        for (int s = 0; s < SN; ++s) ci[a][s] = MF::run(nai[a], br[s], ci[a][s]);
    }
  }
#pragma unroll
  for (int a = 0; a < SM; ++a)
#pragma unroll
    for (int s = 0; s < SN; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = rw + 16 * a + MF::row(lane, i), col = cw + 16 * s + l16;
        if (r < t.N && col < cend) {
          const T v = kEarlyC ? cv[a][s][i] : W[(size_t)r * ld + col];
          W[(size_t)r * ld + col] = T{v.x + cr[a][s][i], v.y + ci[a][s][i]};
        }
      }
}

// Split-BF16 form of the complex64 trailing update (PXD_PREC_MIXED_BF16):
// every operand x = hi + lo with hi = bf16(x) and lo = bf16(x - hi), each
// real product X Y as Xh Yh + Xh Yl + Xl Yh on the 16x16x32 BF16 MFMA with
// FP32 accumulation (the dropped Xl Yl is ~2^-16 relative).  BF16 keeps
// FP32's exponent range, so no scaling is needed.  A stage is one 32-deep
// k-chunk: L21 and U12 are split once when staged (two k at a time, one
// v_cvt_pk_bf16_f32 per pair and plane), into hi/lo planes of the real and
// imaginary parts, L21 as [row][k] and U12 transposed as [col][k], so that
// every fragment is eight consecutive k of one row or column: one 16-byte
// LDS read, the 80-byte row stride putting sixteen lanes' reads on distinct
// banks.  The next stage's operands are read from memory during this stage's
// products.
template <int TM, int TN, int OCC>
__global__ __launch_bounds__(256, OCC) void k_tl_update_bf16x3(TlParams p, int K, int tiles_m, int tiles_n, int cb,
                                                               int ce) {
  using T = float2;
  using MF = Mfma<float>;
  typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
  typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
  constexpr int KC = 32, SW = 20;  // k per stage; LDS row stride in 32-bit words (two BF16 each)
  constexpr int WM = TM / 2, WN = TN / 2, SM = WM / 16, SN = WN / 16;
  constexpr int NA = TM * KC / 2 / kThreads, NBV = KC * TN / 2 / kThreads;  // k pairs staged per thread
  static_assert(TM * KC / 2 % kThreads == 0 && KC * TN / 2 % kThreads == 0, "stage split");
  // planes: 0 re hi, 1 re lo, 2 im hi, 3 im lo (of -L21 and of U12); word w of a row holds k = 2 w, 2 w + 1
  __shared__ __align__(16) unsigned As[4][TM * SW], Bs[4][TN * SW];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  const int total = gridDim.x * gridDim.y;
  const int lid = blockIdx.x + blockIdx.y * gridDim.x;
  const int gid = (lid & 7) * (total >> 3) + (lid >> 3);
  const int b = gid / gridDim.x, tile = gid - b * gridDim.x;
  if (b >= p.B || tile >= tiles_m * tiles_n) return;
  const TlItem t = tl_item(p, b);
  if (K >= t.Ne) return;
  const int kbb = min(p.kb, t.Ne - K), Kend = K + kbb;
  const int tm = tile % tiles_m, tn = tile / tiles_m;
  const int cend = min(t.ncols, Kend + ce);
  const int r0 = Kend + tm * TM, c0 = Kend + cb + tn * TN;
  if (r0 >= t.N || c0 >= cend) return;
  const int ld = p.lay.ld;
  T* W = reinterpret_cast<T*>(p.ws + (size_t)b * p.slot_bytes);
  T ra[NA][2], rb[NBV][2];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = tid + kThreads * i, row = e / (KC / 2), kp = e - row * (KC / 2);
      const int r = r0 + row, k = k0 + 2 * kp;
      const bool in = r < t.N;
      ra[i][0] = (in && k < Kend) ? W[(size_t)r * ld + k] : T{0, 0};
      ra[i][1] = (in && k + 1 < Kend) ? W[(size_t)r * ld + k + 1] : T{0, 0};
    }
#pragma unroll
    for (int i = 0; i < NBV; ++i) {
      const int e = tid + kThreads * i, kp = e / TN, col = e - kp * TN;
      const int k = k0 + 2 * kp, cc = c0 + col;
      const bool in = cc < cend;
      rb[i][0] = (in && k < Kend) ? W[(size_t)k * ld + cc] : T{0, 0};
      rb[i][1] = (in && k + 1 < Kend) ? W[(size_t)(k + 1) * ld + cc] : T{0, 0};
    }
  };
  // (x0, x1) -> hi and lo words, round to nearest even
  auto split2 = [](float x0, float x1, unsigned& hi, unsigned& lo) {
    const bf2 h = {(__bf16)x0, (__bf16)x1};
    hi = __builtin_bit_cast(unsigned, h);
    const float r0 = x0 - __uint_as_float(hi << 16), r1 = x1 - __uint_as_float(hi & 0xffff0000u);
    const bf2 l = {(__bf16)r0, (__bf16)r1};
    lo = __builtin_bit_cast(unsigned, l);
  };
  fetch(K);
  const int wm = wid & 1, wn = wid >> 1;
  const int rw = r0 + wm * WM, cw = c0 + wn * WN;
  // C is read with the first stage's operands, so its latency is not paid after the products
  T cv[SM][SN][4];
#pragma unroll
  for (int a = 0; a < SM; ++a)
#pragma unroll
    for (int s = 0; s < SN; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = rw + 16 * a + MF::row(lane, i), col = cw + 16 * s + l16;
        cv[a][s][i] = (r < t.N && col < cend) ? W[(size_t)r * ld + col] : T{0, 0};
      }
  fx4 cr[SM][SN], ci[SM][SN];
#pragma unroll
  for (int a = 0; a < SM; ++a)
#pragma unroll
    for (int s = 0; s < SN; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        cr[a][s][i] = 0;  // the products are summed apart from C (one rounding into C)
        ci[a][s][i] = 0;
      }
  for (int k0 = K; k0 < Kend; k0 += KC) {
    __syncthreads();  // the previous stage is consumed
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = tid + kThreads * i, row = e / (KC / 2), kp = e - row * (KC / 2);
      split2(-ra[i][0].x, -ra[i][1].x, As[0][row * SW + kp], As[1][row * SW + kp]);  // -A (exact)
      split2(-ra[i][0].y, -ra[i][1].y, As[2][row * SW + kp], As[3][row * SW + kp]);
    }
#pragma unroll
    for (int i = 0; i < NBV; ++i) {
      const int e = tid + kThreads * i, kp = e / TN, col = e - kp * TN;
      split2(rb[i][0].x, rb[i][1].x, Bs[0][col * SW + kp], Bs[1][col * SW + kp]);
      split2(rb[i][0].y, rb[i][1].y, Bs[2][col * SW + kp], Bs[3][col * SW + kp]);
    }
    __syncthreads();
    if (k0 + KC < Kend) fetch(k0 + KC);  // in flight during this stage's products
    // lane (lk, l16): row (column) l16 of its sub-tile, k = 8 lk .. + 7
    uint4 fa[4][SM], fb[4][SN];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int a = 0; a < SM; ++a)
        fa[q][a] = *reinterpret_cast<const uint4*>(&As[q][(wm * WM + 16 * a + l16) * SW + 4 * lk]);
#pragma unroll
      for (int s = 0; s < SN; ++s)
        fb[q][s] = *reinterpret_cast<const uint4*>(&Bs[q][(wn * WN + 16 * s + l16) * SW + 4 * lk]);
    }
    uint4 nbh[SN], nbl[SN];  // -Bi (sign bits flipped)
#pragma unroll
    for (int s = 0; s < SN; ++s) {
      nbh[s] = make_uint4(fb[2][s].x ^ 0x80008000u, fb[2][s].y ^ 0x80008000u, fb[2][s].z ^ 0x80008000u,
                          fb[2][s].w ^ 0x80008000u);
      nbl[s] = make_uint4(fb[3][s].x ^ 0x80008000u, fb[3][s].y ^ 0x80008000u, fb[3][s].z ^ 0x80008000u,
                          fb[3][s].w ^ 0x80008000u);
    }
    auto mma = [](uint4 x, uint4 y, fx4 c) {
      return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, x), __builtin_bit_cast(bf8, y), c, 0, 0,
                                                     0);
    };
    // with -A staged: Cr += (-Ar) Br + (-Ai)(-Bi),  Ci += (-Ar) Bi + (-Ai) Br,
    // each product in three parts, issued part by part over all of the wave's tiles
#define PXD_SPLIT3(ACC, XH, XL, YH, YL)                                                    \
  _Pragma("unroll") for (int a = 0; a < SM; ++a) _Pragma("unroll") for (int s = 0; s < SN; ++s) \
      ACC[a][s] = mma(XH[a], YH[s], ACC[a][s]);                                          \
  _Pragma("unroll") for (int a = 0; a < SM; ++a) _Pragma("unroll") for (int s = 0; s < SN; ++s) \
      ACC[a][s] = mma(XH[a], YL[s], ACC[a][s]);                                          \
  _Pragma("unroll") for (int a = 0; a < SM; ++a) _Pragma("unroll") for (int s = 0; s < SN; ++s) \
      ACC[a][s] = mma(XL[a], YH[s], ACC[a][s]);
    PXD_SPLIT3(cr, fa[0], fa[1], fb[0], fb[1])
    PXD_SPLIT3(ci, fa[0], fa[1], fb[2], fb[3])
    PXD_SPLIT3(cr, fa[2], fa[3], nbh, nbl)
    PXD_SPLIT3(ci, fa[2], fa[3], fb[0], fb[1])
#undef PXD_SPLIT3
  }
#pragma unroll
  for (int a = 0; a < SM; ++a)
#pragma unroll
    for (int s = 0; s < SN; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = rw + 16 * a + MF::row(lane, i), col = cw + 16 * s + l16;
        if (r < t.N && col < cend)
          W[(size_t)r * ld + col] = T{cv[a][s][i].x + cr[a][s][i], cv[a][s][i].y + ci[a][s][i]};
      }
}

// ------------------------------------------------------------------ per-item finish

// FP64 augmented system: the P x P port block left after eliminating the
// first N - P columns, then S (Eqs. 6-7).
__global__ __launch_bounds__(256) void k_tl_finish_plain(TlParams p) {
  const int b = blockIdx.x, tid = threadIdx.x;
  const TlItem t = tl_item(p, b);
  const double2* W = reinterpret_cast<const double2*>(p.ws + (size_t)b * p.slot_bytes);
  const int* aux = tl_aux(p, b);
  double2* Sout = p.S + ((size_t)t.c * p.F + t.f) * p.P * p.P;
  int st = port_solve_and_s(W, p.lay.ld, t.N, p.P, p.port_len, p.z0, Sout);
  if (tid == 0) {
    if (aux[0] && st == PXD_STATUS_OK) st = PXD_STATUS_SINGULAR;
    if (p.fallback_mode && st == PXD_STATUS_OK) st = PXD_STATUS_FALLBACK;
    p.status[(size_t)t.c * p.F + t.f] = st;
  }
}

// Mixed modes: complex64 solve and FP64 refinement of the factored item.
__global__ __launch_bounds__(256) void k_tl_finish_mixed(TlParams p, int nmax) {
  extern __shared__ char dyn[];
  int* sI = reinterpret_cast<int*>(dyn);
  float2* bvec = reinterpret_cast<float2*>(dyn + ((size_t)nmax * 4 + 15) / 16 * 16);
  const int b = blockIdx.x, tid = threadIdx.x;
  const TlItem t = tl_item(p, b);
  char* slot = p.ws + (size_t)b * p.slot_bytes;
  const float2* W = reinterpret_cast<const float2*>(slot);
  const int* piv = reinterpret_cast<const int*>(slot + p.lay.piv_off);
  const int* aux = reinterpret_cast<const int*>(slot + p.lay.aux_off);
  double2* x = reinterpret_cast<double2*>(slot + p.lay.x_off);
  for (int s = tid; s < t.N; s += kThreads) sI[s] = p.Ilist[(size_t)t.c * p.M + s];
  const int bad = aux[0];
  __syncthreads();
  const size_t item = (size_t)t.c * p.F + t.f;
  refine_item(W, p.lay.ld, t.N, piv, p.kb, bvec, sI, x, p.Z128 + (size_t)t.f * p.M * p.M, p.M, p.P, p.port_len,
              p.z0, p.ir_max, p.ir_tol, bad, (int)item, p.S + item * p.P * p.P, p.status + item, p.ir_iters,
              p.fb_count, p.fb_list);
}

// ------------------------------------------------------------------ lock-step refinement
//
// The mixed modes' refinement of a chunk, all items a step at a time.  The
// FP64 residual r = V - (Z_A + loads) x of every item of one frequency comes
// from one product R = Z_f[U, U] X over the union U of the batch's active
// sets: the parent rows are read once per group and step instead of once
// per item and step.  The stop test, the complex64 solve and the update are
// those of the per-item form (refine_verdict, lu_solve_c64).

__device__ __forceinline__ double* ir_mprev(int* aux) { return reinterpret_cast<double*>(aux + kAuxIr + 2); }

// x0 = (LU)^-1 V for one item, into its slot and into its group's X block.
__global__ __launch_bounds__(256) void k_ir_init(TlParams p, IrParams q, int nmax) {
  extern __shared__ char dyn[];
  float2* bvec = reinterpret_cast<float2*>(dyn);  // ir_lds(nmax, P): the right-hand sides only
  const int b = blockIdx.x, tid = threadIdx.x;
  const TlItem t = tl_item(p, b);
  char* slot = p.ws + (size_t)b * p.slot_bytes;
  const float2* W = reinterpret_cast<const float2*>(slot);
  const int* piv = reinterpret_cast<const int*>(slot + p.lay.piv_off);
  int* aux = reinterpret_cast<int*>(slot + p.lay.aux_off);
  double2* x = reinterpret_cast<double2*>(slot + p.lay.x_off);
  const int N = t.N, P = p.P;
  for (int e = tid; e < N * P; e += kThreads) {
    const int i = e / P, jr = e - i * P;
    bvec[e] = float2{(i == N - P + jr) ? (float)p.port_len[jr] : 0.0f, 0.0f};
  }
  __syncthreads();
  lu_solve_c64(W, p.lay.ld, N, piv, bvec, P, p.kb);
  const int g = q.item_grp[b], col = q.item_col[b];
  double2* X = q.X + (size_t)g * q.U * q.ldx;
  const int* I = p.Ilist + (size_t)t.c * p.M;
  for (int e = tid; e < N * P; e += kThreads) {
    const int i = e / P, jr = e - i * P;
    const double2 v = double2{(double)bvec[e].x, (double)bvec[e].y};
    x[e] = v;
    X[(size_t)q.upos[I[i]] * q.ldx + col + jr] = v;
  }
  if (tid == 0) {
    aux[kAuxIr] = 1;
    aux[kAuxIr + 1] = 0;
    *ir_mprev(aux) = 0.0;
    atomicAdd(q.grp_active + g, 1);
  }
}

// R = Z_f[U, U] X for one 64 x 64 tile of one group.  Four waves, each 16 rows
// by 64 columns (four 16 x 16 FP64 MFMA tiles, real and imaginary
// accumulators); Z rows and columns are gathered from the parent through U,
// eight k per LDS stage.
constexpr int kIrTM = 64, kIrTN = 64, kIrKC = 8;
__global__ __launch_bounds__(256) void k_ir_residual(TlParams p, IrParams q) {
  using MF = Mfma<double>;
  using acc_t = typename MF::acc_t;
  constexpr int TM = kIrTM, TN = kIrTN, KC = kIrKC, SA = KC + 1, SBS = TN + 2;
  constexpr int NA = TM * KC / kThreads, NBV = KC * TN / kThreads;
  static_assert(TM * KC % kThreads == 0 && KC * TN % kThreads == 0 && TM == 16 * kWaves, "tile split");
  __shared__ double Ar[TM * SA], Ai[TM * SA], Br[KC * SBS], Bi[KC * SBS];
  const int g = blockIdx.z;
  if (q.grp_active[g] == 0) return;
  const int ncol = q.grp_ncol[g];
  const int r0 = blockIdx.x * TM, c0 = blockIdx.y * TN;
  if (r0 >= q.U || c0 >= ncol) return;
  const double2* Zf = p.Z128 + (size_t)q.grp_f[g] * p.M * p.M;
  const double2* X = q.X + (size_t)g * q.U * q.ldx;
  double2* R = q.R + (size_t)g * q.U * q.ldx;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  acc_t cr[4], ci[4];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int i = 0; i < 4; ++i) cr[s][i] = ci[s][i] = 0.0;
  for (int k0 = 0; k0 < q.U; k0 += KC) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = tid + kThreads * i, row = e / KC, kk = e - row * KC;
      const int r = r0 + row, k = k0 + kk;
      const double2 v = (r < q.U && k < q.U) ? Zf[(size_t)q.ulist[r] * p.M + q.ulist[k]] : double2{0.0, 0.0};
      Ar[row * SA + kk] = v.x;
      Ai[row * SA + kk] = v.y;
    }
#pragma unroll
    for (int i = 0; i < NBV; ++i) {
      const int e = tid + kThreads * i, kr = e / TN, col = e - kr * TN;
      const int k = k0 + kr, c = c0 + col;
      const double2 v = (k < q.U && c < ncol) ? X[(size_t)k * q.ldx + c] : double2{0.0, 0.0};
      Br[kr * SBS + col] = v.x;
      Bi[kr * SBS + col] = v.y;
    }
    __syncthreads();
#pragma unroll
    for (int kq = 0; kq < KC / 4; ++kq) {
      const int row = wid * 16 + l16;
      const double ar = Ar[row * SA + 4 * kq + lk], ai = Ai[row * SA + 4 * kq + lk], nai = -ai;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double br = Br[(4 * kq + lk) * SBS + 16 * s + l16], bi = Bi[(4 * kq + lk) * SBS + 16 * s + l16];
        cr[s] = MF::run(ar, br, cr[s]);
        ci[s] = MF::run(ar, bi, ci[s]);
        cr[s] = MF::run(nai, bi, cr[s]);
        ci[s] = MF::run(ai, br, ci[s]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + wid * 16 + MF::row(lane, i), c = c0 + 16 * s + l16;
      if (r < q.U && c < ncol) R[(size_t)r * q.ldx + c] = double2{cr[s][i], ci[s][i]};
    }
}

// One refinement step of one item still refining: its residual from R, the
// port corrections and the stop test; converged: S and the status; given up
// (or the step budget spent): handed to the FP64 path; else the complex64
// solve of the correction, x += d, and x back into X.
__global__ __launch_bounds__(256) void k_ir_step(TlParams p, IrParams q, int nmax) {
  extern __shared__ char dyn[];
  float2* bvec = reinterpret_cast<float2*>(dyn);  // ir_lds(nmax, P): the right-hand sides only
  __shared__ int s_v;
  __shared__ double s_ds[16], s_sabs[16];
  __shared__ double2 s_delta[16], s_part[kWaves * 16];
  const int b = blockIdx.x, tid = threadIdx.x;
  char* slot = p.ws + (size_t)b * p.slot_bytes;
  int* aux = reinterpret_cast<int*>(slot + p.lay.aux_off);
  if (aux[kAuxIr] == 0) return;  // the same word for every thread
  const TlItem t = tl_item(p, b);
  const float2* W = reinterpret_cast<const float2*>(slot);
  const int* piv = reinterpret_cast<const int*>(slot + p.lay.piv_off);
  double2* x = reinterpret_cast<double2*>(slot + p.lay.x_off);
  const int N = t.N, P = p.P;
  const int g = q.item_grp[b], col = q.item_col[b];
  const double2* R = q.R + (size_t)g * q.U * q.ldx;
  double2* X = q.X + (size_t)g * q.U * q.ldx;
  const int* I = p.Ilist + (size_t)t.c * p.M;  // row i of the item is row upos[I[i]] of U
  for (int e = tid; e < N * P; e += kThreads) {
    const int i = e / P, jr = e - i * P;
    const double2 zx = R[(size_t)q.upos[I[i]] * q.ldx + col + jr];
    double2 r = double2{-zx.x, -zx.y};
    const int pi = i - (N - P);  // port index of this row, if it is a port row
    if (pi >= 0) {
      const double load = p.z0 * p.port_len[pi] * p.port_len[pi];
      const double2 xv = x[e];
      r.x -= load * xv.x;
      r.y -= load * xv.y;
      if (pi == jr) r.x += p.port_len[pi];  // V: 1 V source EMF in the gap of port jr
    }
    bvec[e] = float2{(float)r.x, (float)r.y};
  }
  __syncthreads();
  const int iters = aux[kAuxIr + 1] + 1;
  port_corrections(x, bvec, N, P, p.port_len, s_delta, s_part);
  if (tid == 0) {
    double m = 0.0;
    for (int qq = 0; qq < P * P; ++qq) {
      const int i = qq / P, j = qq - i * P;
      const double gg = 2.0 * p.z0 * p.port_len[i];
      const double ds = gg * sqrt(s_delta[qq].x * s_delta[qq].x + s_delta[qq].y * s_delta[qq].y);
      m = (ds > m || ds != ds) ? ds : m;
      const double2 xv = x[(size_t)(N - P + i) * P + j];
      const double sr = (i == j ? 1.0 : 0.0) - gg * (xv.x + s_delta[qq].x), si = -gg * (xv.y + s_delta[qq].y);
      s_sabs[qq] = sqrt(sr * sr + si * si);
    }
    double target = 1e300;
    for (int qq = 0; qq < P * P; ++qq) target = fmin(target, p.ir_tol * s_sabs[qq] + kIrAbsFloor);
    int v = refine_verdict(iters, p.ir_max, m, *ir_mprev(aux), target);
    if (v == 0 && iters >= p.ir_max) v = 2;  // no step left
    s_v = v;
  }
  __syncthreads();
  const int v = s_v;
  const size_t item = (size_t)t.c * p.F + t.f;
  if (v == 1) {  // converged: the port corrections finish the step
    if (tid < P * P) {
      double2* xv = x + (size_t)(N - P + tid / P) * P + tid % P;
      xv->x += s_delta[tid].x;
      xv->y += s_delta[tid].y;
    }
    __syncthreads();
    if (tid == 0) {
      bool finite = true;
      double2* Sout = p.S + item * P * P;
      for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j) {
          const double2 xv = x[(size_t)(N - P + i) * P + j];
          const double2 sv = double2{(i == j ? 1.0 : 0.0) - 2.0 * p.z0 * p.port_len[i] * xv.x,
                                     -2.0 * p.z0 * p.port_len[i] * xv.y};
          finite = finite && isfinite(sv.x) && isfinite(sv.y);
          Sout[i * P + j] = sv;
        }
      int st = PXD_STATUS_OK;
      if (!finite) st = PXD_STATUS_NONFINITE;
      else if (aux[0]) st = PXD_STATUS_SINGULAR;
      p.status[item] = st;
      aux[kAuxIr] = 0;
      atomicSub(q.grp_active + g, 1);
      atomicAdd(p.ir_iters, iters);
    }
    return;
  }
  if (v == 2) {  // the FP64 path takes the item
    if (tid == 0) {
      p.status[item] = PXD_STATUS_FALLBACK;
      p.fb_list[atomicAdd(p.fb_count, 1)] = (int)item;
      aux[kAuxIr] = 0;
      atomicSub(q.grp_active + g, 1);
      atomicAdd(p.ir_iters, iters);
    }
    return;
  }
  lu_solve_c64(W, p.lay.ld, N, piv, bvec, P, p.kb);
  for (int e = tid; e < N * P; e += kThreads) {
    const int i = e / P, jr = e - i * P;
    const double2 d = double2{(double)bvec[e].x, (double)bvec[e].y};
    double2 xv = x[e];
    xv.x += d.x;
    xv.y += d.y;
    x[e] = xv;
    X[(size_t)q.upos[I[i]] * q.ldx + col + jr] = xv;
    if (i >= N - P) s_ds[(i - (N - P)) * P + jr] = 2.0 * p.z0 * p.port_len[i - (N - P)] * sqrt(d.x * d.x + d.y * d.y);
  }
  __syncthreads();
  if (tid == 0) {
    double m = 0.0;
    for (int qq = 0; qq < P * P; ++qq) m = (s_ds[qq] > m || s_ds[qq] != s_ds[qq]) ? s_ds[qq] : m;
    *ir_mprev(aux) = m;
    aux[kAuxIr + 1] = iters;
  }
}

// Union of the batch's active sets: marks, then one workgroup's prefix sum.
__global__ void k_union_mark(const int* __restrict__ Nc, const int* __restrict__ Ilist, int M, int* mark) {
  const int c = blockIdx.x;
  const int* I = Ilist + (size_t)c * M;
  for (int i = threadIdx.x; i < Nc[c]; i += blockDim.x) mark[I[i]] = 1;
}

__global__ __launch_bounds__(1024) void k_union_scan(const int* __restrict__ mark, int M, int* upos, int* ulist,
                                                     int* count) {
  __shared__ int part[1024];
  const int tid = threadIdx.x, per = (M + 1023) / 1024;
  const int lo = min(M, tid * per), hi = min(M, lo + per);
  int n = 0;
  for (int m = lo; m < hi; ++m) n += mark[m] ? 1 : 0;
  part[tid] = n;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan
    const int v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int pos = part[tid] - n;
  for (int m = lo; m < hi; ++m) {
    if (mark[m]) {
      upos[m] = pos;
      ulist[pos++] = m;
    } else {
      upos[m] = -1;
    }
  }
  if (tid == 1023) count[0] = part[1023];
}

__global__ void k_zero_c128(double2* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = double2{0.0, 0.0};
}

template <typename R, int Q>
constexpr int tl_sb() {
  // register sub-panel width: Q x SB entries per thread; measured on the 24x24x3,
  // 20x20x2 and 32x32x3 stacks, wider sub-panels pay for FP64 at every Q
  // and for complex64 from 12 rows per thread on (fewer passes over the panel
  // outweigh the lower occupancy there)
  constexpr int w = sizeof(R) == 8 ? 32 / Q : (Q >= 12 ? 64 / Q : 32 / Q);
  return w < 1 ? 1 : (w > 16 && sizeof(R) == 8 ? 16 : (w > 32 ? 32 : w));
}

template <typename R>
hipError_t panel_variant(hipStream_t s, const TlParams& p, int K, int q) {
  const dim3 g(p.B), blk(kThreads);
  if (q <= 1) hipLaunchKernelGGL((k_tl_panel<R, 1, tl_sb<R, 1>()>), g, blk, 0, s, p, K);
  else if (q <= 2) hipLaunchKernelGGL((k_tl_panel<R, 2, tl_sb<R, 2>()>), g, blk, 0, s, p, K);
  else if (q <= 4) hipLaunchKernelGGL((k_tl_panel<R, 4, tl_sb<R, 4>()>), g, blk, 0, s, p, K);
  else if (q <= 8) hipLaunchKernelGGL((k_tl_panel<R, 8, tl_sb<R, 8>()>), g, blk, 0, s, p, K);
  else if (q <= 12) hipLaunchKernelGGL((k_tl_panel<R, 12, tl_sb<R, 12>()>), g, blk, 0, s, p, K);
  else if (q <= 16) hipLaunchKernelGGL((k_tl_panel<R, 16, tl_sb<R, 16>()>), g, blk, 0, s, p, K);
  else if (q <= 24) hipLaunchKernelGGL((k_tl_panel<R, 24, 1>), g, blk, 0, s, p, K);
  else if (q <= 32) hipLaunchKernelGGL((k_tl_panel<R, 32, 1>), g, blk, 0, s, p, K);
  else if (q <= 40) hipLaunchKernelGGL((k_tl_panel<R, 40, 1>), g, blk, 0, s, p, K);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

constexpr int kTrsmCols64 = 64, kTrsmCols128 = 32;

// Output-tile shapes of the trailing update (TlParams.shape): 0 = 128 x 64 at
// two workgroups per CU, 1 = 64 x 64 at three (more waves to hide latency,
// more L21/U12 re-reads).
template <typename R>
struct UpdShape;
template <>
struct UpdShape<float> {
  template <int S>
  static void launch(hipStream_t s, dim3 g, const TlParams& p, int K, int tm, int tn, int cb, int ce) {
    if (S == 0) hipLaunchKernelGGL((k_tl_update<float, 128, 64, 16, 2>), g, dim3(kThreads), 0, s, p, K, tm, tn, cb, ce);
    else if (S == 1) hipLaunchKernelGGL((k_tl_update<float, 64, 64, 16, 3>), g, dim3(kThreads), 0, s, p, K, tm, tn, cb, ce);
    else if (S == 2)
      hipLaunchKernelGGL((k_tl_update<float, 128, 64, 16, 2, 4, 2>), g, dim3(512), 0, s, p, K, tm, tn, cb, ce);
    else hipLaunchKernelGGL((k_tl_update<float, 128, 128, 16, 1, 4, 2>), g, dim3(512), 0, s, p, K, tm, tn, cb, ce);
  }
};
template <>
struct UpdShape<double> {
  template <int S>
  static void launch(hipStream_t s, dim3 g, const TlParams& p, int K, int tm, int tn, int cb, int ce) {
    if (S == 0) hipLaunchKernelGGL((k_tl_update<double, 128, 64, 8, 2>), g, dim3(kThreads), 0, s, p, K, tm, tn, cb, ce);
    else if (S == 1) hipLaunchKernelGGL((k_tl_update<double, 64, 64, 8, 3>), g, dim3(kThreads), 0, s, p, K, tm, tn, cb, ce);
    else if (S == 2)
      hipLaunchKernelGGL((k_tl_update<double, 128, 64, 8, 2, 4, 2>), g, dim3(512), 0, s, p, K, tm, tn, cb, ce);
    else hipLaunchKernelGGL((k_tl_update<double, 128, 128, 8, 1, 4, 2>), g, dim3(512), 0, s, p, K, tm, tn, cb, ce);
  }
};
}  // namespace

int tl_max_active() { return 256 * 40; }

int tl_max_active_mixed(int P) {
  // the complex64 solves keep the item's active list and its right-hand sides
  // in LDS (eval_mixed_lds), next to the refinement's static LDS
  int n = tl_max_active();
  while (n > 0 && eval_mixed_lds(n, P) + 4096 > 160 * 1024) n -= 64;
  return n;
}

hipError_t tl_gather(hipStream_t s, const TlParams& p, int nmax) {
  const dim3 g((nmax + 15) / 16, p.B), blk(kThreads);
  if (!p.mixed) hipLaunchKernelGGL((k_tl_gather<double2, double2>), g, blk, 0, s, p, p.Z128);
  else if (p.Z64) hipLaunchKernelGGL((k_tl_gather<float2, float2>), g, blk, 0, s, p, p.Z64);
  else hipLaunchKernelGGL((k_tl_gather<float2, double2>), g, blk, 0, s, p, p.Z128);
  return hipGetLastError();
}

hipError_t tl_panel(hipStream_t s, const TlParams& p, int K, int nmax) {
  const int q = (nmax - K + 255) / 256;
  return p.mixed ? panel_variant<float>(s, p, K, q) : panel_variant<double>(s, p, K, q);
}

hipError_t tl_trsm(hipStream_t s, const TlParams& p, int K, int nmax) {
  const int ncols = p.mixed ? nmax : nmax + p.P;
  if (ncols <= K) return hipSuccess;
  if (p.mixed) {
    const dim3 g((ncols - K + kTrsmCols64 - 1) / kTrsmCols64, p.B), blk(kThreads);
    hipLaunchKernelGGL((k_tl_trsm<float, kTrsmCols64>), g, blk, 0, s, p, K);
  } else {
    const dim3 g((ncols - K + kTrsmCols128 - 1) / kTrsmCols128, p.B), blk(kThreads);
    hipLaunchKernelGGL((k_tl_trsm<double, kTrsmCols128>), g, blk, 0, s, p, K);
  }
  return hipGetLastError();
}

hipError_t tl_update(hipStream_t s, const TlParams& p, int K, int nmax, int cb, int ce) {
  const int ncols = p.mixed ? nmax : nmax + p.P;
  const int mr = nmax - K;                      // bounds of every item's trailing block
  const int nc = std::min(ncols - K, ce) - cb;  // and of this launch's column range
  if (mr <= 0 || nc <= 0) return hipSuccess;
  const bool split = p.mixed && p.half == PXD_HALF_BF16;  // split-BF16 kernels: 128 x 64 or 64 x 64 only
  const int shape = (split && p.shape > 1) ? 0 : p.shape;
  const int TM = shape == 1 ? 64 : 128, TN = shape == 3 ? 128 : 64;
  const int tiles_m = (mr + TM - 1) / TM, tiles_n = (nc + TN - 1) / TN;
  const int gx = (tiles_m * tiles_n + 7) / 8 * 8;  // a multiple of 8: the XCD grouping needs it
  const dim3 g(gx, p.B);
  if (split) {
    if (shape == 1)
      hipLaunchKernelGGL((k_tl_update_bf16x3<64, 64, 2>), g, dim3(kThreads), 0, s, p, K, tiles_m, tiles_n, cb, ce);
    else
      hipLaunchKernelGGL((k_tl_update_bf16x3<128, 64, 1>), g, dim3(kThreads), 0, s, p, K, tiles_m, tiles_n, cb, ce);
  } else if (p.mixed) {
    if (shape == 1) UpdShape<float>::launch<1>(s, g, p, K, tiles_m, tiles_n, cb, ce);
    else if (shape == 2) UpdShape<float>::launch<2>(s, g, p, K, tiles_m, tiles_n, cb, ce);
    else if (shape == 3) UpdShape<float>::launch<3>(s, g, p, K, tiles_m, tiles_n, cb, ce);
    else UpdShape<float>::launch<0>(s, g, p, K, tiles_m, tiles_n, cb, ce);
  } else {
    if (shape == 1) UpdShape<double>::launch<1>(s, g, p, K, tiles_m, tiles_n, cb, ce);
    else if (shape == 2) UpdShape<double>::launch<2>(s, g, p, K, tiles_m, tiles_n, cb, ce);
    else if (shape == 3) UpdShape<double>::launch<3>(s, g, p, K, tiles_m, tiles_n, cb, ce);
    else UpdShape<double>::launch<0>(s, g, p, K, tiles_m, tiles_n, cb, ce);
  }
  return hipGetLastError();
}

hipError_t tl_prepare(const TlParams& p, int nmax) {
  if (!p.mixed) return hipSuccess;
  const int lds = (int)eval_mixed_lds(nmax, p.P);
  for (const void* k : {reinterpret_cast<const void*>(&k_tl_finish_mixed), reinterpret_cast<const void*>(&k_ir_init),
                        reinterpret_cast<const void*>(&k_ir_step)}) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// LDS of the lock-step refinement kernels: the right-hand sides (nmax x P
// complex64), small enough at the 32x32x3 sizes for two workgroups per CU
static size_t ir_lds(int nmax, int P) { return (size_t)nmax * P * sizeof(float2); }

hipError_t tl_ir_init(hipStream_t s, const TlParams& p, const IrParams& q, int nmax) {
  hipLaunchKernelGGL(k_ir_init, dim3(p.B), dim3(kThreads), ir_lds(nmax, p.P), s, p, q, nmax);
  return hipGetLastError();
}

hipError_t tl_ir_residual(hipStream_t s, const TlParams& p, const IrParams& q, int max_ncol) {
  if (q.U <= 0 || max_ncol <= 0 || q.n_grp <= 0) return hipSuccess;
  const dim3 g((q.U + kIrTM - 1) / kIrTM, (max_ncol + kIrTN - 1) / kIrTN, q.n_grp);
  hipLaunchKernelGGL(k_ir_residual, g, dim3(kThreads), 0, s, p, q);
  return hipGetLastError();
}

hipError_t tl_ir_step(hipStream_t s, const TlParams& p, const IrParams& q, int nmax) {
  hipLaunchKernelGGL(k_ir_step, dim3(p.B), dim3(kThreads), ir_lds(nmax, p.P), s, p, q, nmax);
  return hipGetLastError();
}

hipError_t launch_union(hipStream_t s, const int* Nc, const int* Ilist, int C, int M, int* mark, int* upos,
                        int* ulist, int* count) {
  hipError_t e = launch_fill_int(s, mark, M, 0);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_union_mark, dim3(C), dim3(256), 0, s, Nc, Ilist, M, mark);
  hipLaunchKernelGGL(k_union_scan, dim3(1), dim3(1024), 0, s, mark, M, upos, ulist, count);
  return hipGetLastError();
}

hipError_t launch_zero_c128(hipStream_t s, double2* p, size_t n) {
  if (n == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_zero_c128, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t tl_finish(hipStream_t s, const TlParams& p, int nmax) {
  if (p.mixed)
    hipLaunchKernelGGL(k_tl_finish_mixed, dim3(p.B), dim3(kThreads), eval_mixed_lds(nmax, p.P), s, p, nmax);
  else
    hipLaunchKernelGGL(k_tl_finish_plain, dim3(p.B), dim3(kThreads), 0, s, p);
  return hipGetLastError();
}

}  // namespace pxd
