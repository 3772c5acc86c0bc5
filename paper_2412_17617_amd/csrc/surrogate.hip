// CNN surrogate of the evaluation: forward, backward, AdamW and ranking on
// gfx950.  Every product (convolutions as implicit GEMMs, the dense head and
// all their gradients) runs through one tiled MFMA GEMM whose operands are
// fetched by small address functors; the elementwise parts (bias, ReLU,
// pooling, loss, reductions, optimiser) are separate kernels.  Reductions are
// done in a fixed order, so results are reproducible run to run.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pxd.h"
#include "status.hpp"
#include "sur_infer.hpp"
#include "surrogate.hpp"

namespace pxd {
namespace sur {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int TM = 64, TN = 64, TK = 16;

// FP32 -> BF16 bits, round to nearest even (one v_cvt_pk_bf16_f32 on gfx950,
// the conversion the fused inference kernels use too)
__device__ __forceinline__ short to_bf16(float f) { return __builtin_bit_cast(short, (__bf16)f); }

// Problems whose A operand is cheaper with a per-row context computed once
// per tile (Prob::Row, row(m), a_row(row, k)) instead of a(m, k) per element.
template <typename Prob, typename = void>
struct HasRows {
  static constexpr bool value = false;
};
template <typename Prob>
struct HasRows<Prob, std::void_t<typename Prob::Row>> {
  static constexpr bool value = true;
};
struct Dummy {  // row type of the problems without a row context
  struct Row {};
};

// C = A B over a 64 x 64 output tile per workgroup (four waves of 32 x 32,
// each 2 x 2 MFMA tiles).  Prob supplies M, N, K, a(m, k), b(k, n) and
// store(m, n, value, split); blockIdx.z selects a slice of K (split-K, the
// caller reduces the slices).  Each thread stages the same column kk of A for
// the rows r = tid / TK + (256 / TK) i, so a problem with a row context
// decodes its rows once per tile.
template <typename Prob, bool BF16>
__global__ __launch_bounds__(256) void k_gemm(Prob pr, int k_per_split) {
  __shared__ float As[TM][TK + 1];
  __shared__ float Bs[TK][TN + 1];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
  const int kb = blockIdx.z * k_per_split, ke = min(pr.K, kb + k_per_split);
  const int wr = (wid >> 1) * 32, wc = (wid & 1) * 32;
  const int l16 = lane & 15, lq = lane >> 4;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0, 0, 0, 0};
  constexpr int RPT = TM * TK / 256;  // A elements staged per thread
  constexpr int RSTEP = 256 / TK;     // row stride between them
  static_assert(TM * TK % 256 == 0 && 256 % TK == 0, "staging layout");
  const int kk_a = tid % TK, r_a = tid / TK;
  [[maybe_unused]] typename std::conditional<HasRows<Prob>::value, Prob, Dummy>::type::Row rows[RPT];
  if constexpr (HasRows<Prob>::value) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) rows[i] = pr.row(m0 + r_a + RSTEP * i);
  }
  for (int k0 = kb; k0 < ke; k0 += TK) {
    if constexpr (HasRows<Prob>::value) {
      const int k = k0 + kk_a;
      const auto kc = pr.col(k < ke ? k : 0);
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = r_a + RSTEP * i;
        As[r][kk_a] = (m0 + r < pr.M && k < ke) ? pr.a_row(rows[i], kc) : 0.0f;
      }
    } else {
#pragma unroll
      for (int e = tid; e < TM * TK; e += 256) {
        const int r = e / TK, kk = e - r * TK;
        const int m = m0 + r, k = k0 + kk;
        As[r][kk] = (m < pr.M && k < ke) ? pr.a(m, k) : 0.0f;
      }
    }
#pragma unroll
    for (int e = tid; e < TK * TN; e += 256) {
      const int kk = e / TN, c = e - kk * TN;
      const int n = n0 + c, k = k0 + kk;
      Bs[kk][c] = (n < pr.N && k < ke) ? pr.b(k, n) : 0.0f;
    }
    __syncthreads();
    if constexpr (BF16) {
      // 16x16x16: lane l holds A[l % 16][4 (l / 16) + j] and B[4 (l / 16) + j][l % 16]
      s4 av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          av[t][j] = to_bf16(As[wr + 16 * t + l16][4 * lq + j]);
          bv[t][j] = to_bf16(Bs[4 * lq + j][wc + 16 * t + l16]);
        }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[i], bv[j], acc[i][j], 0, 0, 0);
    } else {
      // 16x16x4 steps: lane l holds A[l % 16][4 s + l / 16] and B[4 s + l / 16][l % 16]
#pragma unroll
      for (int s = 0; s < TK / 4; ++s) {
        float a0 = As[wr + l16][4 * s + lq], a1 = As[wr + 16 + l16][4 * s + lq];
        float b0 = Bs[4 * s + lq][wc + l16], b1 = Bs[4 * s + lq][wc + 16 + l16];
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // accumulator element i of lane l: row 4 (l / 16) + i, column l % 16
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wr + 16 * i + 4 * lq + q, n = n0 + wc + 16 * j + l16;
        if (m < pr.M && n < pr.N) pr.store(m, n, acc[i][j][q], blockIdx.z);
      }
}

// ---------------------------------------------------------------- problems

// Image geometry of one conv layer (NHWC activations, B images of H x W).
struct Img {
  int B, H, W, C;
};


// Input of the first conv: the map bytes themselves.
struct MapSrc {
  const uint8_t* maps;
  int n_cells;
  __device__ float at(int b, int y, int x, int c, const Img& g) const {
    return maps[(size_t)b * n_cells + ((size_t)c * g.H + y) * g.W + x] ? 1.0f : 0.0f;
  }
};
struct ActSrc {
  const float* x;
  __device__ float at(int b, int y, int x0, int c, const Img& g) const {
    return x[(((size_t)b * g.H + y) * g.W + x0) * g.C + c];
  }
};

// z = conv3x3(x) + bias: M = B H W, N = Cout, K = 9 Cin.
template <typename Src>
struct ConvFwd {
  int M, N, K;
  Src src;
  Img g;
  const float* w;  // [9][Cin][Cout]
  const float* bias;
  float* z;
  __device__ float a(int m, int k) const {
    const int tap = k / g.C, ci = k - tap * g.C;
    const int x = m % g.W, t = m / g.W, y = t % g.H, b = t / g.H;
    const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
    return (yy >= 0 && yy < g.H && xx >= 0 && xx < g.W) ? src.at(b, yy, xx, ci, g) : 0.0f;
  }
  // row context: the pixel (b, y, x) of output row m (rows past M decode to
  // pixels that a_row never reads: the caller masks them)
  struct Row {
    int b, y, x;
  };
  struct Col {
    int dy, dx, ci;
  };
  __device__ Row row(int m) const {
    const int x = m % g.W, t = m / g.W;
    return Row{t / g.H, t % g.H, x};
  }
  __device__ Col col(int k) const {
    const int tap = k / g.C;
    return Col{tap / 3 - 1, tap % 3 - 1, k - tap * g.C};
  }
  __device__ float a_row(const Row& r, const Col& c) const {
    const int yy = r.y + c.dy, xx = r.x + c.dx;
    return (yy >= 0 && yy < g.H && xx >= 0 && xx < g.W) ? src.at(r.b, yy, xx, c.ci, g) : 0.0f;
  }
  __device__ float b(int k, int n) const { return w[(size_t)k * N + n]; }
  __device__ void store(int m, int n, float v, int) const { z[(size_t)m * N + n] = v + bias[n]; }
};

// dX = conv3x3 transposed: dX[b, y, x, ci] = sum dZ[b, y - dy + 1, x - dx + 1, co] W[tap, ci, co].
// M = B H W, N = Cin, K = 9 Cout.
struct ConvBwdData {
  int M, N, K;
  Img g;  // geometry of dZ (C = Cout)
  const float* dz;
  const float* w;
  float* dx;
  __device__ float a(int m, int k) const {
    const int tap = k / g.C, co = k - tap * g.C;
    const int x = m % g.W, t = m / g.W, y = t % g.H, b = t / g.H;
    const int yy = y - tap / 3 + 1, xx = x - tap % 3 + 1;
    return (yy >= 0 && yy < g.H && xx >= 0 && xx < g.W) ? dz[(((size_t)b * g.H + yy) * g.W + xx) * g.C + co] : 0.0f;
  }
  __device__ float b(int k, int n) const {
    const int tap = k / g.C, co = k - tap * g.C;
    return w[((size_t)tap * N + n) * g.C + co];
  }
  __device__ void store(int m, int n, float v, int) const { dx[(size_t)m * N + n] = v; }
};

// dW[tap, ci, co] = sum over pixels of x[b, y + dy - 1, x + dx - 1, ci] dZ[b, y, x, co].
// M = 9 Cin, N = Cout, K = B H W; split-K slices go to part[split][M][N].
template <typename Src>
struct ConvBwdWeight {
  int M, N, K;
  Src src;
  Img g;  // geometry of the layer input (C = Cin)
  const float* dz;
  float* part;
  __device__ float a(int m, int k) const {
    const int tap = m / g.C, ci = m - tap * g.C;
    const int x = k % g.W, t = k / g.W, y = t % g.H, b = t / g.H;
    const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
    return (yy >= 0 && yy < g.H && xx >= 0 && xx < g.W) ? src.at(b, yy, xx, ci, g) : 0.0f;
  }
  __device__ float b(int k, int n) const { return dz[(size_t)k * N + n]; }
  __device__ void store(int m, int n, float v, int s) const { part[((size_t)s * M + m) * N + n] = v; }
};

// Plain row-major products with optional transposes: C[m, n] = sum A[m, k] B[k, n]
// where A is read as a[m lda + k] (or a[k lda + m] when ta) and likewise B.
struct Dense {
  int M, N, K;
  const float* A;
  const float* Bm;
  int lda, ldb;
  bool ta, tb;
  float* out;  // out[split][M][N] (or M x N with accumulate = false and one split)
  const float* bias;     // added to every row when set (single split only)
  const float* relu_of;  // when set, multiply by (relu_of[m N + n] > 0) (single split only)
  __device__ float a(int m, int k) const { return ta ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k]; }
  __device__ float b(int k, int n) const { return tb ? Bm[(size_t)n * ldb + k] : Bm[(size_t)k * ldb + n]; }
  __device__ void store(int m, int n, float v, int s) const {
    if (bias) v += bias[n];
    if (relu_of && !(relu_of[(size_t)m * N + n] > 0.0f)) v = 0.0f;
    out[((size_t)s * M + m) * N + n] = v;
  }
};

template <typename Prob>
hipError_t gemm(hipStream_t s, const Prob& p, bool bf16, int splits = 1) {
  if (p.M <= 0 || p.N <= 0) return hipSuccess;
  splits = std::max(1, std::min(splits, (p.K + TK - 1) / TK));
  const int per = ((p.K + splits - 1) / splits + TK - 1) / TK * TK;
  splits = (p.K + per - 1) / per;
  dim3 grid((p.M + TM - 1) / TM, (p.N + TN - 1) / TN, std::max(1, splits));
  if (bf16)
    hipLaunchKernelGGL((k_gemm<Prob, true>), grid, dim3(256), 0, s, p, per);
  else
    hipLaunchKernelGGL((k_gemm<Prob, false>), grid, dim3(256), 0, s, p, per);
  return hipGetLastError();
}

// Number of K slices for a reduction-heavy product (gradient of a weight).
inline int splits_for(int M, int N, int K) {
  const int tiles = ((M + TM - 1) / TM) * ((N + TN - 1) / TN);
  int s = std::max(1, 256 / tiles);
  return std::min(s, std::max(1, K / 256));
}

// ---------------------------------------------------------------- elementwise

// a = pool2(relu(z)) (pooled) or relu(z): z is B x H x W x C.
__global__ void k_relu_pool(const float* z, Img g, bool pool, float* a) {
  const int Ho = pool ? g.H / 2 : g.H, Wo = pool ? g.W / 2 : g.W;
  const size_t n = (size_t)g.B * Ho * Wo * g.C;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int c = i % g.C;
    size_t t = i / g.C;
    const int x = t % Wo;
    t /= Wo;
    const int y = t % Ho, b = t / Ho;
    if (!pool) {
      a[i] = fmaxf(z[i], 0.0f);
    } else {
      auto Z = [&](int yy, int xx) { return fmaxf(z[(((size_t)b * g.H + yy) * g.W + xx) * g.C + c], 0.0f); };
      a[i] = 0.25f * ((Z(2 * y, 2 * x) + Z(2 * y + 1, 2 * x)) + (Z(2 * y, 2 * x + 1) + Z(2 * y + 1, 2 * x + 1)));
    }
  }
}

// dz = (pool2 backward of da, or da) * (z > 0); z, dz are B x H x W x C.
__global__ void k_relu_pool_bwd(const float* z, const float* da, Img g, bool pool, float* dz) {
  const size_t n = (size_t)g.B * g.H * g.W * g.C;
  const int Ho = g.H / 2, Wo = g.W / 2;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    float d;
    if (!pool) {
      d = da[i];
    } else {
      const int c = i % g.C;
      size_t t = i / g.C;
      const int x = t % g.W;
      t /= g.W;
      const int y = t % g.H, b = t / g.H;
      const int yo = y / 2, xo = x / 2;
      d = (yo < Ho && xo < Wo) ? 0.25f * da[(((size_t)b * Ho + yo) * Wo + xo) * g.C + c] : 0.0f;
    }
    dz[i] = (z[i] > 0.0f) ? d : 0.0f;
  }
}

// zh[b, f, :] = U[b] + V[f] + bh;  h = relu(zh)
__global__ void k_head_hidden(const float* U, const float* V, const float* bh, int B, int F, int Hd, float* zh,
                              float* h) {
  const size_t n = (size_t)B * F * Hd;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int c = i % Hd;
    const size_t bf = i / Hd;
    const int f = bf % F, b = bf / F;
    const float v = (U[(size_t)b * Hd + c] + V[(size_t)f * Hd + c]) + bh[c];
    zh[i] = v;
    h[i] = fmaxf(v, 0.0f);
  }
}

// e[f, 2j] = sin((j+1) pi u_f), e[f, 2j+1] = cos((j+1) pi u_f)
__global__ void k_embed(const double* u, int F, int E, float* e) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= F * E) return;
  const int f = i / E, j = i % E;
  const double arg = (j / 2 + 1) * M_PI * u[f];
  e[i] = (float)((j & 1) ? cos(arg) : sin(arg));
}

// out[g][c] = sum_{r < R} X[(r sr + g sg) C + c], in order of r.
__global__ void k_group_sum(const float* X, int G, int R, int C, size_t sr, size_t sg, float* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G * C) return;
  const int g = i / C, c = i % C;
  float acc = 0.0f;
  for (int r = 0; r < R; ++r) acc += X[((size_t)r * sr + (size_t)g * sg) * C + c];
  out[i] = acc;
}

// out[i] = sum over s of part[s][i]
__global__ void k_sum_splits(const float* part, int S, size_t n, float* out) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    float acc = 0.0f;
    for (int s = 0; s < S; ++s) acc += part[(size_t)s * n + i];
    out[i] = acc;
  }
}

// dout = 2 (out - target) / n and loss = mean (out - target)^2 (one block, fixed order).
__global__ void k_mse(const float* out, const float* target, size_t n, float* dout, float* loss) {
  __shared__ float red[256];
  float acc = 0.0f;
  const float scale = 2.0f / (float)n;
  for (size_t i = threadIdx.x; i < n; i += 256) {
    const float d = out[i] - target[i];
    dout[i] = scale * d;
    acc += d * d;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = red[0] / (float)n;
}

__global__ void k_adamw(float* p, const float* g, float* m, float* v, size_t n, float lr, float b1, float b2, float eps,
                        float wd, float c1, float c2) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    p[i] -= lr * (mh / (sqrtf(vh) + eps) + wd * p[i]);
  }
}

// maps[c - c0] = base with candidate c's cells toggled
__global__ void k_candidate_maps(const uint8_t* base, const int* off, const int* cells, int c0, int n, int n_cells,
                                 uint8_t* maps) {
  const int r = blockIdx.x;
  if (r >= n) return;
  uint8_t* m = maps + (size_t)r * n_cells;
  for (int i = threadIdx.x; i < n_cells; i += blockDim.x) m[i] = base[i] ? 1 : 0;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int i = off[c0 + r]; i < off[c0 + r + 1]; ++i) {
      const int cell = cells[i];
      if (cell >= 0 && cell < n_cells) m[cell] ^= 1;
    }
}

// FoM (Eqs. 8-9 in closed form) of predicted S: terms on entries that are not
// predicted are skipped.  pred: n x F x (3 n_entries), per entry ln|S| first.
// A term's |S|^power with |S|^2 floored at 1e-30 is exp(power max(ln|S|,
// ln(1e-30) / 2)).
__global__ void k_pred_fom(const float* pred, int n, int F, int n_ent, const int* ent_i, const int* ent_j,
                           FomTable t, double* fom) {
  // one wave per map: terms in turn, lanes over the frequencies, then a
  // fixed-order wave reduction
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (r >= n) return;  // whole waves leave together
  const double floor_log = 0.5 * log(1e-30);
  const float* pr = pred + (size_t)r * F * 3 * n_ent;
  double acc = 0.0;
  for (int q = 0; q < t.n_terms; ++q) {
    const pxd_fom_term tq = t.terms[q];
    int e = -1;
    for (int k = 0; k < n_ent; ++k)
      if (ent_i[k] == tq.i && ent_j[k] == tq.j) e = k;
    if (e < 0) continue;
    const double fac = t.term_fac[q];
    for (int f = lane; f < F; f += 64) {
      if (t.band[f] != tq.band) continue;
      const double ls = fmax((double)pr[(size_t)f * 3 * n_ent + 3 * e], floor_log);  // ln|S|
      acc += fac * exp(tq.power * ls);
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) fom[r] = acc;
}

// k smallest (value, id) pairs in increasing order; pass j takes the least
// pair above the one pass j - 1 took, so no scratch is needed.  NaN counts as
// +inf.  Block g takes positions [g per, (g + 1) per) of v; ids are idx[pos]
// (or pos when idx is null).  Writes out_v[g k + j] and out_i[g k + j]
// (INT_MAX where fewer than k pairs exist).  One block over all of v gives
// the top k; blocks over slices, then one block over their k each, give the
// same k (every pair of the top k is in the top k of its slice).
__global__ void k_topk(const double* v, const int* idx, int n, int k, int per, double* out_v, int* out_i) {
  __shared__ double sv[1024];
  __shared__ int si[1024];
  const int lo = blockIdx.x * per, hi = min(n, lo + per);
  double pv = -__builtin_inf();
  int pi = -1;
  for (int j = 0; j < k; ++j) {
    double best = __builtin_inf();
    int bi = 0x7fffffff;
    for (int p = lo + (int)threadIdx.x; p < hi; p += 1024) {
      double x = v[p];
      if (x != x) x = __builtin_inf();
      const int i = idx ? idx[p] : p;
      const bool above = (x > pv) || (x == pv && i > pi);
      if (above && (x < best || (x == best && i < bi))) best = x, bi = i;
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
        const double ov = sv[threadIdx.x + s];
        const int oi = si[threadIdx.x + s];
        if (ov < sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < si[threadIdx.x]))
          sv[threadIdx.x] = ov, si[threadIdx.x] = oi;
      }
      __syncthreads();
    }
    pv = sv[0];
    pi = si[0];
    if (threadIdx.x == 0) {
      if (out_v) out_v[(size_t)blockIdx.x * k + j] = pv;
      out_i[(size_t)blockIdx.x * k + j] = pi;
    }
    __syncthreads();
  }
}

// INT_MAX (fewer than k candidates) -> -1
__global__ void k_topk_ids(int k, int* top) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < k && top[j] == 0x7fffffff) top[j] = -1;
}

inline dim3 grid1(size_t n) { return dim3((unsigned)std::min<size_t>((n + 255) / 256, 4096)); }

}  // namespace sur
}  // namespace pxd

// ---------------------------------------------------------------- host object

namespace {

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t n) {
    if (n <= bytes) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipMalloc(&p, std::max<size_t>(n, 16));
    if (e == hipSuccess) bytes = n;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

struct Tensor {
  size_t off, n;
};

}  // namespace

// Training targets from exact S (n x F x P x P complex128): per (map,
// frequency) and predicted entry (i, j): ln max(|S_ij|, 1e-30) and the unit
// phasor S_ij / |S_ij|, in entry order.
__global__ void k_encode(const double2* __restrict__ S, int n, int F, int P, int n_ent, const int* __restrict__ ei,
                         const int* __restrict__ ej, float* __restrict__ out) {
  const size_t total = (size_t)n * F * n_ent;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (size_t)gridDim.x * blockDim.x) {
    const int e = (int)(q % n_ent);
    const size_t bf = q / n_ent;
    const double2 v = S[bf * P * P + (size_t)ei[e] * P + ej[e]];
    const double a = fmax(sqrt(v.x * v.x + v.y * v.y), 1e-30);
    float* o = out + bf * (3 * n_ent) + 3 * e;
    o[0] = (float)log(a);
    o[1] = (float)(v.x / a);
    o[2] = (float)(v.y / a);
  }
}

struct pxd_sur {
  pxd_sur_config cfg{};
  std::string err;
  int F = 0, n_out = 0, ch[5] = {}, H[3] = {}, W[3] = {}, feat = 0;
  bool bf16 = false;
  pxd::sur::InferPlan plan;  // fused inference layout (plan.ok: in use)
  Buf frag;                  // its packed BF16 weight fragments
  Tensor t[13];  // W1 b1 W2 b2 W3 b3 W4 b4 Wf We bh Wo bo
  size_t n_params = 0;
  long step = 0;
  Buf params, grad, m, v, u, e, ent;
  // activations and their gradients, sized for max_batch
  Buf z[4], act[4], dz, da, U, V, zh, h, out, dout, dh, dU, dV, part, maps, pred, loss;
  Buf tk_v, tk_i;  // per-slice top-k candidates of the ranking

  int fail(int rc, const std::string& msg) {
    err = msg;
    pxd::set_thread_error(rc, msg);
    return rc;
  }
};

#define SURCHK(s, expr)                                                                     \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return (s)->fail(PXD_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace {

using namespace pxd::sur;

float* P(pxd_sur* s, int i) { return s->params.as<float>() + s->t[i].off; }
float* G(pxd_sur* s, int i) { return s->grad.as<float>() + s->t[i].off; }

// Forward pass of B maps; leaves z[l], act[l], U, zh, h, out.
int forward(pxd_sur* s, hipStream_t st, int B, const uint8_t* maps) {
  const int F = s->F, Hd = s->cfg.hidden;
  for (int l = 0; l < 4; ++l) {
    const int r = l / 2;  // resolution index: layers 0,1 at full size, 2,3 at half
    Img gi{B, s->H[r], s->W[r], s->ch[l]};
    const int M = B * gi.H * gi.W, N = s->ch[l + 1], K = 9 * s->ch[l];
    if (l == 0) {
      ConvFwd<MapSrc> pr{M, N, K, MapSrc{maps, s->cfg.n_layers * s->cfg.ny * s->cfg.nx}, gi, P(s, 0), P(s, 1),
                         s->z[0].as<float>()};
      SURCHK(s, gemm(st, pr, s->bf16));
    } else {
      ConvFwd<ActSrc> pr{M, N, K, ActSrc{s->act[l - 1].as<float>()}, gi, P(s, 2 * l), P(s, 2 * l + 1),
                         s->z[l].as<float>()};
      SURCHK(s, gemm(st, pr, s->bf16));
    }
    Img go{B, gi.H, gi.W, N};
    const bool pool = (l == 1 || l == 3);
    hipLaunchKernelGGL(k_relu_pool, grid1((size_t)M * N), dim3(256), 0, st, s->z[l].as<float>(), go, pool,
                       s->act[l].as<float>());
    SURCHK(s, hipGetLastError());
  }
  // head: U = feat Wf, V = e We, zh = U + V + bh, out = relu(zh) Wo + bo
  Dense pu{B, Hd, s->feat, s->act[3].as<float>(), P(s, 8), s->feat, Hd, false, false, s->U.as<float>(), nullptr,
           nullptr};
  SURCHK(s, gemm(st, pu, s->bf16));
  Dense pv{F, Hd, s->cfg.emb, s->e.as<float>(), P(s, 9), s->cfg.emb, Hd, false, false, s->V.as<float>(), nullptr,
           nullptr};
  SURCHK(s, gemm(st, pv, s->bf16));
  hipLaunchKernelGGL(k_head_hidden, grid1((size_t)B * F * Hd), dim3(256), 0, st, s->U.as<float>(), s->V.as<float>(),
                     P(s, 10), B, F, Hd, s->zh.as<float>(), s->h.as<float>());
  SURCHK(s, hipGetLastError());
  Dense po{B * F, s->n_out, Hd, s->h.as<float>(), P(s, 11), Hd, s->n_out, false, false, s->out.as<float>(), P(s, 12),
           nullptr};
  SURCHK(s, gemm(st, po, s->bf16));
  return PXD_OK;
}

// Packs the current weights into the fused kernels' fragments.
int pack_fused(pxd_sur* s, hipStream_t st) {
  const float* w[4] = {P(s, 0), P(s, 2), P(s, 4), P(s, 6)};
  SURCHK(s, infer_pack(st, s->plan, w, P(s, 8), P(s, 11), s->frag.p));
  return PXD_OK;
}

// V = e We (the frequency half of the head's first layer).
int head_v(pxd_sur* s, hipStream_t st) {
  Dense pv{s->F, s->cfg.hidden, s->cfg.emb, s->e.as<float>(), P(s, 9), s->cfg.emb, s->cfg.hidden, false, false,
           s->V.as<float>(), nullptr, nullptr};
  SURCHK(s, gemm(st, pv, s->bf16));
  return PXD_OK;
}

// Fused forward of B maps (weights packed and V formed beforehand): trunk ->
// act[3] (BF16), U = act[3] Wf, out = relu((U + V) + bh) Wo + bo.
int forward_fused(pxd_sur* s, hipStream_t st, int B, const uint8_t* maps) {
  const float* bias[4] = {P(s, 1), P(s, 3), P(s, 5), P(s, 7)};
  SURCHK(s, infer_trunk(st, s->plan, B, maps, s->cfg.n_layers * s->cfg.ny * s->cfg.nx, s->frag.p, bias,
                        s->act[3].p));  // BF16 here
  SURCHK(s, infer_u(st, s->plan, B, s->act[3].p, s->frag.p, s->U.as<float>()));
  SURCHK(s, infer_head(st, s->plan, B, s->F, s->U.as<float>(), s->V.as<float>(), P(s, 10), s->frag.p, P(s, 12),
                       s->out.as<float>()));
  return PXD_OK;
}

// Weight gradient product with split-K partials, then their fixed-order sum into dst.
template <typename Prob>
int weight_grad(pxd_sur* s, hipStream_t st, Prob pr, float* dst) {
  const int S = splits_for(pr.M, pr.N, pr.K);
  const size_t n = (size_t)pr.M * pr.N;
  SURCHK(s, s->part.ensure(sizeof(float) * n * S));
  pr.part = s->part.as<float>();
  const int per = ((pr.K + S - 1) / S + TK - 1) / TK * TK;
  const int used = (pr.K + per - 1) / per;
  SURCHK(s, gemm(st, pr, s->bf16, S));
  hipLaunchKernelGGL(k_sum_splits, grid1(n), dim3(256), 0, st, s->part.as<float>(), used, n, dst);
  SURCHK(s, hipGetLastError());
  return PXD_OK;
}

int dense_weight_grad(pxd_sur* s, hipStream_t st, int M, int N, int K, const float* A, int lda, const float* Bm,
                      int ldb, float* dst) {
  // dst[M x N] = A^T B with A stored K x M (lda) and B stored K x N (ldb)
  Dense pr{M, N, K, A, Bm, lda, ldb, true, false, nullptr, nullptr, nullptr};
  const int S = splits_for(M, N, K);
  const size_t n = (size_t)M * N;
  SURCHK(s, s->part.ensure(sizeof(float) * n * S));
  pr.out = s->part.as<float>();
  const int per = ((K + S - 1) / S + TK - 1) / TK * TK;
  const int used = (K + per - 1) / per;
  SURCHK(s, gemm(st, pr, s->bf16, S));
  hipLaunchKernelGGL(k_sum_splits, grid1(n), dim3(256), 0, st, s->part.as<float>(), used, n, dst);
  SURCHK(s, hipGetLastError());
  return PXD_OK;
}

int group_sum(pxd_sur* s, hipStream_t st, const float* X, int G, int R, int C, size_t sr, size_t sg, float* out) {
  hipLaunchKernelGGL(k_group_sum, dim3((G * C + 255) / 256), dim3(256), 0, st, X, G, R, C, sr, sg, out);
  SURCHK(s, hipGetLastError());
  return PXD_OK;
}

// Loss and gradient of B maps against target (forward included).
int backward(pxd_sur* s, hipStream_t st, int B, const uint8_t* maps, const float* target, float* loss) {
  int rc = forward(s, st, B, maps);
  if (rc) return rc;
  const int F = s->F, Hd = s->cfg.hidden, no = s->n_out;
  const size_t n_out = (size_t)B * F * no;
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, st, s->out.as<float>(), target, n_out, s->dout.as<float>(), loss);
  SURCHK(s, hipGetLastError());
  // output layer
  if ((rc = dense_weight_grad(s, st, Hd, no, B * F, s->h.as<float>(), Hd, s->dout.as<float>(), no, G(s, 11)))) return rc;
  if ((rc = group_sum(s, st, s->dout.as<float>(), 1, B * F, no, 1, 0, G(s, 12)))) return rc;
  // dzh = (dout Wo^T) * (zh > 0)
  Dense pdh{B * F, Hd, no, s->dout.as<float>(), P(s, 11), no, no, false, true, s->dh.as<float>(), nullptr,
            s->zh.as<float>()};
  SURCHK(s, gemm(st, pdh, s->bf16));
  if ((rc = group_sum(s, st, s->dh.as<float>(), 1, B * F, Hd, 1, 0, G(s, 10)))) return rc;
  if ((rc = group_sum(s, st, s->dh.as<float>(), B, F, Hd, 1, F, s->dU.as<float>()))) return rc;  // sum over f
  if ((rc = group_sum(s, st, s->dh.as<float>(), F, B, Hd, F, 1, s->dV.as<float>()))) return rc;  // sum over b
  if ((rc = dense_weight_grad(s, st, s->feat, Hd, B, s->act[3].as<float>(), s->feat, s->dU.as<float>(), Hd, G(s, 8))))
    return rc;
  if ((rc = dense_weight_grad(s, st, s->cfg.emb, Hd, F, s->e.as<float>(), s->cfg.emb, s->dV.as<float>(), Hd, G(s, 9))))
    return rc;
  // dfeat = dU Wf^T  (into da, the gradient of the pooled a4)
  Dense pdf{B, s->feat, Hd, s->dU.as<float>(), P(s, 8), Hd, Hd, false, true, s->da.as<float>(), nullptr, nullptr};
  SURCHK(s, gemm(st, pdf, s->bf16));
  for (int l = 3; l >= 0; --l) {
    const int r = l / 2;
    Img gz{B, s->H[r], s->W[r], s->ch[l + 1]};
    const bool pool = (l == 1 || l == 3);
    const size_t nz = (size_t)B * gz.H * gz.W * gz.C;
    // dz_l from da (gradient of act[l])
    hipLaunchKernelGGL(k_relu_pool_bwd, grid1(nz), dim3(256), 0, st, s->z[l].as<float>(), s->da.as<float>(), gz, pool,
                       s->dz.as<float>());
    SURCHK(s, hipGetLastError());
    Img gin{B, s->H[r], s->W[r], s->ch[l]};
    const int K = B * gin.H * gin.W;
    if (l == 0) {
      ConvBwdWeight<MapSrc> pw{9 * s->ch[0], s->ch[1], K, MapSrc{maps, s->cfg.n_layers * s->cfg.ny * s->cfg.nx}, gin,
                               s->dz.as<float>(), nullptr};
      if ((rc = weight_grad(s, st, pw, G(s, 0)))) return rc;
    } else {
      ConvBwdWeight<ActSrc> pw{9 * s->ch[l], s->ch[l + 1], K, ActSrc{s->act[l - 1].as<float>()}, gin,
                               s->dz.as<float>(), nullptr};
      if ((rc = weight_grad(s, st, pw, G(s, 2 * l)))) return rc;
    }
    if ((rc = group_sum(s, st, s->dz.as<float>(), 1, K, s->ch[l + 1], 1, 0, G(s, 2 * l + 1)))) return rc;
    if (l > 0) {
      ConvBwdData pd{K, s->ch[l], 9 * s->ch[l + 1], gz, s->dz.as<float>(), P(s, 2 * l), s->da.as<float>()};
      SURCHK(s, gemm(st, pd, s->bf16));
    }
  }
  return PXD_OK;
}

int check_batch(pxd_sur* s, int B) {
  if (B < 1 || B > s->cfg.max_batch) return s->fail(PXD_EINVAL, "batch size outside [1, max_batch]");
  return PXD_OK;
}

uint64_t splitmix_next(uint64_t& st) {
  st += 0x9E3779B97F4A7C15ull;
  uint64_t z = st;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

extern "C" {

int pxd_sur_create(const pxd_sur_config* cfg, int32_t F, const double* freqs_hz, double f_lo, double f_hi,
                   pxd_sur** out) {
  if (!cfg || !out || F < 1 || !freqs_hz || !(f_hi > f_lo)) return pxd::set_thread_error(PXD_EINVAL, "invalid surrogate arguments");
  *out = nullptr;
  const pxd_sur_config& c = *cfg;
  if (c.n_layers < 1 || c.ny < 4 || c.nx < 4 || c.hidden < 1 || c.emb < 2 || (c.emb & 1) || c.n_entries < 1 ||
      c.n_entries > 4 || c.max_batch < 1 || (c.precision != PXD_SUR_FP32 && c.precision != PXD_SUR_BF16) ||
      c.inference < PXD_SUR_INFER_AUTO || c.inference > PXD_SUR_INFER_FUSED)
    return pxd::set_thread_error(PXD_EINVAL, "invalid surrogate configuration");
  if (c.inference == PXD_SUR_INFER_FUSED &&
      (c.precision != PXD_SUR_BF16 || !pxd::sur::infer_plan(c.n_layers, c.ny, c.nx, c.channels, c.hidden,
                                                            3 * c.n_entries).ok))
    return pxd::set_thread_error(PXD_EINVAL, "fused inference does not cover this configuration");
  for (int i = 0; i < 4; ++i)
    if (c.channels[i] < 1 || c.channels[i] > 256) return pxd::set_thread_error(PXD_EINVAL, "channel count outside [1, 256]");
  for (int k = 0; k < c.n_entries; ++k)
    if (c.entry_i[k] < 0 || c.entry_j[k] < 0) return pxd::set_thread_error(PXD_EINVAL, "negative S entry index");
  if (hipSetDevice(c.device) != hipSuccess) return pxd::set_thread_error(PXD_EDEVICE, "no usable HIP device");
  auto* s = new (std::nothrow) pxd_sur();
  if (!s) return pxd::set_thread_error(PXD_ENOMEM, "out of host memory");
  s->cfg = c;
  s->F = F;
  s->n_out = 3 * c.n_entries;
  s->bf16 = c.precision == PXD_SUR_BF16;
  s->ch[0] = c.n_layers;
  for (int i = 0; i < 4; ++i) s->ch[i + 1] = c.channels[i];
  s->H[0] = c.ny, s->W[0] = c.nx;
  s->H[1] = c.ny / 2, s->W[1] = c.nx / 2;
  s->H[2] = s->H[1] / 2, s->W[2] = s->W[1] / 2;
  s->feat = s->H[2] * s->W[2] * s->ch[4];
  const size_t sizes[13] = {
      (size_t)9 * s->ch[0] * s->ch[1], (size_t)s->ch[1], (size_t)9 * s->ch[1] * s->ch[2], (size_t)s->ch[2],
      (size_t)9 * s->ch[2] * s->ch[3], (size_t)s->ch[3], (size_t)9 * s->ch[3] * s->ch[4], (size_t)s->ch[4],
      (size_t)s->feat * c.hidden,      (size_t)c.emb * c.hidden, (size_t)c.hidden,
      (size_t)c.hidden * s->n_out,     (size_t)s->n_out};
  size_t o = 0;
  for (int i = 0; i < 13; ++i) {
    s->t[i] = Tensor{o, sizes[i]};
    o += sizes[i];
  }
  s->n_params = o;
  const size_t B = c.max_batch, Hd = c.hidden;
  const size_t full = B * s->H[0] * s->W[0], half = B * s->H[1] * s->W[1];
  std::vector<double> u(F);
  for (int f = 0; f < F; ++f) u[f] = (freqs_hz[f] - f_lo) / (f_hi - f_lo);
  std::vector<int> ent(8);
  for (int k = 0; k < 4; ++k) ent[k] = c.entry_i[k], ent[4 + k] = c.entry_j[k];
  const size_t maxact = std::max(full * std::max(s->ch[1], s->ch[2]), half * std::max(s->ch[3], s->ch[4]));
  hipError_t e = hipSuccess;
  auto ok = [&](hipError_t r) { if (e == hipSuccess) e = r; };
  ok(s->params.ensure(4 * o));
  ok(s->grad.ensure(4 * o));
  ok(s->m.ensure(4 * o));
  ok(s->v.ensure(4 * o));
  ok(s->u.ensure(8 * F));
  ok(s->e.ensure(4 * (size_t)F * c.emb));
  ok(s->ent.ensure(4 * 8));
  for (int l = 0; l < 4; ++l) {
    const size_t n = (l < 2 ? full : half) * s->ch[l + 1];
    ok(s->z[l].ensure(4 * n));
    ok(s->act[l].ensure(4 * n));
  }
  ok(s->dz.ensure(4 * maxact));
  ok(s->da.ensure(4 * maxact));
  ok(s->U.ensure(4 * B * Hd));
  ok(s->dU.ensure(4 * B * Hd));
  ok(s->V.ensure(4 * (size_t)F * Hd));
  ok(s->dV.ensure(4 * (size_t)F * Hd));
  ok(s->zh.ensure(4 * B * F * Hd));
  ok(s->h.ensure(4 * B * F * Hd));
  ok(s->dh.ensure(4 * B * F * Hd));
  ok(s->out.ensure(4 * B * F * s->n_out));
  ok(s->dout.ensure(4 * B * F * s->n_out));
  ok(s->maps.ensure(B * c.n_layers * c.ny * c.nx));
  ok(s->pred.ensure(4 * B * F * s->n_out));
  ok(s->loss.ensure(4));
  if (s->bf16 && c.inference != PXD_SUR_INFER_GENERIC)
    s->plan = pxd::sur::infer_plan(c.n_layers, c.ny, c.nx, c.channels, c.hidden, s->n_out);
  if (s->plan.ok) {
    ok(s->frag.ensure(16 * 64 * (size_t)s->plan.n_frag));
    ok(pxd::sur::infer_prepare(s->plan));
  }
  if (e == hipSuccess) e = hipMemcpy(s->u.p, u.data(), 8 * F, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->ent.p, ent.data(), 4 * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_embed, dim3((F * c.emb + 255) / 256), dim3(256), 0, 0, s->u.as<double>(), F, c.emb,
                       s->e.as<float>());
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    std::string msg = std::string("surrogate setup: ") + hipGetErrorString(e);
    pxd_sur_destroy(s);
    return pxd::set_thread_error(PXD_ENOMEM, msg);
  }
  if (int rc = pxd_sur_init_params(s, 1)) {
    pxd_sur_destroy(s);
    return rc;
  }
  *out = s;
  return PXD_OK;
}

void pxd_sur_destroy(pxd_sur* s) {
  if (!s) return;
  (void)hipSetDevice(s->cfg.device);
  (void)hipDeviceSynchronize();
  for (Buf* b : {&s->params, &s->grad, &s->m, &s->v, &s->u, &s->e, &s->ent, &s->dz, &s->da, &s->U, &s->V, &s->zh,
                 &s->h, &s->out, &s->dout, &s->dh, &s->dU, &s->dV, &s->part, &s->maps, &s->pred, &s->loss, &s->frag,
                 &s->tk_v, &s->tk_i})
    b->release();
  for (int l = 0; l < 4; ++l) {
    s->z[l].release();
    s->act[l].release();
  }
  delete s;
}

const char* pxd_sur_last_error(const pxd_sur* s) { return s ? s->err.c_str() : pxd::thread_error(); }

int pxd_sur_num_params(const pxd_sur* s, int64_t* n) {
  if (!s || !n) return pxd::set_thread_error(PXD_EINVAL, "null argument");
  *n = (int64_t)s->n_params;
  return PXD_OK;
}

int pxd_sur_inference_path(const pxd_sur* s, int32_t* path) {
  if (!s || !path) return pxd::set_thread_error(PXD_EINVAL, "null argument");
  *path = s->plan.ok ? PXD_SUR_INFER_FUSED : PXD_SUR_INFER_GENERIC;
  return PXD_OK;
}

int pxd_sur_set_params(pxd_sur* s, const float* params, int64_t n) {
  if (!s) return pxd::set_thread_error(PXD_EINVAL, "surrogate is NULL");
  if (!params || n != (int64_t)s->n_params) return s->fail(PXD_EINVAL, "parameter vector of the wrong length");
  SURCHK(s, hipSetDevice(s->cfg.device));
  SURCHK(s, hipMemcpy(s->params.p, params, 4 * s->n_params, hipMemcpyHostToDevice));
  SURCHK(s, hipMemset(s->m.p, 0, 4 * s->n_params));
  SURCHK(s, hipMemset(s->v.p, 0, 4 * s->n_params));
  s->step = 0;
  return PXD_OK;
}

int pxd_sur_get_params(const pxd_sur* s, float* params, int64_t n) {
  if (!s || !params || n != (int64_t)s->n_params) return pxd::set_thread_error(PXD_EINVAL, "invalid arguments");
  if (hipSetDevice(s->cfg.device) != hipSuccess ||
      hipMemcpy(params, s->params.p, 4 * s->n_params, hipMemcpyDeviceToHost) != hipSuccess)
    return pxd::set_thread_error(PXD_EDEVICE, "parameter copy failed");
  return PXD_OK;
}

int pxd_sur_init_params(pxd_sur* s, uint64_t seed) {
  if (!s) return pxd::set_thread_error(PXD_EINVAL, "surrogate is NULL");
  std::vector<float> p(s->n_params);
  for (int i = 0; i < 13; ++i) {
    const bool weight = (i < 8) ? (i % 2 == 0) : (i == 8 || i == 9 || i == 11);
    double bound = 0.05;
    if (weight) {
      size_t fan_in;
      if (i < 8) fan_in = (size_t)9 * s->ch[i / 2];
      else if (i == 8) fan_in = s->feat;
      else if (i == 9) fan_in = s->cfg.emb;
      else fan_in = s->cfg.hidden;
      bound = std::sqrt(3.0 / (double)fan_in);
    }
    uint64_t st = seed * 1000 + (uint64_t)i;
    for (size_t k = 0; k < s->t[i].n; ++k) {
      const double unit = (double)(splitmix_next(st) >> 11) * (1.0 / 9007199254740992.0);
      p[s->t[i].off + k] = (float)((2.0 * unit - 1.0) * bound);
    }
  }
  return pxd_sur_set_params(s, p.data(), (int64_t)s->n_params);
}

int pxd_sur_forward(pxd_sur* s, void* stream, int32_t B, const uint8_t* maps, float* out) {
  if (!s) return pxd::set_thread_error(PXD_EINVAL, "surrogate is NULL");
  if (!maps || !out) return s->fail(PXD_EINVAL, "null device pointer");
  if (int rc = check_batch(s, B)) return rc;
  SURCHK(s, hipSetDevice(s->cfg.device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (s->plan.ok) {
    int rc = pack_fused(s, st);
    if (!rc) rc = head_v(s, st);
    if (!rc) rc = forward_fused(s, st, B, maps);
    if (rc) return rc;
  } else if (int rc = forward(s, st, B, maps)) {
    return rc;
  }
  SURCHK(s, hipMemcpyAsync(out, s->out.p, 4 * (size_t)B * s->F * s->n_out, hipMemcpyDeviceToDevice, st));
  return PXD_OK;
}

int pxd_sur_gradient(pxd_sur* s, void* stream, int32_t B, const uint8_t* maps, const float* target, float* grad,
                     float* loss) {
  if (!s) return pxd::set_thread_error(PXD_EINVAL, "surrogate is NULL");
  if (!maps || !target) return s->fail(PXD_EINVAL, "null device pointer");
  if (int rc = check_batch(s, B)) return rc;
  SURCHK(s, hipSetDevice(s->cfg.device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int rc = backward(s, st, B, maps, target, loss)) return rc;
  if (grad) SURCHK(s, hipMemcpyAsync(grad, s->grad.p, 4 * s->n_params, hipMemcpyDeviceToDevice, st));
  return PXD_OK;
}

int pxd_sur_train_step(pxd_sur* s, void* stream, int32_t B, const uint8_t* maps, const float* target,
                       const pxd_adamw* hp, float* loss) {
  if (!s) return pxd::set_thread_error(PXD_EINVAL, "surrogate is NULL");
  if (!maps || !target || !hp || !(hp->lr > 0) || hp->beta1 < 0 || hp->beta1 >= 1 || hp->beta2 < 0 || hp->beta2 >= 1)
    return s->fail(PXD_EINVAL, "invalid training arguments");
  if (int rc = check_batch(s, B)) return rc;
  SURCHK(s, hipSetDevice(s->cfg.device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int rc = backward(s, st, B, maps, target, loss)) return rc;
  ++s->step;
  const float c1 = (float)(1.0 - std::pow(hp->beta1, (double)s->step));
  const float c2 = (float)(1.0 - std::pow(hp->beta2, (double)s->step));
  hipLaunchKernelGGL(k_adamw, grid1(s->n_params), dim3(256), 0, st, s->params.as<float>(), s->grad.as<float>(),
                     s->m.as<float>(), s->v.as<float>(), s->n_params, (float)hp->lr, (float)hp->beta1,
                     (float)hp->beta2, (float)hp->eps, (float)hp->weight_decay, c1, c2);
  SURCHK(s, hipGetLastError());
  return PXD_OK;
}

int pxd_sur_rank(pxd_sur* s, const pxd_ctx* ctx, void* stream, const uint8_t* base_map, int32_t n_cand,
                 const int32_t* offsets, const int32_t* cells, int32_t k, double* fom_pred, int32_t* top) {
  if (!s) return pxd::set_thread_error(PXD_EINVAL, "surrogate is NULL");
  if (!base_map || !offsets || !cells || n_cand < 1 || !fom_pred || (k > 0 && !top) || k < 0 || k > n_cand)
    return s->fail(PXD_EINVAL, "invalid ranking arguments");
  pxd::FomTable t{};
  if (pxd::fom_table(ctx, &t) != PXD_OK) return s->fail(PXD_ENOTLOADED, "the context has no FoM table");
  if (t.F != s->F) return s->fail(PXD_ESHAPE, "the context's frequency grid differs from the surrogate's");
  SURCHK(s, hipSetDevice(s->cfg.device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int n_cells = s->cfg.n_layers * s->cfg.ny * s->cfg.nx;
  if (s->plan.ok) {
    int rc = pack_fused(s, st);
    if (!rc) rc = head_v(s, st);
    if (rc) return rc;
  }
  for (int c0 = 0; c0 < n_cand; c0 += s->cfg.max_batch) {
    const int n = std::min(s->cfg.max_batch, n_cand - c0);
    hipLaunchKernelGGL(k_candidate_maps, dim3(n), dim3(256), 0, st, base_map, offsets, cells, c0, n, n_cells,
                       s->maps.as<uint8_t>());
    SURCHK(s, hipGetLastError());
    const int rc = s->plan.ok ? forward_fused(s, st, n, s->maps.as<uint8_t>()) : forward(s, st, n, s->maps.as<uint8_t>());
    if (rc) return rc;
    const int* ei = s->ent.as<int>();
    hipLaunchKernelGGL(k_pred_fom, dim3((n + 3) / 4), dim3(256), 0, st, s->out.as<float>(), n, s->F,
                       s->cfg.n_entries, ei, ei + 4, t, fom_pred + c0);
    SURCHK(s, hipGetLastError());
  }
  if (k > 0) {
    // slices of 4,096 candidates (at most 256 of them), then one block over their top k each
    const int G = std::min(256, (n_cand + 4095) / 4096);
    if (G > 1 && k <= 256) {
      const int per = (n_cand + G - 1) / G;
      SURCHK(s, s->tk_v.ensure(sizeof(double) * (size_t)G * k));
      SURCHK(s, s->tk_i.ensure(sizeof(int) * (size_t)G * k));
      hipLaunchKernelGGL(k_topk, dim3(G), dim3(1024), 0, st, fom_pred, nullptr, n_cand, k, per, s->tk_v.as<double>(),
                         s->tk_i.as<int>());
      SURCHK(s, hipGetLastError());
      hipLaunchKernelGGL(k_topk, dim3(1), dim3(1024), 0, st, s->tk_v.as<double>(), s->tk_i.as<int>(), G * k, k,
                         G * k, nullptr, top);
    } else {
      hipLaunchKernelGGL(k_topk, dim3(1), dim3(1024), 0, st, fom_pred, nullptr, n_cand, k, n_cand, nullptr, top);
    }
    SURCHK(s, hipGetLastError());
    hipLaunchKernelGGL(k_topk_ids, dim3((k + 255) / 256), dim3(256), 0, st, k, top);
    SURCHK(s, hipGetLastError());
  }
  return PXD_OK;
}

int pxd_sur_encode(pxd_sur* s, void* stream, int32_t n, const double* S, int32_t P, float* target) {
  if (!s) return pxd::set_thread_error(PXD_EINVAL, "surrogate is NULL");
  if (n < 0 || (n > 0 && (!S || !target)) || P < 1) return s->fail(PXD_EINVAL, "invalid encoding arguments");
  for (int k = 0; k < s->cfg.n_entries; ++k)
    if (s->cfg.entry_i[k] >= P || s->cfg.entry_j[k] >= P) return s->fail(PXD_ESHAPE, "predicted entry beyond P");
  if (n == 0) return PXD_OK;
  SURCHK(s, hipSetDevice(s->cfg.device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t total = (size_t)n * s->F * s->cfg.n_entries;
  const int* ei = s->ent.as<int>();
  hipLaunchKernelGGL(k_encode, dim3((unsigned)std::min<size_t>((total + 255) / 256, 4096)), dim3(256), 0, st,
                     reinterpret_cast<const double2*>(S), n, s->F, P, s->cfg.n_entries, ei, ei + 4, target);
  SURCHK(s, hipGetLastError());
  return PXD_OK;
}

}  // extern "C"
