// Fused BF16 inference kernels of the CNN surrogate (see sur_infer.hpp).
//
// Trunk: one workgroup per map.  Activations live in LDS as BF16, NHWC, with
// a one-pixel zero border so that every 3x3 tap is a plain offset; the pixel
// stride is an odd number of 16-byte chunks and the row stride 4 (mod 16)
// chunks, so the sixteen pixels of a 4 x 4 block that one MFMA row tile reads
// fall in sixteen different bank groups.  Two LDS regions alternate between
// the layers (input of layer l in one, output in the other).  Each wave task
// is mb row tiles x nb column tiles: per 32-deep k step it reads mb A
// fragments from LDS (16 bytes per lane, one tap and eight channels) and nb
// weight fragments from global memory (packed in operand order, L2-resident),
// and issues mb x nb v_mfma_f32_16x16x32_bf16.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sur_infer.hpp"

namespace pxd {
namespace sur {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;  // waves per trunk workgroup
constexpr int kMB = 5;     // most row tiles per wave task (column tiles per task: 2)
constexpr int kHeadFT = 8;       // frequency tiles (16 each) per head pass

// FP32 -> BF16 bits, round to nearest even (v_cvt_pk_bf16_f32)
__device__ __forceinline__ unsigned short bf16_bits(float f) { return __builtin_bit_cast(unsigned short, (__bf16)f); }

// two FP32 -> packed BF16 (low half first)
__device__ __forceinline__ unsigned bf16_pair(float lo, float hi) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  const bf16x2 v = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(unsigned, v);
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

// floor(i / d) with m = ceil(2^20 / d), exact for 0 <= i < 4096 and
// 2 <= d <= 64 (the error i (m - 2^20 / d) / 2^20 stays below 1 / d), and for
// i < 2048 when d = 1 (the product stays below 2^31)
__device__ __forceinline__ int div_small(int i, int m) { return (i * m) >> 20; }

// Zero the one-pixel border of an H x W buffer (pixel stride cs, row stride rs).
__device__ void zero_border(unsigned short* lds, int off, int H, int W, int cs, int rs, int tid) {
  const int cpp = cs >> 3, npix = 2 * (W + 2) + 2 * H;
  for (int pix = tid; pix < npix; pix += 64 * kWaves) {
    int y, x;
    if (pix < W + 2) {
      y = 0, x = pix;
    } else if (pix < 2 * (W + 2)) {
      y = H + 1, x = pix - (W + 2);
    } else {
      const int r = pix - 2 * (W + 2);
      y = 1 + (r >> 1), x = (r & 1) ? W + 1 : 0;
    }
    for (int c = 0; c < cpp; ++c) *reinterpret_cast<uint4*>(lds + off + y * rs + x * cs + 8 * c) = make_uint4(0, 0, 0, 0);
  }
}

struct TrunkArgs {
  InferLayer l[4];
  const uint8_t* maps;
  int n_layers, n_cells, m_w, zero_off;
  const uint4* frag;
  const float* bias[4];
  unsigned short* a4;  // BF16 [B][H/4][W/4][channels[3]]
};

// One convolution layer of one map, all waves of the workgroup.  The task
// shape is compile-time: KS k steps (9 x 8, 32 or 64 padded input channels),
// MB row tiles, two column tiles, so the k loop is unrolled with no branch
// around a load or an MFMA.  The weight fragments of up to nine steps sit in
// registers: loaded once per column group when the whole layer fits, else
// per half of the k range.  A partial last chunk of row tiles repeats its
// last tile (the repeat is not stored); padding taps read a zero chunk.
template <int KS, int MB>
__device__ __forceinline__ void conv_layer(const InferLayer& L, const uint4* __restrict__ wf,
                                           const float* __restrict__ bias, unsigned short* lds, int zero_off,
                                           unsigned short* __restrict__ a4_map, bool last, int wave, int lane) {
  constexpr int NB = 2;
  constexpr int KH = KS > 9 ? 9 : KS;                          // k steps whose weights are held at once
  constexpr int CSH = KS == 3 ? 3 : (KS == 9 ? 5 : 6);         // log2 of the padded input channels
  constexpr bool PAD = 32 * KS > 9 * (1 << CSH);               // steps reach past the nine taps
  static_assert(KS % KH == 0 && (KS == 3 || KS == 9 || KS == 18), "k steps");
  const int wt = L.W >> 2, T = (L.H >> 2) * wt;
  const int nch = (T + MB - 1) / MB, ngr = L.nt / NB;
  const int r = lane & 15, q = lane >> 4;
  bf16x8 bw[KH][NB];
  int loaded = -1;
  for (int task = wave; task < nch * ngr; task += kWaves) {
    const int gi = div_small(task, L.m_nch), t0 = (task - gi * nch) * MB, n0 = gi * NB;
    if (KS != KH || n0 != loaded) {
#pragma unroll
      for (int h = 0; h < KH; ++h)
#pragma unroll
        for (int n = 0; n < NB; ++n) bw[h][n] = as_bf16x8(wf[((size_t)(n0 + n) * KS + h) * 64 + lane]);
      loaded = n0;
    }
    // A row r of tile t is pixel (4 by + r / 4, 4 bx + r % 4); lanes q take channels 8 q .. + 7
    int abase[MB];
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      const int t = min(t0 + m, T - 1);
      const int by = div_small(t, L.m_wt), bx = t - by * wt;
      abase[m] = L.in_off + (4 * by + (r >> 2) + 1) * L.in_rs + (4 * bx + (r & 3) + 1) * L.in_cs +
                 (CSH >= 5 ? 8 * q : 0);
    }
    float bcol[NB];  // the columns' biases, read before the products so the epilogue does not wait on them
#pragma unroll
    for (int n = 0; n < NB; ++n) bcol[n] = bias[16 * (n0 + n) + r];
    __builtin_amdgcn_sched_barrier(0);  // keep these loads ahead of the products
    f4 acc[MB][NB];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int n = 0; n < NB; ++n) acc[m][n] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < KS / KH; ++c) {
      if (c > 0) {  // second half of an 18-step layer
#pragma unroll
        for (int h = 0; h < KH; ++h)
#pragma unroll
          for (int n = 0; n < NB; ++n) bw[h][n] = as_bf16x8(wf[((size_t)(n0 + n) * KS + c * KH + h) * 64 + lane]);
        loaded = -1;
      }
      // A fragments of step h + 1 are read while the MFMAs of step h run
      uint4 acur[MB], anext[MB];
      auto load_a = [&](uint4(&dst)[MB], int s) {
        // k = 32 s + 8 q .. + 7 is one tap and eight consecutive (padded) channels
        int toff;
        bool ok = true;
        if constexpr (CSH >= 5) {  // the tap and channel base are the same for every lane
          const int tap = (32 * s) >> CSH, ty = tap / 3, tx = tap - 3 * ty;
          toff = (ty - 1) * L.in_rs + (tx - 1) * L.in_cs + ((32 * s) & ((1 << CSH) - 1));
        } else {  // eight channels per tap: lane group q takes tap 4 s + q
          const int tap = 4 * s + q;
          const int ty = (tap * 11) >> 5, tx = tap - 3 * ty;  // tap / 3 for tap < 12
          if (PAD) ok = tap < 9;
          toff = (ty - 1) * L.in_rs + (tx - 1) * L.in_cs;
        }
#pragma unroll
        for (int m = 0; m < MB; ++m) dst[m] = *reinterpret_cast<const uint4*>(lds + (ok ? abase[m] + toff : zero_off));
      };
      load_a(acur, c * KH);
#pragma unroll
      for (int h = 0; h < KH; ++h) {
        if (h + 1 < KH) load_a(anext, c * KH + h + 1);
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
          for (int n = 0; n < NB; ++n)
            acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(acur[m]), bw[h][n], acc[m][n], 0, 0, 0);
        if (h + 1 < KH) {
#pragma unroll
          for (int m = 0; m < MB; ++m) acur[m] = anext[m];
        }
      }
    }
    // accumulator element i of lane (q, r): pixel (4 by + q, 4 bx + i), channel 16 tile + r
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      if (t0 + m >= T) continue;  // repeated tile
      const int t = t0 + m, by = div_small(t, L.m_wt), bx = t - by * wt;
#pragma unroll
      for (int n = 0; n < NB; ++n) {
        const int col = 16 * (n0 + n) + r;
        const float bc = bcol[n];
        const f4 z = acc[m][n];
        const float v0 = fmaxf(z[0] + bc, 0.0f), v1 = fmaxf(z[1] + bc, 0.0f);
        const float v2 = fmaxf(z[2] + bc, 0.0f), v3 = fmaxf(z[3] + bc, 0.0f);
        if (!L.pool) {
          unsigned short* o = lds + L.out_off + (4 * by + q + 1) * L.out_rs + (4 * bx + 1) * L.out_cs + col;
          o[0] = bf16_bits(v0);
          o[L.out_cs] = bf16_bits(v1);
          o[2 * L.out_cs] = bf16_bits(v2);
          o[3 * L.out_cs] = bf16_bits(v3);
        } else {
          // pixel rows 4 by + q and + 1 sit in lanes q and q ^ 1 (16 apart)
          const float w0 = __shfl_xor(v0, 16), w1 = __shfl_xor(v1, 16);
          const float w2 = __shfl_xor(v2, 16), w3 = __shfl_xor(v3, 16);
          if (!(q & 1)) {
            const float p0 = 0.25f * ((v0 + w0) + (v1 + w1));
            const float p1 = 0.25f * ((v2 + w2) + (v3 + w3));
            const int yo = 2 * by + (q >> 1), xo = 2 * bx;
            unsigned short* o;
            int step;
            if (last) {  // NHWC, no border: the head's input row of this map
              o = a4_map + ((size_t)yo * (L.W >> 1) + xo) * L.cout + col;
              step = L.cout;
            } else {
              o = lds + L.out_off + (yo + 1) * L.out_rs + (xo + 1) * L.out_cs + col;
              step = L.out_cs;
            }
            o[0] = bf16_bits(p0);
            o[step] = bf16_bits(p1);
          }
        }
      }
    }
  }
}

template <int KS>
__device__ __forceinline__ void conv_mb(const InferLayer& L, const uint4* wf, const float* bias, unsigned short* lds,
                                        int zero_off, unsigned short* a4_map, bool last, int wave, int lane) {
  switch (L.mb) {
    case 1: conv_layer<KS, 1>(L, wf, bias, lds, zero_off, a4_map, last, wave, lane); break;
    case 2: conv_layer<KS, 2>(L, wf, bias, lds, zero_off, a4_map, last, wave, lane); break;
    case 3: conv_layer<KS, 3>(L, wf, bias, lds, zero_off, a4_map, last, wave, lane); break;
    case 4: conv_layer<KS, 4>(L, wf, bias, lds, zero_off, a4_map, last, wave, lane); break;
    default: conv_layer<KS, 5>(L, wf, bias, lds, zero_off, a4_map, last, wave, lane); break;
  }
}

__global__ __launch_bounds__(64 * kWaves) void k_trunk(TrunkArgs p) {
  extern __shared__ __align__(16) unsigned short lds[];
  const int b = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int zero_off = p.zero_off;  // a 16-byte zero chunk after the two regions
  if (tid == 0) *reinterpret_cast<uint4*>(lds + zero_off) = make_uint4(0, 0, 0, 0);
  // input planes -> layer 0's buffer (eight channels, the first n_layers used)
  {
    const InferLayer& L = p.l[0];
    const uint8_t* mp = p.maps + (size_t)b * p.n_cells;
    const int hw = L.H * L.W;
    for (int i = tid; i < hw; i += 64 * kWaves) {
      const int y = div_small(i, p.m_w), x = i - y * L.W;
      unsigned short v[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) v[c] = (c < p.n_layers && mp[(size_t)c * hw + i]) ? 0x3F80 : 0;  // BF16 1.0
      uint4 w;
      w.x = v[0] | ((unsigned)v[1] << 16);
      w.y = v[2] | ((unsigned)v[3] << 16);
      w.z = v[4] | ((unsigned)v[5] << 16);
      w.w = v[6] | ((unsigned)v[7] << 16);
      *reinterpret_cast<uint4*>(lds + L.in_off + (y + 1) * L.in_rs + (x + 1) * L.in_cs) = w;
    }
    zero_border(lds, L.in_off, L.H, L.W, L.in_cs, L.in_rs, tid);
  }
  __syncthreads();
  unsigned short* a4_map = p.a4 + (size_t)b * (p.l[3].H >> 1) * (p.l[3].W >> 1) * p.l[3].cout;
#pragma unroll 1
  for (int li = 0; li < 4; ++li) {
    const InferLayer& L = p.l[li];
    if (li < 3) {
      const int ho = L.pool ? L.H >> 1 : L.H, wo = L.pool ? L.W >> 1 : L.W;
      zero_border(lds, L.out_off, ho, wo, L.out_cs, L.out_rs, tid);
    }
    const uint4* wf = p.frag + (size_t)L.frag * 64;
    switch (L.ks) {  // 9 x (8, 32, 64) padded input channels in 32-deep steps
      case 3: conv_mb<3>(L, wf, p.bias[li], lds, zero_off, a4_map, li == 3, wave, lane); break;
      case 9: conv_mb<9>(L, wf, p.bias[li], lds, zero_off, a4_map, li == 3, wave, lane); break;
      default: conv_mb<18>(L, wf, p.bias[li], lds, zero_off, a4_map, li == 3, wave, lane); break;
    }
    __syncthreads();
  }
}

// Weight fragments: fragment (column tile j, k step s), lane (q, r) holds
// W[k][16 j + r] for k = 32 s + 8 q .. + 7, where k = tap 2^sh + c and the
// source is w[(tap cin + c) cout + n] (zero outside tap < taps, c < cin, n < cout);
// sh = 31 makes k the source row itself.
__global__ void k_pack(const float* __restrict__ w, int taps, int cin, int sh, int cout, int nt, int ks,
                       uint4* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nt * ks * 64) return;
  const int lane = i & 63, fr = i >> 6;
  const int j = fr / ks, s = fr - j * ks;
  const int n = 16 * j + (lane & 15), k0 = 32 * s + 8 * (lane >> 4);
  unsigned short v[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int k = k0 + e, tap = k >> sh, c = k & ((1 << sh) - 1);
    v[e] = (tap < taps && c < cin && n < cout) ? bf16_bits(w[((size_t)tap * cin + c) * cout + n]) : 0;
  }
  uint4 o;
  o.x = v[0] | ((unsigned)v[1] << 16);
  o.y = v[2] | ((unsigned)v[3] << 16);
  o.z = v[4] | ((unsigned)v[5] << 16);
  o.w = v[6] | ((unsigned)v[7] << 16);
  dst[i] = o;
}

// First head layer without its bias: U = a4 Wf, rows the maps, k the
// features in NHWC order, columns the hidden units.  A wave takes 16 maps x
// kUNT column tiles; the four waves of a block take four consecutive map
// tiles of the same columns, so their weight fragments are shared in L1.  The
// k loop runs in stages of kUC steps with the next stage's loads in flight.
constexpr int kUNT = 2, kUC = 4;
__global__ __launch_bounds__(256) void k_head_u(int B, int feat, int ks, int nt, const unsigned short* __restrict__ a4,
                                                const uint4* __restrict__ wf, float* __restrict__ U) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ngr = nt / kUNT;  // nt is even (hidden a power of two >= 32)
  const int g = blockIdx.x % ngr, mt = (blockIdx.x / ngr) * 4 + wave;
  if (16 * mt >= B) return;  // whole waves leave together
  const int r = lane & 15, q = lane >> 4;
  // lane (q, r): map 16 mt + r, k = 32 s + 8 q .. + 7
  const uint4* arow = reinterpret_cast<const uint4*>(a4 + (size_t)min(16 * mt + r, B - 1) * feat) + q;
  const uint4* wcol = wf + (size_t)kUNT * g * ks * 64 + lane;  // fragment (kUNT g + n, s) at (n ks + s) 64
  f4 acc[kUNT];
#pragma unroll
  for (int n = 0; n < kUNT; ++n) acc[n] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  uint4 A0[kUC], B0[kUC][kUNT], A1[kUC], B1[kUC][kUNT];
  auto load = [&](uint4(&A)[kUC], uint4(&Bw)[kUC][kUNT], int s0) {
#pragma unroll
    for (int h = 0; h < kUC; ++h) {
      A[h] = arow[4 * (s0 + h)];
#pragma unroll
      for (int n = 0; n < kUNT; ++n) Bw[h][n] = wcol[((size_t)n * ks + s0 + h) * 64];
    }
  };
  auto mul = [&](const uint4(&A)[kUC], const uint4(&Bw)[kUC][kUNT]) {
#pragma unroll
    for (int h = 0; h < kUC; ++h)
#pragma unroll
      for (int n = 0; n < kUNT; ++n)
        acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(A[h]), as_bf16x8(Bw[h][n]), acc[n], 0, 0, 0);
  };
  const int nc = ks / kUC;  // ks is a multiple of 4: (H / 4) (W / 4) is
  load(A0, B0, 0);
  for (int c = 0; c < nc; c += 2) {
    if (c + 1 < nc) load(A1, B1, (c + 1) * kUC);
    mul(A0, B0);
    if (c + 2 < nc) load(A0, B0, (c + 2) * kUC);
    if (c + 1 < nc) mul(A1, B1);
  }
  const int hd = 16 * nt;
#pragma unroll
  for (int n = 0; n < kUNT; ++n) {
    const int col = 16 * (kUNT * g + n) + r;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = 16 * mt + 4 * q + i;
      if (m < B) U[(size_t)m * hd + col] = acc[n][i];
    }
  }
}

// Head output layer, one wave per map: rows are frequencies (16 per MFMA
// tile), k the hidden units, columns the outputs (one 16-wide tile); the
// hidden activations relu((U[b] + V[f]) + bh) are formed in registers.
__global__ __launch_bounds__(256) void k_head(int B, int F, int hd, int ks, int n_out, const float* __restrict__ U,
                                              const float* __restrict__ V, const float* __restrict__ bh,
                                              const uint4* __restrict__ wf, const float* __restrict__ bo,
                                              float* __restrict__ out) {
  const int lane = threadIdx.x & 63, b = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= B) return;  // whole waves leave together
  const int r = lane & 15, q = lane >> 4;
  for (int f0 = 0; f0 < F; f0 += 16 * kHeadFT) {
    f4 acc[kHeadFT];
#pragma unroll
    for (int t = 0; t < kHeadFT; ++t) acc[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int s = 0; s < ks; ++s) {
      const int k = 32 * s + 8 * q;
      const bf16x8 w = as_bf16x8(wf[(size_t)s * 64 + lane]);
      const float4 u0 = *reinterpret_cast<const float4*>(U + (size_t)b * hd + k);
      const float4 u1 = *reinterpret_cast<const float4*>(U + (size_t)b * hd + k + 4);
      float c[8];  // the parameter vector need not be 16-byte aligned
#pragma unroll
      for (int e = 0; e < 8; ++e) c[e] = bh[k + e];
#pragma unroll
      for (int t = 0; t < kHeadFT; ++t) {  // rows past F are zero and not stored
        const int f = f0 + 16 * t + r;
        const float* vr = V + (size_t)min(f, F - 1) * hd + k;
        const float4 v0 = *reinterpret_cast<const float4*>(vr);
        const float4 v1 = *reinterpret_cast<const float4*>(vr + 4);
        uint4 a;
        a.x = bf16_pair(fmaxf((u0.x + v0.x) + c[0], 0.0f), fmaxf((u0.y + v0.y) + c[1], 0.0f));
        a.y = bf16_pair(fmaxf((u0.z + v0.z) + c[2], 0.0f), fmaxf((u0.w + v0.w) + c[3], 0.0f));
        a.z = bf16_pair(fmaxf((u1.x + v1.x) + c[4], 0.0f), fmaxf((u1.y + v1.y) + c[5], 0.0f));
        a.w = bf16_pair(fmaxf((u1.z + v1.z) + c[6], 0.0f), fmaxf((u1.w + v1.w) + c[7], 0.0f));
        if (f >= F) a = make_uint4(0, 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a), w, acc[t], 0, 0, 0);
      }
    }
    // element i of lane (q, r): frequency f0 + 16 t + 4 q + i, output r
    if (r < n_out) {
      const float bias = bo[r];
#pragma unroll
      for (int t = 0; t < kHeadFT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int f = f0 + 16 * t + 4 * q + i;
          if (f < F) out[((size_t)b * F + f) * n_out + r] = acc[t][i] + bias;
        }
    }
  }
}

// Pixel stride: an odd number of 16-byte chunks; row stride 4 (mod 16) chunks.
void buffer_layout(int H, int W, int C, int* cs, int* rs, int* elems) {
  int c8 = (C + 7) / 8;
  if (c8 % 2 == 0) ++c8;
  int rc = (W + 2) * c8;
  rc += ((4 - rc) % 16 + 16) % 16;
  *cs = 8 * c8;
  *rs = 8 * rc;
  *elems = (H + 2) * *rs;
}

int magic(int d) { return ((1 << 20) + d - 1) / d; }

int log2_exact(int v) {
  int s = 0;
  while ((1 << s) < v) ++s;
  return (1 << s) == v ? s : -1;
}

// Row tiles per task: the fewest rounds of tasks over the waves times the
// task length, ties to the longer task (fewer weight loads).
int pick_mb(int T, int ngr) {
  int best = 1, best_cost = 1 << 30;
  for (int mb = 1; mb <= kMB; ++mb) {
    const int tasks = (T + mb - 1) / mb * ngr;
    const int cost = (tasks + kWaves - 1) / kWaves * mb;
    if (cost <= best_cost) best = mb, best_cost = cost;
  }
  return best;
}

}  // namespace

InferPlan infer_plan(int n_layers, int ny, int nx, const int channels[4], int hidden, int n_out) {
  InferPlan p;
  if (n_layers < 1 || n_layers > 8 || ny % 8 || nx % 8 || ny < 8 || nx < 8) return p;
  for (int i = 0; i < 4; ++i) {
    const int c = channels[i];
    if (c != 32 && c != 64) return p;
  }
  if (hidden < 32 || log2_exact(hidden) < 0 || n_out < 1 || n_out > 16) return p;
  p.L = n_layers, p.H = ny, p.W = nx;
  const int cin[4] = {8, channels[0], channels[1], channels[2]};
  int frag = 0;
  // buffers: in0 (H x W x 8), a1 (H x W x c1), a2 (H/2 x W/2 x c2), a3 (H/2 x W/2 x c3)
  int cs[4], rs[4], el[4];
  buffer_layout(ny, nx, 8, &cs[0], &rs[0], &el[0]);
  buffer_layout(ny, nx, channels[0], &cs[1], &rs[1], &el[1]);
  buffer_layout(ny / 2, nx / 2, channels[1], &cs[2], &rs[2], &el[2]);
  buffer_layout(ny / 2, nx / 2, channels[2], &cs[3], &rs[3], &el[3]);
  // region A (a1, then a3) at 0, region B (in0, then a2) after it
  const int regA = std::max(el[1], el[3]), regB = std::max(el[0], el[2]);
  const int off[4] = {regA, 0, regA, 0};
  p.zero_off = regA + regB;
  p.lds_bytes = 2 * (regA + regB) + 16;
  if (p.lds_bytes > 160 * 1024) return p;
  for (int i = 0; i < 4; ++i) {
    InferLayer& L = p.l[i];
    L.H = i < 2 ? ny : ny / 2;
    L.W = i < 2 ? nx : nx / 2;
    L.cin = i == 0 ? n_layers : channels[i - 1];
    L.cin_sh = log2_exact(cin[i]);
    L.cout = channels[i];
    L.nt = channels[i] / 16;
    L.ks = (9 * cin[i] + 31) / 32;
    L.in_off = off[i], L.in_cs = cs[i], L.in_rs = rs[i];
    if (i < 3) L.out_off = off[i + 1], L.out_cs = cs[i + 1], L.out_rs = rs[i + 1];
    L.pool = (i == 1 || i == 3);
    L.nb = 2;
    const int T = (L.H / 4) * (L.W / 4);
    L.mb = pick_mb(T, L.nt / 2);
    L.m_wt = magic(L.W / 4);
    L.m_nch = magic((T + L.mb - 1) / L.mb);
    L.frag = frag;
    frag += L.nt * L.ks;
  }
  p.feat = (ny / 4) * (nx / 4) * channels[3];
  p.ks_u = p.feat / 32;
  p.u_frag = frag;
  frag += (hidden / 16) * p.ks_u;
  p.hidden = hidden, p.ks_head = hidden / 32, p.n_out = n_out;
  p.head_frag = frag;
  p.n_frag = frag + p.ks_head;
  p.ok = true;
  return p;
}

hipError_t infer_pack(hipStream_t st, const InferPlan& p, const float* const conv_w[4], const float* wf,
                      const float* wo, void* frag) {
  uint4* f = static_cast<uint4*>(frag);
  for (int i = 0; i < 4; ++i) {
    const InferLayer& L = p.l[i];
    const int n = L.nt * L.ks * 64;
    hipLaunchKernelGGL(k_pack, dim3((n + 255) / 256), dim3(256), 0, st, conv_w[i], 9, L.cin, L.cin_sh, L.cout, L.nt,
                       L.ks, f + (size_t)L.frag * 64);
  }
  const int nu = (p.hidden / 16) * p.ks_u * 64;
  hipLaunchKernelGGL(k_pack, dim3((nu + 255) / 256), dim3(256), 0, st, wf, 1, p.feat, 31, p.hidden, p.hidden / 16,
                     p.ks_u, f + (size_t)p.u_frag * 64);
  const int n = p.ks_head * 64;
  hipLaunchKernelGGL(k_pack, dim3((n + 255) / 256), dim3(256), 0, st, wo, 1, p.hidden, log2_exact(p.hidden), p.n_out,
                     1, p.ks_head, f + (size_t)p.head_frag * 64);
  return hipGetLastError();
}

hipError_t infer_prepare(const InferPlan& p) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k_trunk), hipFuncAttributeMaxDynamicSharedMemorySize,
                             p.lds_bytes);
}

hipError_t infer_trunk(hipStream_t st, const InferPlan& p, int B, const uint8_t* maps, int n_cells, const void* frag,
                       const float* const bias[4], void* a4) {
  if (B <= 0) return hipSuccess;
  TrunkArgs a;
  for (int i = 0; i < 4; ++i) a.l[i] = p.l[i], a.bias[i] = bias[i];
  a.maps = maps, a.n_layers = p.L, a.n_cells = n_cells, a.m_w = magic(p.W), a.zero_off = p.zero_off;
  a.frag = static_cast<const uint4*>(frag);
  a.a4 = static_cast<unsigned short*>(a4);
  hipLaunchKernelGGL(k_trunk, dim3(B), dim3(64 * kWaves), p.lds_bytes, st, a);
  return hipGetLastError();
}

hipError_t infer_u(hipStream_t st, const InferPlan& p, int B, const void* a4, const void* frag, float* U) {
  if (B <= 0) return hipSuccess;
  const int nt = p.hidden / 16, ngr = (nt + kUNT - 1) / kUNT, mtiles = (B + 15) / 16;
  hipLaunchKernelGGL(k_head_u, dim3((mtiles + 3) / 4 * ngr), dim3(256), 0, st, B, p.feat, p.ks_u, nt,
                     static_cast<const unsigned short*>(a4), static_cast<const uint4*>(frag) + (size_t)p.u_frag * 64,
                     U);
  return hipGetLastError();
}

hipError_t infer_head(hipStream_t st, const InferPlan& p, int B, int F, const float* U, const float* V,
                      const float* bh, const void* frag, const float* bo, float* out) {
  if (B <= 0 || F <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_head, dim3((B + 3) / 4), dim3(256), 0, st, B, F, p.hidden, p.ks_head, p.n_out, U, V, bh,
                     static_cast<const uint4*>(frag) + (size_t)p.head_frag * 64, bo, out);
  return hipGetLastError();
}

}  // namespace sur
}  // namespace pxd
