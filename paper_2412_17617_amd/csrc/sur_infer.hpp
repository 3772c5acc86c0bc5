// Fused BF16 inference of the CNN surrogate: the four 3x3 convolutions of one
// map (bias, ReLU and the two 2 x 2 average pools included) inside one
// workgroup's LDS, and the head's output layer with its hidden activations
// formed in registers.  The training path's products give the same values up
// to FP32 summation order: operands are rounded to BF16 at the same points
// (every activation and weight that enters a product), sums are FP32.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace pxd {
namespace sur {

// One convolution of the trunk as an implicit GEMM: rows are output pixels in
// 4 x 4 blocks (one 16-row MFMA tile per block), columns output channels in
// 16-wide tiles, k = (tap, input channel) in 32-deep steps.
struct InferLayer {
  int H, W;                      // input = pre-pool output resolution
  int cin, cin_sh;               // input channels; log2 of the padded count
  int cout, nt, ks;              // output channels, column tiles, k steps
  int in_off, in_cs, in_rs;      // input buffer in LDS (elements): base, pixel stride, row stride
  int out_off, out_cs, out_rs;   // output buffer in LDS (not used by the last layer)
  int pool;                      // 2 x 2 average pool after the ReLU
  int mb, nb;                    // row tiles and column tiles per wave task
  int m_wt, m_nch;               // ceil(2^20 / d) for d = W / 4 and the row chunks (division by multiply)
  int frag;                      // first weight fragment (64 lanes x 16 bytes each)
};

struct InferPlan {
  bool ok = false;
  InferLayer l[4];
  int L = 0, H = 0, W = 0;       // map shape
  int lds_bytes = 0;
  int zero_off = 0;              // LDS element offset of a 16-byte zero chunk
  int feat = 0, ks_u = 0;         // head input features (NHWC of the last pooled plane), k steps
  int u_frag = 0;                // first fragment of the head's first-layer weights
  int hidden = 0, ks_head = 0, n_out = 0;
  int head_frag = 0;             // first fragment of the output layer's weights
  int n_frag = 0;                // fragments in all
};

// Layout and task split for a map shape and network; ok = false when the
// fused kernels do not cover it (then the generic products are used).
InferPlan infer_plan(int n_layers, int ny, int nx, const int channels[4], int hidden, int n_out);
// Lets the trunk kernel take the LDS its plans need (current device).
hipError_t infer_prepare(const InferPlan& p);
// Weight fragments (BF16, MFMA operand order) from the FP32 parameters:
// conv_w[l] is [9][cin][cout], wf [feat][hidden], wo [hidden][n_out].
hipError_t infer_pack(hipStream_t st, const InferPlan& p, const float* const conv_w[4], const float* wf,
                      const float* wo, void* frag);
// a4[b] = trunk(maps[b]) as BF16 NHWC (H/4 x W/4 x channels[3]) for B maps.
hipError_t infer_trunk(hipStream_t st, const InferPlan& p, int B, const uint8_t* maps, int n_cells, const void* frag,
                       const float* const bias[4], void* a4);
// U[b] = a4[b] Wf (FP32, B x hidden).
hipError_t infer_u(hipStream_t st, const InferPlan& p, int B, const void* a4, const void* frag, float* U);
// out[b, f, :] = relu((U[b] + V[f]) + bh) Wo + bo for B maps and F frequencies.
hipError_t infer_head(hipStream_t st, const InferPlan& p, int B, int F, const float* U, const float* V,
                      const float* bh, const void* frag, const float* bo, float* out);

}  // namespace sur
}  // namespace pxd
