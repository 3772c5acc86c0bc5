// Device-side helpers for gfx950: complex arithmetic on interleaved pairs,
// wave reductions and MFMA wrappers.
#pragma once

#include <hip/hip_runtime.h>

namespace pxd {

constexpr int kThreads = 256;  // workgroup size of the evaluator (4 waves of 64)
constexpr int kWaves = kThreads / 64;

template <typename R>
struct Cx;
template <>
struct Cx<double> {
  using T = double2;
};
template <>
struct Cx<float> {
  using T = float2;
};

template <typename T>
__device__ __forceinline__ T cmul(T a, T b) {
  return T{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ T csub(T a, T b) {
  return T{a.x - b.x, a.y - b.y};
}
template <typename T>
__device__ __forceinline__ T cadd(T a, T b) {
  return T{a.x + b.x, a.y + b.y};
}
// a - b*c
template <typename T>
__device__ __forceinline__ T cfms(T a, T b, T c) {
  return T{a.x - (b.x * c.x - b.y * c.y), a.y - (b.x * c.y + b.y * c.x)};
}
// 1 / a (exactly-zero input gives zero; the caller flags it)
template <typename T>
__device__ __forceinline__ T crecip(T a) {
  auto d = a.x * a.x + a.y * a.y;
  if (d == 0) return T{0, 0};
  return T{a.x / d, -a.y / d};
}

// (value, index) arg-max over a wave; ties resolve to the smaller index.
template <typename R>
__device__ __forceinline__ void wave_argmax(R& v, int& i) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    R ov = __shfl_xor(v, off, 64);
    int oi = __shfl_xor(i, off, 64);
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
}

typedef double dx4 __attribute__((ext_vector_type(4)));
typedef float fx4 __attribute__((ext_vector_type(4)));

// 16x16x4 MFMA: A operand lane l holds A[l % 16][l / 16]; B operand lane l
// holds B[l / 16][l % 16].  Accumulator element i of lane l is
//   f64: row 4*i + l/16, column l % 16
//   f32: row 4*(l/16) + i, column l % 16
template <typename R>
struct Mfma;
template <>
struct Mfma<double> {
  using acc_t = dx4;
  static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * i + (lane >> 4); }
};
template <>
struct Mfma<float> {
  using acc_t = fx4;
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

}  // namespace pxd
