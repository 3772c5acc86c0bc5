// gfx950 kernels of the per-candidate evaluation.
//
//  expand   : candidate map -> ascending active index set (Eqs. 3-4, Section II-C)
//  order    : candidates by decreasing active size (largest first)
//  eval     : persistent workgroups; per (candidate, frequency) item:
//             gather Z_A = Z_f[I, I] (Eq. 5) with the port loads and the
//             excitation columns, blocked LU with partial pivoting (Eq. 2),
//             S-parameters from the port currents (Eqs. 6-7)
//  fom      : Eqs. 8-9 reduced over frequency, one thread per candidate
//  argmin   : lowest-index minimum (Algorithm 1)
//
// LU layout: each workgroup owns one workspace slot holding the item's
// matrix row-major (leading dimension ld).  The active functions keep their
// parent order, so the P port functions are the last P unknowns.  Eliminating
// the first N-P columns of the augmented [Z_A | V] leaves the P x P Schur
// system of the port unknowns, which is solved directly: no back substitution
// and no storage of L or U is needed for the FP64 path.
//
// Panel factorisation: panels of NB = 32 columns, factored in sub-blocks of
// SB columns held in registers (Q rows per thread, N <= 256 Q, Q SB <= 16 for
// complex128 and <= 32 for complex64); the pivot
// search is a wave shuffle reduction plus one LDS exchange per column.  Row
// interchanges are applied to the trailing columns lazily, fused with the
// triangular solve of the U block.  The trailing update A22 -= L21 U12 is a
// complex GEMM made of four real 16x16x4 MFMAs per complex product; each
// wave owns 32 x 32 output tiles and keeps its L21 fragments in registers
// across a run of tiles of the same block row.
#include "device.hpp"
#include "kernels.hpp"
#include "lu_device.hpp"

// lu_solve_c64 replays a block column's interchanges from a table of this size
static_assert(pxd::kTlKbMax <= pxd::kTlKbMaxSolve && pxd::KB_MIXED <= pxd::kTlKbMaxSolve,
              "block columns wider than the solve's pivot table");

namespace pxd {

// ------------------------------------------------------------------ expand

__global__ __launch_bounds__(256) void k_expand(const uint8_t* __restrict__ base, int n_cells, size_t base_stride,
                                                const int* __restrict__ off, const int* __restrict__ cells,
                                                const int* __restrict__ cell_a, const int* __restrict__ cell_b,
                                                int M, int* __restrict__ Nc, int* __restrict__ Ilist) {
  extern __shared__ uint8_t smap[];
  __shared__ int wave_tot[4];
  const int c = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const uint8_t* cmap = base + (size_t)c * base_stride;  // stride 0: one base map for every candidate
  for (int i = tid; i < n_cells; i += 256) smap[i] = cmap[i] ? 1 : 0;
  __syncthreads();
  if (tid == 0 && off)  // no flip list: the candidate is its own map
    for (int i = off[c]; i < off[c + 1]; ++i) {
      const int cell = cells[i];
      if (cell >= 0 && cell < n_cells) smap[cell] ^= 1;
    }
  __syncthreads();
  int running = 0;
  int* out = Ilist + (size_t)c * M;
  for (int m0 = 0; m0 < M; m0 += 256) {
    const int m = m0 + tid;
    bool on = false;
    if (m < M) {
      const int a = cell_a[m], b = cell_b[m];
      on = (a < 0 || smap[a]) && (b < 0 || smap[b]);
    }
    const unsigned long long mask = __ballot(on);
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wave_tot[wid] = __popcll(mask);
    __syncthreads();
    int pre = running;
    for (int w = 0; w < wid; ++w) pre += wave_tot[w];
    if (on) out[pre + before] = m;
    running += wave_tot[0] + wave_tot[1] + wave_tot[2] + wave_tot[3];
    __syncthreads();
  }
  if (tid == 0) Nc[c] = running;
}

// rank of candidate c when sorted by decreasing N, ties by index
__global__ void k_order(const int* __restrict__ Nc, int C, int* __restrict__ order) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const int n = Nc[c];
  int rank = 0;
  for (int j = 0; j < C; ++j) {
    const int nj = Nc[j];
    rank += (nj > n) || (nj == n && j < c);
  }
  order[rank] = c;
}

// out[0] = min, out[1] = max of v[0 .. n), one workgroup
__global__ __launch_bounds__(256) void k_minmax(const int* __restrict__ v, int n, int* __restrict__ out) {
  __shared__ int lo[256], hi[256];
  const int tid = threadIdx.x;
  int a = 0x7fffffff, b = -0x7fffffff - 1;
  for (int i = tid; i < n; i += 256) a = min(a, v[i]), b = max(b, v[i]);
  lo[tid] = a, hi[tid] = b;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) lo[tid] = min(lo[tid], lo[tid + st]), hi[tid] = max(hi[tid], hi[tid + st]);
    __syncthreads();
  }
  if (tid == 0) out[0] = lo[0], out[1] = hi[0];
}

__global__ void k_fill_int(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ gather

__global__ void k_gather(const double2* __restrict__ Zf, int M, const int* __restrict__ idx, int N,
                         double2* __restrict__ out) {
  const int r = blockIdx.x;
  if (r >= N) return;
  const double2* zrow = Zf + (size_t)idx[r] * M;
  for (int s = threadIdx.x; s < N; s += blockDim.x) out[(size_t)r * N + s] = zrow[idx[s]];
}

__global__ void k_to_c64(const double2* __restrict__ in, float2* __restrict__ out, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double2 v = in[i];
    out[i] = float2{(float)v.x, (float)v.y};
  }
}

// ------------------------------------------------------------------ evaluator (FP64)

// Item index -> (candidate, frequency).  Frequency-major: all candidates of
// one frequency (largest first) before the next frequency, so concurrent
// workgroups gather from the same parent.  Size-major: all frequencies of the
// largest candidate first (longest-processing-time order for uneven batches).
__device__ __forceinline__ void decode_item(const EvalParams& p, int it, int& c, int& f) {
  if (p.item_list) {
    const int e = p.item_list[it];
    c = e / p.F;
    f = e - c * p.F;
  } else if (p.schedule == PXD_SCHED_SIZE_MAJOR) {
    const int r = it / p.F;
    f = it - r * p.F;
    c = p.order[r];
  } else {
    f = it / p.C;
    c = p.order[it - f * p.C];
  }
}

template <int Q, int SB>
__global__ __launch_bounds__(kThreads, 2) void k_eval_plain(EvalParams p) {
  using T = double2;
  __shared__ LuShared<double> sm;
  __shared__ int sI[kThreads * Q];
  __shared__ int s_item;
  const int tid = threadIdx.x;
  const int ld = p.ld;
  const int n_items = p.n_items_dev ? *p.n_items_dev : p.n_items;
  T* W = reinterpret_cast<T*>(p.ws + (size_t)blockIdx.x * p.slot_bytes);
  for (;;) {
    if (tid == 0) s_item = atomicAdd(p.counter, 1);
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= n_items) break;
    int c, f;
    decode_item(p, it, c, f);
    const int N = p.Nc[c];
    double2* Sout = p.S + ((size_t)c * p.F + f) * p.P * p.P;
    if (N > kThreads * Q || N > p.nmax || N < p.P) {  // outside the size the launch was built for
      // no solve: S is marked not-a-number and the status makes the FoM +inf
      if (tid < p.P * p.P) Sout[tid] = double2{__builtin_nan(""), __builtin_nan("")};
      if (tid == 0) p.status[(size_t)c * p.F + f] = PXD_STATUS_SIZE;
      continue;
    }
    for (int s = tid; s < N; s += kThreads) sI[s] = p.Ilist[(size_t)c * p.M + s];
    if (tid == 0) sm.bad = 0;
    __syncthreads();
    gather_item<T, double2>(W, ld, p.Z128 + (size_t)f * p.M * p.M, p.M, sI, N, p.P, p.port_len, p.z0, true);
    lu_factor<double, Q, SB, KB_PLAIN, 1>(W, ld, N, N - p.P, N + p.P, sm, nullptr);
    int st = port_solve_and_s(W, ld, N, p.P, p.port_len, p.z0, Sout);
    if (tid == 0) {
      if (sm.bad && st == PXD_STATUS_OK) st = PXD_STATUS_SINGULAR;
      if (p.fallback_mode && st == PXD_STATUS_OK) st = PXD_STATUS_FALLBACK;
      p.status[(size_t)c * p.F + f] = st;
    }
    __syncthreads();
  }
}


// ------------------------------------------------------------------ base inverse

// G_f = Z_B(f)^-1 of the base map's active set (port loads included), one
// item per frequency: [Z_B | I] is factored with the two-level LU over all N
// columns, then U X = (L^-1 P) is solved upwards, one thread per column of X
// in blocks of 8 rows, and X is written to G (F x N x N, row-major; Z_B is
// symmetric, so G is too).
template <int Q, int SB>
__global__ __launch_bounds__(kThreads, 2) void k_base_inverse(InvParams p) {
  using T = double2;
  __shared__ LuShared<double> sm;
  __shared__ int sI[kThreads * Q];
  __shared__ int s_item;
  const int tid = threadIdx.x;
  const int N = p.N, ld = p.ld;
  T* W = reinterpret_cast<T*>(p.ws + (size_t)blockIdx.x * p.slot_bytes);
  for (int s = tid; s < N && s < kThreads * Q; s += kThreads) sI[s] = p.IB[s];
  __syncthreads();
  for (;;) {
    if (tid == 0) s_item = atomicAdd(p.counter, 1);
    __syncthreads();
    const int f = s_item;
    __syncthreads();
    if (f >= p.F) break;
    if (N > kThreads * Q) {
      if (tid == 0) p.status[f] = PXD_STATUS_SIZE;
      continue;
    }
    if (tid == 0) sm.bad = 0;
    const double2* Zf = p.Z128 + (size_t)f * p.M * p.M;
    for (int r = tid >> 6; r < N; r += kWaves) {
      const double2* zrow = Zf + (size_t)sI[r] * p.M;
      for (int c = tid & 63; c < N; c += 64) {
        W[(size_t)r * ld + c] = zrow[sI[c]];
        W[(size_t)r * ld + N + c] = T{(r == c) ? 1.0 : 0.0, 0.0};
      }
    }
    __syncthreads();
    if (tid < p.P) {
      const int r = N - p.P + tid;
      W[(size_t)r * ld + r].x += p.z0 * p.port_len[tid] * p.port_len[tid];
    }
    __syncthreads();
    lu_factor<double, Q, SB, KB_PLAIN, 1>(W, ld, N, N, 2 * N, sm, nullptr);
    constexpr int B = 8;
    for (int col = N + tid; col < 2 * N; col += kThreads) {
      for (int b1 = N; b1 > 0; b1 -= B) {
        const int b0 = max(0, b1 - B), nb = b1 - b0;
        T u[B];
#pragma unroll
        for (int i = 0; i < B; ++i) u[i] = (i < nb) ? W[(size_t)(b0 + i) * ld + col] : T{0, 0};
        for (int j = b1; j < N; ++j) {  // solved rows below the block
          const T xj = W[(size_t)j * ld + col];
#pragma unroll
          for (int i = 0; i < B; ++i)
            if (i < nb) u[i] = cfms(u[i], W[(size_t)(b0 + i) * ld + j], xj);
        }
#pragma unroll
        for (int i = B - 1; i >= 0; --i) {
          if (i < nb) {
#pragma unroll
            for (int jj = i + 1; jj < B; ++jj)
              if (jj < nb) u[i] = cfms(u[i], W[(size_t)(b0 + i) * ld + b0 + jj], u[jj]);
            u[i] = cmul(u[i], crecip(W[(size_t)(b0 + i) * ld + b0 + i]));
          }
        }
#pragma unroll
        for (int i = 0; i < B; ++i)
          if (i < nb) W[(size_t)(b0 + i) * ld + col] = u[i];
      }
    }
    __syncthreads();
    double2* G = p.G + (size_t)f * N * N;
    for (int r = tid >> 6; r < N; r += kWaves)
      for (int c = tid & 63; c < N; c += 64) G[(size_t)r * N + c] = W[(size_t)r * ld + N + c];
    if (tid == 0) p.status[f] = sm.bad ? PXD_STATUS_SINGULAR : PXD_STATUS_OK;
    __syncthreads();
  }
}

hipError_t launch_base_inverse(hipStream_t s, const InvParams& p, int grid) {
  const int Q = rows_per_thread(p.N);
  if (Q <= 1) hipLaunchKernelGGL((k_base_inverse<1, 16>), dim3(grid), dim3(kThreads), 0, s, p);
  else if (Q <= 2) hipLaunchKernelGGL((k_base_inverse<2, 8>), dim3(grid), dim3(kThreads), 0, s, p);
  else if (Q <= 4) hipLaunchKernelGGL((k_base_inverse<4, 4>), dim3(grid), dim3(kThreads), 0, s, p);
  else if (Q <= 8) hipLaunchKernelGGL((k_base_inverse<8, 2>), dim3(grid), dim3(kThreads), 0, s, p);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// Mixed precision item: complex64 LU of Z_A, initial complex64 solve, then
// refinement with FP64 residuals.  After each step the error left in every
// S_ij = delta_ij - 2 Z0 l_i x_ij is bounded by rho / (1 - rho) times the
// largest change the step made to any S entry, rho being the contraction, the
// ratio of the last two largest changes (so at least two steps are taken).
// Each step first forms the FP64 residual and the port corrections it implies
// (port_corrections, no solve); when the stop test passes on those, they are
// applied and the step ends there, otherwise the full correction is solved.
// The stop test: the estimate is below ir_tol |S_ij| + kIrAbsFloor for every
// entry.  Items that do not converge are queued for the FP64 path.
template <int Q, int SB>
__global__ __launch_bounds__(kThreads, 2) void k_eval_mixed(EvalParams p) {
  using T = float2;
  __shared__ LuShared<float> sm;
  __shared__ int s_item;
  extern __shared__ char dyn[];
  int* sI = reinterpret_cast<int*>(dyn);
  float2* b = reinterpret_cast<float2*>(dyn + ((size_t)p.nmax * 4 + 15) / 16 * 16);
  const int tid = threadIdx.x;
  const int ld = p.ld;
  const SlotLayout lay = slot_layout(p.nmax, p.P, true);
  char* slot = p.ws + (size_t)blockIdx.x * p.slot_bytes;
  T* W = reinterpret_cast<T*>(slot + lay.w_off);
  int* piv = reinterpret_cast<int*>(slot + lay.piv_off);
  double2* x = reinterpret_cast<double2*>(slot + lay.x_off);
  const int P = p.P;
  for (;;) {
    if (tid == 0) s_item = atomicAdd(p.counter, 1);
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= p.n_items) break;
    int c, f;
    decode_item(p, it, c, f);
    const int N = p.Nc[c];
    double2* Sout = p.S + ((size_t)c * p.F + f) * P * P;
    if (N > kThreads * Q || N > p.nmax || N < P) {
      if (tid < P * P) Sout[tid] = double2{__builtin_nan(""), __builtin_nan("")};
      if (tid == 0) p.status[(size_t)c * p.F + f] = PXD_STATUS_SIZE;
      continue;
    }
    for (int s = tid; s < N; s += kThreads) sI[s] = p.Ilist[(size_t)c * p.M + s];
    if (tid == 0) sm.bad = 0;
    __syncthreads();
    const double2* Zf128 = p.Z128 + (size_t)f * p.M * p.M;
    gather_item<T, float2>(W, ld, p.Z64 + (size_t)f * p.M * p.M, p.M, sI, N, P, p.port_len, p.z0, false);
    lu_factor<float, Q, SB, KB_MIXED, 2>(W, ld, N, N, N, sm, piv, p.half);
    refine_item(W, ld, N, piv, KB_MIXED, b, sI, x, Zf128, p.M, P, p.port_len, p.z0, p.ir_max, p.ir_tol, sm.bad,
                c * p.F + f, Sout, p.status + (size_t)c * p.F + f, p.ir_iters, p.fb_count, p.fb_list);
    __syncthreads();
  }
}

size_t eval_mixed_lds(int nmax, int P) { return ((size_t)nmax * 4 + 15) / 16 * 16 + (size_t)nmax * P * 8; }

// ------------------------------------------------------------------ FoM and argmin

__global__ void k_fom(const double2* __restrict__ S, int C, int F, int P, const pxd_fom_term* __restrict__ terms,
                      const double* __restrict__ term_fac, int n_terms, const int8_t* __restrict__ band,
                      const int* __restrict__ item_status, double* __restrict__ fom, int* __restrict__ cand_status) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  double acc = 0.0;
  int worst = 0;
  for (int f = 0; f < F; ++f) {
    const int st = item_status[(size_t)c * F + f];
    if (st < 0) worst = (worst < 0) ? min(worst, st) : st;
    else if (worst >= 0) worst = max(worst, st);
    const int b = band[f];
    if (b < 0) continue;
    const double2* s = S + ((size_t)c * F + f) * P * P;
    for (int t = 0; t < n_terms; ++t) {
      if (terms[t].band != b) continue;
      const double2 v = s[terms[t].i * P + terms[t].j];
      const double m2 = fmax(v.x * v.x + v.y * v.y, 1e-30);
      acc += term_fac[t] * pow(m2, 0.5 * terms[t].power);
    }
  }
  // a candidate with any failed item (singular, non-finite, outside the
  // launch's size bound) has no valid S at that frequency: it can never be
  // selected, so its FoM is +inf
  fom[c] = (worst < 0) ? __builtin_inf() : acc;
  if (cand_status) cand_status[c] = worst;
}

__global__ void k_argmin(const double* __restrict__ fom, int C, int* __restrict__ out) {
  __shared__ double sv[256];
  __shared__ int si[256];
  const int tid = threadIdx.x;
  double best = __builtin_inf();
  int bi = 0x7fffffff;
  for (int c = tid; c < C; c += 256) {
    const double v = fom[c];
    if (!(v < __builtin_inf())) continue;  // +inf (failed candidate) or NaN: never selected
    if (v < best || (v == best && c < bi)) best = v, bi = c;
  }
  sv[tid] = best;
  si[tid] = bi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      const double ov = sv[tid + s];
      const int oi = si[tid + s];
      if (ov < sv[tid] || (ov == sv[tid] && oi < si[tid])) sv[tid] = ov, si[tid] = oi;
    }
    __syncthreads();
  }
  if (tid == 0) *out = (si[0] == 0x7fffffff) ? -1 : si[0];  // -1: no candidate has a finite FoM
}

// ------------------------------------------------------------------ launchers

hipError_t launch_expand(hipStream_t s, const uint8_t* base, int n_cells, size_t base_stride, const int* off,
                         const int* cells, int C, const int* cell_a, const int* cell_b, int M, int* Nc, int* Ilist) {
  if (C <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_expand, dim3(C), dim3(256), (size_t)n_cells, s, base, n_cells, base_stride, off, cells, cell_a,
                     cell_b, M, Nc, Ilist);
  return hipGetLastError();
}

hipError_t launch_order(hipStream_t s, const int* Nc, int C, int* order) {
  if (C <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_order, dim3((C + 255) / 256), dim3(256), 0, s, Nc, C, order);
  return hipGetLastError();
}

hipError_t launch_minmax(hipStream_t s, const int* v, int n, int* out) {
  hipLaunchKernelGGL(k_minmax, dim3(1), dim3(256), 0, s, v, n, out);
  return hipGetLastError();
}

hipError_t launch_fill_int(hipStream_t s, int* p, int n, int v) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// Sub-panel width of a variant: the full register budget (Q SB = 16) or half of it.
template <int Q>
constexpr int sb_of(int half) { return half ? (16 / Q > 1 ? 8 / Q : 1) : 16 / Q; }

template <int Q, int SB>
static hipError_t launch_plain_variant(hipStream_t s, const EvalParams& p, int grid) {
  hipLaunchKernelGGL((k_eval_plain<Q, SB>), dim3(grid), dim3(kThreads), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_eval_plain(hipStream_t s, const EvalParams& p, int grid, int half_sb) {
  const int Q = rows_per_thread(p.nmax);
  if (Q <= 1) return half_sb ? launch_plain_variant<1, sb_of<1>(1)>(s, p, grid) : launch_plain_variant<1, sb_of<1>(0)>(s, p, grid);
  if (Q <= 2) return half_sb ? launch_plain_variant<2, sb_of<2>(1)>(s, p, grid) : launch_plain_variant<2, sb_of<2>(0)>(s, p, grid);
  if (Q <= 4) return half_sb ? launch_plain_variant<4, sb_of<4>(1)>(s, p, grid) : launch_plain_variant<4, sb_of<4>(0)>(s, p, grid);
  if (Q <= 8) return half_sb ? launch_plain_variant<8, sb_of<8>(1)>(s, p, grid) : launch_plain_variant<8, sb_of<8>(0)>(s, p, grid);
  return hipErrorInvalidValue;
}

template <int Q, int SB>
static hipError_t prepare_mixed_variant(size_t lds) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_eval_mixed<Q, SB>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int Q, int SB>
static hipError_t launch_mixed_variant(hipStream_t s, const EvalParams& p, int grid, size_t lds) {
  hipLaunchKernelGGL((k_eval_mixed<Q, SB>), dim3(grid), dim3(kThreads), lds, s, p);
  return hipGetLastError();
}

// The complex64 kernel holds twice as many sub-panel columns in the same registers.
template <int Q>
constexpr int msb_of(int half) { return half ? 16 / Q : 32 / Q; }

// Raise the dynamic LDS limit of the mixed kernel variant the launch will use
// (host-side attribute; called outside any stream capture).
hipError_t prepare_eval_mixed(const EvalParams& p, int half_sb) {
  const int Q = rows_per_thread(p.nmax);
  const size_t lds = eval_mixed_lds(p.nmax, p.P);
  if (Q <= 1) return half_sb ? prepare_mixed_variant<1, msb_of<1>(1)>(lds) : prepare_mixed_variant<1, msb_of<1>(0)>(lds);
  if (Q <= 2) return half_sb ? prepare_mixed_variant<2, msb_of<2>(1)>(lds) : prepare_mixed_variant<2, msb_of<2>(0)>(lds);
  if (Q <= 4) return half_sb ? prepare_mixed_variant<4, msb_of<4>(1)>(lds) : prepare_mixed_variant<4, msb_of<4>(0)>(lds);
  if (Q <= 8) return half_sb ? prepare_mixed_variant<8, msb_of<8>(1)>(lds) : prepare_mixed_variant<8, msb_of<8>(0)>(lds);
  return hipErrorInvalidValue;
}

hipError_t launch_eval_mixed(hipStream_t s, const EvalParams& p, int grid, int half_sb) {
  const int Q = rows_per_thread(p.nmax);
  const size_t lds = eval_mixed_lds(p.nmax, p.P);
  if (Q <= 1) return half_sb ? launch_mixed_variant<1, msb_of<1>(1)>(s, p, grid, lds) : launch_mixed_variant<1, msb_of<1>(0)>(s, p, grid, lds);
  if (Q <= 2) return half_sb ? launch_mixed_variant<2, msb_of<2>(1)>(s, p, grid, lds) : launch_mixed_variant<2, msb_of<2>(0)>(s, p, grid, lds);
  if (Q <= 4) return half_sb ? launch_mixed_variant<4, msb_of<4>(1)>(s, p, grid, lds) : launch_mixed_variant<4, msb_of<4>(0)>(s, p, grid, lds);
  if (Q <= 8) return half_sb ? launch_mixed_variant<8, msb_of<8>(1)>(s, p, grid, lds) : launch_mixed_variant<8, msb_of<8>(0)>(s, p, grid, lds);
  return hipErrorInvalidValue;
}

hipError_t launch_fom(hipStream_t s, const double2* S, int C, int F, int P, const pxd_fom_term* terms,
                      const double* term_fac, int n_terms, const int8_t* band, const int* item_status, double* fom,
                      int* cand_status) {
  if (C <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fom, dim3((C + 255) / 256), dim3(256), 0, s, S, C, F, P, terms, term_fac, n_terms, band,
                     item_status, fom, cand_status);
  return hipGetLastError();
}

hipError_t launch_argmin(hipStream_t s, const double* fom, int C, int* argmin) {
  hipLaunchKernelGGL(k_argmin, dim3(1), dim3(256), 0, s, fom, C, argmin);
  return hipGetLastError();
}

hipError_t launch_gather(hipStream_t s, const double2* Zf, int M, const int* idx, int N, double2* out) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather, dim3(N), dim3(256), 0, s, Zf, M, idx, N, out);
  return hipGetLastError();
}

hipError_t launch_to_c64(hipStream_t s, const double2* in, float2* out, size_t n) {
  hipLaunchKernelGGL(k_to_c64, dim3(4096), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

}  // namespace pxd
