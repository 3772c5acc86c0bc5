// Launch interface between the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cmath>
#include <cstdint>

#include "pxd.h"

namespace pxd {

// Everything one persistent evaluator launch needs.  All pointers are device
// pointers.
struct EvalParams {
  const double2* Z128;  // F x M x M parent matrices (complex128)
  const float2* Z64;    // F x M x M complex64 copy (mixed precision only)
  int M, F, P, C;
  const int* Nc;        // active size per candidate
  const int* Ilist;     // C x M active indices, ascending
  const int* order;     // candidates sorted by decreasing active size
  const double* port_len;
  double z0;
  int n_items;          // items to process in this launch
  const int* n_items_dev; // if set, the item count is read from device memory instead
  const int* item_list; // explicit items (c * F + f), or null for the implicit frequency-major order
  int fallback_mode;    // FP64 re-solve of items the mixed path could not refine: report FALLBACK
  int* counter;         // persistent work counter (zeroed before the launch)
  char* ws;             // workspace, one slot per workgroup
  size_t slot_bytes;
  int nmax;             // largest active size in the batch
  double2* S;           // C x F x P x P
  int* status;          // C x F
  int* fb_list;         // mixed: items handed to the FP64 path
  int* fb_count;
  int* ir_iters;        // mixed: refinement iterations summed (one counter)
  int ld;               // leading dimension of the slot matrix
  int ir_max;
  double ir_tol;
  int schedule;         // PXD_SCHED_FREQ_MAJOR or PXD_SCHED_SIZE_MAJOR (implicit order only)
  int half;             // mixed: operands of the rank-KB trailing updates (PXD_HALF_*)
};

// Operand precision of the complex64 factor's block-column updates.
#define PXD_HALF_NONE 0
#define PXD_HALF_BF16 1
#define PXD_HALF_F16 2

// Base-map inverse: one item per frequency.
struct InvParams {
  const double2* Z128;  // F x M x M parents
  int M, F, P;
  const int* IB;        // base active list (N ascending parent indices, ports last)
  int N;
  const double* port_len;
  double z0;
  char* ws;             // one N x ld complex128 slot per workgroup (ld >= 2 N)
  size_t slot_bytes;
  int ld;
  double2* G;           // F x N x N output
  int* status;          // F
  int* counter;         // work counter (zeroed before the launch)
};
hipError_t launch_base_inverse(hipStream_t s, const InvParams& p, int grid);

// Low-rank evaluation of flip candidates from the base inverse: one item per
// (candidate, frequency), frequency-major.
struct LrParams {
  const double2* Z128;  // F x M x M parents
  int M, F, P, C;
  const int* Nc;        // candidate active sizes
  const int* Ilist;     // C x M candidate active lists
  const int* order;     // candidate order
  const int* IB;        // base active list (NB entries, ports last)
  int NB;
  const int* pos_of;    // M: base position of each parent function, -1 if inactive
  const double2* G;     // F x NB x NB base inverses
  const int* base_status;  // F
  const double* port_len;
  double z0;
  double2* S;           // C x F x P x P
  int* status;          // C x F
  int* counter;
  int* fb_list;         // items beyond the low-rank limits, for the dense FP64 path
  int* fb_count;
};
hipError_t launch_positions(hipStream_t s, const int* IB, int NB, int M, int* pos_of);
hipError_t launch_lowrank(hipStream_t s, const LrParams& p, int grid);

// Per-slot layout of the workspace (byte offsets).
struct SlotLayout {
  size_t w_off, piv_off, x_off, bytes;
  int ld;
};

// plain: complex128 N x (N + P) augmented system; mixed: complex64 N x N
// factor, pivots and an FP64 solution block.
__host__ __device__ inline SlotLayout slot_layout(int nmax, int P, bool mixed) {
  SlotLayout s{};
  auto up = [](size_t v, size_t a) -> size_t { return (v + a - 1) / a * a; };
  if (!mixed) {
    s.ld = (int)up(nmax + P, 4);
    s.w_off = 0;
    s.bytes = up((size_t)nmax * s.ld * 16, 256);
  } else {
    s.ld = (int)up(nmax, 4);
    s.w_off = 0;
    size_t w = up((size_t)nmax * s.ld * 8, 256);
    s.piv_off = w;
    size_t pv = up((size_t)nmax * 4, 256);
    s.x_off = w + pv;
    s.bytes = s.x_off + up((size_t)nmax * P * 16, 256);
  }
  return s;
}

// One step's verdict of the mixed-precision refinement (the stop and give-up
// rule the kernels apply).  m: the largest change of any S entry the step
// would make; m_prev: the same for the previous step (0 before the first);
// target: the smallest ir_tol |S_ij| + floor over the entries.  The observed
// contraction rho = m / m_prev (1 on the first step, so at least two steps are
// taken) bounds the error left in every entry by m rho / (1 - rho).  Returns
// 1 when that bound is below the target (and rho < 0.9), 2 when from the
// third step on the contraction cannot bring it there within ir_max steps
// (rho >= 1, a NaN, or more steps needed than remain: the FP64 path takes
// the item), else 0 (take another step).
__host__ __device__ inline int refine_verdict(int iters, int ir_max, double m, double m_prev, double target) {
  const double rho = (iters == 1) ? 1.0 : (m_prev > 0.0 ? m / m_prev : 0.0);
  const double left = m * rho / (1.0 - rho);
  const bool ok = rho < 0.9 && left <= target;
  if (ok) return 1;
  if (iters >= 3) {
    if (!(rho < 1.0) || !(left == left)) return 2;
    if (rho > 0.0 && left > 0.0) {
      // after k more steps the estimate is left rho^k
      const double k_needed = log(target / left) / log(rho);
      if (iters + k_needed > (double)ir_max) return 2;
    }
  }
  return 0;
}

// ------------------------------------------------------------------ tiled LU
//
// Large active sizes: the items of a chunk are factored in lock step, one
// kernel launch per step of each block column, many workgroups per item.

constexpr int kTlKbMax = 128;  // widest block column of the tiled LU

// Per-item slot of the tiled path: the item's matrix (row-major, ld), its
// pivots, an auxiliary block (flags, the current block column's touched rows
// and their sources, the lock-step refinement's state), the inverse of the
// block column's unit-lower diagonal block (kTlKbMax x kTlKbMax) and, in the
// mixed modes, the FP64 solution.
struct TlLayout {
  int ld;
  size_t piv_off, aux_off, li_off, x_off, bytes;
};
__host__ __device__ inline TlLayout tl_layout(int nmax, int P, bool mixed) {
  auto up = [](size_t v, size_t a) -> size_t { return (v + a - 1) / a * a; };
  TlLayout s{};
  const size_t es = mixed ? 8 : 16;
  s.ld = (int)up(mixed ? nmax : nmax + P, 4);
  size_t o = up((size_t)nmax * s.ld * es, 256);
  s.piv_off = o;
  o += up((size_t)nmax * 4, 256);
  s.aux_off = o;
  o += up((size_t)(4 + 4 * kTlKbMax) * 4 + 16, 256);  // + the refinement state
  s.li_off = o;
  o += up((size_t)kTlKbMax * kTlKbMax * es, 256);
  s.x_off = o;
  if (mixed) o += up((size_t)nmax * P * 16, 256);
  s.bytes = o;
  return s;
}

struct TlParams {
  const double2* Z128;  // F x M x M parent (complex128)
  const float2* Z64;    // its complex64 copy, or null (the gather then rounds Z128)
  int M, F, P;
  const int* Nc;        // active size per candidate
  const int* Ilist;     // C x M active lists
  const int* items;     // this chunk's items (c * F + f)
  int B;                // items in the chunk
  const double* port_len;
  double z0;
  char* ws;             // B slots of slot_bytes
  size_t slot_bytes;
  TlLayout lay;
  int mixed;            // 0: FP64 augmented [Z_A | V] (eliminate N - P columns), 1: complex64 N x N
  int kb;               // block-column width (64 or 128)
  int shape;            // output tile of the trailing update: 0 = 128 x 64, 1 = 64 x 64 (four waves),
                        // 2 = 128 x 64, 3 = 128 x 128 (eight waves; FP32 and FP64 only)
  int half;             // mixed: operands of the trailing updates (PXD_HALF_*)
  double2* S;           // C x F x P x P
  int* status;          // C x F
  int fallback_mode;    // FP64 re-solve of items the mixed path handed over: report FALLBACK
  int ir_max;
  double ir_tol;
  int* ir_iters;
  int* fb_count;
  int* fb_list;
};

// Launches of one chunk.  K: first column of the block column; nmax: the
// chunk's largest active size (sizes the grids); q: register rows per
// thread of the panel (>= (nmax - K) / 256).
hipError_t tl_gather(hipStream_t s, const TlParams& p, int nmax);
hipError_t tl_panel(hipStream_t s, const TlParams& p, int K, int nmax);
hipError_t tl_trsm(hipStream_t s, const TlParams& p, int K, int nmax);
// trailing update of the columns [Kend + cb, Kend + ce) of every item (Kend the
// end of the item's block column; ce is clipped to the item's last column)
hipError_t tl_update(hipStream_t s, const TlParams& p, int K, int nmax, int cb, int ce);
hipError_t tl_finish(hipStream_t s, const TlParams& p, int nmax);
hipError_t tl_prepare(const TlParams& p, int nmax);  // kernel attributes (outside capture)
int tl_max_active();                                 // largest active size the tiled path takes (FP64)
int tl_max_active_mixed(int P);                      // the same for the complex64 + refinement modes

// Lock-step refinement of a mixed-mode chunk.  U is the union of the batch's
// active sets (ascending parent indices).  The chunk's items are grouped by
// frequency; each group keeps the solutions of its items as columns of one
// U-row block X (a candidate's rows outside its active set stay zero), so
// one product R = Z_f[U, U] X per group and step gives every residual of the
// group (r = V - (Z_A + port loads) x on the item's rows of R).
struct IrParams {
  const int* upos;      // M: position of each parent function in U, -1 outside U
  const int* ulist;     // U entries
  int U;
  int ldx;              // columns of one group's X and R blocks
  double2* X;           // n_grp x U x ldx
  double2* R;           // n_grp x U x ldx
  const int* grp_f;     // per group: frequency
  const int* grp_ncol;  // per group: columns in use (items x P)
  int* grp_active;      // per group: items still refining
  const int* item_grp;  // per chunk item: group
  const int* item_col;  // per chunk item: first column of its solution in the group
  int n_grp;
};
// After the factorisation of a chunk: x0 = (LU)^-1 V per item, into its slot and X.
hipError_t tl_ir_init(hipStream_t s, const TlParams& p, const IrParams& q, int nmax);
// R = Z_f[U, U] X for every group that still has an item refining.
hipError_t tl_ir_residual(hipStream_t s, const TlParams& p, const IrParams& q, int max_ncol);
// One refinement step of every item still refining (stop test, solve, update).
hipError_t tl_ir_step(hipStream_t s, const TlParams& p, const IrParams& q, int nmax);
// U: mark (M ints, zeroed here), upos (M), ulist (M), count[0] = |U|.
hipError_t launch_union(hipStream_t s, const int* Nc, const int* Ilist, int C, int M, int* mark, int* upos,
                        int* ulist, int* count);
hipError_t launch_zero_c128(hipStream_t s, double2* p, size_t n);

// Rows of the register-resident sub-panel per thread for a given active size.
__host__ __device__ inline int rows_per_thread(int nmax) { return (nmax + 255) / 256; }

hipError_t launch_expand(hipStream_t s, const uint8_t* base, int n_cells, size_t base_stride, const int* off,
                         const int* cells, int C, const int* cell_a, const int* cell_b, int M, int* Nc, int* Ilist);
hipError_t launch_order(hipStream_t s, const int* Nc, int C, int* order);
hipError_t launch_fill_int(hipStream_t s, int* p, int n, int v);
// out[0] = min(v), out[1] = max(v) over n >= 1 entries
hipError_t launch_minmax(hipStream_t s, const int* v, int n, int* out);

// The no-allocation entry point's workspace: a static device array of
// kScratchBytes per GPU.  scratch_region() returns its device address on
// `device` (looked up once per device, with that device current) and its size.
constexpr size_t kScratchBytes = size_t(64) << 20;
hipError_t scratch_region(int device, char** ptr, size_t* bytes);
// half_sb selects the variant whose register sub-panel is half as wide.
hipError_t launch_eval_plain(hipStream_t s, const EvalParams& p, int grid, int half_sb);
hipError_t prepare_eval_mixed(const EvalParams& p, int half_sb);
hipError_t launch_eval_mixed(hipStream_t s, const EvalParams& p, int grid, int half_sb);
// dynamic LDS of the mixed evaluator for a given largest active size and port count
size_t eval_mixed_lds(int nmax, int P);
hipError_t launch_fom(hipStream_t s, const double2* S, int C, int F, int P, const pxd_fom_term* terms,
                      const double* term_fac, int n_terms, const int8_t* band, const int* item_status, double* fom,
                      int* cand_status);
hipError_t launch_argmin(hipStream_t s, const double* fom, int C, int* argmin);
hipError_t launch_gather(hipStream_t s, const double2* Zf, int M, const int* idx, int N, double2* out);
hipError_t launch_to_c64(hipStream_t s, const double2* in, float2* out, size_t n);

}  // namespace pxd
