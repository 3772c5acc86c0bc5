// Host runtime of the evaluator: context, device memory, launch sequence and
// the C ABI declared in pxd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "problem.hpp"
#include "pxd.h"
#include "status.hpp"
#include "surrogate.hpp"

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t n) {
    if (n <= bytes) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipMalloc(&p, n);
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

}  // namespace

namespace {

// Per-launch device buffers; the context has one set, every graph its own.
struct EvalBufs {
  DevBuf Nc, Ilist, order, counter, item_status, ws, fb_list;
  void release() {
    for (DevBuf* b : {&Nc, &Ilist, &order, &counter, &item_status, &ws, &fb_list}) b->release();
  }
};

// Launch configuration chosen per (precision, size class Q).
struct Tuning {
  int wg_per_cu = 2, half_sb = 0, schedule = PXD_SCHED_FREQ_MAJOR;
  bool tiled = false;  // dense LU path (PXD_PATH_TILED when true)
  int tile_kb = 0;     // tiled path: block-column width (0 = default 128)
  int tile_shape = 0;  // tiled path: update tile, 1 = 128 x 64, 2 = 64 x 64 (0 = default 2)
  bool valid = false;
  double ms = 0;
};
constexpr int kSizeClasses = 5;  // Q = 1, 2, 4, 8, 16 (active sizes up to 256 Q)
constexpr int kPrecisions = 5;   // PXD_PREC_*
constexpr int kClassQ[kSizeClasses] = {1, 2, 4, 8, 16};
int size_class(int Q) { return Q <= 1 ? 0 : Q <= 2 ? 1 : Q <= 4 ? 2 : Q <= 8 ? 3 : 4; }

}  // namespace

struct pxd_ctx {
  pxd_options opt{};
  std::string err;
  int n_cu = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ev[6] = {};
  // parent
  int M = 0, F = 0;
  std::vector<double> freqs;
  DevBuf Z128, Z64;
  // map
  int n_cells = 0, P = 0;
  double z0 = 50.0;
  std::vector<double> port_len;
  DevBuf cell_a, cell_b, plen;
  // fom
  int n_terms = 0;
  DevBuf terms, term_fac, band;
  // per call
  DevBuf base, off, cells, S, cand_status, fom, argmin;
  EvalBufs eb;
  std::vector<int> hNc;
  pxd_stats stats{};
  bool stats_pending_counts = false;
  bool stats_lowrank = false;  // the last call was a low-rank one (stage events differ)
  const int* stats_counts = nullptr;  // device counters of the last dense call ([1] fallbacks, [2] refinement steps)
  // tiled path: look-ahead stream for the next block column's panel, and the
  // two events that order it against the call's stream
  hipStream_t aux = nullptr;
  hipEvent_t la_ev[2] = {};
  // tiled path: the lock-step refinement of a chunk runs on `ref` beside the
  // next chunk's factorisation (the chunks alternate between two halves of
  // the workspace); pp_ev[h] = chunk factored, pp_ev[2 + h] = chunk refined
  hipStream_t ref = nullptr;
  hipEvent_t pp_ev[4] = {};
  // tiled path, when profiling is on: one event pair per trailing-update launch
  bool profile = false;
  std::vector<hipEvent_t> upd_ev;
  int n_upd = 0;
  double upd_flops = 0, upd_bytes = 0;
  // tiled path: item order of the call (host copy) and its device copy
  std::vector<int> h_items, h_fb;
  DevBuf tl_items;
  // tiled path, mixed modes, lock-step refinement: the union U of the call's
  // active sets (marks, positions, list, size), the chunks' frequency-group
  // tables and the groups' X and R blocks
  DevBuf ir_mark, ir_upos, ir_ulist, ir_cnt, ir_tab, ir_xr;
  std::vector<int> h_ir;
  // the no-allocation entry point's region of the static scratch array on this device
  char* scratch = nullptr;
  size_t scratch_bytes = 0;
  // autotuning: tuned[precision][size class]; `forced` overrides during a tuning sweep
  Tuning tuned[kPrecisions][kSizeClasses];
  const Tuning* forced = nullptr;
  // low-rank flip evaluation: inverse of the last base map, valid while gen == lr_gen
  DevBuf lr_G, lr_IB, lr_NB, lr_pos, lr_bstat, lr_ws, lr_cnt;
  std::vector<uint8_t> lr_map;
  int lr_nb = 0;
  long long gen = 0, lr_gen = -1;

  int fail(int rc, const std::string& m) {
    err = m;
    pxd::set_thread_error(rc, m);
    return rc;
  }
  int hip_fail(hipError_t e, const char* where) {
    return fail(PXD_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
  }
};

struct pxd_graph {
  pxd_ctx* ctx = nullptr;
  EvalBufs eb;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

#define HIPCHK(ctx, expr)                              \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return (ctx)->hip_fail(e_, #expr); \
  } while (0)

namespace {

// The launch configuration for this precision and size class: explicit
// options first, then the tuned table, then the defaults.
Tuning resolve(const pxd_ctx* ctx, int Q) {
  if (ctx->forced) return *ctx->forced;
  const Tuning& t = ctx->tuned[ctx->opt.precision][size_class(Q)];
  Tuning r = t.valid ? t : Tuning{};
  if (r.wg_per_cu < 1) r.wg_per_cu = 2;  // a tuned tiled record says nothing about the persistent grid
  if (ctx->opt.wg_per_cu > 0) r.wg_per_cu = std::min(ctx->opt.wg_per_cu, 2);
  if (ctx->opt.half_subpanel == 1 || ctx->opt.half_subpanel == 2) r.half_sb = ctx->opt.half_subpanel - 1;
  if (ctx->opt.schedule != PXD_SCHED_AUTO) r.schedule = ctx->opt.schedule;
  return r;
}

// Where one evaluation's internal buffers come from: the context's (or a
// graph's) growable device buffers, or, for the no-allocation entry point, a
// fixed region carved in order out of the library's static scratch array.
struct Arena {
  char* base = nullptr;  // null: use the EvalBufs
  size_t cap = 0, used = 0;
  char* take(size_t bytes) {
    const size_t at = (used + 255) / 256 * 256;
    if (at + bytes > cap) return nullptr;
    used = at + bytes;
    return base + at;
  }
};

// Whether the batch's dense solves go to the tiled LU: the option, else the
// tuned choice for the size class, else tiled only above the persistent
// kernels' 2,048 limit.
// may_tile: false where the tiled path cannot run (graphs, the no-allocation
// entry point): a tuned preference for it then yields the persistent path;
// only what needs the tiled path selects it there (and is refused).
bool use_tiled(const pxd_ctx* ctx, int nmax, bool may_tile = true) {
  const int prec = ctx->opt.precision;
  if (prec == PXD_PREC_MIXED_BF16X3) return true;  // split-BF16 updates exist on the tiled path only
  if (prec == PXD_PREC_MIXED_BF16 || prec == PXD_PREC_MIXED_F16) return false;  // plain ones on the persistent
  const bool no_c64 = prec != PXD_PREC_FP64 && !ctx->Z64.p;
  if (ctx->opt.lu_path == PXD_PATH_TILED || nmax > 2048 || no_c64) return true;
  if (ctx->opt.lu_path == PXD_PATH_PERSISTENT || !may_tile) return false;
  if (ctx->forced) return ctx->forced->tiled;
  const Tuning& t = ctx->tuned[ctx->opt.precision][size_class(pxd::rows_per_thread(nmax))];
  return t.valid && t.tiled;
}

int tile_kb(const pxd_ctx* ctx, int nmax) {
  if (ctx->opt.tile_kb == 64 || ctx->opt.tile_kb == 128) return ctx->opt.tile_kb;
  if (ctx->forced && ctx->forced->tile_kb) return ctx->forced->tile_kb;
  const Tuning& t = ctx->tuned[ctx->opt.precision][size_class(pxd::rows_per_thread(nmax))];
  return (t.valid && t.tile_kb) ? t.tile_kb : 128;
}

int tile_shape(const pxd_ctx* ctx, int nmax) {
  if (ctx->opt.tile_shape >= 1 && ctx->opt.tile_shape <= 4) return ctx->opt.tile_shape;
  if (ctx->forced && ctx->forced->tile_shape) return ctx->forced->tile_shape;
  const Tuning& t = ctx->tuned[ctx->opt.precision][size_class(pxd::rows_per_thread(nmax))];
  return (t.valid && t.tile_shape) ? t.tile_shape : 2;
}

// Workspace cap of the tiled path in bytes: the option, else 80 % of the
// device memory that is free or already held as workspace, at most 64 GiB.
size_t tiled_ws_cap(const pxd_ctx* ctx, size_t held) {
  if (ctx->opt.ws_gib > 0) return (size_t)(ctx->opt.ws_gib * (double)(1ull << 30));
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = 0;
  return std::min<size_t>((size_t)(0.8 * (double)(fr + held)), size_t(64) << 30);
}

// One trailing-update launch of the tiled path (columns [Kend + cb, Kend + ce)
// of each item), bracketed by events and counted when profiling is on.
int tiled_update(pxd_ctx* ctx, hipStream_t s, const pxd::TlParams& tp, const std::vector<int>& list, int i0, int B,
                 int K, int nmax, int cb, int ce, bool mixed) {
  if (!ctx->profile) {
    HIPCHK(ctx, pxd::tl_update(s, tp, K, nmax, cb, ce));
    return PXD_OK;
  }
  const int F = ctx->F, P = ctx->P, kb = tp.kb;
  if ((int)ctx->upd_ev.size() < 2 * (ctx->n_upd + 1)) {
    for (int e = 0; e < 2; ++e) {
      hipEvent_t ev;
      HIPCHK(ctx, hipEventCreate(&ev));
      ctx->upd_ev.push_back(ev);
    }
  }
  // algorithmic work: 8 kbb (N - Kend) x (the launch's columns) real flops per item
  for (int i = i0; i < i0 + B; ++i) {
    const int N = ctx->hNc[list[i] / F], Ne = mixed ? N : N - P, nc = mixed ? N : N + P;
    if (K >= Ne) continue;
    const int kend = K + std::min(kb, Ne - K);
    const long long c_lo = kend + (long long)cb, c_hi = std::min<long long>(nc, kend + (long long)ce);
    if (c_hi > c_lo) {
      const double kk = kend - K, m = N - kend, n = (double)(c_hi - c_lo), es = mixed ? 8.0 : 16.0;
      ctx->upd_flops += 8.0 * kk * m * n;
      ctx->upd_bytes += es * (2.0 * m * n + kk * m + kk * n);  // C read and written, L21 and U12 read once
    }
  }
  HIPCHK(ctx, hipEventRecord(ctx->upd_ev[2 * ctx->n_upd], s));
  HIPCHK(ctx, pxd::tl_update(s, tp, K, nmax, cb, ce));
  HIPCHK(ctx, hipEventRecord(ctx->upd_ev[2 * ctx->n_upd + 1], s));
  ++ctx->n_upd;
  return PXD_OK;
}

// Factor and solve the items `list[0 .. n)` (c * F + f) with the tiled LU in
// chunks of at most `bmax` items whose slots fit the workspace.  mixed: the
// complex64 factor and refinement (items that do not settle are appended to
// fb_list); else the FP64 augmented system (fallback: report FALLBACK).
int run_tiled(pxd_ctx* ctx, EvalBufs& b, hipStream_t s, const int* d_list, const std::vector<int>& list,
              const int* Nc, const int* Ilist, int* cnt, int* item_status, int* fb_list, double2* d_S, bool mixed,
              bool fallback_mode, int U = 0) {
  const int F = ctx->F, P = ctx->P;
  const int n = (int)list.size();
  if (n == 0) return PXD_OK;
  int nmax_all = 0;
  for (int it : list) nmax_all = std::max(nmax_all, ctx->hNc[it / F]);
  const pxd::TlLayout lay_all = pxd::tl_layout(nmax_all, P, mixed);
  const size_t cap = tiled_ws_cap(ctx, b.ws.bytes);
  const int bmax = (int)std::min<size_t>({(size_t)n, (size_t)4 * ctx->n_cu, cap / lay_all.bytes});
  if (bmax < 1)
    return ctx->fail(PXD_ENOMEM, "tiled LU: one item's workspace (" + std::to_string(lay_all.bytes) +
                                     " bytes) exceeds the workspace cap (" + std::to_string(cap) + " bytes)");
  HIPCHK(ctx, b.ws.ensure(lay_all.bytes * (size_t)bmax));
  // with the lock-step refinement, chunks of half the workspace: chunk c
  // factors in half c % 2 while chunk c - 1 refines in the other half
  const bool lockstep = U > 0 && mixed && !fallback_mode;
  const int cb = lockstep && bmax >= 2 && n > bmax / 2 ? bmax / 2 : bmax;
  const int kb = tile_kb(ctx, nmax_all);
  pxd::TlParams tp{};
  tp.Z128 = ctx->Z128.as<double2>();
  tp.Z64 = ctx->Z64.as<float2>();
  tp.M = ctx->M, tp.F = F, tp.P = P;
  tp.Nc = Nc;
  tp.Ilist = Ilist;
  tp.port_len = ctx->plen.as<double>();
  tp.z0 = ctx->z0;
  tp.ws = b.ws.as<char>();
  tp.mixed = mixed ? 1 : 0;
  tp.kb = kb;
  tp.shape = tile_shape(ctx, nmax_all) - 1;
  tp.half = ctx->opt.precision == PXD_PREC_MIXED_BF16X3 ? PXD_HALF_BF16 : PXD_HALF_NONE;  // split products
  tp.S = d_S;
  tp.status = item_status;
  tp.fallback_mode = fallback_mode ? 1 : 0;
  tp.ir_max = ctx->opt.ir_max_iter;
  tp.ir_tol = ctx->opt.ir_tol;
  tp.ir_iters = cnt + 2;
  tp.fb_count = cnt + 1;
  tp.fb_list = fb_list;
  HIPCHK(ctx, pxd::tl_prepare(tp, nmax_all));
  // lock-step refinement (U > 0): the chunks' frequency groups.  Per chunk the
  // table holds item_grp[B], item_col[B], then grp_f, grp_ncol and grp_active
  // (zero) for its groups.
  struct ChunkIr {
    size_t off;
    int n_grp, max_ncol;
  };
  std::vector<ChunkIr> cir;
  int ldx = 0, n_grp_max = 0;
  if (lockstep) {
    std::vector<int>& tab = ctx->h_ir;
    tab.clear();
    std::vector<int> gid(ctx->F, -1);
    for (int i0 = 0; i0 < n; i0 += cb) {
      const int B = std::min(cb, n - i0);
      std::vector<int> gf, gn;
      ChunkIr c{tab.size(), 0, 0};
      tab.resize(tab.size() + 2 * (size_t)B);
      for (int i = 0; i < B; ++i) {
        const int f = list[i0 + i] % F;
        if (gid[f] < 0) {
          gid[f] = (int)gf.size();
          gf.push_back(f);
          gn.push_back(0);
        }
        const int g = gid[f];
        tab[c.off + i] = g;
        tab[c.off + B + i] = gn[g];
        gn[g] += P;
      }
      for (int f : gf) gid[f] = -1;
      c.n_grp = (int)gf.size();
      for (int v : gn) c.max_ncol = std::max(c.max_ncol, v);
      tab.insert(tab.end(), gf.begin(), gf.end());
      tab.insert(tab.end(), gn.begin(), gn.end());
      tab.insert(tab.end(), gf.size(), 0);
      cir.push_back(c);
      ldx = std::max(ldx, c.max_ncol);
      n_grp_max = std::max(n_grp_max, c.n_grp);
    }
    const size_t xr = 2 * (size_t)n_grp_max * U * ldx * sizeof(double2);
    if (xr > (size_t(4) << 30)) {
      cir.clear();  // the groups' blocks would be too large: refine per item
    } else {
      HIPCHK(ctx, ctx->ir_tab.ensure(tab.size() * sizeof(int)));
      HIPCHK(ctx, hipMemcpyAsync(ctx->ir_tab.p, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice, s));
      HIPCHK(ctx, ctx->ir_xr.ensure(xr));
    }
  }
  const bool pipelined = !cir.empty() && cb < bmax;
  int n_chunks = 0;
  for (int i0 = 0, chunk = 0; i0 < n; i0 += cb, ++chunk, ++n_chunks) {
    const int B = std::min(cb, n - i0);
    const int h = chunk & 1;  // workspace half (pipelined)
    int nmax = 0;
    for (int i = i0; i < i0 + B; ++i) nmax = std::max(nmax, ctx->hNc[list[i] / F]);
    tp.items = d_list + i0;
    tp.B = B;
    tp.lay = pxd::tl_layout(nmax, P, mixed);
    tp.slot_bytes = tp.lay.bytes;
    tp.ws = b.ws.as<char>() + (pipelined ? (size_t)h * cb * lay_all.bytes : 0);
    // the half's slots are free once the chunk two before has refined
    if (pipelined && chunk >= 2) HIPCHK(ctx, hipStreamWaitEvent(s, ctx->pp_ev[2 + h], 0));
    const int ne_max = mixed ? nmax : nmax - P;
    HIPCHK(ctx, pxd::tl_gather(s, tp, nmax));
    if (ne_max > 0) {
      HIPCHK(ctx, pxd::tl_panel(s, tp, 0, nmax));
      HIPCHK(ctx, pxd::tl_trsm(s, tp, 0, nmax));
    }
    // Look-ahead: the update of the next block column's columns comes first;
    // then the next panel runs on the auxiliary stream while the rest of the
    // update runs here, and the next interchange/U12 step waits for both.
    for (int K = 0; K < ne_max; K += kb) {
      const bool next = K + kb < ne_max;
      int rc = tiled_update(ctx, s, tp, list, i0, B, K, nmax, 0, kb, mixed);
      if (rc) return rc;
      if (next) {
        HIPCHK(ctx, hipEventRecord(ctx->la_ev[0], s));
        HIPCHK(ctx, hipStreamWaitEvent(ctx->aux, ctx->la_ev[0], 0));
        HIPCHK(ctx, pxd::tl_panel(ctx->aux, tp, K + kb, nmax));
        HIPCHK(ctx, hipEventRecord(ctx->la_ev[1], ctx->aux));
      }
      rc = tiled_update(ctx, s, tp, list, i0, B, K, nmax, kb, 1 << 30, mixed);
      if (rc) return rc;
      if (next) {
        HIPCHK(ctx, hipStreamWaitEvent(s, ctx->la_ev[1], 0));
        HIPCHK(ctx, pxd::tl_trsm(s, tp, K + kb, nmax));
      }
    }
    if (!cir.empty()) {
      hipStream_t rs = s;
      if (pipelined) {  // refine beside the next chunk's factorisation
        HIPCHK(ctx, hipEventRecord(ctx->pp_ev[h], s));
        HIPCHK(ctx, hipStreamWaitEvent(ctx->ref, ctx->pp_ev[h], 0));
        rs = ctx->ref;
      }
      const ChunkIr& c = cir[chunk];
      int* tab = ctx->ir_tab.as<int>() + c.off;
      pxd::IrParams q{};
      q.upos = ctx->ir_upos.as<int>();
      q.ulist = ctx->ir_ulist.as<int>();
      q.U = U;
      q.ldx = ldx;
      q.X = ctx->ir_xr.as<double2>();
      q.R = q.X + (size_t)n_grp_max * U * ldx;
      q.item_grp = tab;
      q.item_col = tab + B;
      q.grp_f = tab + 2 * B;
      q.grp_ncol = tab + 2 * B + c.n_grp;
      q.grp_active = tab + 2 * B + 2 * c.n_grp;
      q.n_grp = c.n_grp;
      HIPCHK(ctx, pxd::launch_zero_c128(rs, q.X, (size_t)c.n_grp * U * ldx));
      HIPCHK(ctx, pxd::tl_ir_init(rs, tp, q, nmax));
      for (int it = 0; it < std::max(1, ctx->opt.ir_max_iter); ++it) {
        HIPCHK(ctx, pxd::tl_ir_residual(rs, tp, q, c.max_ncol));
        HIPCHK(ctx, pxd::tl_ir_step(rs, tp, q, nmax));
      }
      if (pipelined) HIPCHK(ctx, hipEventRecord(ctx->pp_ev[2 + h], rs));
    } else {
      HIPCHK(ctx, pxd::tl_finish(s, tp, nmax));
    }
  }
  if (pipelined)  // everything after this call runs on s
    for (int h = 0; h < 2 && h < n_chunks; ++h) HIPCHK(ctx, hipStreamWaitEvent(s, ctx->pp_ev[2 + h], 0));
  return PXD_OK;
}

// The rest of an evaluation whose dense solves go to the tiled LU (active
// sizes known on the host): item order, chunks, FP64 re-solve of the items
// the mixed path hands over, FoM and argmin.
int evaluate_tiled(pxd_ctx* ctx, EvalBufs& b, hipStream_t s, int C, const int* Nc, const int* Ilist, int* cnt,
                   int* item_status, int* fb_list, double2* d_S, double* d_fom, int* d_cand_status, int* d_argmin,
                   int nmin, int nmax) {
  const bool mixed = ctx->opt.precision != PXD_PREC_FP64;
  const int F = ctx->F, P = ctx->P;
  const long long items = (long long)C * F;
  // frequency-major (largest candidate first within a frequency) or size-major
  // (largest first over all items): either way a chunk holds items of close sizes
  std::vector<int>& order = ctx->h_items;
  order.resize(items);
  std::vector<int> cand(C);
  for (int c = 0; c < C; ++c) cand[c] = c;
  std::stable_sort(cand.begin(), cand.end(), [&](int a, int b2) { return ctx->hNc[a] > ctx->hNc[b2]; });
  const Tuning tune = resolve(ctx, pxd::rows_per_thread(std::min(nmax, 2048)));
  if (tune.schedule == PXD_SCHED_SIZE_MAJOR) {
    for (int r = 0; r < C; ++r)
      for (int f = 0; f < F; ++f) order[(size_t)r * F + f] = cand[r] * F + f;
  } else {
    for (int f = 0; f < F; ++f)
      for (int r = 0; r < C; ++r) order[(size_t)f * C + r] = cand[r] * F + f;
  }
  HIPCHK(ctx, ctx->tl_items.ensure(sizeof(int) * (size_t)items));
  HIPCHK(ctx, hipMemcpyAsync(ctx->tl_items.p, order.data(), sizeof(int) * (size_t)items, hipMemcpyHostToDevice, s));
  HIPCHK(ctx, pxd::launch_fill_int(s, cnt, 8, 0));
  int U = 0;  // lock-step refinement: the union of the call's active sets
  if (mixed && ctx->opt.refine != PXD_REFINE_PER_ITEM) {
    const int M = ctx->M;
    HIPCHK(ctx, ctx->ir_mark.ensure(sizeof(int) * (size_t)M));
    HIPCHK(ctx, ctx->ir_upos.ensure(sizeof(int) * (size_t)M));
    HIPCHK(ctx, ctx->ir_ulist.ensure(sizeof(int) * (size_t)M));
    HIPCHK(ctx, ctx->ir_cnt.ensure(sizeof(int)));
    HIPCHK(ctx, pxd::launch_union(s, Nc, Ilist, C, M, ctx->ir_mark.as<int>(), ctx->ir_upos.as<int>(),
                                  ctx->ir_ulist.as<int>(), ctx->ir_cnt.as<int>()));
    HIPCHK(ctx, hipMemcpyAsync(&U, ctx->ir_cnt.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (ctx->opt.refine == PXD_REFINE_AUTO && (double)U > 1.25 * nmax) U = 0;
  }
  int rc = run_tiled(ctx, b, s, ctx->tl_items.as<int>(), order, Nc, Ilist, cnt, item_status, fb_list, d_S, mixed,
                     false, U);
  if (rc) return rc;
  HIPCHK(ctx, hipEventRecord(ctx->ev[2], s));
  if (mixed) {  // FP64 re-solve of the items refinement could not settle
    int nfb = 0;
    HIPCHK(ctx, hipMemcpyAsync(&nfb, cnt + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (nfb > 0) {
      ctx->h_fb.resize(nfb);
      HIPCHK(ctx, hipMemcpyAsync(ctx->h_fb.data(), fb_list, sizeof(int) * nfb, hipMemcpyDeviceToHost, s));
      HIPCHK(ctx, hipStreamSynchronize(s));
      rc = run_tiled(ctx, b, s, fb_list, ctx->h_fb, Nc, Ilist, cnt, item_status, fb_list, d_S, false, true);
      if (rc) return rc;
    }
  }
  HIPCHK(ctx, hipEventRecord(ctx->ev[3], s));
  HIPCHK(ctx, pxd::launch_fom(s, d_S, C, F, P, ctx->terms.as<pxd_fom_term>(), ctx->term_fac.as<double>(),
                              ctx->n_terms, ctx->band.as<int8_t>(), item_status, d_fom, d_cand_status));
  if (d_argmin) HIPCHK(ctx, pxd::launch_argmin(s, d_fom, C, d_argmin));
  HIPCHK(ctx, hipEventRecord(ctx->ev[4], s));
  ctx->stats.items = items;
  ctx->stats.max_active = nmax;
  ctx->stats.min_active = nmin;
  ctx->stats_pending_counts = mixed;
  ctx->stats_counts = cnt;
  return PXD_OK;
}

// Enqueue one evaluation of C candidates on stream s.  nmax_bound > 0: the
// launch is sized for that bound without reading the active sizes back (as a
// graph needs); otherwise they are read back to size it exactly.  Events and
// kernel attributes are set only outside stream capture.  With an arena, no
// buffer is allocated: everything the kernels use beyond the caller's inputs
// and outputs is carved out of it (a call that does not fit is refused).
int evaluate(pxd_ctx* ctx, EvalBufs& b, hipStream_t s, const uint8_t* d_base, size_t base_stride, int C,
             const int* d_off, const int* d_cells, double2* d_S, double* d_fom, int* d_cand_status, int* d_argmin,
             int nmax_bound, bool capturing = false, Arena* arena = nullptr) {
  if (!ctx->Z128.p) return ctx->fail(PXD_ENOTLOADED, "parent matrices not loaded");
  if (!ctx->cell_a.p) return ctx->fail(PXD_ENOTLOADED, "pixel-to-RWG map not loaded");
  if (!ctx->terms.p) return ctx->fail(PXD_ENOTLOADED, "FoM table not set");
  const bool mixed = ctx->opt.precision != PXD_PREC_FP64;
  const bool events = !capturing;
  const int M = ctx->M, F = ctx->F, P = ctx->P;
  if (events) ctx->stats = pxd_stats{}, ctx->stats_lowrank = false;
  ctx->n_upd = 0, ctx->upd_flops = 0, ctx->upd_bytes = 0;
  if (C == 0) return PXD_OK;
  const long long items = (long long)C * F;
  int *Nc, *Ilist, *order, *cnt, *item_status, *fb_list = nullptr, *minmax = nullptr;
  if (arena) {
    Nc = (int*)arena->take(sizeof(int) * C);
    order = (int*)arena->take(sizeof(int) * C);
    cnt = (int*)arena->take(sizeof(int) * 8);
    minmax = (int*)arena->take(sizeof(int) * 2);
    item_status = (int*)arena->take(sizeof(int) * (size_t)items);
    if (mixed) fb_list = (int*)arena->take(sizeof(int) * (size_t)items);
    Ilist = (int*)arena->take(sizeof(int) * (size_t)C * M);
    if (!Nc || !order || !cnt || !minmax || !item_status || (mixed && !fb_list) || !Ilist)
      return ctx->fail(PXD_ESHAPE, "batch does not fit the no-allocation scratch (" + std::to_string(arena->cap) +
                                       " bytes): its active lists alone need " +
                                       std::to_string((size_t)C * (8 + 4 * (size_t)M) +
                                                      (size_t)items * (mixed ? 8 : 4)) + " bytes");
  } else {
    HIPCHK(ctx, b.Nc.ensure(sizeof(int) * C));
    HIPCHK(ctx, b.Ilist.ensure(sizeof(int) * (size_t)C * M));
    HIPCHK(ctx, b.order.ensure(sizeof(int) * C));
    HIPCHK(ctx, b.counter.ensure(sizeof(int) * 8));
    HIPCHK(ctx, b.item_status.ensure(sizeof(int) * (size_t)items));
    if (mixed) HIPCHK(ctx, b.fb_list.ensure(sizeof(int) * (size_t)items));
    Nc = b.Nc.as<int>(), Ilist = b.Ilist.as<int>(), order = b.order.as<int>(), cnt = b.counter.as<int>();
    item_status = b.item_status.as<int>(), fb_list = b.fb_list.as<int>();
  }
  if (events) HIPCHK(ctx, hipEventRecord(ctx->ev[0], s));
  HIPCHK(ctx, pxd::launch_expand(s, d_base, ctx->n_cells, base_stride, d_off, d_cells, C, ctx->cell_a.as<int>(),
                                 ctx->cell_b.as<int>(), M, Nc, Ilist));
  HIPCHK(ctx, pxd::launch_order(s, Nc, C, order));
  int nmax = nmax_bound, nmin = P;
  if (nmax_bound <= 0) {
    // the largest active size picks the kernel variant and the slot size
    if (arena) {  // reduced on the device, two ints read back into stack memory
      int h[2] = {0, 0};
      HIPCHK(ctx, pxd::launch_minmax(s, Nc, C, minmax));
      HIPCHK(ctx, hipMemcpyAsync(h, minmax, sizeof(h), hipMemcpyDeviceToHost, s));
      HIPCHK(ctx, hipStreamSynchronize(s));
      nmin = h[0], nmax = h[1];
    } else {
      ctx->hNc.resize(C);
      HIPCHK(ctx, hipMemcpyAsync(ctx->hNc.data(), Nc, sizeof(int) * C, hipMemcpyDeviceToHost, s));
      HIPCHK(ctx, hipStreamSynchronize(s));
      nmax = *std::max_element(ctx->hNc.begin(), ctx->hNc.end());
      nmin = *std::min_element(ctx->hNc.begin(), ctx->hNc.end());
    }
    if (nmin < P) return ctx->fail(PXD_ESHAPE, "candidate with fewer active functions than ports");
  }
  const bool tiled = use_tiled(ctx, nmax, !(arena || nmax_bound > 0));
  if (tiled) {
    if (arena || nmax_bound > 0)
      return ctx->fail(PXD_ESHAPE, "the tiled LU (active sizes above 2,048) is not available in graphs or the "
                                   "no-allocation entry point");
    if (nmax > pxd::tl_max_active())
      return ctx->fail(PXD_ESHAPE, "active size above " + std::to_string(pxd::tl_max_active()) + " is not supported");
    if (ctx->opt.precision != PXD_PREC_FP64 && nmax > pxd::tl_max_active_mixed(ctx->P))
      return ctx->fail(PXD_ESHAPE, "active size above " + std::to_string(pxd::tl_max_active_mixed(ctx->P)) +
                                       " is not supported in the mixed-precision modes (their solves keep the "
                                       "right-hand sides in LDS); FP64 takes up to " +
                                       std::to_string(pxd::tl_max_active()));
    if (events) HIPCHK(ctx, hipEventRecord(ctx->ev[1], s));
    return evaluate_tiled(ctx, b, s, C, Nc, Ilist, cnt, item_status, fb_list, d_S, d_fom, d_cand_status, d_argmin,
                          nmin, nmax);
  }
  if (nmax > 2048)
    return ctx->fail(PXD_ESHAPE, "active size above 2,048: the plain BF16 and FP16 modes run on the persistent LU "
                                 "only (use PXD_PREC_MIXED32 or PXD_PREC_MIXED_BF16X3)");
  if (mixed && !ctx->Z64.p)
    return ctx->fail(PXD_ENOMEM, "the plain BF16 and FP16 modes need the complex64 parent copy, which did not fit");
  if (events) HIPCHK(ctx, hipEventRecord(ctx->ev[1], s));

  const Tuning tune = resolve(ctx, pxd::rows_per_thread(nmax));
  int grid = (int)std::min<long long>(items, (long long)ctx->n_cu * tune.wg_per_cu);
  const pxd::SlotLayout lay_p = pxd::slot_layout(nmax, P, false);
  const pxd::SlotLayout lay_m = pxd::slot_layout(nmax, P, true);
  // the mixed path re-solves unrefined items with the FP64 kernel in the same slots
  const size_t slot = mixed ? std::max(lay_p.bytes, lay_m.bytes) : lay_p.bytes;
  char* ws;
  if (arena) {  // as many persistent workgroups as slots fit (at least one)
    const size_t room = arena->cap > arena->used + 256 ? arena->cap - arena->used - 256 : 0;
    grid = (int)std::min<long long>(grid, (long long)(room / slot));
    if (grid < 1)
      return ctx->fail(PXD_ESHAPE, "batch does not fit the no-allocation scratch (" + std::to_string(arena->cap) +
                                       " bytes): one workspace slot at active size " + std::to_string(nmax) +
                                       " needs " + std::to_string(slot) + " bytes beyond the active lists");
    ws = arena->take(slot * (size_t)grid);
  } else {
    HIPCHK(ctx, b.ws.ensure(slot * (size_t)grid));
    ws = b.ws.as<char>();
  }

  pxd::EvalParams ep{};
  ep.Z128 = ctx->Z128.as<double2>();
  ep.Z64 = ctx->Z64.as<float2>();
  ep.M = M, ep.F = F, ep.P = P, ep.C = C;
  ep.Nc = Nc;
  ep.Ilist = Ilist;
  ep.order = order;
  ep.port_len = ctx->plen.as<double>();
  ep.z0 = ctx->z0;
  ep.n_items = (int)items;
  ep.item_list = nullptr;
  ep.counter = cnt;
  ep.ws = ws;
  ep.slot_bytes = slot;
  ep.ld = mixed ? lay_m.ld : lay_p.ld;
  ep.nmax = nmax;
  ep.S = d_S;
  ep.status = item_status;
  ep.ir_max = ctx->opt.ir_max_iter;
  ep.ir_tol = ctx->opt.ir_tol;
  ep.schedule = tune.schedule;
  ep.half = ctx->opt.precision == PXD_PREC_MIXED_BF16 ? PXD_HALF_BF16
            : ctx->opt.precision == PXD_PREC_MIXED_F16 ? PXD_HALF_F16 : PXD_HALF_NONE;
  // cnt: [0] work, [1] fallback count, [2] refinement steps, [3] fallback work
  ep.fb_list = fb_list;
  ep.fb_count = cnt + 1;
  ep.ir_iters = cnt + 2;
  HIPCHK(ctx, pxd::launch_fill_int(s, cnt, 8, 0));
  if (!mixed) {
    HIPCHK(ctx, pxd::launch_eval_plain(s, ep, grid, tune.half_sb));
    if (events) HIPCHK(ctx, hipEventRecord(ctx->ev[2], s));
    if (events) HIPCHK(ctx, hipEventRecord(ctx->ev[3], s));
  } else {
    if (!capturing) HIPCHK(ctx, pxd::prepare_eval_mixed(ep, tune.half_sb));
    HIPCHK(ctx, pxd::launch_eval_mixed(s, ep, grid, tune.half_sb));
    if (events) HIPCHK(ctx, hipEventRecord(ctx->ev[2], s));
    pxd::EvalParams fb = ep;  // FP64 re-solve of the items refinement could not settle
    fb.item_list = ep.fb_list;
    fb.n_items_dev = cnt + 1;
    fb.counter = cnt + 3;
    fb.ld = lay_p.ld;
    fb.fallback_mode = 1;
    HIPCHK(ctx, pxd::launch_eval_plain(s, fb, grid, tune.half_sb));
    if (events) HIPCHK(ctx, hipEventRecord(ctx->ev[3], s));
  }
  HIPCHK(ctx, pxd::launch_fom(s, d_S, C, F, P, ctx->terms.as<pxd_fom_term>(), ctx->term_fac.as<double>(),
                              ctx->n_terms, ctx->band.as<int8_t>(), item_status, d_fom, d_cand_status));
  if (d_argmin) HIPCHK(ctx, pxd::launch_argmin(s, d_fom, C, d_argmin));
  if (events) {
    HIPCHK(ctx, hipEventRecord(ctx->ev[4], s));
    ctx->stats.items = items;
    ctx->stats.max_active = nmax;
    ctx->stats.min_active = nmin;
    ctx->stats_pending_counts = mixed;
    ctx->stats_counts = cnt;
  }
  return PXD_OK;
}

// The complex64 copy of the parent the mixed modes gather their factor from,
// made only when it fits beside the complex128 parent with 8 GiB to spare;
// without it the tiled path gathers and rounds the complex128 parent.
hipError_t make_c64_copy(pxd_ctx* ctx, size_t n) {
  if (ctx->opt.precision == PXD_PREC_FP64) return hipSuccess;
  size_t fr = 0, tot = 0;
  hipError_t e = hipMemGetInfo(&fr, &tot);
  if (e != hipSuccess) return e;
  if (fr < n * 8 + (size_t(8) << 30)) return hipSuccess;
  if ((e = ctx->Z64.ensure(n * 8)) != hipSuccess) return e;
  return pxd::launch_to_c64(ctx->stream, ctx->Z128.as<double2>(), ctx->Z64.as<float2>(), n);
}

int check_flips(pxd_ctx* ctx, int n_cand, const int32_t* offsets, const int32_t* cells) {
  if (n_cand < 0 || !offsets || (n_cand > 0 && !cells && offsets[n_cand] > 0))
    return ctx->fail(PXD_EINVAL, "invalid flip list");
  if (offsets[0] != 0) return ctx->fail(PXD_EINVAL, "offsets[0] must be 0");
  for (int c = 0; c < n_cand; ++c)
    if (offsets[c + 1] < offsets[c]) return ctx->fail(PXD_EINVAL, "offsets must be non-decreasing");
  for (int i = 0; i < offsets[n_cand]; ++i)
    if (cells[i] < 0 || cells[i] >= ctx->n_cells) return ctx->fail(PXD_EINVAL, "flip cell out of range");
  return PXD_OK;
}

// Copy a host batch into the context's buffers and enqueue its evaluation on
// the context's stream.  base_stride = 0: one base map plus flips; otherwise
// `base` holds C whole maps and offsets/cells are NULL.
int upload_and_evaluate(pxd_ctx* ctx, const uint8_t* base, size_t base_stride, int C, const int32_t* offsets,
                        const int32_t* cells) {
  hipStream_t s = ctx->stream;
  const size_t nbase = base_stride ? base_stride * std::max(1, C) : (size_t)ctx->n_cells;
  const int nf = offsets ? offsets[C] : 0;
  HIPCHK(ctx, ctx->base.ensure(nbase));
  HIPCHK(ctx, ctx->off.ensure(sizeof(int) * (C + 1)));
  HIPCHK(ctx, ctx->cells.ensure(sizeof(int) * std::max(1, nf)));
  HIPCHK(ctx, ctx->S.ensure(sizeof(double2) * std::max<size_t>(1, (size_t)C * ctx->F * ctx->P * ctx->P)));
  HIPCHK(ctx, ctx->fom.ensure(sizeof(double) * std::max(1, C)));
  HIPCHK(ctx, ctx->cand_status.ensure(sizeof(int) * std::max(1, C)));
  HIPCHK(ctx, ctx->argmin.ensure(sizeof(int)));
  if (C > 0 || !base_stride) HIPCHK(ctx, hipMemcpyAsync(ctx->base.p, base, nbase, hipMemcpyHostToDevice, s));
  if (offsets) HIPCHK(ctx, hipMemcpyAsync(ctx->off.p, offsets, sizeof(int) * (C + 1), hipMemcpyHostToDevice, s));
  if (nf > 0) HIPCHK(ctx, hipMemcpyAsync(ctx->cells.p, cells, sizeof(int) * nf, hipMemcpyHostToDevice, s));
  return evaluate(ctx, ctx->eb, s, ctx->base.as<uint8_t>(), base_stride, C, offsets ? ctx->off.as<int>() : nullptr,
                  offsets ? ctx->cells.as<int>() : nullptr, ctx->S.as<double2>(), ctx->fom.as<double>(),
                  ctx->cand_status.as<int>(), ctx->argmin.as<int>(), 0);
}

int download(pxd_ctx* ctx, int C, double* S_out, double* fom_out, int32_t* status, int32_t* argmin_out) {
  hipStream_t s = ctx->stream;
  const size_t nS = (size_t)C * ctx->F * ctx->P * ctx->P;
  if (S_out && C) HIPCHK(ctx, hipMemcpyAsync(S_out, ctx->S.p, sizeof(double2) * nS, hipMemcpyDeviceToHost, s));
  if (fom_out && C) HIPCHK(ctx, hipMemcpyAsync(fom_out, ctx->fom.p, sizeof(double) * C, hipMemcpyDeviceToHost, s));
  if (status && C) HIPCHK(ctx, hipMemcpyAsync(status, ctx->cand_status.p, sizeof(int) * C, hipMemcpyDeviceToHost, s));
  if (argmin_out && C) HIPCHK(ctx, hipMemcpyAsync(argmin_out, ctx->argmin.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  return PXD_OK;
}

// Low-rank evaluation of C flip candidates of one base map (host inputs): the
// base inverse (unless cached), the low-rank kernel, the dense FP64 kernel on
// the items beyond the rank limits, then FoM and argmin.
int evaluate_lowrank(pxd_ctx* ctx, const uint8_t* base_map, int C, const int32_t* offsets, const int32_t* cells) {
  if (!ctx->Z128.p) return ctx->fail(PXD_ENOTLOADED, "parent matrices not loaded");
  if (!ctx->terms.p) return ctx->fail(PXD_ENOTLOADED, "FoM table not set");
  hipStream_t s = ctx->stream;
  const int M = ctx->M, F = ctx->F, P = ctx->P;
  const int nf = offsets[C];
  ctx->stats = pxd_stats{};
  if (C == 0) return PXD_OK;
  HIPCHK(ctx, ctx->base.ensure(ctx->n_cells));
  HIPCHK(ctx, ctx->off.ensure(sizeof(int) * (C + 1)));
  HIPCHK(ctx, ctx->cells.ensure(sizeof(int) * std::max(1, nf)));
  HIPCHK(ctx, ctx->S.ensure(sizeof(double2) * (size_t)C * F * P * P));
  HIPCHK(ctx, ctx->fom.ensure(sizeof(double) * C));
  HIPCHK(ctx, ctx->cand_status.ensure(sizeof(int) * C));
  HIPCHK(ctx, ctx->argmin.ensure(sizeof(int)));
  EvalBufs& b = ctx->eb;
  HIPCHK(ctx, b.Nc.ensure(sizeof(int) * C));
  HIPCHK(ctx, b.Ilist.ensure(sizeof(int) * (size_t)C * M));
  HIPCHK(ctx, b.order.ensure(sizeof(int) * C));
  HIPCHK(ctx, b.counter.ensure(sizeof(int) * 8));
  HIPCHK(ctx, b.item_status.ensure(sizeof(int) * (size_t)C * F));
  HIPCHK(ctx, b.fb_list.ensure(sizeof(int) * (size_t)C * F));
  HIPCHK(ctx, ctx->lr_IB.ensure(sizeof(int) * M));
  HIPCHK(ctx, ctx->lr_NB.ensure(sizeof(int)));
  HIPCHK(ctx, ctx->lr_pos.ensure(sizeof(int) * M));
  HIPCHK(ctx, ctx->lr_bstat.ensure(sizeof(int) * F));
  HIPCHK(ctx, ctx->lr_cnt.ensure(sizeof(int)));
  HIPCHK(ctx, hipEventRecord(ctx->ev[0], s));
  HIPCHK(ctx, hipMemcpyAsync(ctx->base.p, base_map, ctx->n_cells, hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipMemcpyAsync(ctx->off.p, offsets, sizeof(int) * (C + 1), hipMemcpyHostToDevice, s));
  if (nf > 0) HIPCHK(ctx, hipMemcpyAsync(ctx->cells.p, cells, sizeof(int) * nf, hipMemcpyHostToDevice, s));
  HIPCHK(ctx, pxd::launch_expand(s, ctx->base.as<uint8_t>(), ctx->n_cells, 0, ctx->off.as<int>(),
                                 ctx->cells.as<int>(), C, ctx->cell_a.as<int>(), ctx->cell_b.as<int>(), M,
                                 b.Nc.as<int>(), b.Ilist.as<int>()));
  HIPCHK(ctx, pxd::launch_order(s, b.Nc.as<int>(), C, b.order.as<int>()));
  const bool reuse = ctx->lr_gen == ctx->gen && ctx->lr_G.p &&
                     ctx->lr_map.size() == (size_t)ctx->n_cells &&
                     std::memcmp(ctx->lr_map.data(), base_map, ctx->n_cells) == 0;
  if (!reuse) {  // the base map's own active set, as a one-map batch
    // lr_IB / lr_NB are overwritten below: the cached inverse no longer
    // matches them, whether or not this call gets as far as recomputing it
    ctx->lr_gen = -1;
    ctx->lr_map.clear();
    HIPCHK(ctx, pxd::launch_expand(s, ctx->base.as<uint8_t>(), ctx->n_cells, (size_t)ctx->n_cells, nullptr, nullptr,
                                   1, ctx->cell_a.as<int>(), ctx->cell_b.as<int>(), M, ctx->lr_NB.as<int>(),
                                   ctx->lr_IB.as<int>()));
  }
  ctx->hNc.resize(C + 1);
  HIPCHK(ctx, hipMemcpyAsync(ctx->hNc.data(), b.Nc.p, sizeof(int) * C, hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipMemcpyAsync(ctx->hNc.data() + C, ctx->lr_NB.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  const int nmax = *std::max_element(ctx->hNc.begin(), ctx->hNc.begin() + C);
  const int nmin = *std::min_element(ctx->hNc.begin(), ctx->hNc.begin() + C);
  const int NB = reuse ? ctx->lr_nb : ctx->hNc[C];
  if (nmin < P || NB < P) return ctx->fail(PXD_ESHAPE, "candidate with fewer active functions than ports");
  if (nmax > 2048 || NB > 2048) return ctx->fail(PXD_ESHAPE, "active size above 2048 is not supported");
  HIPCHK(ctx, hipEventRecord(ctx->ev[1], s));
  if (!reuse) {
    HIPCHK(ctx, pxd::launch_positions(s, ctx->lr_IB.as<int>(), NB, M, ctx->lr_pos.as<int>()));
    HIPCHK(ctx, ctx->lr_G.ensure(sizeof(double2) * (size_t)F * NB * NB));
    const int ld = (2 * NB + 3) / 4 * 4;
    const size_t slot = ((size_t)NB * ld * sizeof(double2) + 255) / 256 * 256;
    const int grid = std::min(F, ctx->n_cu * 2);
    HIPCHK(ctx, ctx->lr_ws.ensure(slot * grid));
    HIPCHK(ctx, pxd::launch_fill_int(s, ctx->lr_cnt.as<int>(), 1, 0));
    pxd::InvParams ip{};
    ip.Z128 = ctx->Z128.as<double2>();
    ip.M = M, ip.F = F, ip.P = P;
    ip.IB = ctx->lr_IB.as<int>();
    ip.N = NB;
    ip.port_len = ctx->plen.as<double>();
    ip.z0 = ctx->z0;
    ip.ws = ctx->lr_ws.as<char>();
    ip.slot_bytes = slot;
    ip.ld = ld;
    ip.G = ctx->lr_G.as<double2>();
    ip.status = ctx->lr_bstat.as<int>();
    ip.counter = ctx->lr_cnt.as<int>();
    HIPCHK(ctx, pxd::launch_base_inverse(s, ip, grid));
    ctx->lr_map.assign(base_map, base_map + ctx->n_cells);
    ctx->lr_nb = NB;
    ctx->lr_gen = ctx->gen;
  }
  HIPCHK(ctx, hipEventRecord(ctx->ev[5], s));
  int* cnt = b.counter.as<int>();  // [0] work, [1] items beyond the rank limits, [3] their dense work
  HIPCHK(ctx, pxd::launch_fill_int(s, cnt, 8, 0));
  pxd::LrParams lp{};
  lp.Z128 = ctx->Z128.as<double2>();
  lp.M = M, lp.F = F, lp.P = P, lp.C = C;
  lp.Nc = b.Nc.as<int>();
  lp.Ilist = b.Ilist.as<int>();
  lp.order = b.order.as<int>();
  lp.IB = ctx->lr_IB.as<int>();
  lp.NB = NB;
  lp.pos_of = ctx->lr_pos.as<int>();
  lp.G = ctx->lr_G.as<double2>();
  lp.base_status = ctx->lr_bstat.as<int>();
  lp.port_len = ctx->plen.as<double>();
  lp.z0 = ctx->z0;
  lp.S = ctx->S.as<double2>();
  lp.status = b.item_status.as<int>();
  lp.counter = cnt;
  lp.fb_list = b.fb_list.as<int>();
  lp.fb_count = cnt + 1;
  const long long items = (long long)C * F;
  HIPCHK(ctx, pxd::launch_lowrank(s, lp, (int)std::min<long long>(items, (long long)ctx->n_cu * 2)));
  HIPCHK(ctx, hipEventRecord(ctx->ev[2], s));
  int n_fb = 0;
  HIPCHK(ctx, hipMemcpyAsync(&n_fb, cnt + 1, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  if (n_fb > 0) {  // the dense FP64 kernel on the listed items
    const Tuning tune = resolve(ctx, pxd::rows_per_thread(nmax));
    const pxd::SlotLayout lay = pxd::slot_layout(nmax, P, false);
    const int grid = std::min(n_fb, ctx->n_cu * tune.wg_per_cu);
    HIPCHK(ctx, b.ws.ensure(lay.bytes * (size_t)grid));
    pxd::EvalParams ep{};
    ep.Z128 = ctx->Z128.as<double2>();
    ep.M = M, ep.F = F, ep.P = P, ep.C = C;
    ep.Nc = b.Nc.as<int>();
    ep.Ilist = b.Ilist.as<int>();
    ep.order = b.order.as<int>();
    ep.port_len = ctx->plen.as<double>();
    ep.z0 = ctx->z0;
    ep.n_items = n_fb;
    ep.item_list = b.fb_list.as<int>();
    ep.counter = cnt + 3;
    ep.ws = b.ws.as<char>();
    ep.slot_bytes = lay.bytes;
    ep.ld = lay.ld;
    ep.nmax = nmax;
    ep.S = ctx->S.as<double2>();
    ep.status = b.item_status.as<int>();
    ep.schedule = PXD_SCHED_FREQ_MAJOR;
    HIPCHK(ctx, pxd::launch_eval_plain(s, ep, grid, tune.half_sb));
  }
  HIPCHK(ctx, hipEventRecord(ctx->ev[3], s));
  HIPCHK(ctx, pxd::launch_fom(s, ctx->S.as<double2>(), C, F, P, ctx->terms.as<pxd_fom_term>(),
                              ctx->term_fac.as<double>(), ctx->n_terms, ctx->band.as<int8_t>(),
                              b.item_status.as<int>(), ctx->fom.as<double>(), ctx->cand_status.as<int>()));
  HIPCHK(ctx, pxd::launch_argmin(s, ctx->fom.as<double>(), C, ctx->argmin.as<int>()));
  HIPCHK(ctx, hipEventRecord(ctx->ev[4], s));
  ctx->stats.items = items;
  ctx->stats.fallbacks = n_fb;
  ctx->stats.max_active = nmax;
  ctx->stats.min_active = nmin;
  ctx->stats.base_reused = reuse ? 1 : 0;
  ctx->stats_pending_counts = false;
  ctx->stats_lowrank = true;
  return PXD_OK;
}

}  // namespace

namespace pxd {
int fom_table(const pxd_ctx* ctx, FomTable* out) {
  if (!ctx || !ctx->terms.p) return PXD_ENOTLOADED;
  out->terms = ctx->terms.as<pxd_fom_term>();
  out->term_fac = ctx->term_fac.as<double>();
  out->band = ctx->band.as<int8_t>();
  out->n_terms = ctx->n_terms;
  out->F = ctx->F;
  out->P = ctx->P;
  return PXD_OK;
}
}  // namespace pxd

extern "C" {

const char* pxd_last_error(const pxd_ctx* ctx) { return ctx ? ctx->err.c_str() : pxd::thread_error(); }

int pxd_create(const pxd_options* opt, pxd_ctx** out) {
  if (!out) return pxd::set_thread_error(PXD_EINVAL, "out is NULL");
  *out = nullptr;
  auto* ctx = new (std::nothrow) pxd_ctx();
  if (!ctx) return pxd::set_thread_error(PXD_ENOMEM, "out of host memory");
  if (opt) ctx->opt = *opt;
  if (ctx->opt.ir_max_iter <= 0) ctx->opt.ir_max_iter = 10;
  if (!(ctx->opt.ir_tol > 0)) ctx->opt.ir_tol = 1e-7;
  if (ctx->opt.precision < PXD_PREC_FP64 || ctx->opt.precision > PXD_PREC_MIXED_BF16X3) {
    delete ctx;
    return pxd::set_thread_error(PXD_EINVAL, "unknown precision mode");
  }
  if (ctx->opt.refine < PXD_REFINE_AUTO || ctx->opt.refine > PXD_REFINE_LOCKSTEP) {
    delete ctx;
    return pxd::set_thread_error(PXD_EINVAL, "unknown refinement mode");
  }
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0 || ctx->opt.device < 0 || ctx->opt.device >= ndev) {
    delete ctx;
    return pxd::set_thread_error(PXD_EDEVICE, "no usable HIP device");
  }
  if ((e = hipSetDevice(ctx->opt.device)) != hipSuccess ||
      (e = hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, ctx->opt.device)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking)) != hipSuccess) {
    std::string m = std::string("device setup: ") + hipGetErrorString(e);
    delete ctx;
    return pxd::set_thread_error(PXD_EDEVICE, m);
  }
  for (auto& ev : ctx->ev)
    if ((e = hipEventCreate(&ev)) != hipSuccess) {
      pxd_destroy(ctx);
      return pxd::set_thread_error(PXD_EDEVICE, "event creation failed");
    }
  for (auto& ev : ctx->la_ev)
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) {
      pxd_destroy(ctx);
      return pxd::set_thread_error(PXD_EDEVICE, "event creation failed");
    }
  for (auto& ev : ctx->pp_ev)
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) {
      pxd_destroy(ctx);
      return pxd::set_thread_error(PXD_EDEVICE, "event creation failed");
    }
  if ((e = hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking)) != hipSuccess ||  // default priorities
      (e = hipStreamCreateWithFlags(&ctx->ref, hipStreamNonBlocking)) != hipSuccess) {
    pxd_destroy(ctx);
    return pxd::set_thread_error(PXD_EDEVICE, "stream creation failed");
  }
  // device address of this GPU's scratch array (looked up once per device);
  // if the lookup fails here, the no-allocation entry point retries it
  if (pxd::scratch_region(ctx->opt.device, &ctx->scratch, &ctx->scratch_bytes) != hipSuccess) {
    ctx->scratch = nullptr;
    ctx->scratch_bytes = 0;
  }
  *out = ctx;
  return PXD_OK;
}

void pxd_destroy(pxd_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->opt.device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  for (DevBuf* b : {&ctx->Z128, &ctx->Z64, &ctx->cell_a, &ctx->cell_b, &ctx->plen, &ctx->terms, &ctx->term_fac,
                    &ctx->band, &ctx->base, &ctx->off, &ctx->cells, &ctx->S, &ctx->cand_status, &ctx->fom,
                    &ctx->argmin})
    b->release();
  for (DevBuf* b : {&ctx->lr_G, &ctx->lr_IB, &ctx->lr_NB, &ctx->lr_pos, &ctx->lr_bstat, &ctx->lr_ws, &ctx->lr_cnt,
                    &ctx->tl_items})
    b->release();
  ctx->eb.release();
  for (auto& ev : ctx->ev)
    if (ev) (void)hipEventDestroy(ev);
  for (auto& ev : ctx->upd_ev) (void)hipEventDestroy(ev);
  for (auto& ev : ctx->la_ev)
    if (ev) (void)hipEventDestroy(ev);
  for (auto& ev : ctx->pp_ev)
    if (ev) (void)hipEventDestroy(ev);
  for (hipStream_t* st : {&ctx->aux, &ctx->ref})
    if (*st) {
      (void)hipStreamSynchronize(*st);
      (void)hipStreamDestroy(*st);
    }
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

int pxd_load_parent(pxd_ctx* ctx, int32_t M, int32_t F, const double* freqs_hz, const double* Z) {
  if (!ctx) return pxd::set_thread_error(PXD_EINVAL, "ctx is NULL");
  if (M <= 0 || F <= 0 || !freqs_hz || !Z) return ctx->fail(PXD_EINVAL, "invalid parent arguments");
  if (ctx->cell_a.p && M != ctx->M) return ctx->fail(PXD_ESHAPE, "parent size differs from the loaded map");
  HIPCHK(ctx, hipSetDevice(ctx->opt.device));
  const size_t n = (size_t)F * M * M;
  ctx->Z128.release();
  ctx->Z64.release();
  HIPCHK(ctx, ctx->Z128.ensure(n * 16));
  HIPCHK(ctx, hipMemcpyAsync(ctx->Z128.p, Z, n * 16, hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(ctx, make_c64_copy(ctx, n));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  ctx->M = M;
  ctx->F = F;
  ctx->freqs.assign(freqs_hz, freqs_hz + F);
  ++ctx->gen;
  ctx->terms.release();  // band ids depend on the frequency grid
  ctx->n_terms = 0;
  return PXD_OK;
}

int pxd_load_parent_problem(pxd_ctx* ctx, const pxd_problem* p, int32_t F, const double* freqs_hz) {
  if (!ctx) return pxd::set_thread_error(PXD_EINVAL, "ctx is NULL");
  if (!p || F <= 0 || !freqs_hz) return ctx->fail(PXD_EINVAL, "invalid parent arguments");
  const int M = (int)p->p.rwg.size();
  if (ctx->cell_a.p && M != ctx->M) return ctx->fail(PXD_ESHAPE, "parent size differs from the loaded map");
  HIPCHK(ctx, hipSetDevice(ctx->opt.device));
  const size_t n = (size_t)F * M * M;
  ctx->Z128.release();
  ctx->Z64.release();
  HIPCHK(ctx, ctx->Z128.ensure(n * 16));
  std::string err;
  int rc;
  try {
    rc = pxd::fill_problem_device(p->p, F, freqs_hz, ctx->Z128.as<double>(), ctx->stream, &err);
  } catch (const std::bad_alloc&) {
    rc = PXD_ENOMEM, err = "out of host memory";
  }
  if (rc != PXD_OK) {
    ctx->Z128.release();
    return ctx->fail(rc, err);
  }
  HIPCHK(ctx, make_c64_copy(ctx, n));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  ctx->M = M;
  ctx->F = F;
  ctx->freqs.assign(freqs_hz, freqs_hz + F);
  ctx->terms.release();
  ctx->n_terms = 0;
  ++ctx->gen;
  return PXD_OK;
}

int pxd_load_map(pxd_ctx* ctx, int32_t n_cells, int32_t M, const uint8_t* kind, const int32_t* cell_a,
                 const int32_t* cell_b, int32_t P, const int32_t* port_bf, const double* port_len, double z0) {
  if (!ctx) return pxd::set_thread_error(PXD_EINVAL, "ctx is NULL");
  if (n_cells <= 0 || M <= 0 || !cell_a || !cell_b || P < 1 || P > 4 || !port_bf || !port_len || !(z0 > 0))
    return ctx->fail(PXD_EINVAL, "invalid map arguments (1 <= P <= 4)");
  if (ctx->Z128.p && M != ctx->M) return ctx->fail(PXD_ESHAPE, "map size differs from the loaded parent");
  for (int k = 0; k < P; ++k)
    if (port_bf[k] != M - P + k) return ctx->fail(PXD_EINVAL, "port functions must be the last P, in port order");
  for (int m = 0; m < M; ++m) {
    if (cell_a[m] >= n_cells || cell_b[m] >= n_cells) return ctx->fail(PXD_EINVAL, "cell index out of range");
    if (m >= M - P && (cell_a[m] >= 0 || cell_b[m] >= 0))
      return ctx->fail(PXD_EINVAL, "port functions must be always present");
  }
  (void)kind;
  HIPCHK(ctx, hipSetDevice(ctx->opt.device));
  HIPCHK(ctx, ctx->cell_a.ensure(sizeof(int) * M));
  HIPCHK(ctx, ctx->cell_b.ensure(sizeof(int) * M));
  HIPCHK(ctx, ctx->plen.ensure(sizeof(double) * P));
  HIPCHK(ctx, hipMemcpy(ctx->cell_a.p, cell_a, sizeof(int) * M, hipMemcpyHostToDevice));
  HIPCHK(ctx, hipMemcpy(ctx->cell_b.p, cell_b, sizeof(int) * M, hipMemcpyHostToDevice));
  HIPCHK(ctx, hipMemcpy(ctx->plen.p, port_len, sizeof(double) * P, hipMemcpyHostToDevice));
  ctx->n_cells = n_cells;
  ctx->M = M;
  ctx->P = P;
  ctx->z0 = z0;
  ctx->port_len.assign(port_len, port_len + P);
  ++ctx->gen;
  return PXD_OK;
}

int pxd_set_fom(pxd_ctx* ctx, int32_t n_terms, const pxd_fom_term* terms, const int8_t* band_of_freq) {
  if (!ctx) return pxd::set_thread_error(PXD_EINVAL, "ctx is NULL");
  if (!ctx->Z128.p || !ctx->cell_a.p) return ctx->fail(PXD_ENOTLOADED, "load the parent and the map first");
  if (n_terms < 0 || (n_terms > 0 && !terms) || !band_of_freq) return ctx->fail(PXD_EINVAL, "invalid FoM table");
  std::vector<double> fac(std::max(1, (int)n_terms));
  for (int t = 0; t < n_terms; ++t) {
    if (terms[t].i < 0 || terms[t].i >= ctx->P || terms[t].j < 0 || terms[t].j >= ctx->P)
      return ctx->fail(PXD_EINVAL, "FoM term refers to a missing port");
    fac[t] = std::pow(10.0, terms[t].log10_factor);
  }
  HIPCHK(ctx, hipSetDevice(ctx->opt.device));
  HIPCHK(ctx, ctx->terms.ensure(sizeof(pxd_fom_term) * std::max(1, (int)n_terms)));
  HIPCHK(ctx, ctx->term_fac.ensure(sizeof(double) * fac.size()));
  HIPCHK(ctx, ctx->band.ensure(std::max(1, ctx->F)));
  if (n_terms > 0) HIPCHK(ctx, hipMemcpy(ctx->terms.p, terms, sizeof(pxd_fom_term) * n_terms, hipMemcpyHostToDevice));
  HIPCHK(ctx, hipMemcpy(ctx->term_fac.p, fac.data(), sizeof(double) * fac.size(), hipMemcpyHostToDevice));
  HIPCHK(ctx, hipMemcpy(ctx->band.p, band_of_freq, ctx->F, hipMemcpyHostToDevice));
  ctx->n_terms = n_terms;
  return PXD_OK;
}

int pxd_set_fom_paper(pxd_ctx* ctx) { return pxd_set_fom_variant(ctx, PXD_FOM_PAPER); }

int pxd_set_fom_variant(pxd_ctx* ctx, int32_t variant) {
  if (!ctx) return pxd::set_thread_error(PXD_EINVAL, "ctx is NULL");
  if (variant < PXD_FOM_PAPER || variant > PXD_FOM_ISO) return ctx->fail(PXD_EINVAL, "unknown FoM variant");
  if (!ctx->Z128.p || !ctx->cell_a.p) return ctx->fail(PXD_ENOTLOADED, "load the parent and the map first");
  // Section III-B bands: 0 = channel 1, 1 = channel 2, 2 = between, 3 = rest of 3-9 GHz
  std::vector<int8_t> band(ctx->F);
  for (int f = 0; f < ctx->F; ++f) {
    const double x = ctx->freqs[f];
    int8_t b = -1;
    if (x >= 5.15e9 && x <= 5.925e9) b = 0;
    else if (x >= 6.425e9 && x <= 7.125e9) b = 1;
    else if (x > 5.925e9 && x < 6.425e9) b = 2;
    else if (x >= 3.0e9 && x <= 9.0e9) b = 3;
    band[f] = b;
  }
  // Eq. 9 reciprocals in closed form: 1/rw = 10^c |S_ij|^e (S_dB = 20 log10 |S|)
  struct Row {
    int band, i, j;
    double c, e;
  };
  const Row rows[] = {
      {0, 1, 0, -0.1, -2.0},             // 1/rw_p1 on S21
      {0, 0, 0, 1.5, 2.0},               // 1/rw_m1 on S11
      {0, 2, 0, 35.0 / 15.0, 20.0 / 15.0},  // 1/rw_s2 on S31
      {1, 2, 0, -0.1, -2.0},             // 1/rw_p2 on S31
      {1, 0, 0, 1.5, 2.0},               // 1/rw_m2 on S11
      {1, 1, 0, 35.0 / 15.0, 20.0 / 15.0},  // 1/rw_s1 on S21
      {2, 2, 1, 20.0 / 15.0, 20.0 / 15.0},  // 1/rw_oi on S32
      {3, 1, 0, 20.0 / 18.0, 20.0 / 18.0},  // 1/rw_s3 on S21
      {3, 2, 0, 20.0 / 18.0, 20.0 / 18.0},  // 1/rw_s4 on S31
  };
  std::vector<Row> table(std::begin(rows), std::end(rows));
  if (variant == PXD_FOM_REJ) {  // Section III-D: rw_s1, rw_s2 at -45 dB with a /10 slope
    for (Row& r : table)
      if ((r.band == 0 && r.i == 2 && r.j == 0) || (r.band == 1 && r.i == 1 && r.j == 0)) r.c = 4.5, r.e = 2.0;
  } else if (variant == PXD_FOM_ISO) {  // Section III-D: isolation term in both passbands
    table.push_back(Row{0, 2, 1, 35.0 / 15.0, 20.0 / 15.0});
    table.push_back(Row{1, 2, 1, 35.0 / 15.0, 20.0 / 15.0});
  }
  std::vector<pxd_fom_term> t;
  for (const Row& r : table)
    if (r.i < ctx->P && r.j < ctx->P) t.push_back(pxd_fom_term{r.band, r.i, r.j, r.c, r.e});
  return pxd_set_fom(ctx, (int32_t)t.size(), t.data(), band.data());
}

int pxd_evaluate_flips(pxd_ctx* ctx, const uint8_t* base_map, int32_t n_cand, const int32_t* offsets,
                       const int32_t* cells, double* S_out, double* fom_out, int32_t* status, int32_t* argmin_out) {
  if (!ctx) return pxd::set_thread_error(PXD_EINVAL, "ctx is NULL");
  if (!base_map) return ctx->fail(PXD_EINVAL, "base_map is NULL");
  if (!ctx->cell_a.p) return ctx->fail(PXD_ENOTLOADED, "pixel-to-RWG map not loaded");
  int rc = check_flips(ctx, n_cand, offsets, cells);
  if (rc) return rc;
  HIPCHK(ctx, hipSetDevice(ctx->opt.device));
  rc = upload_and_evaluate(ctx, base_map, 0, n_cand, offsets, cells);
  if (rc) return rc;
  return download(ctx, n_cand, S_out, fom_out, status, argmin_out);
}

int pxd_evaluate_flips_lowrank(pxd_ctx* ctx, const uint8_t* base_map, int32_t n_cand, const int32_t* offsets,
                               const int32_t* cells, double* S_out, double* fom_out, int32_t* status,
                               int32_t* argmin_out) {
  if (!ctx) return pxd::set_thread_error(PXD_EINVAL, "ctx is NULL");
  if (!base_map) return ctx->fail(PXD_EINVAL, "base_map is NULL");
  if (!ctx->cell_a.p) return ctx->fail(PXD_ENOTLOADED, "pixel-to-RWG map not loaded");
  int rc = check_flips(ctx, n_cand, offsets, cells);
  if (rc) return rc;
  HIPCHK(ctx, hipSetDevice(ctx->opt.device));
  rc = evaluate_lowrank(ctx, base_map, n_cand, offsets, cells);
  if (rc) return rc;
  return download(ctx, n_cand, S_out, fom_out, status, argmin_out);
}

int pxd_evaluate_flips_device(pxd_ctx* ctx, void* stream, const uint8_t* base_map, int32_t n_cand,
                              const int32_t* offsets, const int32_t* cells, int32_t n_flips, double* S_out,
                              double* fom_out, int32_t* status, int32_t* argmin_out) {
  if (!ctx) return pxd::set_thread_error(PXD_EINVAL, "ctx is NULL");
  if (!base_map || !offsets || n_cand < 0 || n_flips < 0 || (n_flips > 0 && !cells) || !S_out || !fom_out)
    return ctx->fail(PXD_EINVAL, "invalid device arguments");
  HIPCHK(ctx, hipSetDevice(ctx->opt.device));
  hipStream_t s = static_cast<hipStream_t>(stream);  // NULL is the default stream
  return evaluate(ctx, ctx->eb, s, base_map, 0, n_cand, offsets, cells, reinterpret_cast<double2*>(S_out), fom_out,
                  status, argmin_out, 0);
}

int pxd_evaluate_flips_device_noalloc(pxd_ctx* ctx, void* stream, const uint8_t* base_map, int32_t n_cand,
                                      const int32_t* offsets, const int32_t* cells, int32_t n_flips, double* S_out,
                                      double* fom_out, int32_t* status, int32_t* argmin_out) {
  if (!ctx) return pxd::set_thread_error(PXD_EINVAL, "ctx is NULL");
  if (!base_map || !offsets || n_cand < 0 || n_flips < 0 || (n_flips > 0 && !cells) || !S_out || !fom_out)
    return ctx->fail(PXD_EINVAL, "invalid device arguments");
  HIPCHK(ctx, hipSetDevice(ctx->opt.device));
  if (!ctx->scratch) HIPCHK(ctx, pxd::scratch_region(ctx->opt.device, &ctx->scratch, &ctx->scratch_bytes));
  hipStream_t s = static_cast<hipStream_t>(stream);  // NULL is the default stream
  Arena arena{ctx->scratch, ctx->scratch_bytes, 0};
  return evaluate(ctx, ctx->eb, s, base_map, 0, n_cand, offsets, cells, reinterpret_cast<double2*>(S_out), fom_out,
                  status, argmin_out, 0, false, &arena);
}

int pxd_evaluate_maps(pxd_ctx* ctx, int32_t n_maps, const uint8_t* maps, double* S_out, double* fom_out,
                      int32_t* status, int32_t* argmin_out) {
  if (!ctx) return pxd::set_thread_error(PXD_EINVAL, "ctx is NULL");
  if (n_maps < 0 || (n_maps > 0 && !maps)) return ctx->fail(PXD_EINVAL, "invalid maps");
  if (!ctx->cell_a.p) return ctx->fail(PXD_ENOTLOADED, "pixel-to-RWG map not loaded");
  HIPCHK(ctx, hipSetDevice(ctx->opt.device));
  int rc = upload_and_evaluate(ctx, maps, ctx->n_cells, n_maps, nullptr, nullptr);
  if (rc) return rc;
  return download(ctx, n_maps, S_out, fom_out, status, argmin_out);
}

int pxd_evaluate_maps_device(pxd_ctx* ctx, void* stream, int32_t n_maps, const uint8_t* maps, double* S_out,
                             double* fom_out, int32_t* status, int32_t* argmin_out) {
  if (!ctx) return pxd::set_thread_error(PXD_EINVAL, "ctx is NULL");
  if (n_maps < 0 || (n_maps > 0 && !maps) || !S_out || !fom_out) return ctx->fail(PXD_EINVAL, "invalid device arguments");
  if (!ctx->cell_a.p) return ctx->fail(PXD_ENOTLOADED, "pixel-to-RWG map not loaded");
  HIPCHK(ctx, hipSetDevice(ctx->opt.device));
  hipStream_t s = static_cast<hipStream_t>(stream);  // NULL is the default stream
  return evaluate(ctx, ctx->eb, s, maps, (size_t)ctx->n_cells, n_maps, nullptr, nullptr,
                  reinterpret_cast<double2*>(S_out), fom_out, status, argmin_out, 0);
}

int pxd_autotune(pxd_ctx* ctx, const uint8_t* base_map, int32_t n_cand, const int32_t* offsets,
                 const int32_t* cells, int32_t n_reps, pxd_tune_entry* report, int32_t max_report,
                 int32_t* n_report) {
  if (!ctx) return pxd::set_thread_error(PXD_EINVAL, "ctx is NULL");
  if (n_report) *n_report = 0;
  if (!base_map || n_cand <= 0 || (max_report > 0 && !report)) return ctx->fail(PXD_EINVAL, "invalid tuning batch");
  if (!ctx->cell_a.p) return ctx->fail(PXD_ENOTLOADED, "pixel-to-RWG map not loaded");
  int rc = check_flips(ctx, n_cand, offsets, cells);
  if (rc) return rc;
  HIPCHK(ctx, hipSetDevice(ctx->opt.device));
  n_reps = std::max(1, n_reps);
  std::vector<pxd_tune_entry> tried;
  int Q = 0;
  // options the context fixes explicitly are not searched
  const int wg_hi = ctx->opt.wg_per_cu > 0 ? std::min(ctx->opt.wg_per_cu, 2) : 2;
  const int wg_lo = ctx->opt.wg_per_cu > 0 ? wg_hi : 1;
  const bool half_fixed = ctx->opt.half_subpanel == 1 || ctx->opt.half_subpanel == 2;
  const int half_lo = half_fixed ? ctx->opt.half_subpanel - 1 : 0, half_hi = half_fixed ? half_lo : 1;
  const bool sched_fixed = ctx->opt.schedule != PXD_SCHED_AUTO;
  const int sched_lo = sched_fixed ? ctx->opt.schedule : PXD_SCHED_FREQ_MAJOR;
  const int sched_hi = sched_fixed ? ctx->opt.schedule : PXD_SCHED_SIZE_MAJOR;
  const bool kb_fixed = ctx->opt.tile_kb == 64 || ctx->opt.tile_kb == 128;
  const bool shape_fixed = ctx->opt.tile_shape >= 1 && ctx->opt.tile_shape <= 4;
  // the batch's largest active size decides which paths can take it
  int nmax_batch = 0;
  {
    std::vector<int32_t> Nb(n_cand);
    std::vector<int32_t> idx((size_t)n_cand * ctx->M);
    rc = pxd_expand(ctx, base_map, n_cand, offsets, cells, Nb.data(), idx.data());
    if (rc) return rc;
    nmax_batch = *std::max_element(Nb.begin(), Nb.end());
  }
  const int prec = ctx->opt.precision;
  const bool no_c64 = prec != PXD_PREC_FP64 && !ctx->Z64.p;
  const bool plain_half = prec == PXD_PREC_MIXED_BF16 || prec == PXD_PREC_MIXED_F16;
  const bool try_persistent = ctx->opt.lu_path != PXD_PATH_TILED && nmax_batch <= 2048 && !no_c64 &&
                              prec != PXD_PREC_MIXED_BF16X3;
  const bool try_tiled = ctx->opt.lu_path != PXD_PATH_PERSISTENT && !plain_half;
  if (!try_persistent && !try_tiled) return ctx->fail(PXD_ESHAPE, "no LU path takes this batch in this precision");
  std::vector<Tuning> cands;
  if (try_persistent)
    for (int wg = wg_hi; wg >= wg_lo; --wg)
      for (int half = half_lo; half <= half_hi; ++half)
        for (int sched = sched_lo; sched <= sched_hi; ++sched) {
          Tuning t;
          t.wg_per_cu = wg, t.half_sb = half, t.schedule = sched, t.tiled = false, t.valid = true;
          cands.push_back(t);
        }
  if (try_tiled)
    for (int kb : {64, 128}) {
      if (kb_fixed && kb != ctx->opt.tile_kb) continue;
      for (int shape : {1, 2, 3, 4}) {
        if (shape_fixed && shape != ctx->opt.tile_shape) continue;
        if (shape > 2 && prec == PXD_PREC_MIXED_BF16X3) continue;  // the split-BF16 update has two shapes
        for (int sched = sched_lo; sched <= sched_hi; ++sched) {
          Tuning t;
          t.wg_per_cu = 0, t.schedule = sched, t.tiled = true, t.tile_kb = kb, t.tile_shape = shape, t.valid = true;
          cands.push_back(t);
        }
      }
    }
  for (const Tuning& t : cands) {
    double best = 1e300;
    for (int r = 0; r < n_reps; ++r) {
      ctx->forced = &t;
      rc = upload_and_evaluate(ctx, base_map, 0, n_cand, offsets, cells);
      ctx->forced = nullptr;
      if (rc) return rc;
      HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
      pxd_stats st{};
      pxd_get_stats(ctx, &st);
      best = std::min(best, st.ms_solve + st.ms_fallback);
      Q = pxd::rows_per_thread(st.max_active);
    }
    tried.push_back(pxd_tune_entry{Q, t.wg_per_cu, t.half_sb, t.schedule,
                                   t.tiled ? PXD_PATH_TILED : PXD_PATH_PERSISTENT, t.tile_kb, t.tile_shape, 0, best});
  }
  std::stable_sort(tried.begin(), tried.end(),
                   [](const pxd_tune_entry& a, const pxd_tune_entry& b) { return a.ms < b.ms; });
  const pxd_tune_entry& w = tried.front();
  Tuning& slot = ctx->tuned[ctx->opt.precision][size_class(Q)];
  slot.wg_per_cu = w.wg_per_cu, slot.half_sb = w.half_subpanel, slot.schedule = w.schedule;
  slot.tiled = w.lu_path == PXD_PATH_TILED, slot.tile_kb = w.tile_kb, slot.tile_shape = w.tile_shape;
  slot.ms = w.ms, slot.valid = true;
  const int n = std::min<int>(max_report, (int)tried.size());
  for (int i = 0; i < n; ++i) report[i] = tried[i];
  if (n_report) *n_report = n;
  return PXD_OK;
}

int pxd_tune_save(const pxd_ctx* ctx, const char* path) {
  if (!ctx || !path) return pxd::set_thread_error(PXD_EINVAL, "null argument");
  FILE* f = std::fopen(path, "w");
  if (!f) return pxd::set_thread_error(PXD_EINVAL, std::string("cannot write ") + path);
  std::fprintf(f, "# precision rows_per_thread wg_per_cu half_subpanel schedule ms lu_path tile_kb tile_shape\n");
  for (int prec = 0; prec < kPrecisions; ++prec)
    for (int q = 0; q < kSizeClasses; ++q) {
      const Tuning& t = ctx->tuned[prec][q];
      if (t.valid)
        std::fprintf(f, "%d %d %d %d %d %.6f %d %d %d\n", prec, kClassQ[q], t.wg_per_cu, t.half_sb, t.schedule,
                     t.ms, t.tiled ? PXD_PATH_TILED : PXD_PATH_PERSISTENT, t.tile_kb, t.tile_shape);
    }
  std::fclose(f);
  return PXD_OK;
}

int pxd_tune_load(pxd_ctx* ctx, const char* path) {
  if (!ctx || !path) return pxd::set_thread_error(PXD_EINVAL, "null argument");
  FILE* f = std::fopen(path, "r");
  if (!f) return ctx->fail(PXD_EINVAL, std::string("cannot read ") + path);
  char line[256];
  int rc = PXD_OK;
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    int prec, Q, wg, half, sched, path = PXD_PATH_PERSISTENT, kb = 0, shape = 0;
    double ms;
    const int got =
        std::sscanf(line, "%d %d %d %d %d %lf %d %d %d", &prec, &Q, &wg, &half, &sched, &ms, &path, &kb, &shape);
    if ((got != 6 && got != 8 && got != 9) || prec < 0 || prec >= kPrecisions || shape < 0 || shape > 2 ||
        (Q != 1 && Q != 2 && Q != 4 && Q != 8 && Q != 16) || wg < 0 || wg > 2 || half < 0 || half > 1 ||
        sched < PXD_SCHED_FREQ_MAJOR || sched > PXD_SCHED_SIZE_MAJOR ||
        (path != PXD_PATH_PERSISTENT && path != PXD_PATH_TILED) || (kb != 0 && kb != 64 && kb != 128) ||
        (path == PXD_PATH_PERSISTENT && wg < 1)) {
      rc = ctx->fail(PXD_EINVAL, std::string("malformed tuning line: ") + line);
      break;
    }
    Tuning& t = ctx->tuned[prec][size_class(Q)];
    t.wg_per_cu = wg, t.half_sb = half, t.schedule = sched, t.ms = ms, t.valid = true;
    t.tiled = path == PXD_PATH_TILED, t.tile_kb = kb, t.tile_shape = shape;
  }
  std::fclose(f);
  return rc;
}

int pxd_graph_create(pxd_ctx* ctx, const uint8_t* base_map, int64_t base_stride, int32_t n_cand,
                     const int32_t* offsets, const int32_t* cells, int32_t n_max_active, double* S_out,
                     double* fom_out, int32_t* status, int32_t* argmin_out, pxd_graph** out) {
  if (!ctx) return pxd::set_thread_error(PXD_EINVAL, "ctx is NULL");
  if (!out) return ctx->fail(PXD_EINVAL, "out is NULL");
  *out = nullptr;
  if (!base_map || n_cand <= 0 || !S_out || !fom_out || base_stride < 0 ||
      (base_stride == 0 && (!offsets || !cells)) || (base_stride != 0 && base_stride != ctx->n_cells))
    return ctx->fail(PXD_EINVAL, "invalid graph arguments");
  if (base_stride != 0)  // switched off: its one GPU run stalled with no cause found
    return ctx->fail(PXD_EINVAL, "graphs of whole-map batches are not supported; capture a flip batch");
  if (n_max_active < ctx->P || n_max_active > std::min(2048, ctx->M))
    return ctx->fail(PXD_EINVAL, "n_max_active must lie in [P, min(M, 2048)]");
  HIPCHK(ctx, hipSetDevice(ctx->opt.device));
  auto* g = new (std::nothrow) pxd_graph();
  if (!g) return ctx->fail(PXD_ENOMEM, "out of host memory");
  g->ctx = ctx;
  hipStream_t s = ctx->stream;
  // allocate everything and set kernel attributes before capture begins
  int rc = evaluate(ctx, g->eb, s, base_map, (size_t)base_stride, n_cand, base_stride ? nullptr : offsets,
                    base_stride ? nullptr : cells, reinterpret_cast<double2*>(S_out), fom_out, status, argmin_out,
                    n_max_active);
  if (rc == PXD_OK) {
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) rc = ctx->hip_fail(e, "hipStreamBeginCapture");
  }
  if (rc == PXD_OK) {
    rc = evaluate(ctx, g->eb, s, base_map, (size_t)base_stride, n_cand, base_stride ? nullptr : offsets,
                  base_stride ? nullptr : cells, reinterpret_cast<double2*>(S_out), fom_out, status, argmin_out,
                  n_max_active, true);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (rc == PXD_OK && e != hipSuccess) rc = ctx->hip_fail(e, "hipStreamEndCapture");
    g->graph = graph;
    if (rc == PXD_OK) {
      e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
      if (e != hipSuccess) rc = ctx->hip_fail(e, "hipGraphInstantiate");
    }
  }
  if (rc != PXD_OK) {
    pxd_graph_destroy(g);
    return rc;
  }
  *out = g;
  return PXD_OK;
}

int pxd_graph_launch(pxd_graph* g, void* stream) {
  if (!g || !g->exec) return pxd::set_thread_error(PXD_EINVAL, "graph is NULL");
  pxd_ctx* ctx = g->ctx;
  HIPCHK(ctx, hipSetDevice(ctx->opt.device));
  hipStream_t s = static_cast<hipStream_t>(stream);  // NULL is the default stream
  HIPCHK(ctx, hipGraphLaunch(g->exec, s));
  return PXD_OK;
}

void pxd_graph_destroy(pxd_graph* g) {
  if (!g) return;
  if (g->ctx) {
    (void)hipSetDevice(g->ctx->opt.device);
    (void)hipStreamSynchronize(g->ctx->stream);
    (void)hipDeviceSynchronize();
  }
  if (g->ctx && g->ctx->stats_counts == g->eb.counter.as<int>()) {  // the counters go with the graph
    g->ctx->stats_counts = nullptr;
    g->ctx->stats_pending_counts = false;
  }
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  g->eb.release();
  delete g;
}

int pxd_expand(pxd_ctx* ctx, const uint8_t* base_map, int32_t n_cand, const int32_t* offsets, const int32_t* cells,
               int32_t* N_out, int32_t* idx_out) {
  if (!ctx) return pxd::set_thread_error(PXD_EINVAL, "ctx is NULL");
  if (!base_map || !N_out || !idx_out) return ctx->fail(PXD_EINVAL, "null argument");
  if (!ctx->cell_a.p) return ctx->fail(PXD_ENOTLOADED, "pixel-to-RWG map not loaded");
  int rc = check_flips(ctx, n_cand, offsets, cells);
  if (rc) return rc;
  HIPCHK(ctx, hipSetDevice(ctx->opt.device));
  const int C = n_cand, nf = offsets[n_cand];
  if (C == 0) return PXD_OK;
  hipStream_t s = ctx->stream;
  HIPCHK(ctx, ctx->base.ensure(ctx->n_cells));
  HIPCHK(ctx, ctx->off.ensure(sizeof(int) * (C + 1)));
  HIPCHK(ctx, ctx->cells.ensure(sizeof(int) * std::max(1, nf)));
  HIPCHK(ctx, ctx->eb.Nc.ensure(sizeof(int) * C));
  HIPCHK(ctx, ctx->eb.Ilist.ensure(sizeof(int) * (size_t)C * ctx->M));
  HIPCHK(ctx, hipMemcpyAsync(ctx->base.p, base_map, ctx->n_cells, hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipMemcpyAsync(ctx->off.p, offsets, sizeof(int) * (C + 1), hipMemcpyHostToDevice, s));
  if (nf > 0) HIPCHK(ctx, hipMemcpyAsync(ctx->cells.p, cells, sizeof(int) * nf, hipMemcpyHostToDevice, s));
  HIPCHK(ctx, pxd::launch_expand(s, ctx->base.as<uint8_t>(), ctx->n_cells, 0, ctx->off.as<int>(), ctx->cells.as<int>(),
                                 C, ctx->cell_a.as<int>(), ctx->cell_b.as<int>(), ctx->M, ctx->eb.Nc.as<int>(),
                                 ctx->eb.Ilist.as<int>()));
  HIPCHK(ctx, hipMemcpyAsync(N_out, ctx->eb.Nc.p, sizeof(int) * C, hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipMemcpyAsync(idx_out, ctx->eb.Ilist.p, sizeof(int) * (size_t)C * ctx->M, hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  return PXD_OK;
}

int pxd_gather(pxd_ctx* ctx, int32_t f, int32_t N, const int32_t* idx, double* ZA_out) {
  if (!ctx) return pxd::set_thread_error(PXD_EINVAL, "ctx is NULL");
  if (!ctx->Z128.p) return ctx->fail(PXD_ENOTLOADED, "parent matrices not loaded");
  if (f < 0 || f >= ctx->F || N <= 0 || N > ctx->M || !idx || !ZA_out) return ctx->fail(PXD_EINVAL, "invalid gather arguments");
  for (int i = 0; i < N; ++i)
    if (idx[i] < 0 || idx[i] >= ctx->M || (i > 0 && idx[i] <= idx[i - 1]))
      return ctx->fail(PXD_EINVAL, "idx must be ascending parent indices");
  HIPCHK(ctx, hipSetDevice(ctx->opt.device));
  hipStream_t s = ctx->stream;
  DevBuf didx, dout;
  HIPCHK(ctx, didx.ensure(sizeof(int) * N));
  if (dout.ensure(sizeof(double2) * (size_t)N * N) != hipSuccess) {
    didx.release();
    return ctx->fail(PXD_ENOMEM, "device allocation failed");
  }
  int rc = PXD_OK;
  hipError_t e = hipMemcpyAsync(didx.p, idx, sizeof(int) * N, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = pxd::launch_gather(s, ctx->Z128.as<double2>() + (size_t)f * ctx->M * ctx->M, ctx->M, didx.as<int>(), N,
                           dout.as<double2>());
  if (e == hipSuccess) e = hipMemcpyAsync(ZA_out, dout.p, sizeof(double2) * (size_t)N * N, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) rc = ctx->hip_fail(e, "gather");
  didx.release();
  dout.release();
  return rc;
}

int pxd_set_profiling(pxd_ctx* ctx, int32_t on) {
  if (!ctx) return pxd::set_thread_error(PXD_EINVAL, "ctx is NULL");
  ctx->profile = on != 0;
  return PXD_OK;
}

int pxd_refine_verdict(int32_t iters, int32_t ir_max, double m, double m_prev, double target) {
  if (iters < 1 || ir_max < 1) return pxd::set_thread_error(PXD_EINVAL, "iters and ir_max must be >= 1");
  return pxd::refine_verdict(iters, ir_max, m, m_prev, target);
}

int pxd_get_stats(const pxd_ctx* ctx, pxd_stats* out) {
  if (!ctx || !out) return pxd::set_thread_error(PXD_EINVAL, "null argument");
  *out = ctx->stats;
  // stage times of the last call: wait for its final event, then read the events
  if (ctx->stats.items > 0 && hipEventSynchronize(ctx->ev[4]) == hipSuccess) {
    float a = 0, b = 0, c = 0;
    if (hipEventElapsedTime(&a, ctx->ev[0], ctx->ev[1]) == hipSuccess) out->ms_expand = a;
    if (ctx->stats_lowrank) {
      float g = 0, h = 0;
      if (hipEventElapsedTime(&g, ctx->ev[1], ctx->ev[5]) == hipSuccess) out->ms_base_inverse = g;
      if (hipEventElapsedTime(&h, ctx->ev[5], ctx->ev[2]) == hipSuccess) out->ms_solve = h;
      if (hipEventElapsedTime(&h, ctx->ev[2], ctx->ev[3]) == hipSuccess) out->ms_fallback = h;
    } else if (hipEventElapsedTime(&b, ctx->ev[1], ctx->ev[2]) == hipSuccess) {
      out->ms_solve = b;
    }
    if (hipEventElapsedTime(&c, ctx->ev[3], ctx->ev[4]) == hipSuccess) out->ms_fom = c;
    out->update_launches = ctx->n_upd;
    out->update_gflop = ctx->upd_flops / 1e9;
    out->update_gbyte = ctx->upd_bytes / 1e9;
    for (int i = 0; i < ctx->n_upd; ++i) {
      float u = 0;
      if (hipEventElapsedTime(&u, ctx->upd_ev[2 * i], ctx->upd_ev[2 * i + 1]) == hipSuccess) out->ms_update += u;
    }
    float d = 0;
    if (ctx->stats_pending_counts && hipEventElapsedTime(&d, ctx->ev[2], ctx->ev[3]) == hipSuccess) {
      out->ms_fallback = d;
      int h[4] = {0, 0, 0, 0};
      if (ctx->stats_counts && hipMemcpy(h, ctx->stats_counts, sizeof(h), hipMemcpyDeviceToHost) == hipSuccess) {
        out->fallbacks = h[1];
        out->ir_iterations = h[2];
      }
    }
  }
  return PXD_OK;
}

}  // extern "C"
