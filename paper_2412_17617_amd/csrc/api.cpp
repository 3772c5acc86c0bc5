// Host runtime of the evaluator: context, device memory, launch sequence and
// the C ABI declared in pxd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "pxd.h"
#include "status.hpp"

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
  DevBuf base, off, cells, Nc, Ilist, order, counter, S, item_status, cand_status, fom, argmin, ws, fb_list;
  std::vector<int> hNc;
  pxd_stats stats{};
  bool stats_pending_counts = false;

  int fail(int rc, const std::string& m) {
    err = m;
    pxd::set_thread_error(rc, m);
    return rc;
  }
  int hip_fail(hipError_t e, const char* where) {
    return fail(PXD_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
  }
};

#define HIPCHK(ctx, expr)                              \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return (ctx)->hip_fail(e_, #expr); \
  } while (0)

namespace {

int evaluate(pxd_ctx* ctx, hipStream_t s, const uint8_t* d_base, int C, const int* d_off, const int* d_cells,
             double2* d_S, double* d_fom, int* d_cand_status, int* d_argmin) {
  if (!ctx->Z128.p) return ctx->fail(PXD_ENOTLOADED, "parent matrices not loaded");
  if (!ctx->cell_a.p) return ctx->fail(PXD_ENOTLOADED, "pixel-to-RWG map not loaded");
  if (!ctx->terms.p) return ctx->fail(PXD_ENOTLOADED, "FoM table not set");
  const bool mixed = ctx->opt.precision == PXD_PREC_MIXED32;
  const int M = ctx->M, F = ctx->F, P = ctx->P;
  ctx->stats = pxd_stats{};
  if (C == 0) return PXD_OK;
  HIPCHK(ctx, ctx->Nc.ensure(sizeof(int) * C));
  HIPCHK(ctx, ctx->Ilist.ensure(sizeof(int) * (size_t)C * M));
  HIPCHK(ctx, ctx->order.ensure(sizeof(int) * C));
  HIPCHK(ctx, ctx->counter.ensure(sizeof(int) * 8));
  HIPCHK(ctx, ctx->item_status.ensure(sizeof(int) * (size_t)C * F));
  HIPCHK(ctx, hipEventRecord(ctx->ev[0], s));
  HIPCHK(ctx, pxd::launch_expand(s, d_base, ctx->n_cells, d_off, d_cells, C, ctx->cell_a.as<int>(),
                                 ctx->cell_b.as<int>(), M, ctx->Nc.as<int>(), ctx->Ilist.as<int>()));
  HIPCHK(ctx, pxd::launch_order(s, ctx->Nc.as<int>(), C, ctx->order.as<int>()));
  // the largest active size picks the kernel variant and the slot size
  ctx->hNc.resize(C);
  HIPCHK(ctx, hipMemcpyAsync(ctx->hNc.data(), ctx->Nc.p, sizeof(int) * C, hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  const int nmax = *std::max_element(ctx->hNc.begin(), ctx->hNc.end());
  const int nmin = *std::min_element(ctx->hNc.begin(), ctx->hNc.end());
  if (nmax > 2048) return ctx->fail(PXD_ESHAPE, "active size above 2048 is not supported");
  if (nmin < P) return ctx->fail(PXD_ESHAPE, "candidate with fewer active functions than ports");
  HIPCHK(ctx, hipEventRecord(ctx->ev[1], s));

  const int wg_per_cu = ctx->opt.wg_per_cu > 0 ? ctx->opt.wg_per_cu : 2;
  const long long items = (long long)C * F;
  int grid = (int)std::min<long long>(items, (long long)ctx->n_cu * wg_per_cu);
  const pxd::SlotLayout lay_p = pxd::slot_layout(nmax, P, false);
  const pxd::SlotLayout lay_m = pxd::slot_layout(nmax, P, true);
  // the mixed path re-solves unrefined items with the FP64 kernel in the same slots
  const size_t slot = mixed ? std::max(lay_p.bytes, lay_m.bytes) : lay_p.bytes;
  HIPCHK(ctx, ctx->ws.ensure(slot * (size_t)grid));
  if (mixed) HIPCHK(ctx, ctx->fb_list.ensure(sizeof(int) * (size_t)items));

  pxd::EvalParams ep{};
  ep.Z128 = ctx->Z128.as<double2>();
  ep.Z64 = ctx->Z64.as<float2>();
  ep.M = M, ep.F = F, ep.P = P, ep.C = C;
  ep.Nc = ctx->Nc.as<int>();
  ep.Ilist = ctx->Ilist.as<int>();
  ep.order = ctx->order.as<int>();
  ep.port_len = ctx->plen.as<double>();
  ep.z0 = ctx->z0;
  ep.n_items = (int)items;
  ep.item_list = nullptr;
  ep.counter = ctx->counter.as<int>();
  ep.ws = ctx->ws.as<char>();
  ep.slot_bytes = slot;
  ep.ld = mixed ? lay_m.ld : lay_p.ld;
  ep.nmax = nmax;
  ep.S = d_S;
  ep.status = ctx->item_status.as<int>();
  ep.ir_max = ctx->opt.ir_max_iter;
  ep.ir_tol = ctx->opt.ir_tol;
  int* cnt = ctx->counter.as<int>();  // [0] work, [1] fallback count, [2] refinement steps, [3] fallback work
  ep.fb_list = ctx->fb_list.as<int>();
  ep.fb_count = cnt + 1;
  ep.ir_iters = cnt + 2;
  HIPCHK(ctx, pxd::launch_fill_int(s, cnt, 8, 0));
  if (!mixed) {
    HIPCHK(ctx, pxd::launch_eval_plain(s, ep, grid));
    HIPCHK(ctx, hipEventRecord(ctx->ev[2], s));
    HIPCHK(ctx, hipEventRecord(ctx->ev[3], s));
  } else {
    HIPCHK(ctx, pxd::launch_eval_mixed(s, ep, grid));
    HIPCHK(ctx, hipEventRecord(ctx->ev[2], s));
    pxd::EvalParams fb = ep;  // FP64 re-solve of the items refinement could not settle
    fb.item_list = ep.fb_list;
    fb.n_items_dev = cnt + 1;
    fb.counter = cnt + 3;
    fb.ld = lay_p.ld;
    fb.fallback_mode = 1;
    HIPCHK(ctx, pxd::launch_eval_plain(s, fb, grid));
    HIPCHK(ctx, hipEventRecord(ctx->ev[3], s));
  }
  HIPCHK(ctx, pxd::launch_fom(s, d_S, C, F, P, ctx->terms.as<pxd_fom_term>(), ctx->term_fac.as<double>(),
                              ctx->n_terms, ctx->band.as<int8_t>(), ctx->item_status.as<int>(), d_fom,
                              d_cand_status));
  if (d_argmin) HIPCHK(ctx, pxd::launch_argmin(s, d_fom, C, d_argmin));
  HIPCHK(ctx, hipEventRecord(ctx->ev[4], s));
  ctx->stats.items = items;
  ctx->stats.max_active = nmax;
  ctx->stats.min_active = nmin;
  ctx->stats_pending_counts = mixed;
  return PXD_OK;
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

}  // namespace

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
  if (ctx->opt.precision != PXD_PREC_FP64 && ctx->opt.precision != PXD_PREC_MIXED32) {
    delete ctx;
    return pxd::set_thread_error(PXD_EINVAL, "unknown precision mode");
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
  *out = ctx;
  return PXD_OK;
}

void pxd_destroy(pxd_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->opt.device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  for (DevBuf* b : {&ctx->Z128, &ctx->Z64, &ctx->cell_a, &ctx->cell_b, &ctx->plen, &ctx->terms, &ctx->term_fac,
                    &ctx->band, &ctx->base, &ctx->off, &ctx->cells, &ctx->Nc, &ctx->Ilist, &ctx->order,
                    &ctx->counter, &ctx->S, &ctx->item_status, &ctx->cand_status, &ctx->fom, &ctx->argmin,
                    &ctx->ws, &ctx->fb_list})
    b->release();
  for (auto& ev : ctx->ev)
    if (ev) (void)hipEventDestroy(ev);
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
  if (ctx->opt.precision == PXD_PREC_MIXED32) {
    HIPCHK(ctx, ctx->Z64.ensure(n * 8));
    HIPCHK(ctx, pxd::launch_to_c64(ctx->stream, ctx->Z128.as<double2>(), ctx->Z64.as<float2>(), n));
  }
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  ctx->M = M;
  ctx->F = F;
  ctx->freqs.assign(freqs_hz, freqs_hz + F);
  ctx->terms.release();  // band ids depend on the frequency grid
  ctx->n_terms = 0;
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

int pxd_set_fom_paper(pxd_ctx* ctx) {
  if (!ctx) return pxd::set_thread_error(PXD_EINVAL, "ctx is NULL");
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
  std::vector<pxd_fom_term> t;
  for (const Row& r : rows)
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
  const int C = n_cand, nf = offsets[n_cand];
  hipStream_t s = ctx->stream;
  HIPCHK(ctx, ctx->base.ensure(ctx->n_cells));
  HIPCHK(ctx, ctx->off.ensure(sizeof(int) * (C + 1)));
  HIPCHK(ctx, ctx->cells.ensure(sizeof(int) * std::max(1, nf)));
  HIPCHK(ctx, ctx->S.ensure(sizeof(double2) * std::max<size_t>(1, (size_t)C * ctx->F * ctx->P * ctx->P)));
  HIPCHK(ctx, ctx->fom.ensure(sizeof(double) * std::max(1, C)));
  HIPCHK(ctx, ctx->cand_status.ensure(sizeof(int) * std::max(1, C)));
  HIPCHK(ctx, ctx->argmin.ensure(sizeof(int)));
  HIPCHK(ctx, hipMemcpyAsync(ctx->base.p, base_map, ctx->n_cells, hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipMemcpyAsync(ctx->off.p, offsets, sizeof(int) * (C + 1), hipMemcpyHostToDevice, s));
  if (nf > 0) HIPCHK(ctx, hipMemcpyAsync(ctx->cells.p, cells, sizeof(int) * nf, hipMemcpyHostToDevice, s));
  rc = evaluate(ctx, s, ctx->base.as<uint8_t>(), C, ctx->off.as<int>(), ctx->cells.as<int>(), ctx->S.as<double2>(),
                ctx->fom.as<double>(), ctx->cand_status.as<int>(), ctx->argmin.as<int>());
  if (rc) return rc;
  const size_t nS = (size_t)C * ctx->F * ctx->P * ctx->P;
  if (S_out && C) HIPCHK(ctx, hipMemcpyAsync(S_out, ctx->S.p, sizeof(double2) * nS, hipMemcpyDeviceToHost, s));
  if (fom_out && C) HIPCHK(ctx, hipMemcpyAsync(fom_out, ctx->fom.p, sizeof(double) * C, hipMemcpyDeviceToHost, s));
  if (status && C) HIPCHK(ctx, hipMemcpyAsync(status, ctx->cand_status.p, sizeof(int) * C, hipMemcpyDeviceToHost, s));
  if (argmin_out && C) HIPCHK(ctx, hipMemcpyAsync(argmin_out, ctx->argmin.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  return PXD_OK;
}

int pxd_evaluate_flips_device(pxd_ctx* ctx, void* stream, const uint8_t* base_map, int32_t n_cand,
                              const int32_t* offsets, const int32_t* cells, int32_t n_flips, double* S_out,
                              double* fom_out, int32_t* status, int32_t* argmin_out) {
  if (!ctx) return pxd::set_thread_error(PXD_EINVAL, "ctx is NULL");
  if (!base_map || !offsets || n_cand < 0 || n_flips < 0 || (n_flips > 0 && !cells) || !S_out || !fom_out)
    return ctx->fail(PXD_EINVAL, "invalid device arguments");
  HIPCHK(ctx, hipSetDevice(ctx->opt.device));
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : ctx->stream;
  return evaluate(ctx, s, base_map, n_cand, offsets, cells, reinterpret_cast<double2*>(S_out), fom_out, status,
                  argmin_out);
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
  HIPCHK(ctx, ctx->Nc.ensure(sizeof(int) * C));
  HIPCHK(ctx, ctx->Ilist.ensure(sizeof(int) * (size_t)C * ctx->M));
  HIPCHK(ctx, hipMemcpyAsync(ctx->base.p, base_map, ctx->n_cells, hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipMemcpyAsync(ctx->off.p, offsets, sizeof(int) * (C + 1), hipMemcpyHostToDevice, s));
  if (nf > 0) HIPCHK(ctx, hipMemcpyAsync(ctx->cells.p, cells, sizeof(int) * nf, hipMemcpyHostToDevice, s));
  HIPCHK(ctx, pxd::launch_expand(s, ctx->base.as<uint8_t>(), ctx->n_cells, ctx->off.as<int>(), ctx->cells.as<int>(), C,
                                 ctx->cell_a.as<int>(), ctx->cell_b.as<int>(), ctx->M, ctx->Nc.as<int>(),
                                 ctx->Ilist.as<int>()));
  HIPCHK(ctx, hipMemcpyAsync(N_out, ctx->Nc.p, sizeof(int) * C, hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipMemcpyAsync(idx_out, ctx->Ilist.p, sizeof(int) * (size_t)C * ctx->M, hipMemcpyDeviceToHost, s));
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

int pxd_get_stats(const pxd_ctx* ctx, pxd_stats* out) {
  if (!ctx || !out) return pxd::set_thread_error(PXD_EINVAL, "null argument");
  *out = ctx->stats;
  // stage times of the last call: wait for its final event, then read the events
  if (ctx->stats.items > 0 && hipEventSynchronize(ctx->ev[4]) == hipSuccess) {
    float a = 0, b = 0, c = 0;
    if (hipEventElapsedTime(&a, ctx->ev[0], ctx->ev[1]) == hipSuccess) out->ms_expand = a;
    if (hipEventElapsedTime(&b, ctx->ev[1], ctx->ev[2]) == hipSuccess) out->ms_solve = b;
    if (hipEventElapsedTime(&c, ctx->ev[3], ctx->ev[4]) == hipSuccess) out->ms_fom = c;
    float d = 0;
    if (ctx->stats_pending_counts && hipEventElapsedTime(&d, ctx->ev[2], ctx->ev[3]) == hipSuccess) {
      out->ms_fallback = d;
      int h[4] = {0, 0, 0, 0};
      if (hipMemcpy(h, ctx->counter.p, sizeof(h), hipMemcpyDeviceToHost) == hipSuccess) {
        out->fallbacks = h[1];
        out->ir_iterations = h[2];
      }
    }
  }
  return PXD_OK;
}

}  // extern "C"
