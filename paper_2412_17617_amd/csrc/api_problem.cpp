// C ABI for the structure builder and the parent fill (host and device).
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>

#include "problem.hpp"
#include "pxd.h"
#include "status.hpp"

extern "C" {

int pxd_problem_create(const pxd_geometry* g, pxd_problem** out) {
  if (!out) return pxd::set_thread_error(PXD_EINVAL, "out is NULL");
  *out = nullptr;
  auto* h = new (std::nothrow) pxd_problem();
  if (!h) return pxd::set_thread_error(PXD_ENOMEM, "out of host memory");
  std::string err;
  int rc;
  try {
    rc = pxd::build_problem(g, &h->p, &err);
  } catch (const std::bad_alloc&) {
    rc = PXD_ENOMEM, err = "out of host memory";
  }
  if (rc != PXD_OK) {
    delete h;
    return pxd::set_thread_error(rc, err);
  }
  *out = h;
  return PXD_OK;
}

void pxd_problem_destroy(pxd_problem* p) { delete p; }

int pxd_problem_sizes(const pxd_problem* p, int32_t* M, int32_t* n_cells, int32_t* n_ports) {
  if (!p) return pxd::set_thread_error(PXD_EINVAL, "problem is NULL");
  if (M) *M = (int32_t)p->p.rwg.size();
  if (n_cells) *n_cells = p->p.n_cells;
  if (n_ports) *n_ports = p->p.g.n_ports;
  return PXD_OK;
}

int pxd_problem_classification(const pxd_problem* p, uint8_t* kind, int32_t* cell_a, int32_t* cell_b,
                               int32_t* port_bf, double* port_len) {
  if (!p) return pxd::set_thread_error(PXD_EINVAL, "problem is NULL");
  const auto& R = p->p.rwg;
  for (size_t i = 0; i < R.size(); ++i) {
    if (kind) kind[i] = (uint8_t)R[i].kind;
    if (cell_a) cell_a[i] = R[i].cell_a;
    if (cell_b) cell_b[i] = R[i].cell_b;
  }
  for (int k = 0; k < p->p.g.n_ports; ++k) {
    int m = p->p.port_bf[k];
    if (port_bf) port_bf[k] = m;
    if (port_len) {
      auto a = p->p.xyz(R[m].e0), b = p->p.xyz(R[m].e1);
      double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
      port_len[k] = __builtin_sqrt(dx * dx + dy * dy + dz * dz);
    }
  }
  return PXD_OK;
}

int pxd_problem_fill(const pxd_problem* p, int32_t F, const double* freqs_hz, double* Z_out, int32_t n_threads) {
  if (!p) return pxd::set_thread_error(PXD_EINVAL, "problem is NULL");
  std::string err;
  int rc;
  try {
    rc = pxd::fill_problem(p->p, F, freqs_hz, Z_out, n_threads, &err);
  } catch (const std::bad_alloc&) {
    rc = PXD_ENOMEM, err = "out of host memory";
  }
  if (rc != PXD_OK) return pxd::set_thread_error(rc, err);
  return PXD_OK;
}

int pxd_problem_fill_device(const pxd_problem* p, int32_t device, void* stream, int32_t F, const double* freqs_hz,
                            double* Z_out) {
  if (!p) return pxd::set_thread_error(PXD_EINVAL, "problem is NULL");
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return pxd::set_thread_error(PXD_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
  std::string err;
  int rc;
  try {
    rc = pxd::fill_problem_device(p->p, F, freqs_hz, Z_out, stream, &err);
  } catch (const std::bad_alloc&) {
    rc = PXD_ENOMEM, err = "out of host memory";
  }
  if (rc != PXD_OK) return pxd::set_thread_error(rc, err);
  return PXD_OK;
}

}  // extern "C"
