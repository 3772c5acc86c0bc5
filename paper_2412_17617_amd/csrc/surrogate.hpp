// Internal interface between the surrogate module and the evaluator context.
#pragma once

#include <hip/hip_runtime.h>

#include "pxd.h"

namespace pxd {

// FoM table of a context (device pointers), for ranking by predicted S.
struct FomTable {
  const pxd_fom_term* terms;
  const double* term_fac;
  const int8_t* band;
  int n_terms, F, P;
};
int fom_table(const pxd_ctx* ctx, FomTable* out);

}  // namespace pxd
